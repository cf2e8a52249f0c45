// Uniform-filter approximation of a Gaussian blur (Related Work: the
// Gaussian scale space can also be generated with separable uniform 1D
// filters). Along x, then y, then z, `passes` clamp-to-edge uniform passes
// of width w = 2h+1 are applied; an output is the FP32 sum of its w inputs
// in index order, times 1/w.
//
// One launch per axis. A workgroup owns 64 lines x 64 outputs along the
// axis. It stages the lines' 64 + 2*passes*h inputs in LDS (indices clamped
// to the volume), runs every pass there in place, and writes the 64 outputs
// of each line. Pass k is evaluated at
// local positions [k h, E - k h) that lie inside the volume; its taps are
// clamped to the volume before they are looked up, so every pass sees the
// volume's edges, never the tile's, and every looked-up position was
// written by pass k-1 (a clamped tap q satisfies (k-1) h <= q - p0 <
// E - (k-1) h, and q lies inside the volume).
// Lines of the x axis are rows, staged and written with consecutive lanes on
// consecutive x. Lines of the y and z axes are 64 consecutive x at one z
// (y axis) or one y (z axis), staged and written one 64-wide row segment per
// position.
#include "sift3d_internal.h"

namespace s3d {
namespace {

constexpr int kBoxT = 64;          // outputs per line per workgroup
constexpr int kBoxLines = 64;      // lines per workgroup
constexpr int kBoxThreads = 256;
constexpr int kBoxMaxReach = 28;   // passes * h
constexpr int kBoxPerLane = (kBoxT + 2 * kBoxMaxReach + 3) / 4;   // positions a lane computes per pass

struct BoxArgs {
    const float *in;
    float *out;
    int nx, ny, nz;
    int h, passes;
    float inv_w;
    int n_tiles;    // 64-position tiles along the axis
    int x_groups;   // 64-wide x groups (y and z axes)
};

// Base offset of line l of workgroup group `grp`, clamped into the volume;
// `valid` tells whether the line exists.
template <int AXIS>
__device__ __forceinline__ size_t line_base(const BoxArgs &a, int grp, int l, bool &valid)
{
    if constexpr (AXIS == 0) {
        const long long rows = (long long)a.ny * a.nz;
        long long r = (long long)grp * kBoxLines + l;
        valid = r < rows;
        r = r < rows ? r : rows - 1;
        return (size_t)r * a.nx;
    } else {
        const int xg = grp % a.x_groups, o = grp / a.x_groups;   // o: z (y axis) or y (z axis)
        int x = xg * kBoxLines + l;
        valid = x < a.nx;
        x = min(x, a.nx - 1);
        return AXIS == 1 ? (size_t)o * a.nx * a.ny + x : (size_t)o * a.nx + x;
    }
}

// H: the half-width, a template parameter so that the taps unroll. The
// staged lines live in one LDS buffer of 64 x (E + 1) floats (an odd pitch
// puts the lines on distinct banks); a pass keeps its outputs in registers
// until every lane has read its taps, then writes them back in place.
template <int AXIS, int H>
__global__ void __launch_bounds__(kBoxThreads) box_axis_kernel(const BoxArgs a)
{
    extern __shared__ float buf[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tile = blockIdx.x % a.n_tiles, grp = blockIdx.x / a.n_tiles;
    const int n = AXIS == 0 ? a.nx : AXIS == 1 ? a.ny : a.nz;
    const size_t stride = AXIS == 0 ? 1 : AXIS == 1 ? (size_t)a.nx : (size_t)a.nx * a.ny;
    const int reach = a.passes * H;
    const int E = kBoxT + 2 * reach;     // staged positions per line
    const int pitch = E + 1;
    const int p0 = tile * kBoxT - reach; // axis position of local index 0

    // stage: x axis, a wavefront per line with lanes on consecutive
    // positions; y and z axes, a lane per line (consecutive x) with the
    // wavefronts on interleaved positions
    if constexpr (AXIS == 0) {
        for (int l = wave; l < kBoxLines; l += 4) {
            bool v;
            const size_t b = line_base<AXIS>(a, grp, l, v);
            for (int i = lane; i < E; i += 64) buf[l * pitch + i] = a.in[b + min(max(p0 + i, 0), n - 1)];
        }
    } else {
        bool v;
        const size_t b = line_base<AXIS>(a, grp, lane, v);
        for (int i = wave; i < E; i += 4)
            buf[lane * pitch + i] = a.in[b + (size_t)min(max(p0 + i, 0), n - 1) * stride];
    }
    __syncthreads();

    // Each wavefront takes a contiguous quarter of the pass's positions on
    // every line and slides a register window of the 2H+1 (clamped) taps
    // along it: one LDS read per output for the incoming tap, the sum still
    // taken over the window in index order.
    float *s = buf + lane * pitch;
    for (int k = 1; k <= a.passes; ++k) {
        const int lo = max(k * H, -p0), hi = min(E - k * H, n - p0);
        const int chunk = (hi - lo + 3) >> 2;
        const int c0 = lo + wave * chunk;
        const int len = min(chunk, hi - c0);   // positions of this wavefront (may be <= 0)
        float o[kBoxPerLane];
        if (len > 0) {
            const int pb = p0 + c0;            // its first axis position
            float win[2 * H + 1];
#pragma unroll
            for (int j = 0; j < 2 * H + 1; ++j) win[j] = s[min(max(pb - H + j, 0), n - 1) - p0];
#pragma unroll
            for (int q = 0; q < kBoxPerLane; ++q) {
                if (q < len) {
                    float acc = 0.f;
#pragma unroll
                    for (int j = 0; j < 2 * H + 1; ++j) acc += win[j];
                    o[q] = acc * a.inv_w;
#pragma unroll
                    for (int j = 0; j < 2 * H; ++j) win[j] = win[j + 1];
                    // the next tap; after the last output this reads at most
                    // local index E, the row's padding slot, and is unused
                    win[2 * H] = s[min(max(pb + q + 1 + H, 0), n - 1) - p0];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kBoxPerLane; ++q)
            if (q < len) s[c0 + q] = o[q];
        __syncthreads();
    }

    if constexpr (AXIS == 0) {
        const int p = tile * kBoxT + lane;
        for (int l = wave; l < kBoxLines; l += 4) {
            bool v;
            const size_t b = line_base<AXIS>(a, grp, l, v);
            if (v && p < n) a.out[b + p] = buf[l * pitch + reach + lane];
        }
    } else {
        bool v;
        const size_t b = line_base<AXIS>(a, grp, lane, v);
        for (int t = wave; t < kBoxT; t += 4) {
            const int p = tile * kBoxT + t;
            if (v && p < n) a.out[b + (size_t)p * stride] = s[reach + t];
        }
    }
}

template <int AXIS>
void launch_axis(const BoxArgs &a, unsigned blocks, hipStream_t st)
{
    const dim3 g(blocks), b(kBoxThreads);
    const size_t lds = (size_t)kBoxLines * (kBoxT + 2 * a.passes * a.h + 1) * sizeof(float);
    switch (a.h) {
#define S3D_BOX(H) \
    case H: hipLaunchKernelGGL((box_axis_kernel<AXIS, H>), g, b, lds, st, a); break;
        S3D_BOX(0) S3D_BOX(1) S3D_BOX(2) S3D_BOX(3) S3D_BOX(4) S3D_BOX(5) S3D_BOX(6) S3D_BOX(7) S3D_BOX(8)
#undef S3D_BOX
    default: break;
    }
}

static_assert(kBoxThreads == 4 * kBoxLines && kBoxLines == 64 && kBoxT == 64,
              "a lane per line or position, four wavefronts");
constexpr int kBoxMaxH = 8;

}  // namespace

// x: in -> out, y: out -> tmp, z: tmp -> out. Sizes are checked by the caller.
hipError_t launch_box(const float *in, float *out, float *tmp, int nx, int ny, int nz, int h, int passes,
                      hipStream_t st)
{
    if (h < 0 || h > kBoxMaxH || passes < 1 || passes * h > kBoxMaxReach) return hipErrorInvalidValue;
    BoxArgs a{};
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.h = h;
    a.passes = passes;
    a.inv_w = 1.0f / (float)(2 * h + 1);
    a.x_groups = (nx + kBoxLines - 1) / kBoxLines;
    const long long rows = (long long)ny * nz;
    const long long blocks[3] = {
        (long long)((nx + kBoxT - 1) / kBoxT) * ((rows + kBoxLines - 1) / kBoxLines),
        (long long)((ny + kBoxT - 1) / kBoxT) * a.x_groups * nz,
        (long long)((nz + kBoxT - 1) / kBoxT) * a.x_groups * ny,
    };
    for (long long b : blocks)
        if (b < 1 || b > 0x7fffffffLL) return hipErrorInvalidValue;
    a.in = in;
    a.out = out;
    a.n_tiles = (nx + kBoxT - 1) / kBoxT;
    launch_axis<0>(a, (unsigned)blocks[0], st);
    a.in = out;
    a.out = tmp;
    a.n_tiles = (ny + kBoxT - 1) / kBoxT;
    launch_axis<1>(a, (unsigned)blocks[1], st);
    a.in = tmp;
    a.out = out;
    a.n_tiles = (nz + kBoxT - 1) / kBoxT;
    launch_axis<2>(a, (unsigned)blocks[2], st);
    return hipGetLastError();
}

}  // namespace s3d
