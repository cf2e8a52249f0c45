// One-launch Gaussian level for small octaves (Section 3.2.2, Gaussian
// Convolution / Difference-of-Gaussian / Sub-sampling): each workgroup
// computes a 32 x 8 x 4 output tile of G_i = g_sigma * G_{i-1} from the
// tile's whole (32+2R) x (8+2R) x (4+2R) source footprint, with no serial
// chain inside the block and no intermediate level in memory:
//   z pass: one thread per footprint column loads its 4+2R samples (clamped
//           to the volume) and writes 4 z-blurred values to LDS;
//   y pass: one thread per (plane, footprint x) slides down the column and
//           writes 8 y-blurred values to LDS;
//   x pass: one thread per (plane, row, 4 consecutive x) reads its row as
//           float4 and writes 4 outputs, with D_{i-1} = G_{i-1} - G_i (the
//           centre values come from the z pass's samples) and, on levels
//           that feed the next octave, the 2x2x2 mean of G_i (pairs in x
//           inside a thread, in z and y across lanes).
// The footprint is re-read by neighbouring tiles (through the cache), so
// the pass suits octaves that sit in the last-level cache, where the
// streaming pass spends its time on its serial plane chain and the xy + z
// pair on its second launch.
//
// Every tap is a symmetric stencil evaluated in a fixed order, so results
// do not depend on the tile a voxel falls in or on the other jobs of the
// launch.
#include "sift3d_internal.h"

namespace s3d {
namespace {

constexpr int TX = kCTX, TY = kCTY, TZ = kCTZ, NT = kCompactThreads;

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

template <int R, typename F>
__device__ __forceinline__ float sym_stencil(const float (&w)[2 * R + 1], F at)
{
    if constexpr (R == 0) {
        return w[0] * at(0);
    } else {
        float s = w[0] * (at(0) + at(2 * R));
#pragma unroll
        for (int k = 1; k < R; ++k) s = __builtin_fmaf(w[k], at(k) + at(2 * R - k), s);
        return __builtin_fmaf(w[R], at(R), s);
    }
}

template <typename J>
__device__ __forceinline__ int find_job(const J *jobs, int n, int bid)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].block0 <= bid)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Footprint geometry of radius R: FX x FY columns of WN samples; LDS rows
// of PX floats (a multiple of 4, for the x pass's float4 reads).
template <int R>
struct CGeom {
    static constexpr int FX = TX + 2 * R, FY = TY + 2 * R, NC = FX * FY, WN = TZ + 2 * R;
    static constexpr int PX = (FX + 3) & ~3;
    static constexpr int XIN = 4 + ((2 * R + 3) & ~3);   // floats the x pass reads per row segment
};
constexpr int kZbFloats = TZ * CGeom<kCompactMaxR>::FY * CGeom<kCompactMaxR>::PX;
constexpr int kYbFloats = TZ * TY * CGeom<kCompactMaxR>::PX;
constexpr int kCFloats = TZ * TY * TX;

struct CompactSmem {
    float zb[kZbFloats];   // [TZ][FY][PX] z-blurred footprint
    float yb[kYbFloats];   // [TZ][TY][PX] z- then y-blurred
    float c[kCFloats];     // [TZ][TY][TX] centre values G_{i-1} (DoG jobs)
};

template <int R>
__device__ __forceinline__ void compact_body(const float *__restrict__ wt, const float *__restrict__ src,
                                             float *__restrict__ dst, float *__restrict__ dog,
                                             float *__restrict__ sub, const DCJob &jb, int local, CompactSmem &sm)
{
    using Gm = CGeom<R>;
    constexpr int M = 2 * R + 1, FX = Gm::FX, FY = Gm::FY, NC = Gm::NC, WN = Gm::WN, PX = Gm::PX;
    const int tid = threadIdx.x;
    const int nx = jb.nx, ny = jb.ny, nz = jb.nz;
    const size_t nxy = (size_t)nx * ny;
    const int txy = jb.tiles_x * jb.tiles_y;
    const int tz = local / txy, t2 = local - tz * txy;
    const int ty = t2 / jb.tiles_x, tx = t2 - ty * jb.tiles_x;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;

    float w[M];
#pragma unroll
    for (int t = 0; t < M; ++t) w[t] = wt[t];

    // z pass over the footprint columns
    int zoff[WN];
#pragma unroll
    for (int q = 0; q < WN; ++q) zoff[q] = clampi(z0 - R + q, 0, nz - 1);
#pragma unroll 2
    for (int c = tid; c < NC; c += NT) {
        const int cy = c / FX, cx = c - cy * FX;
        const int gx = clampi(x0 - R + cx, 0, nx - 1), gy = clampi(y0 - R + cy, 0, ny - 1);
        const float *col = src + (size_t)gy * nx + gx;
        float v[WN];
#pragma unroll
        for (int q = 0; q < WN; ++q) v[q] = col[(size_t)zoff[q] * nxy];
#pragma unroll
        for (int k = 0; k < TZ; ++k)
            sm.zb[(k * FY + cy) * PX + cx] = sym_stencil<R>(w, [&](int t) { return v[k + t]; });
        if (dog != nullptr && cx >= R && cx < R + TX && cy >= R && cy < R + TY) {
#pragma unroll
            for (int k = 0; k < TZ; ++k) sm.c[(k * TY + cy - R) * TX + cx - R] = v[k + R];
        }
    }
    __syncthreads();

    // y pass: one (plane, footprint x) column of FY values -> TY outputs
    for (int item = tid; item < TZ * FX; item += NT) {
        const int k = item / FX, cx = item - k * FX;
        float col[FY];
#pragma unroll
        for (int j = 0; j < FY; ++j) col[j] = sm.zb[(k * FY + j) * PX + cx];
#pragma unroll
        for (int y = 0; y < TY; ++y)
            sm.yb[(k * TY + y) * PX + cx] = sym_stencil<R>(w, [&](int t) { return col[y + t]; });
    }
    __syncthreads();

    // x pass: thread -> (4 consecutive x, plane k, row y); lane ^ 8 is the
    // other plane of a z pair, lane ^ 32 the other row of a y pair
    const int xq = tid & 7, k = (tid >> 3) & 3, y = tid >> 5;
    const int xb = 4 * xq;
    float in[Gm::XIN];
    const float4 *s4 = reinterpret_cast<const float4 *>(&sm.yb[(k * TY + y) * PX + xb]);
#pragma unroll
    for (int q = 0; q < Gm::XIN / 4; ++q) {
        const float4 v = s4[q];
        in[4 * q + 0] = v.x;
        in[4 * q + 1] = v.y;
        in[4 * q + 2] = v.z;
        in[4 * q + 3] = v.w;
    }
    float o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = sym_stencil<R>(w, [&](int t) { return in[j + t]; });

    const int gz = z0 + k, gy = y0 + y;
    if (gz < nz && gy < ny) {
        const size_t row = (size_t)gz * nxy + (size_t)gy * nx;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gx = x0 + xb + j;
            if (gx < nx) {
                dst[row + gx] = o[j];
                if (dog != nullptr) dog[row + gx] = sm.c[(k * TY + y) * TX + xb + j] - o[j];
            }
        }
    }
    if (sub != nullptr) {
#pragma unroll
        for (int j = 0; j < 4; j += 2) {
            float s = o[j] + o[j + 1];
            s += __shfl_xor(s, 8);    // z pair
            s += __shfl_xor(s, 32);   // y pair
            const int X = (x0 + xb + j) >> 1, Y = gy >> 1, Z = gz >> 1;
            if ((k & 1) == 0 && (y & 1) == 0 && X < jb.mx && Y < jb.my && Z < jb.mz)
                sub[((size_t)Z * jb.my + Y) * jb.mx + X] = s * 0.125f;
        }
    }
}

template <bool INL>
__global__ void __launch_bounds__(NT) blur_compact_kernel(const CompactLaunch a)
{
    __shared__ __align__(16) CompactSmem sm;
    const DCJob jb = INL ? a.inl[find_job(a.inl, a.n_jobs, blockIdx.x)]
                         : a.jobs[find_job(a.jobs, a.n_jobs, blockIdx.x)];
    const float *wt = a.taps + (size_t)jb.taps * kMaxTaps;
    const float *src = jb.src_input ? a.in + jb.src : reinterpret_cast<const float *>(a.ws + jb.src);
    float *dst = reinterpret_cast<float *>(a.ws + jb.dst);
    float *dog = jb.dog < 0 ? nullptr : reinterpret_cast<float *>(a.ws + jb.dog);
    float *sub = jb.sub < 0 ? nullptr : reinterpret_cast<float *>(a.ws + jb.sub);
    const int local = blockIdx.x - jb.block0;
    switch (jb.r) {
#define S3D_C(R) \
    case R: compact_body<R>(wt, src, dst, dog, sub, jb, local, sm); break;
        S3D_C(0) S3D_C(1) S3D_C(2) S3D_C(3) S3D_C(4) S3D_C(5) S3D_C(6) S3D_C(7) S3D_C(8) S3D_C(9) S3D_C(10)
#undef S3D_C
    default: break;
    }
}

static_assert(kCompactMaxR == 10, "radius cases above cover 0..10");
static_assert(TX == 32 && TY == 8 && TZ == 4 && NT == 256, "x pass thread map: 8 x-quads, 4 planes, 8 rows");

}  // namespace

hipError_t launch_blur_compact(const CompactLaunch &a, int max_r, hipStream_t st)
{
    if (a.n_blocks <= 0) return hipSuccess;
    if (max_r < 0 || max_r > kCompactMaxR) return hipErrorInvalidValue;
    const dim3 g(a.n_blocks), b(NT);
    if (a.n_jobs <= kInlineJobs)
        hipLaunchKernelGGL(blur_compact_kernel<true>, g, b, 0, st, a);
    else
        hipLaunchKernelGGL(blur_compact_kernel<false>, g, b, 0, st, a);
    return hipGetLastError();
}

}  // namespace s3d
