// Keypoint descriptors on gfx950: upright 3D SIFT-Rank (Section 2: 2x2x2
// spatial x 8 orientation bins, normalised by ranking) and the BRIEF /
// RRIEF descriptors (Section 3.2.3). One workgroup (4 wavefronts) per
// keypoint; workgroups loop over the keypoint list, whose length is read
// from device memory, so the launch never waits on the host.
//
// Floating-point sums are accumulated in double precision in a fixed order
// (no atomics), so results are bit-reproducible run to run.
#include "sift3d_internal.h"

namespace s3d {
namespace {

constexpr int kDescThreads = 256;

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// One (dx, dy) column of the SIFT-Rank window: all loads of the column are
// issued first (4 per sample for the x/y differences, the column itself for
// z), then |g| is accumulated per (z half, orientation octant) in double.
template <int R>
__device__ __forceinline__ void sift_column(const float *G, int nx, int ny, int nz, int cx, int cy, int cz,
                                            double (&acc)[16])
{
    constexpr int W = 2 * R + 1;
    const int qx = clampi(cx, 0, nx - 1), qy = clampi(cy, 0, ny - 1);
    const int xm = clampi(qx - 1, 0, nx - 1), xp = clampi(qx + 1, 0, nx - 1);
    const int ym = clampi(qy - 1, 0, ny - 1), yp = clampi(qy + 1, 0, ny - 1);
    const size_t nxy = (size_t)nx * ny;
    float fxp[W], fxm[W], fyp[W], fym[W], fzp[W], fzm[W];
#pragma unroll
    for (int i = 0; i < W; ++i) {
        const int qz = clampi(cz + i - R, 0, nz - 1);
        const int zm = clampi(qz - 1, 0, nz - 1), zp = clampi(qz + 1, 0, nz - 1);
        const size_t rc = (size_t)qz * nxy + (size_t)qy * nx;
        fxp[i] = G[rc + xp];
        fxm[i] = G[rc + xm];
        fyp[i] = G[(size_t)qz * nxy + (size_t)yp * nx + qx];
        fym[i] = G[(size_t)qz * nxy + (size_t)ym * nx + qx];
        fzp[i] = G[(size_t)zp * nxy + (size_t)qy * nx + qx];
        fzm[i] = G[(size_t)zm * nxy + (size_t)qy * nx + qx];
    }
#pragma unroll
    for (int i = 0; i < W; ++i) {
        const int dz = i - R;
        const double gx = 0.5 * ((double)fxp[i] - (double)fxm[i]);
        const double gy = 0.5 * ((double)fyp[i] - (double)fym[i]);
        const double gz = 0.5 * ((double)fzp[i] - (double)fzm[i]);
        const double m = sqrt(gx * gx + gy * gy + gz * gz);
        const int bo = (gx > 0.0) + 2 * (gy > 0.0) + 4 * (gz > 0.0);
        const double w0 = dz < 0 ? m : (dz == 0 ? 0.5 * m : 0.0);
        const double w1 = dz > 0 ? m : (dz == 0 ? 0.5 * m : 0.0);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            acc[b] += bo == b ? w0 : 0.0;
            acc[8 + b] += bo == b ? w1 : 0.0;
        }
    }
}

// SIFT-Rank. Each lane owns one (dx, dy) column of the (2R+1)^3 window and
// walks dz, accumulating |g| per (z half, orientation octant); the centre
// plane dz = 0 adds half to each z half. The 64 bins are then summed over
// columns with the column's x/y half weights (1, or 1/2 on the centre
// planes), and ranked.
template <bool INL>
__global__ void __launch_bounds__(kDescThreads) siftrank_kernel(const DescLaunch a)
{
    __shared__ double part[kDescThreads][17];
    __shared__ double hist[64];
    const int tid = threadIdx.x;
    for (int v = 0; v < a.n_vol; ++v) {
    const int count = min(a.counts[v], a.cap);
    const DVol vol = a.vols[v];
    for (int kk = blockIdx.x; kk < count; kk += gridDim.x) {
        const size_t k = (size_t)v * a.cap + kk;
        const sift3d_keypoint kp = a.kp[k];
        if (kp.octave < 0 || kp.octave >= vol.n_units || kp.scale < 1 || kp.scale > a.S) {
            if (tid < 64) a.siftrank[k * 64 + tid] = 0;  // not a keypoint of this plan
            continue;
        }
        const DUnit &oc = (INL ? a.inl[vol.unit0 + kp.octave] : a.units[vol.unit0 + kp.octave]);
        const float *G = reinterpret_cast<const float *>(a.ws + oc.g0) + oc.lstride * kp.scale;
        const int nx = oc.nx, ny = oc.ny, nz = oc.nz;
        const int R = a.sift_R[kp.scale];
        const int W = 2 * R + 1;
        double acc[16];
#pragma unroll
        for (int b = 0; b < 16; ++b) acc[b] = 0.0;
        if (tid < W * W) {
            const int dx = tid % W - R, dy = tid / W - R;
            switch (R) {
            case 1: sift_column<1>(G, nx, ny, nz, kp.x + dx, kp.y + dy, kp.z, acc); break;
            case 2: sift_column<2>(G, nx, ny, nz, kp.x + dx, kp.y + dy, kp.z, acc); break;
            case 3: sift_column<3>(G, nx, ny, nz, kp.x + dx, kp.y + dy, kp.z, acc); break;
            case 4: sift_column<4>(G, nx, ny, nz, kp.x + dx, kp.y + dy, kp.z, acc); break;
            case 5: sift_column<5>(G, nx, ny, nz, kp.x + dx, kp.y + dy, kp.z, acc); break;
            case 6: sift_column<6>(G, nx, ny, nz, kp.x + dx, kp.y + dy, kp.z, acc); break;
            default: sift_column<7>(G, nx, ny, nz, kp.x + dx, kp.y + dy, kp.z, acc); break;
            }
        }
#pragma unroll
        for (int b = 0; b < 16; ++b) part[tid][b] = acc[b];
        __syncthreads();
        if (tid < 64) {
            const int bs = tid >> 3, bo = tid & 7;
            const int bx = bs & 1, by = (bs >> 1) & 1, bz = bs >> 2;
            double h = 0.0;
            for (int c = 0; c < W * W; ++c) {
                const int dx = c % W - R, dy = c / W - R;
                const double wx = dx == 0 ? 0.5 : ((dx > 0) == (bx == 1) ? 1.0 : 0.0);
                const double wy = dy == 0 ? 0.5 : ((dy > 0) == (by == 1) ? 1.0 : 0.0);
                h += (wx * wy) * part[c][8 * bz + bo];
            }
            hist[tid] = h;
        }
        __syncthreads();
        if (tid < 64) {
            const double h = hist[tid];
            int r = 0;
#pragma unroll 8
            for (int e = 0; e < 64; ++e) {
                const double o = hist[e];
                r += (int)(o < h) | ((int)(o == h) & (int)(e < tid));
            }
            a.siftrank[k * 64 + tid] = (uint8_t)r;
        }
        __syncthreads();
    }
    }
}

// BRIEF / RRIEF. B_s is G_s already blurred by the sigma_b pre-blur (a
// whole-level separable pass with the same clamp-to-edge rule, so B_s at a
// voxel equals the pre-blur stencil evaluated there). One wavefront per
// keypoint: lane l owns pairs l, l+64, ...; d_i = B_s(p1) - B_s(p2) is the
// exact double difference of the two samples; bit words come from ballots
// and each rank from a comparison against all n differences in LDS.
template <bool INL>
__global__ void __launch_bounds__(kDescThreads) brief_kernel(const DescLaunch a)
{
    constexpr int WAVES = kDescThreads / 64;
    __shared__ double dd[WAVES][kMaxPairs];
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int n = a.brief_n, nw = n / 64;
    for (int v = 0; v < a.n_vol; ++v) {
    const int count = min(a.counts[v], a.cap);
    const DVol vol = a.vols[v];
    for (int k0 = blockIdx.x * WAVES; k0 < count; k0 += gridDim.x * WAVES) {
        const int kk = k0 + wave;
        const bool live = kk < count;
        const size_t k = (size_t)v * a.cap + kk;
        sift3d_keypoint kp{};
        if (live) kp = a.kp[k];
        const bool valid = live && kp.octave >= 0 && kp.octave < vol.n_units && kp.scale >= 1 && kp.scale <= a.S;
        double d[kMaxPairs / 64] = {0.0, 0.0, 0.0, 0.0};
        if (valid) {
            const DUnit &oc = (INL ? a.inl[vol.unit0 + kp.octave] : a.units[vol.unit0 + kp.octave]);
            const float *B = reinterpret_cast<const float *>(a.ws + oc.b1) + oc.lstride * (kp.scale - 1);
            const int nx = oc.nx, ny = oc.ny, nz = oc.nz;
            const int32_t *off = a.pairs + (size_t)(kp.scale - 1) * n * 6;
            for (int q = 0; q < nw; ++q) {
                const int32_t *o = off + (size_t)(lane + 64 * q) * 6;
                const int x1 = clampi(kp.x + o[0], 0, nx - 1), y1 = clampi(kp.y + o[1], 0, ny - 1);
                const int z1 = clampi(kp.z + o[2], 0, nz - 1);
                const int x2 = clampi(kp.x + o[3], 0, nx - 1), y2 = clampi(kp.y + o[4], 0, ny - 1);
                const int z2 = clampi(kp.z + o[5], 0, nz - 1);
                const float b1 = B[((size_t)z1 * ny + y1) * nx + x1];
                const float b2 = B[((size_t)z2 * ny + y2) * nx + x2];
                d[q] = (double)b1 - (double)b2;
                dd[wave][lane + 64 * q] = d[q];
            }
        }
        __syncthreads();
        if (live) {
            int r[kMaxPairs / 64] = {0, 0, 0, 0};
            if (valid && a.rrief != nullptr) {
                // rank of d_i among the n: #{j : d_j < d_i or (d_j == d_i and j < i)}
                for (int j0 = 0; j0 < n; j0 += 8) {
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int jj = j0 + u;
                        const double o = dd[wave][jj];
#pragma unroll
                        for (int q = 0; q < kMaxPairs / 64; ++q)  // branch-free; q >= nw is unused
                            r[q] += (int)(o < d[q]) | ((int)(o == d[q]) & (int)(jj < lane + 64 * q));
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < kMaxPairs / 64; ++q) {
                if (q >= nw) break;
                const unsigned long long m = __ballot(valid && d[q] > 0.0);
                if (a.brief != nullptr && lane == 0) a.brief[k * nw + q] = m;
                if (a.rrief != nullptr) a.rrief[k * n + lane + 64 * q] = (uint8_t)r[q];
            }
        }
        __syncthreads();
    }
    }
}

}  // namespace

hipError_t launch_describe(const DescLaunch &a, int grid, hipStream_t st)
{
    if (grid <= 0) return hipSuccess;
    if (a.siftrank != nullptr) {
        if (a.n_units <= kInlineUnits)
            hipLaunchKernelGGL(siftrank_kernel<true>, dim3(grid), dim3(kDescThreads), 0, st, a);
        else
            hipLaunchKernelGGL(siftrank_kernel<false>, dim3(grid), dim3(kDescThreads), 0, st, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if ((a.brief != nullptr || a.rrief != nullptr) && a.brief_n > 0) {
        const int g = (grid + kDescThreads / 64 - 1) / (kDescThreads / 64);
        if (a.n_units <= kInlineUnits)
            hipLaunchKernelGGL(brief_kernel<true>, dim3(g), dim3(kDescThreads), 0, st, a);
        else
            hipLaunchKernelGGL(brief_kernel<false>, dim3(g), dim3(kDescThreads), 0, st, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace s3d
