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

// SIFT-Rank. Each lane owns one (dx, dy) column of the (2R+1)^3 window and
// walks dz, accumulating |g| per (z half, orientation octant); the centre
// plane dz = 0 adds half to each z half. The 64 bins are then summed over
// columns with the column's x/y half weights (1, or 1/2 on the centre
// planes), and ranked.
__global__ void __launch_bounds__(kDescThreads) siftrank_kernel(const DescribeArgs a)
{
    __shared__ double part[kDescThreads][17];
    __shared__ double hist[64];
    const int count = min(*a.d_count, a.cap);
    const int tid = threadIdx.x;
    for (int k = blockIdx.x; k < count; k += gridDim.x) {
        const sift3d_keypoint kp = a.kp[k];
        if (kp.octave < 0 || kp.octave >= a.n_oct || kp.scale < 1 || kp.scale > a.S) {
            if (tid < 64) a.siftrank[(size_t)k * 64 + tid] = 0;  // not a keypoint of this plan
            continue;
        }
        const DescOctave &oc = a.oc[kp.octave];
        const float *G = oc.G + oc.lstride * kp.scale;
        const int nx = oc.nx, ny = oc.ny, nz = oc.nz;
        const int R = a.sift_R[kp.scale];
        const int W = 2 * R + 1;
        double acc[16];
#pragma unroll
        for (int b = 0; b < 16; ++b) acc[b] = 0.0;
        if (tid < W * W) {
            const int dx = tid % W - R, dy = tid / W - R;
            const int qx = clampi(kp.x + dx, 0, nx - 1), qy = clampi(kp.y + dy, 0, ny - 1);
            const int xm = clampi(qx - 1, 0, nx - 1), xp = clampi(qx + 1, 0, nx - 1);
            const int ym = clampi(qy - 1, 0, ny - 1), yp = clampi(qy + 1, 0, ny - 1);
            for (int dz = -R; dz <= R; ++dz) {
                const int qz = clampi(kp.z + dz, 0, nz - 1);
                const int zm = clampi(qz - 1, 0, nz - 1), zp = clampi(qz + 1, 0, nz - 1);
                const size_t rc = ((size_t)qz * ny + qy) * nx;
                const double gx = 0.5 * ((double)G[rc + xp] - (double)G[rc + xm]);
                const double gy = 0.5 * ((double)G[((size_t)qz * ny + yp) * nx + qx] -
                                         (double)G[((size_t)qz * ny + ym) * nx + qx]);
                const double gz = 0.5 * ((double)G[((size_t)zp * ny + qy) * nx + qx] -
                                         (double)G[((size_t)zm * ny + qy) * nx + qx]);
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
            for (int e = 0; e < 64; ++e) {
                const double o = hist[e];
                r += (o < h) || (o == h && e < tid);
            }
            a.siftrank[(size_t)k * 64 + tid] = (uint8_t)r;
        }
        __syncthreads();
    }
}

// BRIEF / RRIEF. For each of the 2n sample points p = clamp(v + offset),
// B(p) = sum over the (2rb+1)^3 stencil of wb_a wb_b wb_c G[clamp(p + (a,b,c))]
// is evaluated by one wavefront: lane (a, b) sums its z column, the wave
// then reduces with a fixed xor-butterfly and lane 0's total is kept.
__global__ void __launch_bounds__(kDescThreads) brief_kernel(const DescribeArgs a)
{
    __shared__ double Bv[2 * kMaxPairs];
    __shared__ double dd[kMaxPairs];
    const int count = min(*a.d_count, a.cap);
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int n = a.brief_n, rb = a.brief_rb, W = 2 * rb + 1, W2 = W * W;
    const int nw = n / 64;
    for (int k = blockIdx.x; k < count; k += gridDim.x) {
        const sift3d_keypoint kp = a.kp[k];
        if (kp.octave < 0 || kp.octave >= a.n_oct || kp.scale < 1 || kp.scale > a.S) {
            if (wave < nw && a.brief != nullptr && lane == 0) a.brief[(size_t)k * nw + wave] = 0;
            if (tid < n && a.rrief != nullptr) a.rrief[(size_t)k * n + tid] = 0;
            continue;
        }
        const DescOctave &oc = a.oc[kp.octave];
        const float *G = oc.G + oc.lstride * kp.scale;
        const int nx = oc.nx, ny = oc.ny, nz = oc.nz;
        const int32_t *off = a.pairs + (size_t)(kp.scale - 1) * n * 6;
        for (int q = wave; q < 2 * n; q += kDescThreads / 64) {
            const int px = clampi(kp.x + off[3 * q + 0], 0, nx - 1);
            const int py = clampi(kp.y + off[3 * q + 1], 0, ny - 1);
            const int pz = clampi(kp.z + off[3 * q + 2], 0, nz - 1);
            double part = 0.0;
            for (int ab = lane; ab < W2; ab += 64) {
                const int ai = ab % W, bi = ab / W;
                const int xx = clampi(px + ai - rb, 0, nx - 1), yy = clampi(py + bi - rb, 0, ny - 1);
                const float *col = G + (size_t)yy * nx + xx;
                double acc = 0.0;
                for (int c = 0; c < W; ++c) {
                    const int zz = clampi(pz + c - rb, 0, nz - 1);
                    acc += a.wb[c] * (double)col[(size_t)zz * nx * ny];
                }
                part += (a.wb[ai] * a.wb[bi]) * acc;
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o);
            if (lane == 0) Bv[q] = part;
        }
        __syncthreads();
        if (tid < n) dd[tid] = Bv[2 * tid] - Bv[2 * tid + 1];
        __syncthreads();
        if (wave < nw) {
            const double d = dd[tid];
            const unsigned long long m = __ballot(d > 0.0);
            if (a.brief != nullptr && lane == 0) a.brief[(size_t)k * nw + wave] = m;
            if (a.rrief != nullptr) {
                int r = 0;
                for (int j = 0; j < n; ++j) {
                    const double o = dd[j];
                    r += (o < d) || (o == d && j < tid);
                }
                a.rrief[(size_t)k * n + tid] = (uint8_t)r;
            }
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_describe(const DescribeArgs &a, int grid, hipStream_t st)
{
    if (grid <= 0) return hipSuccess;
    if (a.siftrank != nullptr) {
        hipLaunchKernelGGL(siftrank_kernel, dim3(grid), dim3(kDescThreads), 0, st, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if ((a.brief != nullptr || a.rrief != nullptr) && a.brief_n > 0) {
        hipLaunchKernelGGL(brief_kernel, dim3(grid), dim3(kDescThreads), 0, st, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace s3d
