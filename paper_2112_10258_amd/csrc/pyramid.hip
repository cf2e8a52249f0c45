// Fused scale-space pass for gfx950: one launch computes
//   G_i = G_{i-1} blurred by a separable Gaussian (x, then y, then z),
//   D_{i-1} = G_{i-1} - G_i                     (optional),
//   the 2x2x2 mean of G_i into the next octave's G_0 (optional),
// reading G_{i-1} from HBM once (Section 3.2.2: Gaussian Convolution,
// Difference-of-Gaussian and Sub-sampling, fused here into one pass).
//
// Work decomposition: a workgroup owns a 32 x 16 (x, y) tile and a slab of
// L output planes in z. It streams the input planes of its slab plus R
// halo planes on each side through LDS: each plane's (16+2R) x (32+2R)
// halo tile is staged in LDS (coalesced row loads, clamp-to-edge), blurred
// along x into a second LDS tile, then along y into registers. The z pass
// keeps the last 2R+1 y-blurred values of each output column in a
// per-thread register ring; the ring slot is a compile-time constant in
// each of the 2R+1 unrolled phases, so the ring never leaves registers.
#include "sift3d_internal.h"

namespace s3d {
namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8). Remap so that each XCD receives one contiguous range of logical
// tiles: neighbouring tiles then share their halo rows in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int n)
{
    const int per = n / 8, rem = n % 8;
    const int xcd = bid % 8, idx = bid / 8;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// One symmetric 1D stencil: sum_t w[t] * at(t), t = 0..2R, with w[t] = w[2R-t].
// Taps are paired and summed from the outermost inward, so the partial sum
// stays small until the last (largest) terms: fewer roundings at full
// magnitude than a straight left-to-right chain, same instruction count.
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

template <int R, int NY, bool DOG, int P>
__device__ __forceinline__ void ring_step(float (&ring)[NY][2 * R + 1], float (&cen)[NY][2 * R + 1],
                                          const float (&yv)[NY], const float (&cv)[NY],
                                          const float (&w)[2 * R + 1], float (&zo)[NY], float (&co)[NY])
{
    constexpr int M = 2 * R + 1;
#pragma unroll
    for (int j = 0; j < NY; ++j) {
        ring[j][P] = yv[j];
        if constexpr (DOG) cen[j][P] = cv[j];
    }
    // slot (P + 1 + t) % M holds input plane (current - 2R + t)
#pragma unroll
    for (int j = 0; j < NY; ++j) {
        zo[j] = sym_stencil<R>(w, [&](int t) { return ring[j][(P + 1 + t) % M]; });
        if constexpr (DOG) co[j] = cen[j][(P + 1 + R) % M];  // input plane (current - R)
    }
}

template <int R, int NY, bool DOG, int P = 0>
__device__ __forceinline__ void ring_dispatch(int phase, float (&ring)[NY][2 * R + 1],
                                              float (&cen)[NY][2 * R + 1], const float (&yv)[NY],
                                              const float (&cv)[NY], const float (&w)[2 * R + 1],
                                              float (&zo)[NY], float (&co)[NY])
{
    if constexpr (P < 2 * R + 1) {
        if (phase == P)
            ring_step<R, NY, DOG, P>(ring, cen, yv, cv, w, zo, co);
        else
            ring_dispatch<R, NY, DOG, P + 1>(phase, ring, cen, yv, cv, w, zo, co);
    }
}

template <int R, bool DOG>
__global__ void __launch_bounds__(kBlurThreads) blur_level_kernel(const BlurArgs a)
{
    constexpr int TX = kBlurTX, TY = kBlurTY, NY = kBlurNY, NT = kBlurThreads;
    constexpr int M = 2 * R + 1;
    constexpr int AWL = TX + 2 * R;                 // staged width
    constexpr int AW = (AWL + 3) & ~3;              // LDS row pitch (16-byte rows)
    constexpr int AH = TY + 2 * R;                  // staged height
    constexpr int AE = AH * AWL;
    constexpr int KL = (AE + NT - 1) / NT;          // staged elements per thread
    constexpr int XQ = TX / 4;                      // x-pass items per row (4 outputs each)
    constexpr int XIN = 4 + ((2 * R + 3) & ~3);     // x-pass inputs per item, multiple of 4
    static_assert(NY == 2, "sub-sampling pairs rows inside a thread");
    __shared__ __align__(16) float A[AH * AW];
    __shared__ __align__(16) float B[AH * TX];

    const int tid = threadIdx.x;
    const int logical = xcd_remap(blockIdx.x, a.n_blocks);
    const int ntile = a.tiles_x * a.tiles_y;
    const int slab = logical / ntile;
    const int t2 = logical - slab * ntile;
    const int tyi = t2 / a.tiles_x;
    const int txi = t2 - tyi * a.tiles_x;
    const int x0 = txi * TX, y0 = tyi * TY, z0 = slab * a.L;
    const int z1 = min(z0 + a.L, a.nz);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const size_t nxy = (size_t)nx * ny;

    // Per-thread staging slots: the same in-plane offsets for every plane.
    int goff[KL], loff[KL];
#pragma unroll
    for (int k = 0; k < KL; ++k) {
        const int idx = tid + k * NT;
        if (idx < AE) {
            const int r = idx / AWL, c = idx - r * AWL;
            goff[k] = clampi(y0 - R + r, 0, ny - 1) * nx + clampi(x0 - R + c, 0, nx - 1);
            loff[k] = r * AW + c;
        } else {
            goff[k] = 0;
            loff[k] = -1;
        }
    }
    float pre[KL];
    auto load_plane = [&](int zi) {
        const float *p = a.src + (size_t)clampi(zi, 0, nz - 1) * nxy;
#pragma unroll
        for (int k = 0; k < KL; ++k) pre[k] = p[goff[k]];
    };

    float w[M];
#pragma unroll
    for (int t = 0; t < M; ++t) w[t] = a.w[t];

    const int tx = tid % TX;
    const int tyb = (tid / TX) * NY;
    const int gx = x0 + tx;
    float ring[NY][M], cen[NY][M];
#pragma unroll
    for (int j = 0; j < NY; ++j)
#pragma unroll
        for (int t = 0; t < M; ++t) ring[j][t] = cen[j][t] = 0.f;
    float subacc = 0.f;

    const int nplanes = (z1 - z0) + 2 * R;
    int phase = 0;
    load_plane(z0 - R);
    for (int it = 0; it < nplanes; ++it) {
#pragma unroll
        for (int k = 0; k < KL; ++k)
            if (loff[k] >= 0) A[loff[k]] = pre[k];
        __syncthreads();
        if (it + 1 < nplanes) load_plane(z0 - R + it + 1);

        float cv[NY];
#pragma unroll
        for (int j = 0; j < NY; ++j) cv[j] = DOG ? A[(R + tyb + j) * AW + R + tx] : 0.f;

        // x pass: 4 consecutive outputs per item from one LDS strip
        for (int item = tid; item < AH * XQ; item += NT) {
            const int r = item / XQ, xb = (item - r * XQ) * 4;
            float in[XIN];
            const float4 *s4 = reinterpret_cast<const float4 *>(&A[r * AW + xb]);
#pragma unroll
            for (int q = 0; q < XIN / 4; ++q) {
                const float4 v = s4[q];
                in[4 * q + 0] = v.x;
                in[4 * q + 1] = v.y;
                in[4 * q + 2] = v.z;
                in[4 * q + 3] = v.w;
            }
            float o[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) o[q] = sym_stencil<R>(w, [&](int t) { return in[q + t]; });
            *reinterpret_cast<float4 *>(&B[r * TX + xb]) = make_float4(o[0], o[1], o[2], o[3]);
        }
        __syncthreads();

        // y pass: NY consecutive outputs of column tx
        float yv[NY];
        {
            float col[NY + 2 * R];
#pragma unroll
            for (int q = 0; q < NY + 2 * R; ++q) col[q] = B[(tyb + q) * TX + tx];
#pragma unroll
            for (int j = 0; j < NY; ++j) yv[j] = sym_stencil<R>(w, [&](int t) { return col[j + t]; });
        }

        // z pass from the register ring
        float zo[NY], co[NY];
        ring_dispatch<R, NY, DOG>(phase, ring, cen, yv, cv, w, zo, co);
        phase = (phase + 1 == M) ? 0 : phase + 1;

        if (it >= 2 * R) {
            const int oz = z0 + it - 2 * R;
#pragma unroll
            for (int j = 0; j < NY; ++j) {
                const int gy = y0 + tyb + j;
                if (gx < nx && gy < ny) {
                    const size_t i = (size_t)oz * nxy + (size_t)gy * nx + gx;
                    a.dst[i] = zo[j];
                    if constexpr (DOG) a.dog[i] = co[j] - zo[j];
                }
            }
            if (a.sub != nullptr) {
                const float s2 = zo[0] + zo[1];
                const float s4 = s2 + __shfl_xor(s2, 1);
                if ((oz & 1) == 0) {
                    subacc = s4;
                } else {
                    const int X = gx >> 1, Y = (y0 + tyb) >> 1, Z = oz >> 1;
                    if ((tx & 1) == 0 && X < a.mx && Y < a.my && Z < a.mz)
                        a.sub[((size_t)Z * a.my + Y) * a.mx + X] = (subacc + s4) * 0.125f;
                }
            }
        }
    }
}

template <int R>
hipError_t launch_r(const BlurArgs &a, bool dog, hipStream_t st)
{
    if (dog)
        hipLaunchKernelGGL((blur_level_kernel<R, true>), dim3(a.n_blocks), dim3(kBlurThreads), 0, st, a);
    else
        hipLaunchKernelGGL((blur_level_kernel<R, false>), dim3(a.n_blocks), dim3(kBlurThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_blur(const BlurArgs &a, int r, bool dog, hipStream_t st)
{
    switch (r) {
    case 0: return launch_r<0>(a, dog, st);
    case 1: return launch_r<1>(a, dog, st);
    case 2: return launch_r<2>(a, dog, st);
    case 3: return launch_r<3>(a, dog, st);
    case 4: return launch_r<4>(a, dog, st);
    case 5: return launch_r<5>(a, dog, st);
    case 6: return launch_r<6>(a, dog, st);
    case 7: return launch_r<7>(a, dog, st);
    case 8: return launch_r<8>(a, dog, st);
    case 9: return launch_r<9>(a, dog, st);
    case 10: return launch_r<10>(a, dog, st);
    case 11: return launch_r<11>(a, dog, st);
    case 12: return launch_r<12>(a, dog, st);
    case 13: return launch_r<13>(a, dog, st);
    case 14: return launch_r<14>(a, dog, st);
    case 15: return launch_r<15>(a, dog, st);
    case 16: return launch_r<16>(a, dog, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace s3d
