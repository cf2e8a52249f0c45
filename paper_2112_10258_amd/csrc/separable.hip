// Two-launch separable Gaussian level for volumes that stay resident in the
// last-level cache (Section 3.2.2, Gaussian Convolution / Difference-of-
// Gaussian / Sub-sampling):
//   xy launch: per (64x16 tile, a few consecutive planes), stage each
//              plane's (16+2R) x (64+2R) halo tile in LDS, blur along x into
//              a second LDS tile, then along y, write the xy-blurred plane T;
//   z launch:  per (32x8 columns, 16 output planes), slide a register window
//              of 16+2R samples of T down each column, blur along z, and
//              write G, optionally D = centre - G and the 2x2x2 mean of G.
// Neither launch has a serial plane chain, so every block finishes in a
// few microseconds; the price is the T round trip through the cache.
//
// Both launches take a list of jobs (levels of one or several volumes or
// octaves) that may differ in tap radius: each block reads its job and
// branches once to the body compiled for that radius. Independent levels
// (later levels of octave o, early levels of octave o+1, BRIEF pre-blurs)
// therefore share launches.
#include "sift3d_internal.h"

namespace s3d {
namespace {

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

// Job of a block: the last job whose first block is <= bid (jobs sorted by block0).
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

// Staged elements per thread and the LDS floats of the staging tile (the
// tile plus one dummy slot per unused staging lane, so that every lane
// writes unconditionally).
template <int R>
struct XYGeom {
    static constexpr int AWL = kXYTX + 2 * R;
    static constexpr int AW = (AWL + 3) & ~3;
    static constexpr int AH = kXYTY + 2 * R;
    static constexpr int AE = AH * AWL;
    static constexpr int KL = (AE + kXYThreads - 1) / kXYThreads;
    static constexpr int A_FLOATS = AH * AW + KL * kXYThreads - AE;
    static constexpr int B_FLOATS = AH * kXYTX;
};

// One (64 x 16) tile of `planes` consecutive planes: each plane's halo tile
// is staged in LDS, blurred along x into a second LDS tile, then along y
// into the output. The next plane's staging values are loaded into
// registers while the current plane is blurred.
template <int R>
__device__ __forceinline__ void xy_body(const float *__restrict__ wt, const float *__restrict__ vol,
                                        float *__restrict__ out, const DXYJob &jb, int local, float *smem)
{
    using Gm = XYGeom<R>;
    constexpr int TX = kXYTX, TY = kXYTY, NT = kXYThreads, M = 2 * R + 1;
    constexpr int NYo = TX * TY / NT;               // y outputs per thread
    constexpr int AWL = Gm::AWL, AW = Gm::AW, AH = Gm::AH, AE = Gm::AE, KL = Gm::KL;
    constexpr int XQ = TX / 4;
    constexpr int XIN = 4 + ((2 * R + 3) & ~3);
    float *A = smem;                                // [AH][AW] + dummy slots
    float *B = smem + Gm::A_FLOATS;                 // [AH][TX]

    const int ntile = jb.tiles_x * jb.tiles_y;
    const int zg = local / ntile;
    const int t2 = local - zg * ntile;
    const int tyi = t2 / jb.tiles_x, txi = t2 - tyi * jb.tiles_x;
    const int x0 = txi * TX, y0 = tyi * TY;
    const int nx = jb.nx, ny = jb.ny;
    const int z_first = zg * jb.planes, z_end = min(z_first + jb.planes, jb.nz);
    const size_t nxy = (size_t)nx * ny;
    const int tid = threadIdx.x;

    float w[M];
#pragma unroll
    for (int t = 0; t < M; ++t) w[t] = wt[t];

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
            loff[k] = AH * AW + (idx - AE);
        }
    }
    float pre[KL];
    {
        const float *src = vol + (size_t)z_first * nxy;
#pragma unroll
        for (int k = 0; k < KL; ++k) pre[k] = src[goff[k]];
    }
    const int tx = tid % TX, tyb = (tid / TX) * NYo;
    const int gx = x0 + tx;
    for (int z = z_first; z < z_end; ++z) {
#pragma unroll
        for (int k = 0; k < KL; ++k) A[loff[k]] = pre[k];
        __syncthreads();
        if (z + 1 < z_end) {
            const float *src = vol + (size_t)(z + 1) * nxy;
#pragma unroll
            for (int k = 0; k < KL; ++k) pre[k] = src[goff[k]];
        }
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
        float col[NYo + 2 * R];
#pragma unroll
        for (int q = 0; q < NYo + 2 * R; ++q) col[q] = B[(tyb + q) * TX + tx];
        float *dst = out + (size_t)z * nxy;
#pragma unroll
        for (int k = 0; k < NYo; ++k) {
            const float v = sym_stencil<R>(w, [&](int t) { return col[k + t]; });
            const int gy = y0 + tyb + k;
            if (gx < nx && gy < ny) dst[(size_t)gy * nx + gx] = v;
        }
    }
}

template <int R>
__device__ __forceinline__ void z_body(const float *__restrict__ wt, const float *__restrict__ tin,
                                       const float *__restrict__ center, float *__restrict__ dst,
                                       float *__restrict__ dog, float *__restrict__ sub, const DZJob &jb, int local)
{
    constexpr int ZS = kZPlanes, M = 2 * R + 1, WN = ZS + 2 * R;
    static_assert(ZS % 2 == 0, "sub-sampling pairs planes inside a thread");
    const int gxy = jb.gx * jb.gy;
    const int bz = local / gxy;
    const int t2 = local - bz * gxy;
    const int byi = t2 / jb.gx, bxi = t2 - byi * jb.gx;
    const int tid = threadIdx.x;
    const int tx = tid & 31, ty = tid >> 5;
    const int nx = jb.nx, ny = jb.ny, nz = jb.nz;
    const int x = bxi * 32 + tx, y = byi * 8 + ty, z0 = bz * ZS;
    const int xc = min(x, nx - 1), yc = min(y, ny - 1);
    const size_t nxy = (size_t)nx * ny;
    const size_t col = (size_t)yc * nx + xc;

    float w[M];
#pragma unroll
    for (int t = 0; t < M; ++t) w[t] = wt[t];
    float win[WN];
#pragma unroll
    for (int q = 0; q < WN; ++q) win[q] = tin[(size_t)clampi(z0 - R + q, 0, nz - 1) * nxy + col];
    float g[ZS];
#pragma unroll
    for (int k = 0; k < ZS; ++k) g[k] = sym_stencil<R>(w, [&](int t) { return win[k + t]; });

    const bool in_xy = x < nx && y < ny;
#pragma unroll
    for (int k = 0; k < ZS; ++k) {
        const int z = z0 + k;
        if (in_xy && z < nz) {
            const size_t i = (size_t)z * nxy + col;
            dst[i] = g[k];
            if (dog != nullptr) dog[i] = center[i] - g[k];
        }
    }
    if (sub != nullptr) {
#pragma unroll
        for (int k = 0; k < ZS; k += 2) {
            float s = g[k] + g[k + 1];
            s += __shfl_xor(s, 1);   // x pair: neighbouring lane
            s += __shfl_xor(s, 32);  // y pair: same lane of the other half-wave
            const int X = x >> 1, Y = y >> 1, Z = (z0 + k) >> 1;
            if ((tx & 1) == 0 && (ty & 1) == 0 && X < jb.mx && Y < jb.my && Z < jb.mz)
                sub[((size_t)Z * jb.my + Y) * jb.mx + X] = s * 0.125f;
        }
    }
}

// Radius switch of a kernel instantiated for radii up to RMAX (the host
// launches the RMAX = 10 instantiation when every job's radius allows it:
// its register count, and so its occupancy, is set by the largest body).
#define S3D_RADIUS_CASES(BODY)             \
    case 0: BODY(0); break;                \
    case 1: BODY(1); break;                \
    case 2: BODY(2); break;                \
    case 3: BODY(3); break;                \
    case 4: BODY(4); break;                \
    case 5: BODY(5); break;                \
    case 6: BODY(6); break;                \
    case 7: BODY(7); break;                \
    case 8: BODY(8); break;                \
    case 9: BODY(9); break;                \
    case 10: BODY(10); break;              \
    case 11: if constexpr (RMAX >= 11) BODY(11); break; \
    case 12: if constexpr (RMAX >= 12) BODY(12); break; \
    case 13: if constexpr (RMAX >= 13) BODY(13); break; \
    case 14: if constexpr (RMAX >= 14) BODY(14); break; \
    case 15: if constexpr (RMAX >= 15) BODY(15); break; \
    case 16: if constexpr (RMAX >= 16) BODY(16); break; \
    default: break;

constexpr int kSmallR = 10;

// INL: the jobs are read from the inline copy in the arguments (small
// launches), else from the device table.
template <bool INL, int RMAX>
__global__ void __launch_bounds__(kXYThreads) blur_xy_kernel(const XYLaunch a)
{
    extern __shared__ __align__(16) float smem[];
    const DXYJob jb = INL ? a.inl[find_job(a.inl, a.n_jobs, blockIdx.x)]
                          : a.jobs[find_job(a.jobs, a.n_jobs, blockIdx.x)];
    const float *wt = a.taps + (size_t)jb.taps * kMaxTaps;
    const float *src = jb.src_input ? a.in + jb.src : reinterpret_cast<const float *>(a.ws + jb.src);
    float *dst = reinterpret_cast<float *>(a.ws + jb.dst);
    const int local = blockIdx.x - jb.block0;
#define S3D_XY(R) xy_body<R>(wt, src, dst, jb, local, smem)
    switch (jb.r) { S3D_RADIUS_CASES(S3D_XY) }
#undef S3D_XY
}

template <bool INL, int RMAX>
__global__ void __launch_bounds__(kZThreads) blur_z_kernel(const ZLaunch a)
{
    const DZJob jb = INL ? a.inl[find_job(a.inl, a.n_jobs, blockIdx.x)]
                         : a.jobs[find_job(a.jobs, a.n_jobs, blockIdx.x)];
    const float *wt = a.taps + (size_t)jb.taps * kMaxTaps;
    const float *tin = reinterpret_cast<const float *>(a.ws + jb.t);
    const float *center = jb.center < 0 ? nullptr
                          : jb.center_input ? a.in + jb.center
                                            : reinterpret_cast<const float *>(a.ws + jb.center);
    float *dst = reinterpret_cast<float *>(a.ws + jb.dst);
    float *dog = jb.dog < 0 ? nullptr : reinterpret_cast<float *>(a.ws + jb.dog);
    float *sub = jb.sub < 0 ? nullptr : reinterpret_cast<float *>(a.ws + jb.sub);
    const int local = blockIdx.x - jb.block0;
#define S3D_Z(R) z_body<R>(wt, tin, center, dst, dog, sub, jb, local)
    switch (jb.r) { S3D_RADIUS_CASES(S3D_Z) }
#undef S3D_Z
}

}  // namespace

// LDS bytes of the xy body for radius r.
static size_t xy_lds_bytes(int r)
{
    switch (r) {
#define S3D_LDS(R) \
    case R: return (size_t)(XYGeom<R>::A_FLOATS + XYGeom<R>::B_FLOATS) * sizeof(float);
        S3D_LDS(0) S3D_LDS(1) S3D_LDS(2) S3D_LDS(3) S3D_LDS(4) S3D_LDS(5) S3D_LDS(6) S3D_LDS(7) S3D_LDS(8)
        S3D_LDS(9) S3D_LDS(10) S3D_LDS(11) S3D_LDS(12) S3D_LDS(13) S3D_LDS(14) S3D_LDS(15) S3D_LDS(16)
#undef S3D_LDS
    default: return 0;
    }
}

hipError_t launch_blur_xy(const XYLaunch &a, int max_r, hipStream_t st)
{
    if (a.n_blocks <= 0) return hipSuccess;
    if (max_r < 0 || max_r > kMaxR) return hipErrorInvalidValue;
    const size_t lds = xy_lds_bytes(max_r);
    const bool inl = a.n_jobs <= kInlineJobs, small = max_r <= kSmallR;
    const dim3 g(a.n_blocks), b(kXYThreads);
    if (inl && small)
        hipLaunchKernelGGL((blur_xy_kernel<true, kSmallR>), g, b, lds, st, a);
    else if (inl)
        hipLaunchKernelGGL((blur_xy_kernel<true, kMaxR>), g, b, lds, st, a);
    else if (small)
        hipLaunchKernelGGL((blur_xy_kernel<false, kSmallR>), g, b, lds, st, a);
    else
        hipLaunchKernelGGL((blur_xy_kernel<false, kMaxR>), g, b, lds, st, a);
    return hipGetLastError();
}

hipError_t launch_blur_z(const ZLaunch &a, int max_r, hipStream_t st)
{
    if (a.n_blocks <= 0) return hipSuccess;
    if (max_r < 0 || max_r > kMaxR) return hipErrorInvalidValue;
    const bool inl = a.n_jobs <= kInlineJobs, small = max_r <= kSmallR;
    const dim3 g(a.n_blocks), b(kZThreads);
    if (inl && small)
        hipLaunchKernelGGL((blur_z_kernel<true, kSmallR>), g, b, 0, st, a);
    else if (inl)
        hipLaunchKernelGGL((blur_z_kernel<true, kMaxR>), g, b, 0, st, a);
    else if (small)
        hipLaunchKernelGGL((blur_z_kernel<false, kSmallR>), g, b, 0, st, a);
    else
        hipLaunchKernelGGL((blur_z_kernel<false, kMaxR>), g, b, 0, st, a);
    return hipGetLastError();
}

}  // namespace s3d
