// The fused scale-space kernel template (see pyramid.hip), instantiated by
// pyramid.hip (16-row tiles) and pyramid_tall.hip (32-row tiles) so that the
// two sets of instances compile in parallel.
#pragma once

#include <type_traits>

#include "sift3d_internal.h"

namespace s3d {
namespace fused {


__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// Plane accesses go through buffer resources: a plane's base and size sit
// in scalar registers and each lane adds a 32-bit byte offset, so loads and
// stores cost no per-lane 64-bit address arithmetic. A store whose offset
// is kDropOffset lies past every plane (planes are at most 1 GiB) and is
// discarded by the hardware range check: out-of-volume lanes store
// unconditionally instead of branching around the store.
constexpr int kRawBufferWord3 = 0x00020000;   // dword 3 of a raw (untyped) buffer resource on gfx9
constexpr unsigned kDropOffset = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float *base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(base), (short)0, (int)bytes, kRawBufferWord3);
}
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t rs, unsigned boff)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (int)boff, 0, 0));
}
// Stores carry the non-temporal cache policy (aux bit 1): a level written
// here is read back only by a later launch, after far more than the L2 has
// streamed through on the volumes where it matters (about 3% off the
// 512x512x384 pyramid, no change at 145x174x145 or 256^3).
constexpr int kStoreNonTemporal = 2;
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t rs, unsigned boff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rs, (int)boff, 0, kStoreNonTemporal);
}

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

// f(std::integral_constant<int, P>) for P = I .. N-1: every P is a
// compile-time constant inside f, whatever the unroller's size limits.
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// Job of a block: the last job whose first block is <= bid (jobs sorted by block0).
__device__ __forceinline__ int find_fjob(const DFJob *jobs, int n, int bid)
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

// INL: the jobs are read from the inline copy in the arguments (small
// launches), else from the device table. PB: the jobs also write B_s, the
// BRIEF pre-blur (radius kFusedPreR) of their source level G_s, from the
// same staged planes: x outputs from the x pass's row registers, y into a
// third LDS tile, z through a 2*kFusedPreR+1 register shift ring. Each
// stencil is the one a stand-alone pre-blur pass evaluates, in the same
// order, so B_s is the same either way.
template <int R, bool DOG, bool INL, int TY, bool PB>
__global__ void __launch_bounds__(blur_threads(TY)) blur_level_kernel(const FusedLaunch fl)
{
    constexpr int TX = kBlurTX, NY = kBlurNY, NT = blur_threads(TY);
    constexpr int M = 2 * R + 1;
    constexpr int LR = M + 1;                       // y-ring length: even, so two staging buffers alternate in step
    constexpr int RB = PB ? kFusedPreR : 0;         // pre-blur radius
    constexpr int MB = 2 * RB + 1;
    constexpr int BH = TY + 2 * RB;                 // pre-blur rows of the x pass
    static_assert(!PB || (DOG && R >= kFusedPreR), "the pre-blur rides on level passes with a halo >= its radius");
    constexpr int AWL = TX + 2 * R;                 // staged width
    // LDS row pitches, both 16 (mod 32) floats. The x pass reads A and
    // writes B as float4, 16 lanes at a time covering two rows two apart;
    // the y pass reads B one row per half-wavefront, the halves two rows
    // apart. A pitch of 16 (mod 32) puts those two rows in disjoint halves
    // of the 64 LDS banks, so none of these accesses conflict.
    constexpr int AW = AWL + ((16 - AWL % 32) + 32) % 32;
    constexpr int BW = 48;
    static_assert(AW % 32 == 16 && AW >= AWL && BW % 32 == 16 && BW >= TX, "LDS pitches");
    constexpr int AH = TY + 2 * R;                  // staged height
    constexpr int AE = AH * AWL;
    constexpr int KL = (AE + NT - 1) / NT;          // staged elements per thread
    constexpr int XQ = TX / 4;                      // x-pass items per row (4 outputs each)
    constexpr int XIN = 4 + ((2 * R + 3) & ~3);     // x-pass inputs per item, multiple of 4
    static_assert(NY == 2, "sub-sampling pairs rows inside a thread");
    // staging tile plus one dummy slot per unused staging lane (branch-free writes)
    __shared__ __align__(16) float A[AH * AW + KL * NT - AE];
    __shared__ __align__(16) float B[AH * BW];
    // centre values (G_{i-1} at the thread's output voxels) of the last R+1
    // input planes: private to each thread, kept in LDS because the slot
    // index is not a compile-time constant
    __shared__ float C[DOG ? (R + 1) * NY * NT : 1];
    __shared__ __align__(16) float B2[PB ? BH * BW : 1];

    const int tid = threadIdx.x;
    const int logical = xcd_remap(blockIdx.x, fl.n_blocks);
    const DFJob jb = INL ? fl.inl[find_fjob(fl.inl, fl.n_jobs, logical)]
                         : fl.jobs[find_fjob(fl.jobs, fl.n_jobs, logical)];
    const float *const src = jb.src_input ? fl.in + jb.src : reinterpret_cast<const float *>(fl.ws + jb.src);
    float *const dst = reinterpret_cast<float *>(fl.ws + jb.dst);
    float *const dogp = DOG ? reinterpret_cast<float *>(fl.ws + jb.dog) : nullptr;
    float *const subp = jb.sub < 0 ? nullptr : reinterpret_cast<float *>(fl.ws + jb.sub);
    const float *const wt = fl.taps + (size_t)jb.taps * kMaxTaps;
    const int local = logical - jb.block0;
    const int ntile = jb.tiles_x * jb.tiles_y;
    const int slab = local / ntile;
    const int t2 = local - slab * ntile;
    const int tyi = t2 / jb.tiles_x;
    const int txi = t2 - tyi * jb.tiles_x;
    const int x0 = txi * TX, y0 = tyi * TY, z0 = slab * jb.L;
    const int z1 = min(z0 + jb.L, jb.nz);
    const int nx = jb.nx, ny = jb.ny, nz = jb.nz;
    const size_t nxy = (size_t)nx * ny;
    const unsigned plane_bytes = (unsigned)(nxy * sizeof(float));

    // Per-thread staging slots: the same in-plane byte offsets for every plane.
    unsigned goff[KL];
    int loff[KL];
#pragma unroll
    for (int k = 0; k < KL; ++k) {
        const int idx = tid + k * NT;
        if (idx < AE) {
            const int r = idx / AWL, c = idx - r * AWL;
            goff[k] = 4u * (unsigned)(clampi(y0 - R + r, 0, ny - 1) * nx + clampi(x0 - R + c, 0, nx - 1));
            loff[k] = r * AW + c;
        } else {
            goff[k] = 0;
            loff[k] = AH * AW + (idx - AE);
        }
    }
    // two planes in flight: staging buffer b holds the plane of every step
    // with the parity b
    float pre[2][KL];
    auto load_plane = [&](float(&dstv)[KL], int zi) {
        const auto rs = plane_rsrc(src + (size_t)clampi(zi, 0, nz - 1) * nxy, plane_bytes);
#pragma unroll
        for (int k = 0; k < KL; ++k) dstv[k] = buf_load(rs, goff[k]);
    };

    float w[M];
#pragma unroll
    for (int t = 0; t < M; ++t) w[t] = wt[t];
    float wb[MB];
    float ringb[NY][MB];
    float *const pbp = PB ? reinterpret_cast<float *>(fl.ws + jb.pb) : nullptr;
    if constexpr (PB) {
        const float *wbt = fl.taps + (size_t)jb.pb_taps * kMaxTaps;
#pragma unroll
        for (int t = 0; t < MB; ++t) wb[t] = wbt[t];
#pragma unroll
        for (int j = 0; j < NY; ++j)
#pragma unroll
            for (int t = 0; t < MB; ++t) ringb[j][t] = 0.f;
    }

    const int tx = tid % TX;
    const int tyb = (tid / TX) * NY;
    const int gx = x0 + tx, gy0 = y0 + tyb;
    // byte offsets of the thread's two outputs in a plane (kDropOffset outside the volume)
    const unsigned o0 = gx < nx && gy0 < ny ? 4u * (unsigned)(gy0 * nx + gx) : kDropOffset;
    const unsigned o1 = gx < nx && gy0 + 1 < ny ? 4u * (unsigned)((gy0 + 1) * nx + gx) : kDropOffset;
    // byte offset of the 2x2x2 mean this thread writes in a plane of the next
    // octave's G_0 (even x, the thread holding both rows of the y pair)
    const int sub_plane = jb.mx * jb.my;
    const unsigned so = (tx & 1) == 0 && (gx >> 1) < jb.mx && (gy0 >> 1) < jb.my
                            ? 4u * (unsigned)((gy0 >> 1) * jb.mx + (gx >> 1))
                            : kDropOffset;
    float ring[NY][LR];
#pragma unroll
    for (int j = 0; j < NY; ++j)
#pragma unroll
        for (int t = 0; t < LR; ++t) ring[j][t] = 0.f;
    float subacc = 0.f;
    int cslot = 0;                                  // C slot of the current step (it mod R+1)

    // Input plane z0 - R + it is staged at step it; output plane z0 + it - 2R
    // completes at step it. The plane loop is unrolled by the ring length so
    // that every ring slot is a fixed register.
    //
    // Every step issues the same memory operations: the loads of the next
    // plane (the last input plane again at the final step) and one store per
    // output stream, whose per-lane offset is kDropOffset while the step has
    // nothing to write there. Loads and stores share one completion counter;
    // with a fixed count after each plane's loads, the wait before staging
    // that plane covers its loads only, not the stores issued after them.
    const int nplanes = (z1 - z0) + 2 * R;
    const int zin_last = z1 - 1 + R;               // last input plane of the slab
    const bool has_sub = subp != nullptr;
    float *const subbase = has_sub ? subp : dst;
    const unsigned sub_bytes = has_sub ? 4u * (unsigned)sub_plane : 0u;   // 0: every store dropped
    load_plane(pre[0], z0 - R);
    load_plane(pre[1], z0 - R + 1);
    // Steps past the slab's last (dead steps, only in the final round of the
    // unrolled loop) skip the arithmetic but keep the memory operations and
    // barriers, so the loop body has no early exit and the same operation
    // count on every path.
    // The first round is peeled: there the step number is a constant, and
    // the steps before any output exists (the first 2R for G and D, R + RB
    // for the pre-blur) issue no stores. Every later step issues all of them.
    auto step = [&](auto pc, int base, auto first_round) {
            constexpr int p = decltype(pc)::value;
            constexpr bool FIRST = decltype(first_round)::value;
            constexpr bool ZSTORE = !FIRST || p >= 2 * R;       // G, D and sub-sample stores issued
            constexpr bool PSTORE = !FIRST || p >= R + RB;      // pre-blur stores issued
            constexpr int pb = p & 1;
            const int it = base + p;
            const bool live = it < nplanes;
#pragma unroll
            for (int k = 0; k < KL; ++k) A[loff[k]] = pre[pb][k];
            __syncthreads();
            load_plane(pre[pb], min(z0 - R + it + 2, zin_last));
            const int oz = z0 + it - 2 * R;
            const bool zact = live && it >= 2 * R;  // output plane oz exists
            float cv0 = 0.f, cv1 = 0.f;
            if (live) {
                if constexpr (DOG) {
                    // D_{i-1} needs G_{i-1} at the output voxel: keep this plane's centre
                    // values, and take those of the plane staged R steps ago (slot cslot+1)
                    const int rslot = cslot == R ? 0 : cslot + 1;
                    C[(cslot * NY + 0) * NT + tid] = A[(R + tyb) * AW + R + tx];
                    C[(cslot * NY + 1) * NT + tid] = A[(R + tyb + 1) * AW + R + tx];
                    if (zact) {
                        cv0 = C[(rslot * NY + 0) * NT + tid];
                        cv1 = C[(rslot * NY + 1) * NT + tid];
                    }
                    cslot = rslot;
                }

                // x pass: 4 consecutive outputs per item from one LDS strip. A
                // wavefront covers 8 rows per round, its 16-lane groups the
                // rows {0, 2}, {1, 3}, {4, 6}, {5, 7} (8 items of a row each)
                static_assert(XQ == 8, "8 items per row");
                const int lane = tid & 63, lg = lane >> 4;
                const int rlane = 4 * (lg >> 1) + (lg & 1) + 2 * ((lane >> 3) & 1);
                const int xb = 4 * (lane & 7);
                for (int r = 8 * (tid >> 6) + rlane; r < AH; r += 8 * (NT / 64)) {
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
                    *reinterpret_cast<float4 *>(&B[r * BW + xb]) = make_float4(o[0], o[1], o[2], o[3]);
                    if constexpr (PB) {
                        // rows y0 - RB .. y0 + TY + RB of the pre-blur, x from the same registers
                        if (r >= R - RB && r < R + TY + RB) {
                            float ob[4];
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                ob[q] = sym_stencil<RB>(wb, [&](int t) { return in[q + R - RB + t]; });
                            *reinterpret_cast<float4 *>(&B2[(r - (R - RB)) * BW + xb]) =
                                make_float4(ob[0], ob[1], ob[2], ob[3]);
                        }
                    }
                }
            }
            __syncthreads();

            float pbv[NY], zo[NY];
#pragma unroll
            for (int j = 0; j < NY; ++j) pbv[j] = zo[j] = 0.f;
            if (live) {
                // y pass: NY consecutive outputs of column tx, into ring slot p
                float col[NY + 2 * R];
#pragma unroll
                for (int q = 0; q < NY + 2 * R; ++q) col[q] = B[(tyb + q) * BW + tx];
#pragma unroll
                for (int j = 0; j < NY; ++j) ring[j][p] = sym_stencil<R>(w, [&](int t) { return col[j + t]; });

                if constexpr (PB) {
                    // pre-blur: y pass into the shift ring (oldest plane first), then z
                    float colb[NY + 2 * RB];
#pragma unroll
                    for (int q = 0; q < NY + 2 * RB; ++q) colb[q] = B2[(tyb + q) * BW + tx];
#pragma unroll
                    for (int j = 0; j < NY; ++j) {
#pragma unroll
                        for (int t = 0; t + 1 < MB; ++t) ringb[j][t] = ringb[j][t + 1];
                        ringb[j][MB - 1] = sym_stencil<RB>(wb, [&](int t) { return colb[j + t]; });
                        pbv[j] = sym_stencil<RB>(wb, [&](int t) { return ringb[j][t]; });
                    }
                }
                // z pass: slot (p + 2 + t) % LR holds input plane (it - 2R + t)
                if (zact) {
#pragma unroll
                    for (int j = 0; j < NY; ++j)
                        zo[j] = sym_stencil<R>(w, [&](int t) { return ring[j][(p + 2 + t) % LR]; });
                }
            }
            if constexpr (PB && PSTORE) {
                // the pre-blur ring holds input planes zin - 2RB .. zin (zin = z0 - R + it);
                // its centre plane is an output plane of this slab from step R + RB on
                const int qz = z0 - R + it - RB;
                const bool pact = live && it >= R + RB && qz < z1;
                const auto rs = plane_rsrc(pbp + (size_t)clampi(qz, 0, nz - 1) * nxy, plane_bytes);
                buf_store(rs, pact ? o0 : kDropOffset, pbv[0]);
                buf_store(rs, pact ? o1 : kDropOffset, pbv[1]);
            }
            if constexpr (!ZSTORE) return;
            const int ozc = clampi(oz, 0, nz - 1);
            const unsigned a0 = zact ? o0 : kDropOffset, a1 = zact ? o1 : kDropOffset;
            const auto rd = plane_rsrc(dst + (size_t)ozc * nxy, plane_bytes);
            buf_store(rd, a0, zo[0]);
            buf_store(rd, a1, zo[1]);
            if constexpr (DOG) {
                const auto re = plane_rsrc(dogp + (size_t)ozc * nxy, plane_bytes);
                buf_store(re, a0, cv0 - zo[0]);
                buf_store(re, a1, cv1 - zo[1]);
            }
            // 2x2x2 mean: the even plane's partial sum waits in subacc, the odd
            // plane completes it
            float s4 = 0.f;
            if (has_sub) {
                const float s2 = zo[0] + zo[1];
                s4 = s2 + __shfl_xor(s2, 1);
            }
            const bool sact = zact && (oz & 1) != 0 && (oz >> 1) < jb.mz;
            const auto rsub = plane_rsrc(subbase + (size_t)(ozc >> 1) * sub_plane, sub_bytes);
            buf_store(rsub, sact ? so : kDropOffset, (subacc + s4) * 0.125f);
            if (zact && (oz & 1) == 0) subacc = s4;
    };
    static_for<0, LR>([&](auto pc) { step(pc, 0, std::true_type{}); });
    for (int base = LR; base < nplanes; base += LR)
        static_for<0, LR>([&](auto pc) { step(pc, base, std::false_type{}); });
}


template <int R, int TY>
hipError_t launch_rt(const FusedLaunch &a, bool dog, bool pb, hipStream_t st)
{
    const dim3 g(a.n_blocks), b(blur_threads(TY));
    const bool inl = a.n_jobs <= kInlineJobs;
    if (pb) {
        if constexpr (R >= kFusedPreR) {
            if (!dog) return hipErrorInvalidValue;
            if (inl)
                hipLaunchKernelGGL((blur_level_kernel<R, true, true, TY, true>), g, b, 0, st, a);
            else
                hipLaunchKernelGGL((blur_level_kernel<R, true, false, TY, true>), g, b, 0, st, a);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    if (dog && inl)
        hipLaunchKernelGGL((blur_level_kernel<R, true, true, TY, false>), g, b, 0, st, a);
    else if (dog)
        hipLaunchKernelGGL((blur_level_kernel<R, true, false, TY, false>), g, b, 0, st, a);
    else if (inl)
        hipLaunchKernelGGL((blur_level_kernel<R, false, true, TY, false>), g, b, 0, st, a);
    else
        hipLaunchKernelGGL((blur_level_kernel<R, false, false, TY, false>), g, b, 0, st, a);
    return hipGetLastError();
}

template <int R, int TY>
int occupancy_rt(bool dog, bool pb)
{
    int n = 0;
    hipError_t e;
    if constexpr (R >= kFusedPreR) {
        if (pb && dog)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, blur_level_kernel<R, true, true, TY, true>,
                                                             blur_threads(TY), 0);
        else if (pb)
            return 0;
        else if (dog)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, blur_level_kernel<R, true, true, TY, false>,
                                                             blur_threads(TY), 0);
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, blur_level_kernel<R, false, true, TY, false>,
                                                             blur_threads(TY), 0);
    } else {
        if (pb) return 0;
        e = dog ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, blur_level_kernel<R, true, true, TY, false>,
                                                               blur_threads(TY), 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, blur_level_kernel<R, false, true, TY, false>,
                                                               blur_threads(TY), 0);
    }
    return e == hipSuccess ? n : 0;
}

// Launch (or query the occupancy of) the instance for radius r, tile height TY.
template <int TY>
hipError_t launch_ty(const FusedLaunch &a, int r, bool dog, bool pb, hipStream_t st)
{
    static_assert(kMaxFusedR == 10, "one case per fused radius");
    switch (r) {
    case 0: return launch_rt<0, TY>(a, dog, pb, st);
    case 1: return launch_rt<1, TY>(a, dog, pb, st);
    case 2: return launch_rt<2, TY>(a, dog, pb, st);
    case 3: return launch_rt<3, TY>(a, dog, pb, st);
    case 4: return launch_rt<4, TY>(a, dog, pb, st);
    case 5: return launch_rt<5, TY>(a, dog, pb, st);
    case 6: return launch_rt<6, TY>(a, dog, pb, st);
    case 7: return launch_rt<7, TY>(a, dog, pb, st);
    case 8: return launch_rt<8, TY>(a, dog, pb, st);
    case 9: return launch_rt<9, TY>(a, dog, pb, st);
    case 10: return launch_rt<10, TY>(a, dog, pb, st);
    default: return hipErrorInvalidValue;
    }
}

template <int TY>
int occupancy_ty(int r, bool dog, bool pb)
{
    switch (r) {
    case 0: return occupancy_rt<0, TY>(dog, pb);
    case 1: return occupancy_rt<1, TY>(dog, pb);
    case 2: return occupancy_rt<2, TY>(dog, pb);
    case 3: return occupancy_rt<3, TY>(dog, pb);
    case 4: return occupancy_rt<4, TY>(dog, pb);
    case 5: return occupancy_rt<5, TY>(dog, pb);
    case 6: return occupancy_rt<6, TY>(dog, pb);
    case 7: return occupancy_rt<7, TY>(dog, pb);
    case 8: return occupancy_rt<8, TY>(dog, pb);
    case 9: return occupancy_rt<9, TY>(dog, pb);
    case 10: return occupancy_rt<10, TY>(dog, pb);
    default: return 0;
    }
}

}  // namespace fused
}  // namespace s3d
