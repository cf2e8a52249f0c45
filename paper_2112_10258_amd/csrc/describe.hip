// Keypoint descriptors on gfx950: upright 3D SIFT-Rank (Section 2: 2x2x2
// spatial x 8 orientation bins, normalised by ranking), one workgroup per
// keypoint, and the BRIEF / RRIEF descriptors (Section 3.2.3), one
// wavefront per keypoint. Workgroups (wavefronts) loop over the keypoint
// lists, whose lengths are read from device memory, so the launches never
// wait on the host. The keypoints of all volumes of a plan are dealt to
// them as one flat sequence.
//
// Floating-point sums are accumulated in double precision in a fixed order
// (no atomics), so results are bit-reproducible run to run.
#include <algorithm>
#include <type_traits>

#include "sift3d_internal.h"

namespace s3d {
namespace {

constexpr int kDescThreads = 256;

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// Side of the cube of G_s a SIFT-Rank window reads: the (2R+1)^3 samples
// and their central-difference neighbours.
constexpr int kSiftTile = 2 * kMaxSiftR + 3;

// One (dx, dy) column of the SIFT-Rank window, read from the staged cube T
// (T[k][j][i] = G_s at clamp(corner + (i, j, k)), corner = keypoint - R - 1):
// the sample q = clamp(v + d) and its neighbours clamp(q +- 1) always fall
// inside the cube, so each is one LDS read. |g| is evaluated in single
// precision (relative error <= 4.5 * 2^-24: the differences, squares, sum
// and square root each round once) and accumulated per (z half,
// orientation octant) in double. Bins are sums of positive terms, so each
// carries the same relative error bound and two bins' difference is off by
// at most 5.4e-7 of the largest bin. The octant signs are exact: a float
// difference has the sign of the exact difference.
template <int R>
__device__ __forceinline__ void sift_column(const float *T, int nx, int ny, int nz, int kx, int ky, int kz, int dx,
                                            int dy, double (&acc)[16])
{
    constexpr int W = 2 * R + 1, TW = 2 * R + 3;
    const int cx = kx - R - 1, cy = ky - R - 1, cz = kz - R - 1;
    const int qx = clampi(kx + dx, 0, nx - 1), qy = clampi(ky + dy, 0, ny - 1);
    const int lx = qx - cx, ly = qy - cy;
    const int lxm = clampi(qx - 1, 0, nx - 1) - cx, lxp = clampi(qx + 1, 0, nx - 1) - cx;
    const int lym = clampi(qy - 1, 0, ny - 1) - cy, lyp = clampi(qy + 1, 0, ny - 1) - cy;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        const int dz = i - R;
        const int qz = clampi(kz + dz, 0, nz - 1);
        const int lz = qz - cz, lzm = clampi(qz - 1, 0, nz - 1) - cz, lzp = clampi(qz + 1, 0, nz - 1) - cz;
        const float *row = T + (lz * TW + ly) * TW;
        const float fxp = row[lxp], fxm = row[lxm];
        const float fyp = T[(lz * TW + lyp) * TW + lx], fym = T[(lz * TW + lym) * TW + lx];
        const float fzp = T[(lzp * TW + ly) * TW + lx], fzm = T[(lzm * TW + ly) * TW + lx];
        const float gx = 0.5f * (fxp - fxm);
        const float gy = 0.5f * (fyp - fym);
        const float gz = 0.5f * (fzp - fzm);
        const double m = (double)__builtin_sqrtf(gx * gx + gy * gy + gz * gz);
        const int bo = (gx > 0.0f) + 2 * (gy > 0.0f) + 4 * (gz > 0.0f);
        // dz is a compile-time constant here: a sample feeds only its z half
        // (both halves, with half weight, on the centre plane)
        if (dz < 0) {
#pragma unroll
            for (int b = 0; b < 8; ++b) acc[b] += bo == b ? m : 0.0;
        } else if (dz > 0) {
#pragma unroll
            for (int b = 0; b < 8; ++b) acc[8 + b] += bo == b ? m : 0.0;
        } else {
            const double h = 0.5 * m;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                acc[b] += bo == b ? h : 0.0;
                acc[8 + b] += bo == b ? h : 0.0;
            }
        }
    }
}

// The cube of G_s a window reads, clamp(keypoint - R - 1 .. keypoint + R +
// 1) per axis, passes through registers: element idx = tid + 256 j of the
// (2R+3)^3 cube (x fastest) is slot j of thread tid. cube_fetch issues the
// loads of the next keypoint's cube while the current one is still being
// ranked; cube_stage writes the slots to LDS.
constexpr int kCubeSlots = (kSiftTile * kSiftTile * kSiftTile + kDescThreads - 1) / kDescThreads;
constexpr int kRawBufferWord3 = 0x00020000;   // dword 3 of a raw (untyped) buffer resource on gfx9

// Slot j of thread tid is element idx = tid + 256 j: its (x, y, z) in the
// cube advance from slot to slot by 256 written in base TW (one carry per
// digit at most), so one code path serves every radius.
struct CubeWalk {
    int TW, N, s0, s1, s2;   // side, elements, digits of 256 in base TW
    int i, j, k;             // position of this thread's current slot
    __device__ __forceinline__ CubeWalk(int R, int tid)
    {
        TW = 2 * R + 3;
        N = TW * TW * TW;
        s2 = kDescThreads / (TW * TW);
        const int r2 = kDescThreads - s2 * TW * TW;
        s1 = r2 / TW;
        s0 = r2 - s1 * TW;
        // the slot positions are recomputed per call rather than kept live
        // across the keypoint loop
        int t = tid;
        asm volatile("" : "+v"(t));
        i = t % TW;
        const int jk = t / TW;
        j = jk % TW;
        k = jk / TW;
    }
    __device__ __forceinline__ void next()
    {
        i += s0;
        const int ci = i >= TW;
        i -= ci ? TW : 0;
        j += s1 + ci;
        const int cj = j >= TW;
        j -= cj ? TW : 0;
        k += s2 + cj;
    }
};

__device__ __forceinline__ void cube_fetch(const float *G, int nx, int ny, int nz, int kx, int ky, int kz, int R,
                                           int tid, float (&pre)[kCubeSlots])
{
    CubeWalk w(R, tid);
    const int cx = kx - R - 1, cy = ky - R - 1, cz = kz - R - 1;
    // a buffer resource over the level: each load needs only a 32-bit
    // offset (the level holds at most 2^30 floats)
    const unsigned bytes = (unsigned)min((long long)nx * ny * nz * 4, 0xffffffffLL);
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(G), (short)0, (int)bytes, kRawBufferWord3);
#pragma unroll
    for (int s = 0; s < kCubeSlots; ++s) {
        if (tid + kDescThreads * s < w.N) {
            const int gx = clampi(cx + w.i, 0, nx - 1), gy = clampi(cy + w.j, 0, ny - 1);
            const int gz = clampi(cz + w.k, 0, nz - 1);
            const unsigned off = 4u * (((unsigned)gz * (unsigned)ny + (unsigned)gy) * (unsigned)nx + (unsigned)gx);
            pre[s] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0));
        }
        w.next();
    }
}

__device__ __forceinline__ void cube_stage(float *T, int R, int tid, const float (&pre)[kCubeSlots])
{
    const int TW = 2 * R + 3, N = TW * TW * TW;
#pragma unroll
    for (int s = 0; s < kCubeSlots; ++s) {
        const int idx = tid + kDescThreads * s;
        if (idx < N) T[idx] = pre[s];
    }
}

// f(std::integral_constant<int, R>) for the window half-width R (1..7).
template <typename F>
__device__ __forceinline__ void with_radius(int R, F &&f)
{
    switch (R) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    default: f(std::integral_constant<int, 7>{}); break;
    }
}

// Class of an offset along x or y: 0 for d < 0, 1 for d == 0, 2 for d > 0,
// and the weight a class gives spatial half b (0: d < 0 side, 1: d > 0
// side): the centre plane splits half/half.
__device__ __forceinline__ double half_weight(int cls, int b)
{
    return cls == 1 ? 0.5 : ((cls == 2) == (b == 1) ? 1.0 : 0.0);
}

// First keypoint of volume v that block b handles when the keypoints of all
// volumes are dealt round-robin to the blocks in one flat sequence (base =
// keypoints of the volumes before v).
__device__ __forceinline__ int first_of_block(int b, long long base, int grid)
{
    const long long r = ((long long)b - base) % grid;
    return (int)(r < 0 ? r + grid : r);
}

// SIFT-Rank, one workgroup per keypoint. Each of the first (2R+1)^2 threads
// owns one (dx, dy) column of the (2R+1)^3 window and walks dz,
// accumulating |g| per (z half, orientation octant); the centre plane dz = 0
// adds half to each z half. The column sums are then added up within each
// of the 9 (sign dx, sign dy) classes (row sums per x class, then over the
// rows of each y class, in a fixed order), and each of the 64 bins combines
// the 9 class sums with their x/y half weights, and is ranked.
template <bool INL>
__device__ __forceinline__ void siftrank_body(const DescLaunch &a, int blk, int nblk)
{
    constexpr int kCols = (2 * kMaxSiftR + 1) * (2 * kMaxSiftR + 1);
    static_assert(kCols <= kDescThreads, "one thread per window column");
    constexpr int kTileFloats = kSiftTile * kSiftTile * kSiftTile;
    constexpr int kPartBytes = kCols * 17 * (int)sizeof(double);
    // the staged cube and the per-column sums share LDS (a barrier separates them)
    __shared__ __align__(16) char scratch[kPartBytes > kTileFloats * 4 ? kPartBytes : kTileFloats * 4];
    float *const T = reinterpret_cast<float *>(scratch);
    double(*const part)[17] = reinterpret_cast<double(*)[17]>(scratch);
    __shared__ double rows[2 * kMaxSiftR + 1][3][16];   // per (row, x class) sums
    __shared__ double cls[9][16];
    __shared__ double hist[64];
    __shared__ int rank_part[kDescThreads / 64][64];
    static_assert(kDescThreads == 256, "four wavefronts share the ranking");
    const int tid = threadIdx.x;
    // the window of a keypoint: level, octave dims and radius, or not a
    // keypoint of this plan
    struct Win {
        const float *G;
        int nx, ny, nz, R;
        bool ok;
    };
    auto window_of = [&](const DVol &vol, const sift3d_keypoint &kp) -> Win {
        Win w{};
        w.ok = !(kp.octave < 0 || kp.octave >= vol.n_units || kp.scale < 1 || kp.scale > a.S);
        if (!w.ok) return w;
        const DUnit &oc = (INL ? a.inl[vol.unit0 + kp.octave] : a.units[vol.unit0 + kp.octave]);
        w.nx = oc.nx;
        w.ny = oc.ny;
        w.nz = oc.nz;
        w.G = reinterpret_cast<const float *>(a.ws + oc.g0) + oc.lstride * kp.scale;
        w.R = a.sift_R[kp.scale];
        return w;
    };
    auto fetch = [&](const Win &w, const sift3d_keypoint &kp, float (&pre)[kCubeSlots]) {
        if (w.ok) cube_fetch(w.G, w.nx, w.ny, w.nz, kp.x, kp.y, kp.z, w.R, tid, pre);
    };
    float pre[kCubeSlots];
    long long base = 0;
    for (int v = 0; v < a.n_vol; ++v) {
    const int count = min(a.counts[v], a.cap);
    const DVol vol = a.vols[v];
    int kk = first_of_block(blk, base, nblk);
    sift3d_keypoint kp{};
    Win win{};
    if (kk < count) {
        kp = a.kp[(size_t)v * a.cap + kk];
        win = window_of(vol, kp);
        fetch(win, kp, pre);
    }
    for (; kk < count; kk += nblk) {
        const size_t k = (size_t)v * a.cap + kk;
        if (!win.ok) {
            // not a keypoint of this plan (uniform: the whole workgroup)
            if (tid < 64) a.siftrank[k * 64 + tid] = 0;
            if (kk + nblk < count) {
                kp = a.kp[k + nblk];
                win = window_of(vol, kp);
                fetch(win, kp, pre);
            }
            continue;
        }
        const sift3d_keypoint cur = kp;
        const Win cw = win;
        const int R = cw.R;
        const int W = 2 * R + 1;
        cube_stage(T, R, tid, pre);
        __syncthreads();   // the cube is staged
        double acc[16];
#pragma unroll
        for (int b = 0; b < 16; ++b) acc[b] = 0.0;
        if (tid < W * W) {
            const int dy = tid / W - R, dx = tid - (tid / W) * W - R;
            with_radius(R, [&](auto r) {
                sift_column<decltype(r)::value>(T, cw.nx, cw.ny, cw.nz, cur.x, cur.y, cur.z, dx, dy, acc);
            });
        }
        __syncthreads();   // the column sums overwrite the staged cube
        if (tid < W * W) {
#pragma unroll
            for (int b = 0; b < 16; ++b) part[tid][b] = acc[b];
        }
        __syncthreads();
        // class sums in two steps (each a chain of at most R adds): along x
        // within each row and x class, then over the rows of each y class
        for (int item = tid; item < W * 48; item += kDescThreads) {
            const int yy = item / 48, rem = item - yy * 48;
            const int cx = rem >> 4, j = rem & 15;
            const int x0 = cx == 0 ? 0 : (cx == 1 ? R : R + 1), x1 = cx == 0 ? R : (cx == 1 ? R + 1 : W);
            double sum = 0.0;
            for (int xx = x0; xx < x1; ++xx) sum += part[yy * W + xx][j];
            rows[yy][cx][j] = sum;
        }
        __syncthreads();
        if (tid < 144) {
            // class q = (cy, cx), value j: columns with dx, dy in the class ranges
            const int q = tid >> 4, j = tid & 15;
            const int cy = q / 3, cx = q - cy * 3;
            const int y0 = cy == 0 ? 0 : (cy == 1 ? R : R + 1), y1 = cy == 0 ? R : (cy == 1 ? R + 1 : W);
            double sum = 0.0;
            for (int yy = y0; yy < y1; ++yy) sum += rows[yy][cx][j];
            cls[q][j] = sum;
        }
        __syncthreads();
        if (tid < 64) {
            const int bs = tid >> 3, bo = tid & 7;
            const int bx = bs & 1, by = (bs >> 1) & 1, bz = bs >> 2;
            double h = 0.0;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int cy = q / 3, cx = q - cy * 3;
                h += (half_weight(cx, bx) * half_weight(cy, by)) * cls[q][8 * bz + bo];
            }
            hist[tid] = h;
        }
        __syncthreads();
        // the next keypoint's cube is fetched while this one is ranked
        if (kk + nblk < count) {
            kp = a.kp[k + nblk];
            win = window_of(vol, kp);
            fetch(win, kp, pre);
        }
        {
            // rank of bin e = tid % 64 among the 64 (ties by index): the four
            // wavefronts count over a quarter of the bins each
            const int e = tid & 63, q = tid >> 6;
            const double h = hist[e];
            int r = 0;
#pragma unroll
            for (int o = 16 * q; o < 16 * q + 16; ++o) {
                const double x = hist[o];
                r += (int)(x < h) | ((int)(x == h) & (int)(o < e));
            }
            rank_part[q][e] = r;
        }
        __syncthreads();
        if (tid < 64)
            a.siftrank[k * 64 + tid] =
                (uint8_t)(rank_part[0][tid] + rank_part[1][tid] + rank_part[2][tid] + rank_part[3][tid]);
        __syncthreads();
    }
    base += count;
    }
}

// BRIEF / RRIEF, one wavefront per keypoint (four per workgroup, each on
// its own keypoints). B_s is G_s already blurred by the sigma_b pre-blur (a
// whole-level separable pass with the same clamp-to-edge rule, so B_s at a
// voxel equals the pre-blur stencil evaluated there). Lane l holds pairs
// 64 j + l, j < 4: d = B_s(p1) - B_s(p2) is the exact double difference of
// the two samples; word j of the binary descriptor is the ballot of d > 0
// over register j. RRIEF ranks (position of (d_i, i) in ascending
// lexicographic order, i.e. #{m : d_m < d_i or (d_m == d_i and m < i)})
// come from a bitonic sort of the 256 (difference, index) pairs (n padded
// with +inf keys, which sort after every finite difference) held as
// element 64 j + l: partners 64 or 128 apart are registers of the same
// lane, the others are lanes of the same register. No barriers, no LDS.
constexpr int kBriefRegs = kMaxPairs / 64;

__device__ __forceinline__ bool pair_gt(double ka, int ia, double kb, int ib)
{
    return ka > kb || (ka == kb && ia > ib);
}

template <bool INL>
__device__ __forceinline__ void brief_body(const DescLaunch &a, int blk, int nblk)
{
    const int lane = threadIdx.x & 63;
    // wave index: uniform across the wave
    const int gw = __builtin_amdgcn_readfirstlane(blk * (kDescThreads / 64) + (threadIdx.x >> 6));
    const int nwaves = nblk * (kDescThreads / 64);
    const int n = a.brief_n, nw = n / 64;
    // The two samples of every pair of a keypoint (8 loads per lane) are
    // issued one keypoint ahead: the next keypoint's loads are in flight
    // while the current one is compared and sorted.
    auto gather = [&](const DVol &vol, const sift3d_keypoint &kp, float (&s1)[kBriefRegs],
                      float (&s2)[kBriefRegs]) -> bool {
        if (kp.octave < 0 || kp.octave >= vol.n_units || kp.scale < 1 || kp.scale > a.S) return false;
        const DUnit &oc = (INL ? a.inl[vol.unit0 + kp.octave] : a.units[vol.unit0 + kp.octave]);
        const int nx = oc.nx, ny = oc.ny, nz = oc.nz;
        const float *B = reinterpret_cast<const float *>(a.ws + oc.b1) + oc.lstride * (kp.scale - 1);
#pragma unroll
        for (int j = 0; j < kBriefRegs; ++j) {
            const int i = 64 * j + lane;
            s1[j] = s2[j] = 0.f;
            if (i < n) {
                const int32_t *o = a.pairs + ((size_t)(kp.scale - 1) * n + i) * 6;
                const int x1 = clampi(kp.x + o[0], 0, nx - 1), y1 = clampi(kp.y + o[1], 0, ny - 1);
                const int z1 = clampi(kp.z + o[2], 0, nz - 1);
                const int x2 = clampi(kp.x + o[3], 0, nx - 1), y2 = clampi(kp.y + o[4], 0, ny - 1);
                const int z2 = clampi(kp.z + o[5], 0, nz - 1);
                s1[j] = B[((size_t)z1 * ny + y1) * nx + x1];
                s2[j] = B[((size_t)z2 * ny + y2) * nx + x2];
            }
        }
        return true;
    };
    float n1[kBriefRegs], n2[kBriefRegs];
    long long base = 0;
    for (int v = 0; v < a.n_vol; ++v) {
    const int count = min(a.counts[v], a.cap);
    const DVol vol = a.vols[v];
    int kk = first_of_block(gw, base, nwaves);
    bool nok = false;
    if (kk < count) nok = gather(vol, a.kp[(size_t)v * a.cap + kk], n1, n2);
    for (; kk < count; kk += nwaves) {
        const size_t k = (size_t)v * a.cap + kk;
        const bool ok = nok;
        float b1[kBriefRegs], b2[kBriefRegs];
#pragma unroll
        for (int j = 0; j < kBriefRegs; ++j) {
            b1[j] = n1[j];
            b2[j] = n2[j];
        }
        if (kk + nwaves < count) nok = gather(vol, a.kp[k + nwaves], n1, n2);
        if (!ok) {
            // not a keypoint of this plan
#pragma unroll
            for (int j = 0; j < kBriefRegs; ++j) {
                const int i = 64 * j + lane;
                if (a.rrief != nullptr && i < n) a.rrief[k * n + i] = 0;
            }
            if (a.brief != nullptr && lane < nw) a.brief[k * nw + lane] = 0;
            continue;
        }
        double key[kBriefRegs];
        int idx[kBriefRegs];
#pragma unroll
        for (int j = 0; j < kBriefRegs; ++j) {
            const int i = 64 * j + lane;
            idx[j] = i;
            key[j] = i < n ? (double)b1[j] - (double)b2[j] : __builtin_inf();
        }
        if (a.brief != nullptr) {
#pragma unroll
            for (int j = 0; j < kBriefRegs; ++j) {
                const unsigned long long m = __ballot(key[j] > 0.0);   // +inf pads only past n
                if (j < nw && lane == 0) a.brief[k * nw + j] = m;
            }
        }
        if (a.rrief != nullptr) {
#pragma unroll
            for (int kk2 = 2; kk2 <= kMaxPairs; kk2 <<= 1) {
#pragma unroll
                for (int jj = kk2 >> 1; jj > 0; jj >>= 1) {
                    if (jj >= 64) {
                        const int jr = jj >> 6;
#pragma unroll
                        for (int j = 0; j < kBriefRegs; ++j) {
                            if (j & jr) continue;
                            const int j2 = j | jr;
                            const bool up = ((64 * j + lane) & kk2) == 0;
                            // the lower element keeps the smaller pair on an ascending run
                            if (pair_gt(key[j], idx[j], key[j2], idx[j2]) == up) {
                                const double tk = key[j];
                                const int ti = idx[j];
                                key[j] = key[j2];
                                idx[j] = idx[j2];
                                key[j2] = tk;
                                idx[j2] = ti;
                            }
                        }
                    } else {
                        const bool lower = (lane & jj) == 0;
#pragma unroll
                        for (int j = 0; j < kBriefRegs; ++j) {
                            const double pk = __shfl_xor(key[j], jj);
                            const int pi = __shfl_xor(idx[j], jj);
                            const bool up = ((64 * j + lane) & kk2) == 0;
                            const bool gt = pair_gt(key[j], idx[j], pk, pi);
                            if (lower == up ? gt : !gt) {
                                key[j] = pk;
                                idx[j] = pi;
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < kBriefRegs; ++j)
                if (idx[j] < n) a.rrief[k * n + idx[j]] = (uint8_t)(64 * j + lane);
        }
    }
    base += count;
    }
}

// Both descriptor families in one launch: workgroups [0, sr_blocks) compute
// SIFT-Rank, the others BRIEF / RRIEF, so the two run side by side (the
// roles are uniform per workgroup).
template <bool INL>
__global__ void __launch_bounds__(kDescThreads, 4) describe_kernel(const DescLaunch a)
{
    const int b = blockIdx.x;
    if (b < a.sr_blocks)
        siftrank_body<INL>(a, b, a.sr_blocks);
    else
        brief_body<INL>(a, b - a.sr_blocks, gridDim.x - a.sr_blocks);
}

}  // namespace

// Workgroups of `k` resident on one CU (registers and LDS), at least 1.
template <typename K>
static int blocks_per_cu(K k)
{
    int n = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, kDescThreads, 0) == hipSuccess && n > 0 ? n : 1;
}

// Grid: the device's resident slots filled once (the workgroups loop over
// the keypoints). SIFT-Rank takes one workgroup per keypoint slot and
// BRIEF / RRIEF one per four while both fit; past that they share the
// slots 3 : 1 (a SIFT-Rank keypoint costs about three times a BRIEF one).
hipError_t launch_describe(const DescLaunch &a0, long long kp_slots, int n_cu, hipStream_t st)
{
    if (a0.brief_n < 0 || a0.brief_n > kMaxPairs || a0.brief_n % 64 != 0) return hipErrorInvalidValue;
    if (kp_slots <= 0) return hipSuccess;
    const bool sr = a0.siftrank != nullptr;
    const bool br = (a0.brief != nullptr || a0.rrief != nullptr) && a0.brief_n > 0;
    if (!sr && !br) return hipSuccess;
    static const int per_cu = blocks_per_cu(describe_kernel<true>);
    const long long slots = (long long)per_cu * n_cu;
    const int waves = kDescThreads / 64;
    long long gs = sr ? kp_slots : 0, gb = br ? (kp_slots + waves - 1) / waves : 0;
    if (gs + gb > slots) {
        if (!br)
            gs = slots;
        else if (!sr)
            gb = slots;
        else {
            gb = std::max<long long>(1, std::min(gb, slots / 4));
            gs = std::max<long long>(1, slots - gb);
        }
    }
    DescLaunch a = a0;
    a.sr_blocks = (int)gs;
    const dim3 grid((unsigned)(gs + gb));
    if (a.n_units <= kInlineUnits)
        hipLaunchKernelGGL(describe_kernel<true>, grid, dim3(kDescThreads), 0, st, a);
    else
        hipLaunchKernelGGL(describe_kernel<false>, grid, dim3(kDescThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace s3d
