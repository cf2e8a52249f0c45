// Nearest-neighbour matching of descriptors on gfx950: for every row of A,
// the nearest row of B, its distance and the second-smallest distance (for
// a ratio test). Keypoints are matched by their descriptors (Section 3.3):
//   BRIEF: rows of w 64-bit words, distance = Hamming distance (popcount of
//          the XOR);
//   ranks (SIFT-Rank, RRIEF): rows of m uint8 ranks, distance = squared
//          Euclidean distance = |a|^2 + |b|^2 - 2 a.b, the dot products on
//          the int8 matrix cores; exact integers.
// BRIEF: a workgroup owns 64 rows of A, one per lane, held in registers; B
// streams through LDS in tiles, and wavefront w of the four scans the w-th
// quarter of every tile (broadcast reads), in index order. Ranks: see the
// matrix-core kernel below. Partial results of a row are merged with one
// rule: the smallest distance with the lowest index wins, and the
// second-smallest distance is the smallest of everything but the winner.
#include <climits>
#include <cstdint>

#include "sift3d_internal.h"

namespace s3d {
namespace {

constexpr int kMatchThreads = 256;
constexpr int kMatchWaves = kMatchThreads / 64;   // B quarters per row of A
constexpr int kMatchLdsWords = 8192;   // 32 KB of B rows per tile

struct MatchArgs {
    const uint32_t *a, *b;   // rows of W 32-bit words
    int n_a, n_b;
    int32_t *idx, *d1, *d2;
};

// Running best (index, distance) and second-best distance over B in index order.
struct Best {
    int idx = -1;
    int d1 = INT_MAX, d2 = INT_MAX;
    __device__ __forceinline__ void take(int d, int j)
    {
        if (d < d1) {
            d2 = d1;
            d1 = d;
            idx = j;
        } else if (d < d2) {
            d2 = d;
        }
    }
};

// BRIEF rows of W 32-bit words (W/2 descriptor words).
template <int W>
__global__ void __launch_bounds__(kMatchThreads) match_kernel(const MatchArgs a)
{
    constexpr int TILE = kMatchLdsWords / W;   // rows of B per tile
    __shared__ uint32_t tb[TILE * W];
    __shared__ int pidx[kMatchWaves][64], pd1[kMatchWaves][64], pd2[kMatchWaves][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const bool live = i < a.n_a;
    uint32_t ra[W];
#pragma unroll
    for (int w = 0; w < W; ++w) ra[w] = live ? a.a[(size_t)i * W + w] : 0u;
    Best best;
    for (int j0 = 0; j0 < a.n_b; j0 += TILE) {
        const int rows = min(TILE, a.n_b - j0);
        __syncthreads();   // the previous tile is no longer read
        for (int e = threadIdx.x; e < rows * W; e += kMatchThreads) tb[e] = a.b[(size_t)j0 * W + e];
        __syncthreads();
        // this wavefront's quarter of the tile
        const int q = (rows + kMatchWaves - 1) / kMatchWaves;
        const int r0 = wave * q, r1 = min(rows, r0 + q);
        if (live) {
            for (int r = r0; r < r1; ++r) {
                int d = 0;
#pragma unroll
                for (int w = 0; w < W; ++w) d += __popc(ra[w] ^ tb[r * W + w]);
                best.take(d, j0 + r);
            }
        }
    }
    pidx[wave][lane] = best.idx;
    pd1[wave][lane] = best.d1;
    pd2[wave][lane] = best.d2;
    __syncthreads();
    if (wave == 0 && live) {
        // winner: smallest distance, lowest index among equal ones (each
        // quarter's index is already its lowest at that distance)
        int wb = 0;
        for (int w = 1; w < kMatchWaves; ++w) {
            const bool better = pd1[w][lane] < pd1[wb][lane] ||
                                (pd1[w][lane] == pd1[wb][lane] && pidx[w][lane] >= 0 &&
                                 (pidx[wb][lane] < 0 || pidx[w][lane] < pidx[wb][lane]));
            if (better) wb = w;
        }
        int d2 = pd2[wb][lane];
        for (int w = 0; w < kMatchWaves; ++w)
            if (w != wb) d2 = min(d2, pd1[w][lane]);
        a.idx[i] = pidx[wb][lane];
        a.d1[i] = pd1[wb][lane];
        a.d2[i] = d2;
    }
}

// ---------------------------------------------------------------- ranks on MFMA
// Rank vectors (KB x 32 bytes) on the int8 matrix cores: a rank r becomes
// the signed byte r - 128 (r ^ 0x80), which leaves every difference, and so
// every distance |a|^2 + |b|^2 - 2 a.b, unchanged and exact in int32.
// A workgroup owns 32 (or 64) rows of A; B streams through LDS in tiles
// of 512 rows, and wavefront w of the sixteen takes rows 32 w .. 32 w + 31. One
// v_mfma_i32_32x32x32_i8 per 32 bytes gives the 32 x 32 dot products of a
// block of B rows (matrix rows, the A operand) with the workgroup's A rows
// (matrix columns, the B operand): lane l holds column l % 32 and, in
// accumulator v, row 8 (v / 4) + 4 (l / 32) + v % 4. Both operands take
// the 16 bytes 32 t + 16 (l / 32) .. + 15 of their row for instruction t,
// so the k order is the same on both sides. Each lane keeps the running
// (best, index, second) of its A row over the B rows it holds, in
// increasing index; the lane pair and the four wavefronts are merged with
// the tie rule at the end.
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

struct BestM {
    int idx = -1;
    int d1 = INT_MAX, d2 = INT_MAX;
    // merge another state: smallest distance, then lowest index; the second
    // distance is the smallest over everything but the winner
    __device__ __forceinline__ void merge(int oidx, int od1, int od2)
    {
        const bool other = od1 < d1 || (od1 == d1 && oidx >= 0 && (idx < 0 || oidx < idx));
        if (other) {
            d2 = min(od2, d1);
            d1 = od1;
            idx = oidx;
        } else {
            d2 = min(d2, od1);
        }
    }
};

constexpr int kRankThreads = 1024;                 // sixteen wavefronts
constexpr int kRankWaves = kRankThreads / 64;
constexpr int kRankTile = 32 * kRankWaves;           // B rows per tile: 32 per wavefront

template <int KB, int NA>
__global__ void __launch_bounds__(kRankThreads) match_rank_mfma_kernel(const MatchArgs a)
{
    constexpr int RB = 32 * KB;                        // bytes per row
    constexpr int RW = RB / 4;                         // words per row
    constexpr int PITCH = RB + 16;                     // LDS row pitch (bytes)
    __shared__ __align__(16) unsigned char tb[kRankTile * PITCH];
    __shared__ int tn[kRankTile];                      // |b - 128|^2 of the tile's rows
    __shared__ int pidx[kRankWaves][32 * NA], pd1[kRankWaves][32 * NA], pd2[kRankWaves][32 * NA];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int n = lane & 31, h = lane >> 5;
    // A operands of this lane's NA rows (32 apart): 16 bytes per
    // instruction, shifted to signed bytes
    v4i aop[NA][KB];
    int na[NA];
#pragma unroll
    for (int g = 0; g < NA; ++g) {
        const int i = (blockIdx.x * NA + g) * 32 + n;
        const bool live = i < a.n_a;
        na[g] = 0;
#pragma unroll
        for (int t = 0; t < KB; ++t) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const unsigned w = live ? a.a[(size_t)i * RW + 8 * t + 4 * h + q] : 0x80808080u;
                aop[g][t][q] = (int)(w ^ 0x80808080u);
                na[g] = __builtin_amdgcn_sdot4(aop[g][t][q], aop[g][t][q], na[g], false);
            }
        }
        na[g] += __shfl_xor(na[g], 32);                // the other half of the row
    }
    BestM best[NA];
    for (int j0 = 0; j0 < a.n_b; j0 += kRankTile) {
        const int rows = min(kRankTile, a.n_b - j0);
        __syncthreads();   // the previous tile is no longer read
        for (int e = tid; e < rows * RW; e += kRankThreads) {
            const int r = e / RW, c = e - r * RW;
            *reinterpret_cast<unsigned *>(tb + r * PITCH + 4 * c) = a.b[(size_t)j0 * RW + e] ^ 0x80808080u;
        }
        __syncthreads();
        if (tid < rows) {
            int q = 0;
#pragma unroll
            for (int c = 0; c < RB / 16; ++c) {
                const v4i x = *reinterpret_cast<const v4i *>(tb + tid * PITCH + 16 * c);
#pragma unroll
                for (int k = 0; k < 4; ++k) q = __builtin_amdgcn_sdot4(x[k], x[k], q, false);
            }
            tn[tid] = q;
        }
        __syncthreads();
        const int r0 = 32 * wave;                      // this wavefront's rows of the tile
        if (r0 >= rows) continue;                      // uniform per wavefront
        v16i acc[NA];
#pragma unroll
        for (int g = 0; g < NA; ++g) acc[g] = v16i{};
#pragma unroll
        for (int t = 0; t < KB; ++t) {
            const v4i bop = *reinterpret_cast<const v4i *>(tb + (r0 + n) * PITCH + 32 * t + 16 * h);
#pragma unroll
            for (int g = 0; g < NA; ++g) acc[g] = __builtin_amdgcn_mfma_i32_32x32x32_i8(bop, aop[g][t], acc[g], 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int r = r0 + 8 * (v >> 2) + 4 * h + (v & 3);
            if (r < rows) {
                const int nb = tn[r];
#pragma unroll
                for (int g = 0; g < NA; ++g) {
                    const int d = na[g] + nb - 2 * acc[g][v];
                    if (d < best[g].d1) {
                        best[g].d2 = best[g].d1;
                        best[g].d1 = d;
                        best[g].idx = j0 + r;
                    } else if (d < best[g].d2) {
                        best[g].d2 = d;
                    }
                }
            }
        }
    }
    // the two lanes of each A row, then the wavefronts
#pragma unroll
    for (int g = 0; g < NA; ++g) {
        const int oi = __shfl_xor(best[g].idx, 32), o1 = __shfl_xor(best[g].d1, 32), o2 = __shfl_xor(best[g].d2, 32);
        best[g].merge(oi, o1, o2);
        if (h == 0) {
            pidx[wave][32 * g + n] = best[g].idx;
            pd1[wave][32 * g + n] = best[g].d1;
            pd2[wave][32 * g + n] = best[g].d2;
        }
    }
    __syncthreads();
    if (tid < 32 * NA) {
        const int i = blockIdx.x * 32 * NA + tid;
        if (i < a.n_a) {
            BestM m;
            for (int w = 0; w < kRankWaves; ++w) m.merge(pidx[w][tid], pd1[w][tid], pd2[w][tid]);
            a.idx[i] = m.idx;
            a.d1[i] = m.d1;
            a.d2[i] = m.d2;
        }
    }
}

// Rows of 128 bytes or more: two A blocks per workgroup (half the tile
// traffic per pair; measured 606 -> 414 us for 16384 x 16384 rows of 256).
// Rows of 64 bytes: one block (135 against 142 us with two).
template <int KB>
void launch_rank_mfma(const MatchArgs &m, hipStream_t st)
{
    constexpr int NA = KB >= 4 ? 2 : 1;
    hipLaunchKernelGGL((match_rank_mfma_kernel<KB, NA>), dim3((m.n_a + 32 * NA - 1) / (32 * NA)), dim3(kRankThreads),
                       0, st, m);
}

template <int W>
void launch_w(const MatchArgs &m, hipStream_t st)
{
    const int grid = (m.n_a + 63) / 64;
    hipLaunchKernelGGL((match_kernel<W>), dim3(grid), dim3(kMatchThreads), 0, st, m);
}

}  // namespace

hipError_t launch_match(int kind, const void *a, int n_a, const void *b, int n_b, int row_elems, int32_t *idx,
                        int32_t *d1, int32_t *d2, hipStream_t st)
{
    if (n_a <= 0) return hipSuccess;
    const MatchArgs m{static_cast<const uint32_t *>(a), static_cast<const uint32_t *>(b), n_a, n_b, idx, d1, d2};
    if (kind == 0) {   // row_elems = BRIEF words (64 bits)
        switch (row_elems) {
        case 1: launch_w<2>(m, st); break;
        case 2: launch_w<4>(m, st); break;
        case 3: launch_w<6>(m, st); break;
        case 4: launch_w<8>(m, st); break;
        default: return hipErrorInvalidValue;
        }
    } else {           // row_elems = ranks (bytes)
        switch (row_elems) {
        case 64: launch_rank_mfma<2>(m, st); break;
        case 128: launch_rank_mfma<4>(m, st); break;
        case 192: launch_rank_mfma<6>(m, st); break;
        case 256: launch_rank_mfma<8>(m, st); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

}  // namespace s3d
