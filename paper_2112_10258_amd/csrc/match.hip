// Nearest-neighbour matching of descriptors on gfx950: for every row of A,
// the nearest row of B, its distance and the second-smallest distance (for
// a ratio test). Keypoints are matched by their descriptors (Section 3.3):
//   BRIEF: rows of w 64-bit words, distance = Hamming distance (popcount of
//          the XOR);
//   ranks (SIFT-Rank, RRIEF): rows of m uint8 ranks, distance = squared
//          Euclidean distance = |a|^2 + |b|^2 - 2 a.b, the dot product from
//          unsigned 8-bit dot4 instructions on 32-bit words; exact integers.
// A workgroup owns 64 rows of A, one per lane, held in registers; B streams
// through LDS in tiles, and wavefront w of the four scans the w-th quarter
// of every tile (broadcast reads), in index order. The four partial results
// of a row are merged at the end in a fixed order: the smallest distance
// with the lowest index wins, and the second-smallest distance is the
// smaller of the winner's own second and the other quarters' best.
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

// KIND 0: W 32-bit words = W/2 BRIEF words; KIND 1: W words = 4W ranks.
template <int KIND, int W>
__global__ void __launch_bounds__(kMatchThreads) match_kernel(const MatchArgs a)
{
    constexpr int TILE = kMatchLdsWords / (W + (KIND == 1 ? 1 : 0));   // rows of B per tile
    __shared__ uint32_t tb[TILE * W];
    __shared__ int tn[KIND == 1 ? TILE : 1];                            // |b|^2 of the tile's rows
    __shared__ int pidx[kMatchWaves][64], pd1[kMatchWaves][64], pd2[kMatchWaves][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const bool live = i < a.n_a;
    uint32_t ra[W];
    int na = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) ra[w] = live ? a.a[(size_t)i * W + w] : 0u;
    if constexpr (KIND == 1) {
#pragma unroll
        for (int w = 0; w < W; ++w) na = (int)__builtin_amdgcn_udot4(ra[w], ra[w], (unsigned)na, false);
    }
    Best best;
    for (int j0 = 0; j0 < a.n_b; j0 += TILE) {
        const int rows = min(TILE, a.n_b - j0);
        __syncthreads();   // the previous tile is no longer read
        for (int e = threadIdx.x; e < rows * W; e += kMatchThreads) tb[e] = a.b[(size_t)j0 * W + e];
        if constexpr (KIND == 1) {
            __syncthreads();
            for (int r = threadIdx.x; r < rows; r += kMatchThreads) {
                unsigned s = 0;
#pragma unroll
                for (int w = 0; w < W; ++w) s = __builtin_amdgcn_udot4(tb[r * W + w], tb[r * W + w], s, false);
                tn[r] = (int)s;
            }
        }
        __syncthreads();
        // this wavefront's quarter of the tile
        const int q = (rows + kMatchWaves - 1) / kMatchWaves;
        const int r0 = wave * q, r1 = min(rows, r0 + q);
        if (live) {
            for (int r = r0; r < r1; ++r) {
                int d;
                if constexpr (KIND == 0) {
                    d = 0;
#pragma unroll
                    for (int w = 0; w < W; ++w) d += __popc(ra[w] ^ tb[r * W + w]);
                } else {
                    unsigned dot = 0;
#pragma unroll
                    for (int w = 0; w < W; ++w) dot = __builtin_amdgcn_udot4(ra[w], tb[r * W + w], dot, false);
                    d = na + tn[r] - 2 * (int)dot;
                }
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

template <int KIND, int W>
void launch_w(const MatchArgs &m, hipStream_t st)
{
    const int grid = (m.n_a + 63) / 64;
    hipLaunchKernelGGL((match_kernel<KIND, W>), dim3(grid), dim3(kMatchThreads), 0, st, m);
}

}  // namespace

hipError_t launch_match(int kind, const void *a, int n_a, const void *b, int n_b, int row_elems, int32_t *idx,
                        int32_t *d1, int32_t *d2, hipStream_t st)
{
    if (n_a <= 0) return hipSuccess;
    const MatchArgs m{static_cast<const uint32_t *>(a), static_cast<const uint32_t *>(b), n_a, n_b, idx, d1, d2};
    if (kind == 0) {   // row_elems = BRIEF words (64 bits)
        switch (row_elems) {
        case 1: launch_w<0, 2>(m, st); break;
        case 2: launch_w<0, 4>(m, st); break;
        case 3: launch_w<0, 6>(m, st); break;
        case 4: launch_w<0, 8>(m, st); break;
        default: return hipErrorInvalidValue;
        }
    } else {           // row_elems = ranks (bytes)
        switch (row_elems) {
        case 64: launch_w<1, 16>(m, st); break;
        case 128: launch_w<1, 32>(m, st); break;
        case 192: launch_w<1, 48>(m, st); break;
        case 256: launch_w<1, 64>(m, st); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

}  // namespace s3d
