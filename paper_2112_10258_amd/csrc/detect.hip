// 4D extremum detection and ordered compaction (Section 3.2.2, 4D Peak
// Detection). A voxel of DoG level s is kept when |D_s| exceeds the
// threshold and the sum over its 80 neighbours (3x3x3 blocks of D_{s-1} and
// D_{s+1}, the other 26 of D_s) of sign(D_s(v) - neighbour) reaches
// +votes (peak) or -votes (valley).
//
// The candidate space of all volumes and octaves is cut into "rows": (volume,
// octave, s, z, y) over the x range, enumerated in canonical order, each
// volume starting on a block of kRowBlock rows. Launches turn the per-voxel
// test into per-volume keypoint lists in that order without a sort and
// without atomics:
//   test:  per-row keypoint counts (and, on the strict path, bit masks);
//   scan:  one workgroup scans the per-block counts (exclusive) and writes
//          each volume's total;
//   emit:  blocks with keypoints write each one at (block offset - the
//          volume's first offset) + row prefix + rank within the row.
#include <type_traits>

#include "sift3d_internal.h"

namespace s3d {
namespace {

template <typename F>
__device__ __forceinline__ int last_le(int n, F key, long long v)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (key(mid) <= v)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// INL: units from the inline copy in the arguments, else from the device table.
template <bool INL>
__device__ __forceinline__ const DUnit &unit_at(const DetLaunch &a, int i)
{
    return INL ? a.inl[i] : a.units[i];
}

struct RowPos {
    int u, s, y, z;
    bool valid;
};

// Unit and (s, z, y) of global row g; invalid for padding rows.
template <bool INL>
__device__ __forceinline__ RowPos decode_row(const DetLaunch &a, long long g)
{
    RowPos p;
    p.u = last_le(a.n_units, [&](int i) { return unit_at<INL>(a, i).row_base; }, g);
    const DUnit &un = unit_at<INL>(a, p.u);
    const long long r = g - un.row_base;
    p.valid = r >= 0 && r < un.rows;
    if (!p.valid) {
        p.s = p.y = p.z = 0;
        return p;
    }
    const long long per_s = (long long)(un.nz - 2) * (un.ny - 2);
    p.s = 1 + (int)(r / per_s);
    const long long rem = r - (long long)(p.s - 1) * per_s;
    p.z = 1 + (int)(rem / (un.ny - 2));
    p.y = 1 + (int)(rem - (long long)(p.z - 1) * (un.ny - 2));
    return p;
}

__device__ __forceinline__ const float *unit_D(const DetLaunch &a, const DUnit &un)
{
    return reinterpret_cast<const float *>(a.ws + un.g0) + un.lstride * (a.S + 3);
}

__device__ __forceinline__ void write_keypoint(const DetLaunch &a, const DUnit &un, int idx, int x, int y, int z,
                                               int s, int pol, float v)
{
    sift3d_keypoint k;
    k.x = x;
    k.y = y;
    k.z = z;
    k.octave = (int16_t)un.octave;
    k.scale = (int16_t)s;
    k.polarity = (int8_t)pol;
    k.pad[0] = k.pad[1] = k.pad[2] = 0;
    k.dog = v;
    const float f = (float)(1 << un.octave);
    const float h = 0.5f * (f - 1.f);
    k.xf = f * (float)x + h;
    k.yf = f * (float)y + h;
    k.zf = f * (float)z + h;
    k.sigma = un.sigma[s];
    a.kp[(size_t)un.vol * a.cap + idx] = k;
}

// Offset of the first keypoint of volume v in the global order.
__device__ __forceinline__ int volume_base(const DetLaunch &a, int v)
{
    return a.block_off[a.vols[v].row_base / a.rows_per_block];
}

// ---------------------------------------------------------------- general path (votes < 80)

// +1 peak, -1 valley, 0 otherwise. v = D_s at the voxel; c points at it in D_s.
// Neighbours are read one 3x3 plane at a time; the test stops as soon as
// neither |f| >= votes outcome is reachable.
__device__ __forceinline__ int extremum(const float *c, long long lstride, int nx, long long nxy,
                                        float v, int votes)
{
    int pos = 0, neg = 0, done = 0;
    // plane order: the centre level first (most selective), then below, then above
    const long long lev[3] = {0, -lstride, lstride};
#pragma unroll
    for (int l = 0; l < 3; ++l) {
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz) {
            const float *p = c + lev[l] + dz * nxy;
            float nb[9];
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) nb[(dy + 1) * 3 + dx + 1] = p[dy * nx + dx];
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                if (l == 0 && dz == 0 && q == 4) continue;  // the voxel itself
                pos += v > nb[q];
                neg += v < nb[q];
                ++done;
            }
            const int left = 80 - done;
            if (pos - neg + left < votes && neg - pos + left < votes) return 0;
        }
    }
    const int f = pos - neg;
    return f >= votes ? 1 : (f <= -votes ? -1 : 0);
}

// Count (EMIT = false) or write (EMIT = true) the keypoints of one row.
template <bool EMIT, bool INL>
__device__ int process_row(const DetLaunch &a, long long g, int lane, int base)
{
    const RowPos rp = decode_row<INL>(a, g);
    if (!rp.valid) return 0;
    const DUnit &un = unit_at<INL>(a, rp.u);
    const long long nxy = (long long)un.nx * un.ny;
    const float *Ds = unit_D(a, un) + un.lstride * rp.s;
    const long long row = (long long)rp.z * nxy + (long long)rp.y * un.nx;
    int total = 0;
    for (int xb = 1; xb <= un.nx - 2; xb += 64) {
        const int x = xb + lane;
        int pol = 0;
        float v = 0.f;
        if (x <= un.nx - 2) {
            v = Ds[row + x];
            if (fabsf(v) > a.thr) pol = extremum(Ds + row + x, un.lstride, un.nx, nxy, v, a.votes);
        }
        const unsigned long long m = __ballot(pol != 0);
        if constexpr (EMIT) {
            if (pol != 0) {
                const int idx = base + total + __popcll(m & ((1ull << lane) - 1ull));
                if (idx < a.cap) write_keypoint(a, un, idx, x, rp.y, rp.z, rp.s, pol, v);
            }
        }
        total += __popcll(m);
    }
    return total;
}

template <bool INL>
__global__ void __launch_bounds__(kDetThreads) detect_count_kernel(const DetLaunch a)
{
    __shared__ int wsum[kDetThreads / 64];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const long long row0 = (long long)blockIdx.x * kDetRowsPerBlock + wave * kDetRowsPerWave;
    int sum = 0;
    for (int rr = 0; rr < kDetRowsPerWave; ++rr) {
        const long long g = row0 + rr;
        if (g >= a.total_rows) break;
        const int c = process_row<false, INL>(a, g, lane, 0);
        if (lane == 0) a.row_count[g] = c;
        sum += c;
    }
    if (lane == 0) wsum[wave] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kDetThreads / 64; ++w) t += wsum[w];
        a.block_sum[blockIdx.x] = t;
    }
}

template <bool INL>
__global__ void __launch_bounds__(kDetThreads) detect_emit_kernel(const DetLaunch a)
{
    __shared__ int roff[kDetRowsPerBlock];
    if (a.block_sum[blockIdx.x] == 0) return;
    const long long row0 = (long long)blockIdx.x * kDetRowsPerBlock;
    const RowPos first = decode_row<INL>(a, row0);
    const int vbase = volume_base(a, unit_at<INL>(a, first.u).vol);
    if (a.block_off[blockIdx.x] - vbase >= a.cap) return;
    if (threadIdx.x == 0) {
        int run = a.block_off[blockIdx.x] - vbase;
        for (int r = 0; r < kDetRowsPerBlock; ++r) {
            roff[r] = run;
            if (row0 + r < a.total_rows) run += a.row_count[row0 + r];
        }
    }
    __syncthreads();
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int rr = 0; rr < kDetRowsPerWave; ++rr) {
        const int r = wave * kDetRowsPerWave + rr;
        const long long g = row0 + r;
        if (g >= a.total_rows) break;
        if (a.row_count[g] == 0) continue;
        process_row<true, INL>(a, g, lane, roff[r]);
    }
}

// ---------------------------------------------------------------- scan

// Exclusive scan of the block counts (one workgroup) and per-volume totals.
__global__ void __launch_bounds__(kScanThreads) detect_scan_kernel(const DetLaunch a)
{
    __shared__ int part[kScanThreads];
    const int tid = threadIdx.x;
    const int n = a.n_blocks;
    const int per = (n + kScanThreads - 1) / kScanThreads;
    const int b0 = min(tid * per, n), b1 = min(b0 + per, n);
    int s = 0;
    for (int b = b0; b < b1; ++b) s += a.block_sum[b];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = tid ? part[tid - 1] : 0;
    for (int b = b0; b < b1; ++b) {
        a.block_off[b] = run;
        run += a.block_sum[b];
    }
    // keypoints of volume v = prefix(first block of v+1) - prefix(first block of v),
    // with prefix(b) the exclusive sum of block_sum[0..b): the thread-level
    // partials in LDS plus at most `per` block sums
    auto prefix = [&](long long b) -> int {
        if (b >= n) return part[kScanThreads - 1];
        const int t = (int)(b / per);
        int r = t ? part[t - 1] : 0;
        for (long long q = (long long)t * per; q < b; ++q) r += a.block_sum[q];
        return r;
    };
    for (int v = tid; v < a.n_vol; v += kScanThreads) {
        if (per == 0) {
            a.counts[v] = 0;
            continue;
        }
        const long long f = a.vols[v].row_base / a.rows_per_block;
        const long long l = v + 1 < a.n_vol ? a.vols[v + 1].row_base / a.rows_per_block : n;
        a.counts[v] = prefix(l) - prefix(f);
    }
}

// ---------------------------------------------------------------- strict path (votes == 80)
// With votes == 80 the sum-of-signs test accepts v exactly when v is above
// (peak) or below (valley) every one of its 80 neighbours, i.e. above the
// maximum or below the minimum of them. For scale s that neighbour maximum
// is the max over the 3x3x3 blocks of D_{s-1} and D_{s+1}, the 3x3 (x, y)
// blocks of D_s at z-1 and z+1, and the 8-voxel ring of D_s at z.
//
// One wavefront loads 64 consecutive x (lanes 0 and 63 are halo, lanes
// 1..62 produce) of WY consecutive y rows and streams z through a slab: per
// plane and level it loads the WY + 2 rows y0-1 .. y0+WY (coalesced), takes
// x neighbours from the adjacent lanes with DPP whole-wave shifts, reduces
// each loaded row over x once, and combines three such rows per output row;
// the 3x3 max/min of the last three planes stay in registers. The next
// plane is loaded before the current one is reduced. No LDS, no barriers.
// Ballots of the flags are the 64-bit words of the per-row keypoint bit
// masks (bit l of word t is x = 62 t + l).

// Rows y0-1 .. y0+WY of plane pz of every level, as buffer loads: each
// plane is a buffer resource built in scalar registers (base, size), the
// per-lane part is a 32-bit byte offset inside the plane (a plane is at
// most 2^30 floats), so a load costs no per-lane address arithmetic (plain
// global loads made the compiler add a 64-bit per-lane address for every
// row). Offsets stay inside the plane (clamped rows, clamped x).
constexpr int kRawBufferWord3 = 0x00020000;   // dword 3 of a raw (untyped) buffer resource on gfx9
constexpr unsigned kDropOffset = 0x80000000u;  // past any resource here: the store is dropped
typedef unsigned u32x2 __attribute__((__vector_size__(8)));

template <int NL, int NR>
__device__ __forceinline__ void load_plane_rows(const float *D, long long lstride, long long nxy, int pz,
                                                const unsigned (&boff)[NR], float (&v)[NL][NR])
{
    const int bytes = (int)(unsigned)min(nxy * 4, 0xffffffffLL);   // bound of the offsets (unsigned)
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        const float *pl = D + lstride * l + (long long)pz * nxy;
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(pl), (short)0, bytes, kRawBufferWord3);
#pragma unroll
        for (int r = 0; r < NR; ++r)
            v[l][r] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (int)boff[r], 0, 0));
    }
}

// f(std::integral_constant<int, P>) for P = I .. N-1 (compile-time P in f).
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// Value of the lane to the left / right (whole-wave DPP shift). Lane 0
// (left) and lane 63 (right) have no source and read 0: they are halo
// lanes, whose own results are never used.
__device__ __forceinline__ float from_left(float v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ float from_right(float v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true); }

template <int S, bool INL>
__global__ void __launch_bounds__(256) detect_tile_kernel(const DetLaunch a)
{
    constexpr int NL = S + 2;
    constexpr int WY = kDTWY;          // output rows per wavefront
    constexpr int NR = WY + 2;         // loaded rows per plane and level
    const int u = last_le(a.n_units, [&](int i) { return (long long)unit_at<INL>(a, i).tile_block0; }, blockIdx.x);
    const DUnit &un = unit_at<INL>(a, u);
    const float *D = unit_D(a, un);
    unsigned long long *masks = reinterpret_cast<unsigned long long *>(a.scr + un.masks);
    const int local = blockIdx.x - un.tile_block0;
    const int txi = local % un.tiles_x;
    const int rest = local / un.tiles_x;
    const int tyi = rest % un.tiles_y, tzi = rest / un.tiles_y;
    // the wavefront index is uniform: keep it (and every row address) scalar
    const int lane = threadIdx.x & 63, wy = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nx = un.nx, ny = un.ny, nz = un.nz, words = un.words;
    const int xl = txi * kDTXOut + lane;             // this lane's column
    const int y0 = 1 + tyi * kDTY + wy * WY;         // first output row of this wavefront
    if (y0 > ny - 2) return;                         // whole wavefront: no row here
    const int z0 = 1 + tzi * kDTZ;
    const int z1 = min(z0 + kDTZ, nz - 1);           // outputs z0 .. z1-1 (interior)
    const int x = min(xl, nx - 1);
    const bool in_x = lane >= 1 && lane <= kDTXOut && xl <= nx - 2;
    const float thr = a.thr;

    // Rings over the planes, indexed by plane number: M/m[l][k % 3][r] = 3x3
    // max/min of level l around output row r at plane k, cen/rx/rn[s][k %
    // 2][r] = centre value and 8-ring max/min of D_s at plane k, v[k % 2] =
    // the rows of plane k (the plane loop is unrolled by 6, so every slot is
    // a fixed register).
    float M[NL][3][WY], m[NL][3][WY];
    float cen[S + 1][2][WY], rx[S + 1][2][WY], rn[S + 1][2][WY];
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int r = 0; r < WY; ++r) M[l][q][r] = m[l][q][r] = 0.f;
#pragma unroll
    for (int l = 0; l <= S; ++l)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < WY; ++r) cen[l][q][r] = rx[l][q][r] = rn[l][q][r] = 0.f;

    const long long nxy = (long long)nx * ny;
    unsigned roff[NR];   // byte offsets of rows y0-1 .. y0+WY at column x
#pragma unroll
    for (int r = 0; r < NR; ++r) roff[r] = 4u * (unsigned)(min(max(y0 - 1 + r, 0), ny - 1) * nx + x);
    // Mask words go out through a buffer resource: every plane step issues
    // the same loads and stores (a step past the slab re-reads its last
    // plane, and a store with nothing to write goes to an offset past the
    // resource, which the hardware drops), so the waits before each plane's
    // use count exactly the loads issued after it.
    const unsigned mask_bytes = (unsigned)min((long long)S * (nz - 2) * (ny - 2) * words * 8, 0x7fffffffLL);
    const __amdgpu_buffer_rsrc_t mrs = __builtin_amdgcn_make_buffer_rsrc(masks, (short)0, (int)mask_bytes,
                                                                         kRawBufferWord3);
    // plane k (z = z0 - 1 + k) sits in buffer k % 3: loads run two planes ahead
    float v[3][NL][NR];
    const int nplanes = (z1 - z0) + 2;   // >= 3
    load_plane_rows<NL, NR>(D, un.lstride, nxy, z0 - 1, roff, v[0]);
    load_plane_rows<NL, NR>(D, un.lstride, nxy, z0, roff, v[1]);
    for (int base = 0; base < nplanes; base += 6) {
        static_for<0, 6>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            constexpr int b = p % 3, nb = (p + 2) % 3;          // plane buffers of k, k+2
            constexpr int q0 = (p + 1) % 3, q1 = (p + 2) % 3, q2 = p % 3;   // M slots of k-2, k-1, k
            constexpr int c0 = (p + 1) % 2, c1 = p % 2;          // cen/rx/rn slots of k-1, k
            const int k = base + p;
            load_plane_rows<NL, NR>(D, un.lstride, nxy, z0 - 1 + min(k + 2, nplanes - 1), roff, v[nb]);
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                // each loaded row reduced over x once
                float hx[NR], hn[NR], lf[NR], rt[NR];
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    lf[r] = from_left(v[b][l][r]);
                    rt[r] = from_right(v[b][l][r]);
                    hx[r] = fmaxf(fmaxf(lf[r], rt[r]), v[b][l][r]);
                    hn[r] = fminf(fminf(lf[r], rt[r]), v[b][l][r]);
                }
#pragma unroll
                for (int r = 0; r < WY; ++r) {
                    M[l][q2][r] = fmaxf(fmaxf(hx[r], hx[r + 1]), hx[r + 2]);
                    m[l][q2][r] = fminf(fminf(hn[r], hn[r + 1]), hn[r + 2]);
                    if (l >= 1 && l <= S) {
                        cen[l][c1][r] = v[b][l][r + 1];
                        rx[l][c1][r] = fmaxf(fmaxf(hx[r], hx[r + 2]), fmaxf(lf[r + 1], rt[r + 1]));
                        rn[l][c1][r] = fminf(fminf(hn[r], hn[r + 2]), fminf(lf[r + 1], rt[r + 1]));
                    }
                }
            }
            {
                const int z = z0 + k - 2;                // output plane of this step
                const bool zlive = k >= 2 && k < nplanes;
#pragma unroll
                for (int r = 0; r < WY; ++r) {
                    const int y = y0 + r;
                    const bool live = zlive && y <= ny - 2;   // the same for the whole wavefront
                    const long long row_z = (long long)(z - 1) * (ny - 2) + (y - 1);
                    // 3x3x3 max / min of every level around (x, y, z), once per level
                    float ZX[NL], ZN[NL];
#pragma unroll
                    for (int l = 0; l < NL; ++l) {
                        ZX[l] = fmaxf(fmaxf(M[l][q0][r], M[l][q1][r]), M[l][q2][r]);
                        ZN[l] = fminf(fminf(m[l][q0][r], m[l][q1][r]), m[l][q2][r]);
                    }
#pragma unroll
                    for (int s = 1; s <= S; ++s) {
                        const float vv = cen[s][c0][r];
                        const float mx = fmaxf(fmaxf(ZX[s - 1], ZX[s + 1]),
                                               fmaxf(fmaxf(M[s][q0][r], M[s][q2][r]), rx[s][c0][r]));
                        const float mn = fminf(fminf(ZN[s - 1], ZN[s + 1]),
                                               fminf(fminf(m[s][q0][r], m[s][q2][r]), rn[s][c0][r]));
                        // evaluated in full (no short-circuit branches)
                        const bool flag = in_x & (fabsf(vv) > thr) & ((vv > mx) | (vv < mn));
                        const unsigned long long bits = __ballot(flag);
                        const long long row = (long long)(s - 1) * (nz - 2) * (ny - 2) + row_z;
                        const unsigned woff = (unsigned)((row * words + txi) * 8);
                        const unsigned off = live && lane == 0 ? woff : kDropOffset;
                        const u32x2 w = {(unsigned)bits, (unsigned)(bits >> 32)};
                        __builtin_amdgcn_raw_buffer_store_b64(w, mrs, (int)off, 0, 0);
                    }
                }
            }
        });
    }
}

// Keypoints per row (popcount of its words) and per block of kRowBlock rows.
template <bool INL>
__global__ void __launch_bounds__(kRowBlock) row_count_kernel(const DetLaunch a)
{
    __shared__ int wsum[kRowBlock / 64];
    const long long g = (long long)blockIdx.x * kRowBlock + threadIdx.x;
    int c = 0;
    if (g < a.total_rows) {
        const RowPos rp = decode_row<INL>(a, g);
        if (rp.valid) {
            const DUnit &un = unit_at<INL>(a, rp.u);
            const unsigned long long *w =
                reinterpret_cast<const unsigned long long *>(a.scr + un.masks) + (g - un.row_base) * un.words;
            for (int q = 0; q < un.words; ++q) c += __popcll(w[q]);
        }
        a.row_count[g] = c;
    }
    int t = c;
    for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x / 64] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        int b = 0;
        for (int q = 0; q < kRowBlock / 64; ++q) b += wsum[q];
        a.block_sum[blockIdx.x] = b;
    }
}

// Keypoint records in canonical order: row offset = block offset - volume
// offset + prefix of the block's row counts; within a row, x ascending.
template <bool INL>
__global__ void __launch_bounds__(kRowBlock) emit_rows_kernel(const DetLaunch a)
{
    __shared__ int pre[kRowBlock];
    if (a.block_sum[blockIdx.x] == 0) return;
    const long long row0 = (long long)blockIdx.x * kRowBlock;
    const RowPos first = decode_row<INL>(a, row0);
    const int vbase = volume_base(a, unit_at<INL>(a, first.u).vol);
    if (a.block_off[blockIdx.x] - vbase >= a.cap) return;
    const long long g = row0 + threadIdx.x;
    const int c = g < a.total_rows ? a.row_count[g] : 0;
    pre[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < kRowBlock; off <<= 1) {
        const int v = threadIdx.x >= off ? pre[threadIdx.x - off] : 0;
        __syncthreads();
        pre[threadIdx.x] += v;
        __syncthreads();
    }
    if (c == 0) return;
    int idx = a.block_off[blockIdx.x] - vbase + pre[threadIdx.x] - c;
    const RowPos rp = decode_row<INL>(a, g);
    const DUnit &un = unit_at<INL>(a, rp.u);
    const long long r = g - un.row_base;
    const long long nxy = (long long)un.nx * un.ny;
    const float *Ds = unit_D(a, un) + un.lstride * rp.s;
    const unsigned long long *mw = reinterpret_cast<const unsigned long long *>(a.scr + un.masks) + r * un.words;
    for (int q = 0; q < un.words && idx < a.cap; ++q) {
        unsigned long long w = mw[q];
        while (w != 0ull && idx < a.cap) {
            const int x = kDTXOut * q + (__ffsll((long long)w) - 1);
            w &= w - 1ull;
            const long long vi = (long long)rp.z * nxy + (long long)rp.y * un.nx + x;
            const float v = Ds[vi];
            // a strict extremum differs from every neighbour: one decides peak or valley
            const bool peak = v > Ds[vi + 1];
            write_keypoint(a, un, idx++, x, rp.y, rp.z, rp.s, peak ? 1 : -1, v);
        }
    }
}

template <int S, bool INL>
hipError_t launch_strict(const DetLaunch &a, hipStream_t st)
{
    hipLaunchKernelGGL((detect_tile_kernel<S, INL>), dim3(a.tile_blocks), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(row_count_kernel<INL>, dim3(a.n_blocks), dim3(kRowBlock), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(detect_scan_kernel, dim3(1), dim3(kScanThreads), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(emit_rows_kernel<INL>, dim3(a.n_blocks), dim3(kRowBlock), 0, st, a);
    return hipGetLastError();
}

template <bool INL>
hipError_t launch_general(const DetLaunch &a, hipStream_t st)
{
    hipLaunchKernelGGL(detect_count_kernel<INL>, dim3(a.n_blocks), dim3(kDetThreads), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(detect_scan_kernel, dim3(1), dim3(kScanThreads), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(detect_emit_kernel<INL>, dim3(a.n_blocks), dim3(kDetThreads), 0, st, a);
    return hipGetLastError();
}

template <bool INL>
hipError_t launch_strict_s(const DetLaunch &a, hipStream_t st)
{
    switch (a.S) {
    case 1: return launch_strict<1, INL>(a, st);
    case 2: return launch_strict<2, INL>(a, st);
    case 3: return launch_strict<3, INL>(a, st);
    case 4: return launch_strict<4, INL>(a, st);
    case 5: return launch_strict<5, INL>(a, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_detect(const DetLaunch &in, hipStream_t st)
{
    DetLaunch a = in;
    const bool inl = a.n_units <= kInlineUnits;
    if (a.votes == 80) {
        a.rows_per_block = kRowBlock;
        a.n_blocks = (int)((a.total_rows + kRowBlock - 1) / kRowBlock);
        return inl ? launch_strict_s<true>(a, st) : launch_strict_s<false>(a, st);
    }
    a.rows_per_block = kDetRowsPerBlock;
    a.n_blocks = (int)((a.total_rows + kDetRowsPerBlock - 1) / kDetRowsPerBlock);
    return inl ? launch_general<true>(a, st) : launch_general<false>(a, st);
}

}  // namespace s3d
