// 4D extremum detection and ordered compaction (Section 3.2.2, 4D Peak
// Detection). A voxel of DoG level s is kept when |D_s| exceeds the
// threshold and the sum over its 80 neighbours (3x3x3 blocks of D_{s-1} and
// D_{s+1}, the other 26 of D_s) of sign(D_s(v) - neighbour) reaches
// +votes (peak) or -votes (valley).
//
// The candidate space of all octaves is cut into "rows": (octave, s, z, y)
// over the interior x range, enumerated in canonical order. Three launches
// turn the per-voxel test into a keypoint list in that order without a
// sort and without atomics:
//   count: one wavefront per row, wavefront ballots + popcount, per-row
//          and per-block counts;
//   scan:  one workgroup scans the block counts (exclusive) and writes the
//          total to the device-side count;
//   emit:  blocks with a non-zero count re-test their non-empty rows and
//          write each keypoint at block offset + row prefix + ballot rank.
#include "sift3d_internal.h"

namespace s3d {
namespace {

struct RowPos {
    int o, s, y, z;
};

__device__ __forceinline__ RowPos decode_row(const DetectArgs &a, long long g)
{
    int o = 0;
    for (int k = 1; k < a.n_oct; ++k)
        if (g >= a.oc[k].row_base) o = k;
    const DetOctave &oc = a.oc[o];
    const long long r = g - oc.row_base;
    const long long per_s = (long long)(oc.nz - 2) * (oc.ny - 2);
    RowPos p;
    p.o = o;
    p.s = 1 + (int)(r / per_s);
    const long long rem = r - (long long)(p.s - 1) * per_s;
    p.z = 1 + (int)(rem / (oc.ny - 2));
    p.y = 1 + (int)(rem - (long long)(p.z - 1) * (oc.ny - 2));
    return p;
}

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
template <bool EMIT>
__device__ int process_row(const DetectArgs &a, long long g, int lane, int base)
{
    const RowPos rp = decode_row(a, g);
    const DetOctave &oc = a.oc[rp.o];
    const long long nxy = (long long)oc.nx * oc.ny;
    const float *Ds = oc.D + oc.lstride * rp.s;
    const long long row = (long long)rp.z * nxy + (long long)rp.y * oc.nx;
    int total = 0;
    for (int xb = 1; xb <= oc.nx - 2; xb += 64) {
        const int x = xb + lane;
        int pol = 0;
        float v = 0.f;
        if (x <= oc.nx - 2) {
            v = Ds[row + x];
            if (fabsf(v) > a.thr) pol = extremum(Ds + row + x, oc.lstride, oc.nx, nxy, v, a.votes);
        }
        const unsigned long long m = __ballot(pol != 0);
        if constexpr (EMIT) {
            if (pol != 0) {
                const int idx = base + total + __popcll(m & ((1ull << lane) - 1ull));
                if (idx < a.cap) {
                    sift3d_keypoint k;
                    k.x = x;
                    k.y = rp.y;
                    k.z = rp.z;
                    k.octave = (int16_t)rp.o;
                    k.scale = (int16_t)rp.s;
                    k.polarity = (int8_t)pol;
                    k.pad[0] = k.pad[1] = k.pad[2] = 0;
                    k.dog = v;
                    const float f = (float)(1 << rp.o);
                    const float h = 0.5f * (f - 1.f);
                    k.xf = f * (float)x + h;
                    k.yf = f * (float)rp.y + h;
                    k.zf = f * (float)rp.z + h;
                    k.sigma = oc.sigma[rp.s];
                    a.kp[idx] = k;
                }
            }
        }
        total += __popcll(m);
    }
    return total;
}

__global__ void __launch_bounds__(kDetThreads) detect_count_kernel(const DetectArgs a)
{
    __shared__ int wsum[kDetThreads / 64];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const long long row0 = (long long)blockIdx.x * kDetRowsPerBlock + wave * kDetRowsPerWave;
    int sum = 0;
    for (int rr = 0; rr < kDetRowsPerWave; ++rr) {
        const long long g = row0 + rr;
        if (g >= a.total_rows) break;
        const int c = process_row<false>(a, g, lane, 0);
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

__global__ void __launch_bounds__(kScanThreads) detect_scan_kernel(const DetectArgs a)
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
    if (tid == kScanThreads - 1) *a.d_count = part[kScanThreads - 1];
}

__global__ void __launch_bounds__(kDetThreads) detect_emit_kernel(const DetectArgs a)
{
    __shared__ int roff[kDetRowsPerBlock];
    if (a.block_sum[blockIdx.x] == 0) return;
    if (a.block_off[blockIdx.x] >= a.cap) return;
    const long long row0 = (long long)blockIdx.x * kDetRowsPerBlock;
    if (threadIdx.x == 0) {
        int run = a.block_off[blockIdx.x];
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
        process_row<true>(a, g, lane, roff[r]);
    }
}

// ---------------------------------------------------------------- strict path
// With votes == 80 the sum-of-signs test accepts v exactly when v is above
// (peak) or below (valley) every one of its 80 neighbours, i.e. above the
// maximum or below the minimum of them. For scale s that neighbour maximum
// is the max over the 3x3x3 blocks of D_{s-1} and D_{s+1}, the 3x3 (x, y)
// blocks of D_s at z-1 and z+1, and the 8-voxel ring of D_s at z.
//
// One wavefront owns 64 consecutive x of one y row and streams z through a
// slab: per plane and level it loads rows y-1, y, y+1 (coalesced), takes x
// neighbours from the adjacent lanes (the two edge lanes load theirs), and
// keeps 3x3 max/min of the last three planes in registers. The next plane is
// loaded before the current one is reduced. No LDS, no barriers. Ballots of
// the flags are the 64-bit words of the per-row keypoint bit masks.
template <int NL>
__device__ __forceinline__ void load_plane_rows(const DetOctave &oc, int pz, int x, int xe, int y,
                                                float (&v)[NL][3], float (&e)[NL][3])
{
    const long long nxy = (long long)oc.nx * oc.ny;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        const float *pl = oc.D + oc.lstride * l + pz * nxy;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const float *row = pl + (long long)min(max(y - 1 + r, 0), oc.ny - 1) * oc.nx;
            v[l][r] = row[x];
            e[l][r] = row[xe];
        }
    }
}

template <int S>
__global__ void __launch_bounds__(256) detect_tile_kernel(const DetectArgs a)
{
    constexpr int NL = S + 2;
    int o = 0;
    while (o + 1 < a.n_oct && (int)blockIdx.x >= a.oc[o + 1].block0) ++o;
    const DetOctave &oc = a.oc[o];
    const int local = blockIdx.x - oc.block0;
    const int txi = local % oc.tiles_x;
    const int rest = local / oc.tiles_x;
    const int tyi = rest % oc.tiles_y, tzi = rest / oc.tiles_y;
    const int lane = threadIdx.x & 63, wy = threadIdx.x >> 6;
    const int nx = oc.nx, ny = oc.ny, nz = oc.nz;
    const int x0 = txi * kDTX, y = 1 + tyi * kDTY + wy, z0 = 1 + tzi * kDTZ;
    if (y > ny - 2) return;                          // whole wavefront: no row here
    const int z1 = min(z0 + kDTZ, nz - 1);           // outputs z0 .. z1-1 (interior)
    const int x = min(x0 + lane, nx - 1);
    // lane 0 fetches x0-1, lane 63 fetches x0+64 (clamped); others a duplicate
    const int xe = lane == 0 ? max(x0 - 1, 0) : min(x0 + 64, nx - 1);
    const bool in_x = x0 + lane >= 1 && x0 + lane <= nx - 2;

    float M[NL][3], m[NL][3];
    float cen[S + 1][2], rx[S + 1][2], rn[S + 1][2];   // [.][0] previous plane, [.][1] current
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
        for (int q = 0; q < 3; ++q) M[l][q] = m[l][q] = 0.f;
#pragma unroll
    for (int l = 0; l <= S; ++l) cen[l][0] = cen[l][1] = rx[l][0] = rx[l][1] = rn[l][0] = rn[l][1] = 0.f;

    float v[NL][3], e[NL][3], vn[NL][3], en[NL][3];
    load_plane_rows<NL>(oc, z0 - 1, x, xe, y, v, e);
    const int nplanes = (z1 - z0) + 2;
    for (int k = 0; k < nplanes; ++k) {
        if (k + 1 < nplanes) load_plane_rows<NL>(oc, z0 + k, x, xe, y, vn, en);
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            float hx[3], hn[3], left1 = 0.f, right1 = 0.f;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                float left = __shfl_up(v[l][r], 1);
                float right = __shfl_down(v[l][r], 1);
                if (lane == 0) left = e[l][r];
                if (lane == 63) right = e[l][r];
                hx[r] = fmaxf(fmaxf(left, right), v[l][r]);
                hn[r] = fminf(fminf(left, right), v[l][r]);
                if (r == 1) {
                    left1 = left;
                    right1 = right;
                }
            }
            M[l][0] = M[l][1];
            M[l][1] = M[l][2];
            M[l][2] = fmaxf(fmaxf(hx[0], hx[1]), hx[2]);
            m[l][0] = m[l][1];
            m[l][1] = m[l][2];
            m[l][2] = fminf(fminf(hn[0], hn[1]), hn[2]);
            if (l >= 1 && l <= S) {
                cen[l][0] = cen[l][1];
                cen[l][1] = v[l][1];
                rx[l][0] = rx[l][1];
                rx[l][1] = fmaxf(fmaxf(hx[0], hx[2]), fmaxf(left1, right1));
                rn[l][0] = rn[l][1];
                rn[l][1] = fminf(fminf(hn[0], hn[2]), fminf(left1, right1));
            }
        }
        if (k >= 2) {
            const int z = z0 + k - 2;
            const long long row_z = (long long)(z - 1) * (ny - 2) + (y - 1);
#pragma unroll
            for (int s = 1; s <= S; ++s) {
                const float vv = cen[s][0];
                float mx = fmaxf(fmaxf(M[s - 1][0], M[s - 1][1]), M[s - 1][2]);
                mx = fmaxf(mx, fmaxf(fmaxf(M[s + 1][0], M[s + 1][1]), M[s + 1][2]));
                mx = fmaxf(mx, fmaxf(fmaxf(M[s][0], M[s][2]), rx[s][0]));
                float mn = fminf(fminf(m[s - 1][0], m[s - 1][1]), m[s - 1][2]);
                mn = fminf(mn, fminf(fminf(m[s + 1][0], m[s + 1][1]), m[s + 1][2]));
                mn = fminf(mn, fminf(fminf(m[s][0], m[s][2]), rn[s][0]));
                const bool flag = in_x && fabsf(vv) > a.thr && (vv > mx || vv < mn);
                const unsigned long long bits = __ballot(flag);
                if (lane == 0) {
                    const long long row = (long long)(s - 1) * (nz - 2) * (ny - 2) + row_z;
                    oc.masks[row * oc.words + txi] = bits;
                }
            }
        }
#pragma unroll
        for (int l = 0; l < NL; ++l)
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                v[l][r] = vn[l][r];
                e[l][r] = en[l][r];
            }
    }
}

__device__ __forceinline__ int row_octave(const DetectArgs &a, long long g)
{
    int o = 0;
    for (int k = 1; k < a.n_oct; ++k)
        if (g >= a.oc[k].row_base) o = k;
    return o;
}

// Keypoints per row (popcount of its words) and per block of kRowBlock rows.
__global__ void __launch_bounds__(kRowBlock) row_count_kernel(const DetectArgs a)
{
    __shared__ int wsum[kRowBlock / 64];
    const long long g = (long long)blockIdx.x * kRowBlock + threadIdx.x;
    int c = 0;
    if (g < a.total_rows) {
        const DetOctave &oc = a.oc[row_octave(a, g)];
        const unsigned long long *w = oc.masks + (g - oc.row_base) * oc.words;
        for (int q = 0; q < oc.words; ++q) c += __popcll(w[q]);
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

// Keypoint records in canonical order: row offset = block offset + prefix
// of the block's row counts; within a row, x ascending.
__global__ void __launch_bounds__(kRowBlock) emit_rows_kernel(const DetectArgs a)
{
    __shared__ int pre[kRowBlock];
    if (a.block_sum[blockIdx.x] == 0 || a.block_off[blockIdx.x] >= a.cap) return;
    const long long g = (long long)blockIdx.x * kRowBlock + threadIdx.x;
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
    int idx = a.block_off[blockIdx.x] + pre[threadIdx.x] - c;
    const int o = row_octave(a, g);
    const DetOctave &oc = a.oc[o];
    const long long r = g - oc.row_base;
    const long long per_s = (long long)(oc.nz - 2) * (oc.ny - 2);
    const int s = 1 + (int)(r / per_s);
    const long long rem = r - (long long)(s - 1) * per_s;
    const int z = 1 + (int)(rem / (oc.ny - 2));
    const int y = 1 + (int)(rem - (long long)(z - 1) * (oc.ny - 2));
    const long long nxy = (long long)oc.nx * oc.ny;
    const float *Ds = oc.D + oc.lstride * s;
    const float f = (float)(1 << o);
    const float h = 0.5f * (f - 1.f);
    for (int q = 0; q < oc.words && idx < a.cap; ++q) {
        unsigned long long w = oc.masks[r * oc.words + q];
        while (w != 0ull && idx < a.cap) {
            const int x = 64 * q + (__ffsll((long long)w) - 1);
            w &= w - 1ull;
            const long long vi = (long long)z * nxy + (long long)y * oc.nx + x;
            const float v = Ds[vi];
            // a strict extremum differs from every neighbour: one decides peak or valley
            const bool peak = v > Ds[vi + 1];
            sift3d_keypoint k;
            k.x = x;
            k.y = y;
            k.z = z;
            k.octave = (int16_t)o;
            k.scale = (int16_t)s;
            k.polarity = (int8_t)(peak ? 1 : -1);
            k.pad[0] = k.pad[1] = k.pad[2] = 0;
            k.dog = v;
            k.xf = f * (float)x + h;
            k.yf = f * (float)y + h;
            k.zf = f * (float)z + h;
            k.sigma = oc.sigma[s];
            a.kp[idx++] = k;
        }
    }
}

template <int S>
hipError_t launch_strict(const DetectArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL((detect_tile_kernel<S>), dim3(a.tile_blocks), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(row_count_kernel, dim3(a.row_blocks), dim3(kRowBlock), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    DetectArgs b = a;
    b.n_blocks = a.row_blocks;
    hipLaunchKernelGGL(detect_scan_kernel, dim3(1), dim3(kScanThreads), 0, st, b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(emit_rows_kernel, dim3(a.row_blocks), dim3(kRowBlock), 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_detect(const DetectArgs &a, hipStream_t st)
{
    if (a.votes == 80) {
        switch (a.S) {
        case 1: return launch_strict<1>(a, st);
        case 2: return launch_strict<2>(a, st);
        case 3: return launch_strict<3>(a, st);
        case 4: return launch_strict<4>(a, st);
        case 5: return launch_strict<5>(a, st);
        default: return hipErrorInvalidValue;
        }
    }
    hipLaunchKernelGGL(detect_count_kernel, dim3(a.n_blocks), dim3(kDetThreads), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(detect_scan_kernel, dim3(1), dim3(kScanThreads), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(detect_emit_kernel, dim3(a.n_blocks), dim3(kDetThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace s3d
