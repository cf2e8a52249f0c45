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

}  // namespace

hipError_t launch_detect(const DetectArgs &a, hipStream_t st)
{
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
