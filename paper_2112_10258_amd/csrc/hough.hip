// The matching stage beside the hot path, on gfx950:
//   - unit-length normalisation of descriptors (Section 3.1, step e);
//   - matching units: the oriented (or upright) keypoints of one volume as
//     flat rows of geometry and descriptor, in keypoint order;
//   - the global 7-DoF similarity Hough vote and its inliers (Section 3.3:
//     matches count when they are inliers to a rotation + translation +
//     isotropic scale found by a Hough transform).
//
// The Hough vote runs as a handful of small launches: each valid match
// derives its similarity hypothesis in double precision and the low corner
// of its 2^7 bins; one thread per (match, corner) inserts the bin into an
// open-addressing hash table with 64-bit compare-and-swap and counts the
// vote with an atomic add (counts do not depend on the order of arrival);
// two grid-wide reductions find the largest count and the smallest key
// holding it; a single workgroup then runs the fit / inlier rounds with
// fixed-order reductions in double (wave butterflies, then the 16 wave
// partials in order), so every result is reproducible run to run.
#include <cmath>
#include <cstdint>

#include "sift3d_internal.h"

// The hypothesis and inlier formulas are evaluated as written: no fused
// multiply-adds, so that the rounding follows the plain formulas.
#pragma clang fp contract(off)

namespace s3d {
namespace {

// ------------------------------------------------------------ normalisation

// One wavefront per row, four rows per workgroup. Ranks: each lane holds up
// to four entries, the integer sum of squares is exact, the norm and the
// quotient are taken in double and rounded to float once.
template <int KIND>
__global__ void __launch_bounds__(256) normalize_kernel(const void *in, int n, int row_elems, float *out)
{
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);   // the same for the whole wavefront
    if (row >= n) return;
    if constexpr (KIND == SIFT3D_MATCH_BRIEF) {
        const uint64_t *w = static_cast<const uint64_t *>(in) + (size_t)row * row_elems;
        const float v = (float)(1.0 / sqrt(64.0 * row_elems));
        float *o = out + (size_t)row * 64 * row_elems;
        for (int j = 0; j < row_elems; ++j) {
            const bool bit = (w[j] >> lane) & 1ull;
            o[64 * j + lane] = bit ? v : -v;
        }
    } else {
        const uint8_t *r = static_cast<const uint8_t *>(in) + (size_t)row * row_elems;
        int val[4];
        int ss = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int e = lane + 64 * j;
            val[j] = e < row_elems ? (int)r[e] : 0;
            ss += val[j] * val[j];
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
        const double nrm = sqrt((double)ss);
        float *o = out + (size_t)row * row_elems;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int e = lane + 64 * j;
            if (e < row_elems) o[e] = ss > 0 ? (float)((double)val[j] / nrm) : 0.0f;
        }
    }
}

// ------------------------------------------------------------ matching units

constexpr int kUnitThreads = 1024;
constexpr int kUnitWaves = kUnitThreads / 64;

// One workgroup walks the keypoints in chunks of 1024: a unit count per
// keypoint, an exclusive scan over the chunk (wave scans, then the wave
// totals in order), and each thread writes its keypoint's units.
__global__ void __launch_bounds__(kUnitThreads) units_kernel(const UnitsArgs a)
{
    __shared__ int wsum[kUnitWaves];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int K = min(max(*a.count, 0), a.cap);
    int base = 0;
    for (int k0 = 0; k0 < K; k0 += kUnitThreads) {
        const int k = k0 + t;
        int nf = 0;
        if (k < K) nf = a.nframes ? min(max(a.nframes[k], 0), kMaxOrient) : 1;
        int inc = nf;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(inc, off);
            if (lane >= off) inc += y;
        }
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        int wbase = 0, total = 0;
        for (int w = 0; w < kUnitWaves; ++w) {
            wbase += w < wave ? wsum[w] : 0;
            total += wsum[w];
        }
        const int first = base + wbase + inc - nf;
        for (int f = 0; f < nf; ++f) {
            const int u = first + f;
            a.unit[u] = k * kMaxOrient + f;
            const sift3d_keypoint &p = a.kp[k];
            float *g = a.geo + (size_t)u * 13;
            g[0] = p.xf;
            g[1] = p.yf;
            g[2] = p.zf;
            g[3] = p.sigma;
            if (a.nframes) {
                const float *fr = a.frames + ((size_t)k * kMaxOrient + f) * 9;
                for (int e = 0; e < 9; ++e) g[4 + e] = fr[e];
            } else {
                for (int e = 0; e < 9; ++e) g[4 + e] = e % 4 == 0 ? 1.0f : 0.0f;
            }
            if (a.desc_out) {
                const size_t src = a.nframes ? (size_t)k * kMaxOrient + f : (size_t)k;
                const uint32_t *s = reinterpret_cast<const uint32_t *>(a.desc + src * a.row_bytes);
                uint32_t *d = reinterpret_cast<uint32_t *>(a.desc_out + (size_t)u * a.row_bytes);
                for (int e = 0; e < a.row_bytes / 4; ++e) d[e] = s[e];
            }
        }
        base += total;
        __syncthreads();   // wsum is rewritten by the next chunk
    }
    if (t == 0) *a.n_units = base;
}

// ------------------------------------------------------------ Hough vote

constexpr unsigned long long kEmpty = ~0ull;   // an unused table slot / a match that does not vote
constexpr int kFieldBits = 9;
constexpr int kFieldBias = 256;
constexpr int kDims = 7;
constexpr int kCorners = 1 << kDims;
constexpr int kFitThreads = 1024;
constexpr int kFitWaves = kFitThreads / 64;

__device__ __forceinline__ int key_field(unsigned long long key, int d)
{
    return (int)((key >> (kFieldBits * d)) & ((1u << kFieldBits) - 1));   // biased coordinate
}

__device__ __forceinline__ unsigned slot_of(unsigned long long key, int log2_slots)
{
    return (unsigned)((key * 0x9E3779B97F4A7C15ull) >> (64 - log2_slots));
}

// Match i's B row, or -1 when the match is not valid (index out of range or
// a scale that is not positive).
__device__ __forceinline__ int valid_match(const HoughArgs &a, int i)
{
    const int j = a.match[i];
    if (j < 0 || j >= a.n_b) return -1;
    if (!(a.geo_a[(size_t)i * 13 + 3] > 0.0f) || !(a.geo_b[(size_t)j * 13 + 3] > 0.0f)) return -1;
    return j;
}

// Rotation vector of a 3x3 matrix R (row-major), the inverse of Rodrigues'
// formula: antisymmetric part for cos theta >= -0.99, symmetric part near pi.
__device__ void rotation_vector(const double R[9], double w[3])
{
    const double c = fmin(1.0, fmax(-1.0, (R[0] + R[4] + R[8] - 1.0) / 2.0));
    const double th = acos(c);
    const double v[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]};
    if (c >= -0.99) {
        const double f = th < 1e-4 ? 0.5 * (1.0 + th * th / 6.0) : th / (2.0 * sin(th));
        for (int k = 0; k < 3; ++k) w[k] = v[k] * f;
        return;
    }
    double B[9];
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) B[3 * r + q] = 0.5 * (R[3 * r + q] + R[3 * q + r]) - (r == q ? c : 0.0);
    int i = 0;
    for (int k = 1; k < 3; ++k)
        if (B[4 * k] > B[4 * i]) i = k;
    const double den = sqrt(B[4 * i] * (1.0 - c));
    double ax[3];
    for (int k = 0; k < 3; ++k) ax[k] = B[3 * k + i] / den;
    const double dot = ax[0] * v[0] + ax[1] * v[1] + ax[2] * v[2];
    const double sg = dot < 0.0 ? -1.0 : 1.0;
    for (int k = 0; k < 3; ++k) w[k] = th * sg * ax[k];
}

__global__ void __launch_bounds__(256) hough_clear_kernel(const HoughArgs a)
{
    const size_t slots = (size_t)1 << a.log2_slots;
    for (size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x; s < slots; s += (size_t)gridDim.x * blockDim.x) {
        a.keys[s] = kEmpty;
        a.counts[s] = 0u;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *a.best_count = 0u;
        *a.best_key = kEmpty;
    }
}

// Hypothesis of match i: s = sigma_b / sigma_a, R = R_b R_a^T, the image p
// of A's reference point; vote vector (log2 s, rotation vector, p) over the
// bin widths; per coordinate the lower of floor(q) and its nearer neighbour.
__global__ void __launch_bounds__(256) hough_hypothesis_kernel(const HoughArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_a) return;
    unsigned long long key = kEmpty;
    const int j = valid_match(a, i);
    if (j >= 0) {
        const float *ga = a.geo_a + (size_t)i * 13, *gb = a.geo_b + (size_t)j * 13;
        const double s = (double)gb[3] / (double)ga[3];
        double R[9];
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += (double)gb[4 + 3 * r + k] * (double)ga[4 + 3 * q + k];
                R[3 * r + q] = acc;
            }
        double v[kDims];
        v[0] = log2(s);
        rotation_vector(R, v + 1);
        double d[3];
        for (int k = 0; k < 3; ++k) d[k] = a.centre[k] - (double)ga[k];
        for (int r = 0; r < 3; ++r) {
            const double rd = R[3 * r] * d[0] + R[3 * r + 1] * d[1] + R[3 * r + 2] * d[2];
            v[4 + r] = (double)gb[r] + s * rd;
        }
        unsigned long long k = 0;
        bool ok = true;
        for (int dd = 0; dd < kDims; ++dd) {
            const double q = v[dd] / a.width[dd];
            if (!(q > -257.0 && q < 256.0)) {   // also rejects NaN
                ok = false;
                break;
            }
            const double b = floor(q);
            const double lo = q - b >= 0.5 ? b : b - 1.0;
            if (lo < -256.0 || lo > 254.0) {
                ok = false;
                break;
            }
            k |= (unsigned long long)((int)lo + kFieldBias) << (kFieldBits * dd);
        }
        if (ok) key = k;
    }
    a.lo[i] = key;
}

// One thread per (match, corner): bin lo + corner, inserted by linear probing.
__global__ void __launch_bounds__(256) hough_insert_kernel(const HoughArgs a)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)a.n_a * kCorners) return;
    const unsigned long long lo = a.lo[g / kCorners];
    if (lo == kEmpty) return;
    const int corner = (int)(g % kCorners);
    unsigned long long key = lo;
    for (int d = 0; d < kDims; ++d) key += (unsigned long long)((corner >> d) & 1) << (kFieldBits * d);
    const unsigned mask = (1u << a.log2_slots) - 1u;
    unsigned s = slot_of(key, a.log2_slots);
    // at most 2^7 n_a distinct keys in 2^8 n_a (or more) slots: an empty
    // or equal slot is always found within one sweep of the table
    for (unsigned probe = 0; probe <= mask; ++probe) {
        const unsigned long long prev = atomicCAS(&a.keys[s], kEmpty, key);
        if (prev == kEmpty || prev == key) {
            atomicAdd(&a.counts[s], 1u);
            return;
        }
        s = (s + 1u) & mask;
    }
}

__global__ void __launch_bounds__(256) hough_max_kernel(const HoughArgs a)
{
    const size_t slots = (size_t)1 << a.log2_slots;
    unsigned m = 0;
    for (size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x; s < slots; s += (size_t)gridDim.x * blockDim.x)
        m = max(m, a.counts[s]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, off));
    if ((threadIdx.x & 63) == 0 && m > 0) atomicMax(a.best_count, m);
}

__global__ void __launch_bounds__(256) hough_key_kernel(const HoughArgs a)
{
    const size_t slots = (size_t)1 << a.log2_slots;
    const unsigned best = *a.best_count;
    if (best == 0) return;
    unsigned long long m = kEmpty;
    for (size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x; s < slots; s += (size_t)gridDim.x * blockDim.x)
        if (a.counts[s] == best) m = min(m, a.keys[s]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off);
        m = min(m, o);
    }
    if ((threadIdx.x & 63) == 0 && m != kEmpty) atomicMin(a.best_key, m);
}

// Sum over the workgroup in a fixed order: a butterfly within each
// wavefront (every lane ends with the same value: addition commutes), then
// the wave partials in wave order.
__device__ double block_sum(double v, double *sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kFitWaves; ++w) s += sh[w];
    __syncthreads();
    return s;
}

// Eigen-decomposition of a symmetric 4x4 matrix by cyclic Jacobi rotations;
// returns the eigenvector of the largest eigenvalue (lowest index on ties)
// in q and that eigenvalue.
__device__ double jacobi_top(double A[4][4], double q[4])
{
    double V[4][4];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) V[r][c] = r == c ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) {
                tot += A[r][c] * A[r][c];
                if (c > r) off += A[r][c] * A[r][c];
            }
        if (off <= 1e-32 * tot) break;
        for (int p = 0; p < 3; ++p)
            for (int r = p + 1; r < 4; ++r) {
                if (A[p][r] == 0.0) continue;
                const double th = (A[r][r] - A[p][p]) / (2.0 * A[p][r]);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 4; ++k) {
                    const double akp = A[k][p], akr = A[k][r];
                    A[k][p] = c * akp - s * akr;
                    A[k][r] = s * akp + c * akr;
                }
                for (int k = 0; k < 4; ++k) {
                    const double apk = A[p][k], ark = A[r][k];
                    A[p][k] = c * apk - s * ark;
                    A[r][k] = s * apk + c * ark;
                }
                for (int k = 0; k < 4; ++k) {
                    const double vkp = V[k][p], vkr = V[k][r];
                    V[k][p] = c * vkp - s * vkr;
                    V[k][r] = s * vkp + c * vkr;
                }
            }
    }
    int b = 0;
    for (int k = 1; k < 4; ++k)
        if (A[k][k] > A[b][b]) b = k;
    for (int k = 0; k < 4; ++k) q[k] = V[k][b];
    return A[b][b];
}

struct FitShared {
    double red[kFitWaves];
    double s, R[9], t[3];   // this round's transform
    int stop;
};

// The fit / inlier rounds, one workgroup.
__global__ void __launch_bounds__(kFitThreads) hough_fit_kernel(const HoughArgs a)
{
    __shared__ FitShared sh;
    const int tid = threadIdx.x;
    const unsigned votes = *a.best_count;
    const unsigned long long win = *a.best_key;
    for (int i = tid; i < a.n_a; i += kFitThreads) a.inlier[i] = 0;
    int have = 0, n_fit = 0, n_inl = 0;
    double acc_s = 0.0, acc_R[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, acc_t[3] = {0.0, 0.0, 0.0};
    for (int round = 0; round < a.iterations && votes > 0; ++round) {
        __syncthreads();   // the previous round's inlier flags are complete
        // pass 1: size and sums of the fit set
        double cnt = 0.0, sa[3] = {0.0, 0.0, 0.0}, sb[3] = {0.0, 0.0, 0.0};
        for (int i = tid; i < a.n_a; i += kFitThreads) {
            bool m;
            if (round == 0) {
                const unsigned long long lo = a.lo[i];
                m = lo != kEmpty;
                for (int d = 0; d < kDims && m; ++d) {
                    const int l = key_field(lo, d), w = key_field(win, d);
                    m = l <= w && w <= l + 1;
                }
            } else {
                m = a.inlier[i] != 0;
            }
            if (!m) continue;
            const int j = a.match[i];
            cnt += 1.0;
            for (int k = 0; k < 3; ++k) {
                sa[k] += (double)a.geo_a[(size_t)i * 13 + k];
                sb[k] += (double)a.geo_b[(size_t)j * 13 + k];
            }
        }
        const double n = block_sum(cnt, sh.red);
        if (n < 3.0) break;
        double ma[3], mb[3];
        for (int k = 0; k < 3; ++k) {
            ma[k] = block_sum(sa[k], sh.red) / n;
            mb[k] = block_sum(sb[k], sh.red) / n;
        }
        // pass 2: centred cross-covariance S[r][c] = sum a_r b_c and sum |a|^2
        double S[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, var = 0.0;
        for (int i = tid; i < a.n_a; i += kFitThreads) {
            bool m;
            if (round == 0) {
                const unsigned long long lo = a.lo[i];
                m = lo != kEmpty;
                for (int d = 0; d < kDims && m; ++d) {
                    const int l = key_field(lo, d), w = key_field(win, d);
                    m = l <= w && w <= l + 1;
                }
            } else {
                m = a.inlier[i] != 0;
            }
            if (!m) continue;
            const int j = a.match[i];
            double ca[3], cb[3];
            for (int k = 0; k < 3; ++k) {
                ca[k] = (double)a.geo_a[(size_t)i * 13 + k] - ma[k];
                cb[k] = (double)a.geo_b[(size_t)j * 13 + k] - mb[k];
            }
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) S[3 * r + c] += ca[r] * cb[c];
            var += ca[0] * ca[0] + ca[1] * ca[1] + ca[2] * ca[2];
        }
        for (int k = 0; k < 9; ++k) S[k] = block_sum(S[k], sh.red);
        var = block_sum(var, sh.red);
        if (tid == 0) {
            // Horn's closed form: the rotation is the unit quaternion of the
            // largest eigenvalue of N(S); that eigenvalue over sum |a|^2 is the
            // least-squares scale.
            const double Sxx = S[0], Sxy = S[1], Sxz = S[2], Syx = S[3], Syy = S[4], Syz = S[5], Szx = S[6],
                         Szy = S[7], Szz = S[8];
            double N[4][4] = {{Sxx + Syy + Szz, Syz - Szy, Szx - Sxz, Sxy - Syx},
                              {Syz - Szy, Sxx - Syy - Szz, Sxy + Syx, Szx + Sxz},
                              {Szx - Sxz, Sxy + Syx, -Sxx + Syy - Szz, Syz + Szy},
                              {Sxy - Syx, Szx + Sxz, Syz + Szy, -Sxx - Syy + Szz}};
            double q[4];
            const double lam = jacobi_top(N, q);
            const double q0 = q[0], qx = q[1], qy = q[2], qz = q[3];
            const double R[9] = {q0 * q0 + qx * qx - qy * qy - qz * qz, 2.0 * (qx * qy - q0 * qz),
                                 2.0 * (qx * qz + q0 * qy), 2.0 * (qy * qx + q0 * qz),
                                 q0 * q0 - qx * qx + qy * qy - qz * qz, 2.0 * (qy * qz - q0 * qx),
                                 2.0 * (qz * qx - q0 * qy), 2.0 * (qz * qy + q0 * qx),
                                 q0 * q0 - qx * qx - qy * qy + qz * qz};
            const double s = var > 0.0 ? lam / var : 0.0;
            sh.stop = !(s > 0.0);
            sh.s = s;
            for (int k = 0; k < 9; ++k) sh.R[k] = R[k];
            for (int r = 0; r < 3; ++r)
                sh.t[r] = mb[r] - s * (R[3 * r] * ma[0] + R[3 * r + 1] * ma[1] + R[3 * r + 2] * ma[2]);
        }
        __syncthreads();
        if (sh.stop) break;
        // pass 3: inliers among all valid matches
        double inl = 0.0;
        for (int i = tid; i < a.n_a; i += kFitThreads) {
            const int j = valid_match(a, i);
            uint8_t f = 0;
            if (j >= 0) {
                const float *ga = a.geo_a + (size_t)i * 13, *gb = a.geo_b + (size_t)j * 13;
                double e2 = 0.0;
                for (int r = 0; r < 3; ++r) {
                    const double ra = sh.R[3 * r] * (double)ga[0] + sh.R[3 * r + 1] * (double)ga[1] +
                                      sh.R[3 * r + 2] * (double)ga[2];
                    const double y = sh.s * ra + sh.t[r] - (double)gb[r];
                    e2 += y * y;
                }
                const double e = sqrt(e2);
                const double lim = a.inl_sig * (double)gb[3];
                const double ds = fabs(log2(sh.s * (double)ga[3] / (double)gb[3]));
                f = (e <= lim && ds <= a.inl_log2s) ? 1 : 0;
            }
            a.inlier[i] = f;
            inl += f;
        }
        n_inl = (int)block_sum(inl, sh.red);
        n_fit = (int)n;
        have = 1;
        acc_s = sh.s;   // the transform of the last completed round
        for (int k = 0; k < 9; ++k) acc_R[k] = sh.R[k];
        for (int k = 0; k < 3; ++k) acc_t[k] = sh.t[k];
    }
    if (tid == 0) {
        sift3d_similarity o;
        o.status = have;
        o.votes = (int32_t)votes;
        o.bin = votes > 0 ? (int64_t)win : -1;
        o.n_fit = have ? n_fit : 0;
        o.n_inliers = have ? n_inl : 0;
        o.scale = acc_s;
        for (int k = 0; k < 9; ++k) o.rot[k] = acc_R[k];
        for (int k = 0; k < 3; ++k) o.trans[k] = acc_t[k];
        *a.out = o;
    }
}

}  // namespace

hipError_t launch_normalize(int kind, const void *in, int n, int row_elems, float *out, hipStream_t st)
{
    const int blocks = (n + 3) / 4;
    if (kind == SIFT3D_MATCH_BRIEF)
        hipLaunchKernelGGL(normalize_kernel<SIFT3D_MATCH_BRIEF>, dim3(blocks), dim3(256), 0, st, in, n, row_elems, out);
    else
        hipLaunchKernelGGL(normalize_kernel<SIFT3D_MATCH_RANKS>, dim3(blocks), dim3(256), 0, st, in, n, row_elems, out);
    return hipGetLastError();
}

hipError_t launch_units(const UnitsArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(units_kernel, dim3(1), dim3(kUnitThreads), 0, st, a);
    return hipGetLastError();
}

int hough_log2_slots(int n_a)
{
    int l = 8;
    while (((size_t)1 << l) < (size_t)2 * kCorners * (size_t)n_a) ++l;
    return l;
}

hipError_t launch_hough(const HoughArgs &a, hipStream_t st)
{
    const size_t slots = (size_t)1 << a.log2_slots;
    const int table_blocks = (int)std::min<size_t>((slots + 255) / 256, 4096);
    hipLaunchKernelGGL(hough_clear_kernel, dim3(table_blocks), dim3(256), 0, st, a);
    if (a.n_a > 0) {
        hipLaunchKernelGGL(hough_hypothesis_kernel, dim3((a.n_a + 255) / 256), dim3(256), 0, st, a);
        const long long threads = (long long)a.n_a * kCorners;
        hipLaunchKernelGGL(hough_insert_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, a);
        hipLaunchKernelGGL(hough_max_kernel, dim3(table_blocks), dim3(256), 0, st, a);
        hipLaunchKernelGGL(hough_key_kernel, dim3(table_blocks), dim3(256), 0, st, a);
    }
    hipLaunchKernelGGL(hough_fit_kernel, dim3(1), dim3(kFitThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace s3d
