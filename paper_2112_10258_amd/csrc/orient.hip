// Dominant 3D orientations and SIFT-Rank after reorientation (Related Work,
// 3D SIFT-Rank: peaks of a discrete spherical histogram of gradient
// directions give one or more 3x3 rotations per keypoint; the descriptor is
// computed in each rotated frame).
//
// One workgroup per keypoint, looping over the keypoints of all volumes.
// The clamped (2R+3)^3 cube of G_s around the keypoint is staged in LDS,
// and every pass over the (2R+1)^3 window reads it there: thread (dx, dy)
// walks dz. Gradients are central differences evaluated in double
// precision (a float difference is exact in double).
//
// Histogram sums are accumulated as 64-bit fixed-point integers with LDS
// atomics: every term is the double value times a per-keypoint power of two
// S, rounded to the nearest integer, so the sums do not depend on the order
// in which lanes add them and the results are bit-reproducible. S is chosen
// from the largest |G| of the cube so that no sum can exceed 2^61; a term's
// rounding is at most 2^-50 of that bound.
//
//   pass 1: each sample with |g| > 0 goes to the nearest of the 26
//           directions n/|n|, n in {-1,0,1}^3 \ {0}; the bin keeps the sum
//           of |g| and of g;
//   peaks:  bins with a sum >= tau * the largest, above every neighbour
//           within 60 degrees (equal sums: the lower bin number wins), in
//           decreasing order; the primary axis is the bin's mean gradient;
//   pass 2: per primary axis e1, the same histogram of g - (g.e1) e1; each
//           of its peaks gives e2 (the part orthogonal to e1, normalised)
//           and e3 = e1 x e2;
//   pass 3: for every frame, each sample's offset and gradient in frame
//           coordinates bin as the upright descriptor does (spatial half by
//           the sign of each offset component, half to each side when it
//           is 0; orientation octant of the rotated gradient), weighted by
//           |g|; the 64 sums are ranked (ties by index).
// The nearest direction is found from the sorted gradient magnitudes: the
// best direction with s nonzero components takes the s largest |g_k| with
// their signs, worth their sum over sqrt(s).
#include "sift3d_internal.h"

namespace s3d {
namespace {

constexpr int kOrThreads = 256;
constexpr int kOrTile = 2 * kMaxSiftR + 3;

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// Direction n of bin b: the 27 vectors of {-1,0,1}^3 in (z, y, x) order
// with the zero vector (number 13) left out.
__device__ __forceinline__ void bin_dir(int b, int &nx, int &ny, int &nz)
{
    const int q = b < 13 ? b : b + 1;
    nx = q % 3 - 1;
    ny = (q / 3) % 3 - 1;
    nz = q / 9 - 1;
}

__device__ __forceinline__ int dir_bin(int nx, int ny, int nz)
{
    const int q = (nx + 1) + 3 * (ny + 1) + 9 * (nz + 1);
    return q < 13 ? q : q - 1;
}

// Bins a and b are neighbours: angle at most 60 degrees.
__device__ __forceinline__ bool bins_adjacent(int a, int b)
{
    int ax, ay, az, bx, by, bz;
    bin_dir(a, ax, ay, az);
    bin_dir(b, bx, by, bz);
    const int d = ax * bx + ay * by + az * bz;
    const int qa = ax * ax + ay * ay + az * az, qb = bx * bx + by * by + bz * bz;
    return a != b && d > 0 && 4 * d * d >= qa * qb;
}

// Nearest of the 26 directions to v (|v| > 0).
__device__ __forceinline__ int nearest_dir(double vx, double vy, double vz)
{
    const double ax = fabs(vx), ay = fabs(vy), az = fabs(vz);
    // axes by decreasing magnitude
    int i0 = 0, i1 = 1, i2 = 2;
    double a0 = ax, a1 = ay, a2 = az;
    if (a1 > a0) {
        double t = a0; a0 = a1; a1 = t;
        int u = i0; i0 = i1; i1 = u;
    }
    if (a2 > a1) {
        double t = a1; a1 = a2; a2 = t;
        int u = i1; i1 = i2; i2 = u;
        if (a1 > a0) {
            t = a0; a0 = a1; a1 = t;
            u = i0; i0 = i1; i1 = u;
        }
    }
    const double c1 = a0, c2 = (a0 + a1) * 0.70710678118654752440, c3 = (a0 + a1 + a2) * 0.57735026918962576451;
    const int s = c3 > c2 && c3 > c1 ? 3 : (c2 > c1 ? 2 : 1);
    int n[3] = {0, 0, 0};
    const double v[3] = {vx, vy, vz};
    n[i0] = v[i0] > 0.0 ? 1 : -1;
    if (s >= 2) n[i1] = v[i1] > 0.0 ? 1 : -1;
    if (s >= 3) n[i2] = v[i2] > 0.0 ? 1 : -1;
    return dir_bin(n[0], n[1], n[2]);
}

__device__ __forceinline__ unsigned long long fix(double v, double S)
{
    return (unsigned long long)__double2ll_rn(v * S);
}

__device__ __forceinline__ double unfix(unsigned long long v, double invS) { return (double)(long long)v * invS; }

struct OrientShared {
    float T[kOrTile * kOrTile * kOrTile];
    unsigned long long acc[4][26];                   // sum of weights, then of x, y, z
    unsigned long long hist[kMaxOrient][64];
    double frame[kMaxOrient][9];                      // R[3 i + j] = component i of axis j
    double e1[26][3];                                 // primary axes, in peak order
    double red[kOrThreads / 64];
    int peaks[26], npeaks;
    int nprim;
    int nframes;
    double S;
};

// Register run of one column: the sums of consecutive samples that fall in
// the same direction bin, added to the LDS histogram when the bin changes.
struct BinRun {
    int bin = -1;
    unsigned long long w = 0, x = 0, y = 0, z = 0;
    __device__ __forceinline__ void flush(OrientShared &s)
    {
        if (bin < 0) return;
        atomicAdd(&s.acc[0][bin], w);
        atomicAdd(&s.acc[1][bin], x);
        atomicAdd(&s.acc[2][bin], y);
        atomicAdd(&s.acc[3][bin], z);
    }
    __device__ __forceinline__ void add(OrientShared &s, int b, unsigned long long tw, unsigned long long tx,
                                        unsigned long long ty, unsigned long long tz)
    {
        if (b != bin) {
            flush(s);
            bin = b;
            w = x = y = z = 0;
        }
        w += tw;
        x += tx;
        y += ty;
        z += tz;
    }
};

// Peaks of the histogram in s.acc[0] into s.peaks (called by wavefront 0).
__device__ void find_peaks(OrientShared &s, double tau, int lane)
{
    long long h = lane < 26 ? (long long)s.acc[0][lane] : 0;
    long long hmax = h;
    for (int off = 32; off >= 1; off >>= 1) hmax = max(hmax, (long long)__shfl_xor(hmax, off));
    bool pk = false;
    if (lane < 26 && h > 0 && (double)h >= tau * (double)hmax) {
        pk = true;
        for (int c = 0; c < 26; ++c) {
            if (!bins_adjacent(lane, c)) continue;
            const long long hc = (long long)s.acc[0][c];
            if (!(h > hc || (h == hc && lane < c))) pk = false;
        }
    }
    // order: decreasing sum, lower bin first on ties
    const unsigned long long m = __ballot(pk);
    if (pk) {
        int pos = 0;
        for (int c = 0; c < 26; ++c) {
            if (!((m >> c) & 1ull) || c == lane) continue;
            const long long hc = (long long)s.acc[0][c];
            pos += hc > h || (hc == h && c < lane);
        }
        s.peaks[pos] = lane;
    }
    if (lane == 0) s.npeaks = __popcll(m);
}

template <int R>
__device__ __forceinline__ void stage(OrientShared &s, const float *G, int nx, int ny, int nz, int kx, int ky, int kz,
                                      int tid)
{
    constexpr int TW = 2 * R + 3;
    const int cx = kx - R - 1, cy = ky - R - 1, cz = kz - R - 1;
    const size_t nxy = (size_t)nx * ny;
    float mx = 0.f;
    for (int idx = tid; idx < TW * TW * TW; idx += kOrThreads) {
        const int i = idx % TW, jk = idx / TW;
        const int j = jk % TW, k = jk / TW;
        const float v = G[(size_t)clampi(cz + k, 0, nz - 1) * nxy + (size_t)clampi(cy + j, 0, ny - 1) * nx +
                          clampi(cx + i, 0, nx - 1)];
        s.T[idx] = v;
        mx = fmaxf(mx, fabsf(v));
    }
    for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if ((tid & 63) == 0) s.red[tid >> 6] = mx;
}

// Gradient of window sample (dx, dy, dz) from the staged cube.
template <int R>
__device__ __forceinline__ void grad(const OrientShared &s, int nx, int ny, int nz, int kx, int ky, int kz, int dx,
                                     int dy, int dz, double &gx, double &gy, double &gz)
{
    constexpr int TW = 2 * R + 3;
    const int cx = kx - R - 1, cy = ky - R - 1, cz = kz - R - 1;
    const int qx = clampi(kx + dx, 0, nx - 1), qy = clampi(ky + dy, 0, ny - 1), qz = clampi(kz + dz, 0, nz - 1);
    const int lx = qx - cx, ly = qy - cy, lz = qz - cz;
    const int lxm = clampi(qx - 1, 0, nx - 1) - cx, lxp = clampi(qx + 1, 0, nx - 1) - cx;
    const int lym = clampi(qy - 1, 0, ny - 1) - cy, lyp = clampi(qy + 1, 0, ny - 1) - cy;
    const int lzm = clampi(qz - 1, 0, nz - 1) - cz, lzp = clampi(qz + 1, 0, nz - 1) - cz;
    gx = 0.5 * ((double)s.T[(lz * TW + ly) * TW + lxp] - (double)s.T[(lz * TW + ly) * TW + lxm]);
    gy = 0.5 * ((double)s.T[(lz * TW + lyp) * TW + lx] - (double)s.T[(lz * TW + lym) * TW + lx]);
    gz = 0.5 * ((double)s.T[(lzp * TW + ly) * TW + lx] - (double)s.T[(lzm * TW + ly) * TW + lx]);
}

template <int R>
__device__ void orient_one(OrientShared &s, const OrientLaunch &a, const float *G, int nx, int ny, int nz, int kx,
                           int ky, int kz, size_t k)
{
    constexpr int W = 2 * R + 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    stage<R>(s, G, nx, ny, nz, kx, ky, kz, tid);
    for (int i = tid; i < 4 * 26; i += kOrThreads) (&s.acc[0][0])[i] = 0ull;
    for (int i = tid; i < kMaxOrient * 64; i += kOrThreads) (&s.hist[0][0])[i] = 0ull;
    if (tid == 0) s.nframes = 0;
    __syncthreads();
    if (tid == 0) {
        float mx = 0.f;
        for (int w = 0; w < kOrThreads / 64; ++w) mx = fmaxf(mx, s.red[w]);
        // every term is at most sqrt(3) max|G| and a window has < 2^12
        // samples: S = 2^(61 - 12 - e) with sqrt(3) max|G| <= 2^e
        int e = 0;
        frexp(1.7320508075688772 * (double)mx, &e);
        s.S = mx > 0.f ? ldexp(1.0, 49 - e) : 0.0;
    }
    __syncthreads();
    const double S = s.S;
    if (S == 0.0) {
        // constant cube: no gradient, no frame
        for (int t = tid; t < kMaxOrient * 64; t += kOrThreads) a.siftrank[k * kMaxOrient * 64 + t] = 0;
        for (int t = tid; t < kMaxOrient * 9; t += kOrThreads) a.frames[k * kMaxOrient * 9 + t] = 0.f;
        if (tid == 0) a.nframes[k] = 0;
        return;
    }
    const double invS = 1.0 / S;
    const bool col = tid < W * W;
    const int dy = tid / W - R, dx = tid - (tid / W) * W - R;

    // pass 1: spherical histogram of the gradients. Consecutive samples of a
    // column that fall in the same bin are summed in registers and added to
    // LDS once (integer sums: the result does not depend on the grouping).
    if (col) {
        BinRun run;
        for (int dz = -R; dz <= R; ++dz) {
            double gx, gy, gz;
            grad<R>(s, nx, ny, nz, kx, ky, kz, dx, dy, dz, gx, gy, gz);
            const double m = sqrt(gx * gx + gy * gy + gz * gz);
            if (!(m > 0.0)) continue;
            run.add(s, nearest_dir(gx, gy, gz), fix(m, S), fix(gx, S), fix(gy, S), fix(gz, S));
        }
        run.flush(s);
    }
    __syncthreads();
    if (wave == 0) {
        find_peaks(s, a.tau, lane);
        // primary axis of each peak: the bin's mean gradient
        if (lane < s.npeaks) {
            const int b = s.peaks[lane];
            const double vx = unfix(s.acc[1][b], invS), vy = unfix(s.acc[2][b], invS), vz = unfix(s.acc[3][b], invS);
            const double vn = sqrt(vx * vx + vy * vy + vz * vz);
            s.e1[lane][0] = vx / vn;
            s.e1[lane][1] = vy / vn;
            s.e1[lane][2] = vz / vn;
        }
        if (lane == 0) s.nprim = s.npeaks;
    }
    __syncthreads();
    const int nprim = s.nprim;

    // pass 2 per primary axis
    for (int ip = 0; ip < nprim; ++ip) {
        if (s.nframes >= kMaxOrient) break;      // uniform: read after a barrier
        for (int i = tid; i < 4 * 26; i += kOrThreads) (&s.acc[0][0])[i] = 0ull;
        __syncthreads();
        const double e1x = s.e1[ip][0], e1y = s.e1[ip][1], e1z = s.e1[ip][2];
        if (col) {
            BinRun run;
            for (int dz = -R; dz <= R; ++dz) {
                double gx, gy, gz;
                grad<R>(s, nx, ny, nz, kx, ky, kz, dx, dy, dz, gx, gy, gz);
                const double t = gx * e1x + gy * e1y + gz * e1z;
                const double px = gx - t * e1x, py = gy - t * e1y, pz = gz - t * e1z;
                const double m2 = sqrt(px * px + py * py + pz * pz);
                if (!(m2 > 0.0)) continue;
                run.add(s, nearest_dir(px, py, pz), fix(m2, S), fix(px, S), fix(py, S), fix(pz, S));
            }
            run.flush(s);
        }
        __syncthreads();
        if (wave == 0) find_peaks(s, a.tau, lane);
        __syncthreads();
        if (tid == 0) {
            for (int is = 0; is < s.npeaks && s.nframes < kMaxOrient; ++is) {
                const int b = s.peaks[is];
                const double wx = unfix(s.acc[1][b], invS), wy = unfix(s.acc[2][b], invS), wz = unfix(s.acc[3][b], invS);
                const double t = wx * e1x + wy * e1y + wz * e1z;
                const double ux = wx - t * e1x, uy = wy - t * e1y, uz = wz - t * e1z;
                const double un = sqrt(ux * ux + uy * uy + uz * uz);
                if (!(un > 0.0)) continue;
                const double e2x = ux / un, e2y = uy / un, e2z = uz / un;
                double *F = s.frame[s.nframes++];
                F[0] = e1x; F[3] = e1y; F[6] = e1z;
                F[1] = e2x; F[4] = e2y; F[7] = e2z;
                F[2] = e1y * e2z - e1z * e2y;
                F[5] = e1z * e2x - e1x * e2z;
                F[8] = e1x * e2y - e1y * e2x;
            }
        }
        __syncthreads();
    }
    const int nf = s.nframes;

    // pass 3: SIFT-Rank of every frame
    if (col && nf > 0) {
        // per frame, a run of samples feeding one single bin is summed in
        // registers (integer sums); samples on a frame plane (several bins)
        // go to LDS at once
        int rbin[kMaxOrient];
        unsigned long long racc[kMaxOrient];
#pragma unroll
        for (int f = 0; f < kMaxOrient; ++f) {
            rbin[f] = -1;
            racc[f] = 0ull;
        }
        for (int dz = -R; dz <= R; ++dz) {
            double gx, gy, gz;
            grad<R>(s, nx, ny, nz, kx, ky, kz, dx, dy, dz, gx, gy, gz);
            const double m = sqrt(gx * gx + gy * gy + gz * gz);
            if (!(m > 0.0)) continue;
#pragma unroll
            for (int f = 0; f < kMaxOrient; ++f) {
                if (f >= nf) break;
                const double *F = s.frame[f];
                int bo = 0, lo[3], hi[3];
                double w0[3];
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const double dp = F[j] * dx + F[3 + j] * dy + F[6 + j] * dz;
                    const double gp = F[j] * gx + F[3 + j] * gy + F[6 + j] * gz;
                    bo |= (gp > 0.0) << j;
                    // spatial halves this axis feeds and the weight of the lower one
                    lo[j] = dp > 0.0 ? 1 : 0;
                    hi[j] = dp < 0.0 ? 0 : 1;
                    w0[j] = dp == 0.0 ? 0.5 : 1.0;
                }
                const unsigned long long term = fix(m * w0[0] * w0[1] * w0[2], S);
                if (lo[0] == hi[0] && lo[1] == hi[1] && lo[2] == hi[2]) {
                    const int bin = 8 * (lo[0] + 2 * lo[1] + 4 * lo[2]) + bo;
                    if (bin != rbin[f]) {
                        if (rbin[f] >= 0) atomicAdd(&s.hist[f][rbin[f]], racc[f]);
                        rbin[f] = bin;
                        racc[f] = 0ull;
                    }
                    racc[f] += term;
                } else {
                    for (int bz = lo[2]; bz <= hi[2]; ++bz)
                        for (int by = lo[1]; by <= hi[1]; ++by)
                            for (int bx = lo[0]; bx <= hi[0]; ++bx)
                                atomicAdd(&s.hist[f][8 * (bx + 2 * by + 4 * bz) + bo], term);
                }
            }
        }
#pragma unroll
        for (int f = 0; f < kMaxOrient; ++f)
            if (f < nf && rbin[f] >= 0) atomicAdd(&s.hist[f][rbin[f]], racc[f]);
    }
    __syncthreads();
    // ranks (ties by index) and outputs
    for (int t = tid; t < kMaxOrient * 64; t += kOrThreads) {
        const int f = t >> 6, e = t & 63;
        uint8_t r = 0;
        if (f < nf) {
            const long long h = (long long)s.hist[f][e];
            int c = 0;
            for (int q = 0; q < 64; ++q) {
                const long long o = (long long)s.hist[f][q];
                c += (o < h) || (o == h && q < e);
            }
            r = (uint8_t)c;
        }
        a.siftrank[(k * kMaxOrient + f) * 64 + e] = r;
    }
    for (int t = tid; t < kMaxOrient * 9; t += kOrThreads) {
        const int f = t / 9, q = t - f * 9;
        a.frames[(k * kMaxOrient + f) * 9 + q] = f < nf ? (float)s.frame[f][q] : 0.f;
    }
    if (tid == 0) a.nframes[k] = nf;
}

template <bool INL>
__global__ void __launch_bounds__(kOrThreads) orient_kernel(const OrientLaunch a)
{
    __shared__ OrientShared s;
    const int tid = threadIdx.x;
    long long base = 0;
    for (int v = 0; v < a.n_vol; ++v) {
        const int count = min(a.counts[v], a.cap);
        const DVol vol = a.vols[v];
        long long r0 = ((long long)blockIdx.x - base) % gridDim.x;
        if (r0 < 0) r0 += gridDim.x;
        for (int kk = (int)r0; kk < count; kk += gridDim.x) {
            const size_t k = (size_t)v * a.cap + kk;
            const sift3d_keypoint kp = a.kp[k];
            if (kp.octave < 0 || kp.octave >= vol.n_units || kp.scale < 1 || kp.scale > a.S) {
                // not a keypoint of this plan: no frames
                for (int t = tid; t < kMaxOrient * 64; t += kOrThreads) a.siftrank[k * kMaxOrient * 64 + t] = 0;
                for (int t = tid; t < kMaxOrient * 9; t += kOrThreads) a.frames[k * kMaxOrient * 9 + t] = 0.f;
                if (tid == 0) a.nframes[k] = 0;
                continue;
            }
            const DUnit &oc = INL ? a.inl[vol.unit0 + kp.octave] : a.units[vol.unit0 + kp.octave];
            const float *G = reinterpret_cast<const float *>(a.ws + oc.g0) + oc.lstride * kp.scale;
            switch (a.sift_R[kp.scale]) {
            case 1: orient_one<1>(s, a, G, oc.nx, oc.ny, oc.nz, kp.x, kp.y, kp.z, k); break;
            case 2: orient_one<2>(s, a, G, oc.nx, oc.ny, oc.nz, kp.x, kp.y, kp.z, k); break;
            case 3: orient_one<3>(s, a, G, oc.nx, oc.ny, oc.nz, kp.x, kp.y, kp.z, k); break;
            case 4: orient_one<4>(s, a, G, oc.nx, oc.ny, oc.nz, kp.x, kp.y, kp.z, k); break;
            case 5: orient_one<5>(s, a, G, oc.nx, oc.ny, oc.nz, kp.x, kp.y, kp.z, k); break;
            case 6: orient_one<6>(s, a, G, oc.nx, oc.ny, oc.nz, kp.x, kp.y, kp.z, k); break;
            default: orient_one<7>(s, a, G, oc.nx, oc.ny, oc.nz, kp.x, kp.y, kp.z, k); break;
            }
            __syncthreads();   // the next keypoint overwrites the shared state
        }
        base += count;
    }
}

}  // namespace

hipError_t launch_orient(const OrientLaunch &a, long long kp_slots, int n_cu, hipStream_t st)
{
    if (kp_slots <= 0) return hipSuccess;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, orient_kernel<true>, kOrThreads, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const long long grid = std::min<long long>(kp_slots, (long long)per_cu * n_cu);
    if (a.n_units <= kInlineUnits)
        hipLaunchKernelGGL(orient_kernel<true>, dim3((unsigned)grid), dim3(kOrThreads), 0, st, a);
    else
        hipLaunchKernelGGL(orient_kernel<false>, dim3((unsigned)grid), dim3(kOrThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace s3d
