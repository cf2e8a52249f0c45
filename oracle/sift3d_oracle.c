/*
 * sift3d_oracle.c -- plain, slow, FP64 reference of the 3D SIFT-Rank hot path.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path may call, link or
 * load this file. It shares no code, header, table or constant with the
 * HIP library; only the seeded inputs are common to both.
 *
 * Every routine is the plain definition written out as nested loops, in
 * double precision, with clamp-to-edge sampling wherever a coordinate
 * leaves the volume. Volumes are [z][y][x] with x fastest.
 *
 * Paper: Carluer et al., "GPU optimization of the 3D Scale-invariant
 * Feature Transform Algorithm and a Novel BRIEF-inspired 3D Fast
 * Descriptor" (arXiv 2112.10258).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define VIDX(x, y, z, nx, ny) ((((size_t)(z)) * (size_t)(ny) + (size_t)(y)) * (size_t)(nx) + (size_t)(x))

static long clampl(long v, long lo, long hi) { return v < lo ? lo : (v > hi ? hi : v); }

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Gaussian filter taps (Section 3.2.2, Gaussian Convolution: the filter is
 * a sampled normal density). w[t + r] = exp(-t^2 / (2 sigma^2)) for
 * t = -r..r with r = ceil(trunc * sigma), normalised by their sum.
 * sigma == 0 gives the identity filter (r = 0, w = {1}).
 * Returns r, or -1 if 2r+1 > cap.
 */
int orc_gauss_taps(double sigma, double trunc, double *w, int cap)
{
    int r = sigma > 0.0 ? (int)ceil(trunc * sigma) : 0;
    if (2 * r + 1 > cap) return -1;
    if (r == 0) { w[0] = 1.0; return 0; }
    double sum = 0.0;
    for (int t = -r; t <= r; ++t) {
        w[t + r] = exp(-(double)t * (double)t / (2.0 * sigma * sigma));
        sum += w[t + r];
    }
    for (int t = 0; t <= 2 * r; ++t) w[t] /= sum;
    return r;
}

/* One 1D convolution pass along `axis` (0 = x, 1 = y, 2 = z), clamp-to-edge. */
void orc_blur_axis(const double *in, double *out, int nx, int ny, int nz, int axis,
                   const double *w, int r)
{
    long n_axis = axis == 0 ? nx : (axis == 1 ? ny : nz);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long c = axis == 0 ? x : (axis == 1 ? y : z);
                double s = 0.0;
                for (int t = -r; t <= r; ++t) {
                    long q = clampl(c + t, 0, n_axis - 1);
                    size_t i = axis == 0 ? VIDX(q, y, z, nx, ny)
                             : axis == 1 ? VIDX(x, q, z, nx, ny)
                                         : VIDX(x, y, q, nx, ny);
                    s += w[t + r] * in[i];
                }
                out[VIDX(x, y, z, nx, ny)] = s;
            }
}

/*
 * Separable Gaussian blur: three 1D passes in x, then y, then z
 * (Section 3.2.2, Gaussian Convolution). `tmp` has the volume's size.
 * Returns the tap radius, or -1 if it exceeds 63.
 */
int orc_blur(const double *in, double *out, double *tmp, int nx, int ny, int nz,
             double sigma, double trunc)
{
    double w[127];
    int r = orc_gauss_taps(sigma, trunc, w, 127);
    if (r < 0) return -1;
    orc_blur_axis(in, out, nx, ny, nz, 0, w, r);
    orc_blur_axis(out, tmp, nx, ny, nz, 1, w, r);
    orc_blur_axis(tmp, out, nx, ny, nz, 2, w, r);
    return r;
}

/*
 * Difference of Gaussians (Section 3.2.2, Difference-of-Gaussian):
 * d = a - b voxel by voxel, with a the finer and b the coarser level.
 */
void orc_dog(const double *a, const double *b, double *d, size_t n)
{
    for (size_t i = 0; i < n; ++i) d[i] = a[i] - b[i];
}

/*
 * 2x sub-sampling (Section 3.2.2, Sub-sampling): each output voxel is the
 * mean of the 8 input voxels of its 2x2x2 block. Output dims are floor(n/2).
 */
void orc_subsample(const double *in, int nx, int ny, int nz, double *out)
{
    int mx = nx / 2, my = ny / 2, mz = nz / 2;
    for (int z = 0; z < mz; ++z)
        for (int y = 0; y < my; ++y)
            for (int x = 0; x < mx; ++x) {
                double s = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a)
                            s += in[VIDX(2 * x + a, 2 * y + b, 2 * z + c, nx, ny)];
                out[VIDX(x, y, z, mx, my)] = s / 8.0;
            }
}

static int sgn(double v) { return (v > 0.0) - (v < 0.0); }

/*
 * Sum of signs (Section 3.2.2, 4D Peak Detection): for the voxel (x,y,z)
 * of the middle DoG level d0, the sum over its 80 neighbours -- the 3x3x3
 * blocks of dm and dp and the 26 others of d0 -- of sign(d0(v) - neighbour).
 * The voxel must be interior (1 <= x <= nx-2, same for y and z).
 */
int orc_sum_of_signs(const double *dm, const double *d0, const double *dp,
                     int nx, int ny, int nz, int x, int y, int z)
{
    (void)nz;
    double v = d0[VIDX(x, y, z, nx, ny)];
    int f = 0;
    const double *lv[3] = {dm, d0, dp};
    for (int l = 0; l < 3; ++l)
        for (int k = -1; k <= 1; ++k)
            for (int j = -1; j <= 1; ++j)
                for (int i = -1; i <= 1; ++i) {
                    if (l == 1 && i == 0 && j == 0 && k == 0) continue;
                    f += sgn(v - lv[l][VIDX(x + i, y + j, z + k, nx, ny)]);
                }
    return f;
}

/*
 * Extremum detection on one DoG triple (Section 3.2.2, 4D Peak Detection):
 * interior voxels with |d0| > thr and sum of signs >= votes (peak) or
 * <= -votes (valley). Results in z, y, x order as rows (x, y, z, polarity).
 * Returns the number found; at most `cap` rows are written.
 */
long orc_detect(const double *dm, const double *d0, const double *dp, int nx, int ny, int nz,
                double thr, int votes, int *out, long cap)
{
    long cnt = 0;
    for (int z = 1; z < nz - 1; ++z)
        for (int y = 1; y < ny - 1; ++y)
            for (int x = 1; x < nx - 1; ++x) {
                double v = d0[VIDX(x, y, z, nx, ny)];
                if (!(fabs(v) > thr)) continue;
                int f = orc_sum_of_signs(dm, d0, dp, nx, ny, nz, x, y, z);
                if (f >= votes || f <= -votes) {
                    if (cnt < cap) {
                        out[4 * cnt + 0] = x;
                        out[4 * cnt + 1] = y;
                        out[4 * cnt + 2] = z;
                        out[4 * cnt + 3] = f > 0 ? 1 : -1;
                    }
                    ++cnt;
                }
            }
    return cnt;
}

/* Rank of each element: r_i = #{j : v_j < v_i or (v_j == v_i and j < i)}. */
void orc_rank(const double *v, int n, int *r)
{
    for (int i = 0; i < n; ++i) {
        int c = 0;
        for (int j = 0; j < n; ++j)
            if (v[j] < v[i] || (v[j] == v[i] && j < i)) ++c;
        r[i] = c;
    }
}

/*
 * Upright 3D SIFT-Rank histogram (Related Work: 2x2x2 spatial bins times 8
 * orientation bins, normalised by ranking) for keypoints on one Gaussian
 * level G. For each offset d in [-R, R]^3 around the keypoint:
 *   q = clamp(v + d); g = central-difference gradient at q (neighbours
 *   clamped); m = |g|; orientation bin = [gx>0] + 2[gy>0] + 4[gz>0];
 *   per axis the spatial weight goes to bin 0 if d < 0, bin 1 if d > 0 and
 *   half to each if d == 0; spatial bin = bx + 2 by + 4 bz;
 *   hist[8 * spatial + orientation] += m * wx * wy * wz.
 * Then rank[e] = rank of hist[e] among the 64 (ties by index).
 * `kp` holds K rows (x, y, z). hist is [K][64], rank is [K][64].
 */
void orc_siftrank(const double *G, int nx, int ny, int nz, const int *kp, long K, int R,
                  double *hist, uint8_t *rank)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (long k = 0; k < K; ++k) {
        int vx = kp[3 * k + 0], vy = kp[3 * k + 1], vz = kp[3 * k + 2];
        double h[64];
        for (int e = 0; e < 64; ++e) h[e] = 0.0;
        for (int dz = -R; dz <= R; ++dz)
            for (int dy = -R; dy <= R; ++dy)
                for (int dx = -R; dx <= R; ++dx) {
                    long qx = clampl(vx + dx, 0, nx - 1);
                    long qy = clampl(vy + dy, 0, ny - 1);
                    long qz = clampl(vz + dz, 0, nz - 1);
                    double gx = 0.5 * (G[VIDX(clampl(qx + 1, 0, nx - 1), qy, qz, nx, ny)] -
                                       G[VIDX(clampl(qx - 1, 0, nx - 1), qy, qz, nx, ny)]);
                    double gy = 0.5 * (G[VIDX(qx, clampl(qy + 1, 0, ny - 1), qz, nx, ny)] -
                                       G[VIDX(qx, clampl(qy - 1, 0, ny - 1), qz, nx, ny)]);
                    double gz = 0.5 * (G[VIDX(qx, qy, clampl(qz + 1, 0, nz - 1), nx, ny)] -
                                       G[VIDX(qx, qy, clampl(qz - 1, 0, nz - 1), nx, ny)]);
                    double m = sqrt(gx * gx + gy * gy + gz * gz);
                    int bo = (gx > 0.0) + 2 * (gy > 0.0) + 4 * (gz > 0.0);
                    double wx[2], wy[2], wz[2];
                    wx[0] = dx < 0 ? 1.0 : (dx == 0 ? 0.5 : 0.0); wx[1] = 1.0 - wx[0];
                    wy[0] = dy < 0 ? 1.0 : (dy == 0 ? 0.5 : 0.0); wy[1] = 1.0 - wy[0];
                    wz[0] = dz < 0 ? 1.0 : (dz == 0 ? 0.5 : 0.0); wz[1] = 1.0 - wz[0];
                    for (int bz = 0; bz < 2; ++bz)
                        for (int by = 0; by < 2; ++by)
                            for (int bx = 0; bx < 2; ++bx) {
                                double ws = wx[bx] * wy[by] * wz[bz];
                                if (ws == 0.0) continue;
                                h[8 * (bx + 2 * by + 4 * bz) + bo] += m * ws;
                            }
                }
        int r[64];
        orc_rank(h, 64, r);
        for (int e = 0; e < 64; ++e) {
            hist[64 * k + e] = h[e];
            rank[64 * k + e] = (uint8_t)r[e];
        }
    }
}

/*
 * BRIEF and RRIEF (Section 3.2.3). For keypoint v on Gaussian level G and
 * pair i with integer offsets (o1, o2):
 *   p1 = clamp(v + o1), p2 = clamp(v + o2),
 *   B(p) = sum_{i,j,k in [-rb, rb]} wb_i wb_j wb_k G[clamp(p + (i,j,k))]
 *   (the patch pre-blur, evaluated at the sample points),
 *   d_i = B(p1) - B(p2);
 *   BRIEF bit i = [d_i > 0], packed least-significant-bit first into
 *   64-bit words; RRIEF r_i = rank of d_i among the n (ties by index).
 * off is [n][2][3] (x,y,z) integers, wb has 2 rb + 1 taps.
 * d is [K][n], bits is [K][n/64], ranks is [K][n].
 */
void orc_brief_rrief(const double *G, int nx, int ny, int nz, const int *kp, long K,
                     const int *off, int n, const double *wb, int rb,
                     double *d, uint64_t *bits, uint16_t *ranks)
{
    int nw = (n + 63) / 64;
#pragma omp parallel for schedule(dynamic, 4)
    for (long k = 0; k < K; ++k) {
        int vx = kp[3 * k + 0], vy = kp[3 * k + 1], vz = kp[3 * k + 2];
        double *dk = d + (size_t)k * n;
        for (int i = 0; i < n; ++i) {
            double B[2];
            for (int e = 0; e < 2; ++e) {
                long px = clampl(vx + off[6 * i + 3 * e + 0], 0, nx - 1);
                long py = clampl(vy + off[6 * i + 3 * e + 1], 0, ny - 1);
                long pz = clampl(vz + off[6 * i + 3 * e + 2], 0, nz - 1);
                double s = 0.0;
                for (int c = -rb; c <= rb; ++c)
                    for (int b = -rb; b <= rb; ++b)
                        for (int a = -rb; a <= rb; ++a) {
                            double w = wb[a + rb] * wb[b + rb] * wb[c + rb];
                            s += w * G[VIDX(clampl(px + a, 0, nx - 1), clampl(py + b, 0, ny - 1),
                                            clampl(pz + c, 0, nz - 1), nx, ny)];
                        }
                B[e] = s;
            }
            dk[i] = B[0] - B[1];
        }
        for (int w = 0; w < nw; ++w) bits[(size_t)k * nw + w] = 0;
        for (int i = 0; i < n; ++i)
            if (dk[i] > 0.0) bits[(size_t)k * nw + i / 64] |= (uint64_t)1 << (i % 64);
        int *r = (int *)malloc(sizeof(int) * (size_t)n);
        orc_rank(dk, n, r);
        for (int i = 0; i < n; ++i) ranks[(size_t)k * n + i] = (uint16_t)r[i];
        free(r);
    }
}

/*
 * Dominant orientations and oriented SIFT-Rank (Related Work, 3D SIFT-Rank:
 * dominant peaks of a discrete spherical histogram of gradient directions
 * give one or more 3x3 rotations per keypoint, and the descriptor is
 * computed after reorientation). The paper does not spell the histogram
 * out; the reading taken here:
 *
 *   samples   the SIFT-Rank window: offsets d in [-R, R]^3, gradient g by
 *             central differences at q = clamp(v + d), magnitude |g|;
 *   bins      the 26 directions n/|n|, n in {-1,0,1}^3 \ {0}, numbered in
 *             the order (nz, ny, nx) = (-1,-1,-1), (-1,-1,0), ... skipping
 *             0; a vector goes to the bin of largest n.g/|n| (lowest
 *             number on ties); zero vectors go nowhere;
 *   histogram H[b] = sum of |g| over the bin's samples, V[b] = sum of g;
 *   peaks     b is a peak if H[b] > 0, H[b] >= tau * max H, and for every
 *             neighbour b' (angle <= 60 degrees: 4 (n.n')^2 >= |n|^2 |n'|^2
 *             with n.n' > 0) H[b] > H[b'], or H[b] == H[b'] and b < b';
 *             peaks are taken in decreasing H (lower number first on ties);
 *   axis 1    e1 = V[b] / |V[b]| of a primary peak;
 *   axis 2    the same histogram of p = g - (g.e1) e1 (weights |p|, sums
 *             of p), its peaks in the same order; e2 = the normalised part
 *             of V2[b] orthogonal to e1 (skipped if zero);
 *   axis 3    e3 = e1 x e2; the frame is the rotation with columns e1, e2,
 *             e3; frames are listed primary by primary, secondaries in
 *             order within each, at most kmax;
 *   oriented  SIFT-Rank of each frame: every sample's offset and gradient
 *             in frame coordinates, d' = R^T d and g' = R^T g, then the
 *             upright rule: spatial bin per axis 0 if d'_k < 0, 1 if > 0,
 *             half to each if 0; orientation bin [g'_1>0] + 2[g'_2>0] +
 *             4[g'_3>0]; weight |g|; ranks with ties by index. With the
 *             identity frame this is the upright descriptor exactly.
 *
 * Outputs per keypoint k: nframes[k]; frames[k][f][9] with R[3 i + j] =
 * component i of axis j; hist/rank[k][f][64]; margin[k] = the smallest of
 * the relative decision margins: bin choice (best - second best n.g/|n|)
 * / |g|, peak tests |H[b] - tau max H| / max H and |H[b] - H[b']| / max H
 * over neighbours, |H[b] - H[b']| / max H of peaks next to each other in
 * the order, and, per frame, |d'_k| / R and |g'_k| / |g| of every nonzero
 * sample. A GPU taking the same decisions in another rounding
 * order can only differ where this margin is tiny.
 */
static void orc_dir(int b, int n[3])
{
    int q = b < 13 ? b : b + 1;              /* skip the zero vector (index 13 of 27) */
    n[0] = q % 3 - 1;
    n[1] = (q / 3) % 3 - 1;
    n[2] = q / 9 - 1;
}

/* Bin of vector g (|g| > 0) and the relative margin of the choice. */
static int orc_dirbin(const double g[3], double *margin)
{
    double best = -HUGE_VAL, second = -HUGE_VAL;
    int arg = -1;
    for (int b = 0; b < 26; ++b) {
        int n[3];
        orc_dir(b, n);
        double nn = (double)(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        double c = (n[0] * g[0] + n[1] * g[1] + n[2] * g[2]) / sqrt(nn);
        if (c > best) {
            second = best;
            best = c;
            arg = b;
        } else if (c > second) {
            second = c;
        }
    }
    double m = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    double r = (best - second) / m;
    if (r < *margin) *margin = r;
    return arg;
}

static int orc_neighbours(int a, int b)
{
    int na[3], nb[3];
    orc_dir(a, na);
    orc_dir(b, nb);
    long d = na[0] * nb[0] + na[1] * nb[1] + na[2] * nb[2];
    long qa = na[0] * na[0] + na[1] * na[1] + na[2] * na[2];
    long qb = nb[0] * nb[0] + nb[1] * nb[1] + nb[2] * nb[2];
    return a != b && d > 0 && 4 * d * d >= qa * qb;
}

/* Peaks of H in order; returns their count. */
static int orc_peaks(const double H[26], double tau, int *out, double *margin)
{
    double hmax = 0.0;
    for (int b = 0; b < 26; ++b)
        if (H[b] > hmax) hmax = H[b];
    if (!(hmax > 0.0)) return 0;
    int np = 0;
    for (int b = 0; b < 26; ++b) {
        if (!(H[b] > 0.0)) continue;
        double r = fabs(H[b] - tau * hmax) / hmax;
        if (r < *margin) *margin = r;
        if (H[b] < tau * hmax) continue;
        int peak = 1;
        for (int c = 0; c < 26; ++c) {
            if (!orc_neighbours(b, c)) continue;
            double rc = fabs(H[b] - H[c]) / hmax;
            if (rc < *margin) *margin = rc;
            if (!(H[b] > H[c] || (H[b] == H[c] && b < c))) peak = 0;
        }
        if (peak) out[np++] = b;
    }
    /* decreasing H, lower bin first on ties (insertion sort) */
    for (int i = 1; i < np; ++i)
        for (int j = i; j > 0; --j) {
            int a = out[j - 1], c = out[j];
            if (H[c] > H[a] || (H[c] == H[a] && c < a)) {
                out[j - 1] = c;
                out[j] = a;
            }
        }
    for (int i = 1; i < np; ++i) {
        double r = fabs(H[out[i - 1]] - H[out[i]]) / hmax;   /* the order of two peaks */
        if (r < *margin) *margin = r;
    }
    return np;
}

static void orc_sample_grad(const double *G, int nx, int ny, int nz, long qx, long qy, long qz, double g[3])
{
    g[0] = 0.5 * (G[VIDX(clampl(qx + 1, 0, nx - 1), qy, qz, nx, ny)] - G[VIDX(clampl(qx - 1, 0, nx - 1), qy, qz, nx, ny)]);
    g[1] = 0.5 * (G[VIDX(qx, clampl(qy + 1, 0, ny - 1), qz, nx, ny)] - G[VIDX(qx, clampl(qy - 1, 0, ny - 1), qz, nx, ny)]);
    g[2] = 0.5 * (G[VIDX(qx, qy, clampl(qz + 1, 0, nz - 1), nx, ny)] - G[VIDX(qx, qy, clampl(qz - 1, 0, nz - 1), nx, ny)]);
}

/* SIFT-Rank histogram of keypoint v in frame F (R[3 i + j] = component i of
 * axis j): offsets and gradients in frame coordinates, then the upright
 * binning. Lowers *mg to the smallest |d'_k| / R and |g'_k| / |g|. */
static void orc_frame_hist(const double *G, int nx, int ny, int nz, long vx, long vy, long vz, int R,
                           const double *F, double h[64], double *mg)
{
    for (int e = 0; e < 64; ++e) h[e] = 0.0;
    for (int dz = -R; dz <= R; ++dz)
        for (int dy = -R; dy <= R; ++dy)
            for (int dx = -R; dx <= R; ++dx) {
                double g[3];
                orc_sample_grad(G, nx, ny, nz, clampl(vx + dx, 0, nx - 1), clampl(vy + dy, 0, ny - 1),
                                clampl(vz + dz, 0, nz - 1), g);
                double m = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
                double d[3] = {(double)dx, (double)dy, (double)dz};
                double dp[3], gp[3];
                for (int j = 0; j < 3; ++j) {
                    dp[j] = F[0 + j] * d[0] + F[3 + j] * d[1] + F[6 + j] * d[2];
                    gp[j] = F[0 + j] * g[0] + F[3 + j] * g[1] + F[6 + j] * g[2];
                    if (dp[j] != 0.0 && fabs(dp[j]) / R < *mg) *mg = fabs(dp[j]) / R;
                    if (m > 0.0 && gp[j] != 0.0 && fabs(gp[j]) / m < *mg) *mg = fabs(gp[j]) / m;
                }
                int bo = (gp[0] > 0.0) + 2 * (gp[1] > 0.0) + 4 * (gp[2] > 0.0);
                double w[3][2];
                for (int j = 0; j < 3; ++j) {
                    w[j][0] = dp[j] < 0.0 ? 1.0 : (dp[j] == 0.0 ? 0.5 : 0.0);
                    w[j][1] = 1.0 - w[j][0];
                }
                for (int bz = 0; bz < 2; ++bz)
                    for (int by = 0; by < 2; ++by)
                        for (int bx = 0; bx < 2; ++bx) {
                            double ws = w[0][bx] * w[1][by] * w[2][bz];
                            if (ws == 0.0) continue;
                            h[8 * (bx + 2 * by + 4 * bz) + bo] += m * ws;
                        }
            }
}

/* SIFT-Rank of keypoints in given frames (frames [K][9]); hist [K][64],
 * rank [K][64], margin [K] as in orc_orient. */
void orc_siftrank_frames(const double *G, int nx, int ny, int nz, const int *kp, long K, int R,
                         const double *frames, double *hist, uint8_t *rank, double *margin)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (long k = 0; k < K; ++k) {
        double mg = HUGE_VAL;
        orc_frame_hist(G, nx, ny, nz, kp[3 * k], kp[3 * k + 1], kp[3 * k + 2], R, frames + 9 * k, hist + 64 * k, &mg);
        int r[64];
        orc_rank(hist + 64 * k, 64, r);
        for (int e = 0; e < 64; ++e) rank[64 * k + e] = (uint8_t)r[e];
        margin[k] = mg;
    }
}

void orc_orient(const double *G, int nx, int ny, int nz, const int *kp, long K, int R, double tau, int kmax,
                int *nframes, double *frames, double *hist, uint8_t *rank, double *margin)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (long k = 0; k < K; ++k) {
        long vx = kp[3 * k + 0], vy = kp[3 * k + 1], vz = kp[3 * k + 2];
        double mg = HUGE_VAL;
        double H[26], V[26][3];
        for (int b = 0; b < 26; ++b) H[b] = V[b][0] = V[b][1] = V[b][2] = 0.0;
        /* primary histogram */
        for (int dz = -R; dz <= R; ++dz)
            for (int dy = -R; dy <= R; ++dy)
                for (int dx = -R; dx <= R; ++dx) {
                    double g[3];
                    orc_sample_grad(G, nx, ny, nz, clampl(vx + dx, 0, nx - 1), clampl(vy + dy, 0, ny - 1),
                                    clampl(vz + dz, 0, nz - 1), g);
                    double m = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
                    if (!(m > 0.0)) continue;
                    int b = orc_dirbin(g, &mg);
                    H[b] += m;
                    V[b][0] += g[0];
                    V[b][1] += g[1];
                    V[b][2] += g[2];
                }
        int prim[26];
        int np = orc_peaks(H, tau, prim, &mg);
        int nf = 0;
        for (int ip = 0; ip < np && nf < kmax; ++ip) {
            const double *v = V[prim[ip]];
            double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            double e1[3] = {v[0] / vn, v[1] / vn, v[2] / vn};
            double H2[26], V2[26][3];
            for (int b = 0; b < 26; ++b) H2[b] = V2[b][0] = V2[b][1] = V2[b][2] = 0.0;
            for (int dz = -R; dz <= R; ++dz)
                for (int dy = -R; dy <= R; ++dy)
                    for (int dx = -R; dx <= R; ++dx) {
                        double g[3];
                        orc_sample_grad(G, nx, ny, nz, clampl(vx + dx, 0, nx - 1), clampl(vy + dy, 0, ny - 1),
                                        clampl(vz + dz, 0, nz - 1), g);
                        double a = g[0] * e1[0] + g[1] * e1[1] + g[2] * e1[2];
                        double p[3] = {g[0] - a * e1[0], g[1] - a * e1[1], g[2] - a * e1[2]};
                        double m2 = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
                        if (!(m2 > 0.0)) continue;
                        int b = orc_dirbin(p, &mg);
                        H2[b] += m2;
                        V2[b][0] += p[0];
                        V2[b][1] += p[1];
                        V2[b][2] += p[2];
                    }
            int sec[26];
            int ns = orc_peaks(H2, tau, sec, &mg);
            for (int is = 0; is < ns && nf < kmax; ++is) {
                const double *w = V2[sec[is]];
                double a = w[0] * e1[0] + w[1] * e1[1] + w[2] * e1[2];
                double u[3] = {w[0] - a * e1[0], w[1] - a * e1[1], w[2] - a * e1[2]};
                double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                if (!(un > 0.0)) continue;
                double e2[3] = {u[0] / un, u[1] / un, u[2] / un};
                double e3[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                                e1[0] * e2[1] - e1[1] * e2[0]};
                double *F = frames + ((size_t)k * kmax + nf) * 9;
                for (int i = 0; i < 3; ++i) {
                    F[3 * i + 0] = e1[i];
                    F[3 * i + 1] = e2[i];
                    F[3 * i + 2] = e3[i];
                }
                ++nf;
            }
        }
        nframes[k] = nf;
        /* oriented SIFT-Rank per frame */
        for (int f = 0; f < nf; ++f) {
            double *h = hist + ((size_t)k * kmax + f) * 64;
            orc_frame_hist(G, nx, ny, nz, vx, vy, vz, R, frames + ((size_t)k * kmax + f) * 9, h, &mg);
            int r[64];
            orc_rank(h, 64, r);
            for (int e = 0; e < 64; ++e) rank[((size_t)k * kmax + f) * 64 + e] = (uint8_t)r[e];
        }
        margin[k] = mg;
    }
}
