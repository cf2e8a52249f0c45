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
