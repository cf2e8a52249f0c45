/*
 * Drives every routine of oracle/sift3d_oracle.c on small and edge-case
 * inputs (one-voxel axes, keypoints at corners, offsets far outside the
 * volume) so that a build with the address and undefined-behaviour
 * sanitizers checks the oracle's indexing. Exit status 0 on success; the
 * sanitizers abort with a report otherwise.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_gauss_taps(double sigma, double trunc, double *w, int cap);
void orc_blur_axis(const double *in, double *out, int nx, int ny, int nz, int axis, const double *w, int r);
int orc_blur(const double *in, double *out, double *tmp, int nx, int ny, int nz, double sigma, double trunc);
void orc_dog(const double *a, const double *b, double *d, size_t n);
void orc_subsample(const double *in, int nx, int ny, int nz, double *out);
long orc_detect(const double *dm, const double *d0, const double *dp, int nx, int ny, int nz, double thr,
                int votes, int *out, long cap);
void orc_siftrank(const double *G, int nx, int ny, int nz, const int *kp, long K, int R, double *hist,
                  uint8_t *rank);
void orc_brief_rrief(const double *G, int nx, int ny, int nz, const int *kp, long K, const int *off, int n,
                     const double *wb, int rb, double *d, uint64_t *bits, uint16_t *ranks);

static double frand(unsigned *s)
{
    *s = *s * 1103515245u + 12345u;
    return ((*s >> 8) & 0xffff) / 65536.0 - 0.5;
}

static int run(int nx, int ny, int nz, unsigned seed)
{
    size_t n = (size_t)nx * ny * nz;
    double *a = malloc(n * sizeof(double)), *b = malloc(n * sizeof(double)), *c = malloc(n * sizeof(double));
    double *d = malloc(n * sizeof(double)), *t = malloc(n * sizeof(double));
    for (size_t i = 0; i < n; ++i) a[i] = frand(&seed);
    double w[127];
    int r = orc_gauss_taps(3.09, 3.0, w, 127);
    for (int axis = 0; axis < 3; ++axis) orc_blur_axis(a, b, nx, ny, nz, axis, w, r);
    orc_blur(a, b, t, nx, ny, nz, 1.6, 3.0);
    orc_blur(b, c, t, nx, ny, nz, 1.2263, 3.0);
    orc_dog(b, c, d, n);
    double *sub = malloc(((size_t)(nx / 2) * (ny / 2) * (nz / 2) + 1) * sizeof(double));
    orc_subsample(c, nx, ny, nz, sub);
    int *out = malloc(4 * 64 * sizeof(int));
    long k = orc_detect(a, b, c, nx, ny, nz, 0.0, 80, out, 64);
    k += orc_detect(a, b, c, nx, ny, nz, 0.0, 60, out, 64);
    int kp[3 * 4] = {0, 0, 0, nx - 1, ny - 1, nz - 1, nx / 2, ny / 2, nz / 2, 0, ny - 1, nz / 3};
    double hist[4 * 64];
    uint8_t rank[4 * 64];
    orc_siftrank(c, nx, ny, nz, kp, 4, 7, hist, rank);
    int off[64 * 6];
    for (int i = 0; i < 64 * 6; ++i) off[i] = (int)(frand(&seed) * 80.0);
    double wb[7];
    int rb = orc_gauss_taps(0.95, 3.0, wb, 7);
    double dd[4 * 64];
    uint64_t bits[4];
    uint16_t rr[4 * 64];
    orc_brief_rrief(c, nx, ny, nz, kp, 4, off, 64, wb, rb, dd, bits, rr);
    printf("%dx%dx%d: %ld candidates\n", nx, ny, nz, k);
    free(a); free(b); free(c); free(d); free(t); free(sub); free(out);
    return 0;
}

int main(void)
{
    run(1, 1, 1, 1);
    run(3, 1, 5, 2);
    run(17, 9, 4, 3);
    run(24, 20, 22, 4);
    return 0;
}
