/*
 * sift3d.h -- C ABI of the MI355X (gfx950) 3D SIFT-Rank hot path.
 *
 * Method: Carluer et al., "GPU optimization of the 3D Scale-invariant
 * Feature Transform Algorithm and a Novel BRIEF-inspired 3D Fast
 * Descriptor" (arXiv 2112.10258). The problem statement (Section 3.1):
 * a scalar volume I_x goes to keypoints (sigma_i, x_i) found as 4D extrema
 * of a difference-of-Gaussian scale space, each described by a vector f_i.
 *
 * Conventions
 *   - Volumes are float32, layout [z][y][x] with x fastest, dims (nx,ny,nz).
 *   - All device pointers (prefix d_) are HIP device memory owned by the
 *     caller. The library owns only its host handles and one small device
 *     table per context (pair offsets), freed by sift3d_destroy.
 *   - `stream` is a hipStream_t (NULL = the null stream). Every call that
 *     takes a stream only enqueues work on it and returns without waiting;
 *     no call synchronises the device, so a whole sift3d_extract can be
 *     captured into a HIP graph. Inputs must stay alive until the stream
 *     work completes.
 *   - Functions return SIFT3D_OK (0) or a negative SIFT3D_E_* code; they
 *     never abort. On SIFT3D_E_HIP, sift3d_last_hip_error() gives the
 *     hipError_t of the failing call on this thread.
 *   - Octave o has dims floor(dims_{o-1} / 2). Each octave holds S+3
 *     Gaussian levels G_0..G_{S+2} and S+2 DoG levels D_0..D_{S+1}.
 */
#ifndef SIFT3D_H
#define SIFT3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SIFT3D_OK = 0,
    SIFT3D_E_ARG = -1,        /* null pointer, bad parameter or size       */
    SIFT3D_E_TOO_SMALL = -2,  /* volume gives no octave (min dim < min_dim) */
    SIFT3D_E_WORKSPACE = -3,  /* workspace smaller than the plan needs      */
    SIFT3D_E_HIP = -5,        /* a HIP runtime call failed                  */
    SIFT3D_E_UNSUPPORTED = -6, /* parameter outside what the kernels support */
    SIFT3D_E_SCRATCH = -7,    /* plan needs more than the static scratch    */
    SIFT3D_E_TIMEOUT = -8,    /* server request not admitted in time        */
    SIFT3D_PENDING = 1         /* sift3d_server_result: not finished yet   */
};

/* Method parameters. sift3d_default_params() fills the defaults in []. */
typedef struct sift3d_params {
    int n_octaves;          /* [0] 0 = keep octave o while min(dims_o) >= min_dim;
                               >0 = at most this many octaves                    */
    int min_dim;            /* [16] smallest dimension an octave may have (>= 4) */
    int scales;             /* [3] S, detection scales per octave, 1..5          */
    double sigma0;          /* [1.6] blur of G_0 in its octave's voxels          */
    double sigma_in;        /* [0.0] blur already present in the input           */
    double trunc;           /* [3.0] tap radius r = ceil(trunc * sigma), r <= 16 */
    float dog_threshold;    /* [0.01] keypoints need |D| > dog_threshold         */
    int votes;              /* [80] sum-of-signs acceptance |f| >= votes, 1..80  */
    int brief_n;            /* [256] BRIEF/RRIEF pairs, multiple of 64, <= 256   */
    double brief_blur;      /* [0.95] patch pre-blur sigma_b (0 = none); its tap
                               radius ceil(trunc * sigma_b) <= 10 */
    double siftrank_factor; /* [2.0] SIFT-Rank half-width R = ceil(f * sigma_s), R <= 7 */
    int pyramid_mode;       /* [0] 0 = by size (fused streaming pass for octaves of
                               >= 24M voxels, and for levels of radius <= 8 in
                               octaves of >= 2M voxels; compact one-launch pass
                               below 2M voxels, for radii <= 8 only from 1M
                               voxels on; xy + z launches for the rest),
                               1 = always fused, 2 = always xy + z, 3 = always
                               compact; results agree to rounding. Levels whose
                               tap radius exceeds 10 always run as xy + z
                               launches */
    int brief_method;       /* [3] point-pair selection (Section 3.2.3), sigma the
                               keypoint scale: 1 = p1, p2 uniform in the ball of
                               radius 2 sigma; 2 = p1, p2 ~ N(0, sigma); 3 = p1 ~
                               N(0, sigma), p2 ~ N(p1, sigma); 4 = p1 at the
                               centre, p2 ~ N(0, sigma); 5 = p1 at the centre,
                               p2 on a regular spherical grid. Built from the
                               pair draws as sift3d_pair_offsets describes */
} sift3d_params;

/*
 * One keypoint (40 bytes). (x, y, z) are voxel coordinates in octave
 * `octave`, `scale` is the DoG level s (1..S) it is an extremum of,
 * polarity is +1 for a peak and -1 for a valley, `dog` is D_s at the
 * voxel. (xf, yf, zf) is the position in input voxels,
 * 2^o * x + (2^o - 1) / 2, and sigma = sigma0 * 2^(s/S) * 2^o.
 */
typedef struct sift3d_keypoint {
    int32_t x, y, z;
    int16_t octave, scale;
    int8_t polarity;
    int8_t pad[3];
    float dog, xf, yf, zf, sigma;
} sift3d_keypoint;

typedef struct sift3d_ctx sift3d_ctx;
typedef struct sift3d_plan sift3d_plan;

/* Fill *p with the defaults listed above. */
int sift3d_default_params(sift3d_params *p);

/*
 * Create a context on the current HIP device.
 * pair_draws: host array [n_draws][2][3] of standard-normal draws (z1, z2)
 * for the BRIEF/RRIEF point pairs (Section 3.2.3, method 3: p1 ~ N(0, sigma),
 * p2 ~ N(p1, sigma)); pair i uses u1 = z1, u2 = z1 + z2 and, at scale s,
 * the integer offsets floor(sigma_s * u + 0.5) with sigma_s = sigma0 2^(s/S).
 * n_draws >= brief_n. May be NULL only if brief_n == 0. The draws are
 * copied; the offset tables are uploaded synchronously to device memory
 * that the context owns.
 */
int sift3d_create(const sift3d_params *p, const double *pair_draws, int n_draws, sift3d_ctx **out);
int sift3d_destroy(sift3d_ctx *ctx);

/* Copy of the parameters a context was created with. */
int sift3d_ctx_params(const sift3d_ctx *ctx, sift3d_params *out);

/*
 * Integer pair offsets of scale s (1..S) that a context built from the same
 * parameters and draws uses: out is [brief_n][2][3] (x,y,z). Pure host
 * function (no device needed). pair_draws holds two standard-normal
 * 3-vectors (z1, z2) per pair; with sigma the scale-s sigma in octave
 * voxels, the real-valued points are, by brief_method:
 *   1: p1 = 2 sigma F(|z2|^2)^(1/3) z1/|z1|, p2 = 2 sigma F(|z1|^2)^(1/3) z2/|z2|,
 *      F the chi-square CDF with 3 degrees of freedom (uniform in the ball);
 *   2: p1 = sigma z1, p2 = sigma z2;    3: p1 = sigma z1, p2 = sigma (z1 + z2);
 *   4: p1 = 0, p2 = sigma z2;
 *   5: p1 = 0, p2 = pair 64 k + 8 j + i of a spherical grid: radius
 *      2 sigma (k+1)/(n/64), polar angle pi (j + 1/2)/8, azimuth
 *      2 pi (i + (j mod 2)/2)/8 (z1, z2 unused);
 * each coordinate rounded as floor(c + 0.5).
 */
int sift3d_pair_offsets(const sift3d_params *p, const double *pair_draws, int n_draws, int scale,
                        int32_t *out);

/*
 * Plan extraction for one volume shape (a plan over one volume). Host
 * planning plus one small device table (the plan's job descriptors, holding
 * offsets only) uploaded synchronously; freed by sift3d_plan_destroy.
 * kp_capacity >= 0 is the size of the caller's keypoint and descriptor
 * buffers per volume. The plan keeps a pointer to ctx, which must outlive it.
 * Shapes: nx, ny, nz >= 1, nx * ny <= 2^28 (a plane of at most 1 GiB) and
 * nx * ny * nz <= 2^40; SIFT3D_E_ARG otherwise.
 */
int sift3d_plan_create(sift3d_ctx *ctx, int nx, int ny, int nz, int kp_capacity, sift3d_plan **out);

/*
 * Plan extraction for a batch of n_volumes volumes of any sizes; dims is
 * [n_volumes][3] (nx, ny, nz). Every call on such a plan processes all
 * volumes together: each launch covers the same stage of every volume.
 * Per-volume results are identical to a one-volume plan's. The input is one
 * packed buffer: volume v starts at element offset input_offset(v)
 * (sift3d_plan_volume), 256-byte aligned. Outputs are [n_volumes] blocks:
 * keypoints [n_volumes][kp_capacity], counts [n_volumes], descriptors
 * [n_volumes][kp_capacity][...]. n_volumes <= 4096.
 */
int sift3d_plan_create_batch(sift3d_ctx *ctx, int n_volumes, const int *dims, int kp_capacity,
                             sift3d_plan **out);
int sift3d_plan_destroy(sift3d_plan *plan);

/* Workspace size in bytes, number of volumes, and floats of the packed input. */
int sift3d_plan_info(const sift3d_plan *plan, size_t *workspace_bytes, int *n_volumes, size_t *input_elems);

/* Dims, element offset in the packed input, and octave count of volume v. */
int sift3d_plan_volume(const sift3d_plan *plan, int volume, int dims[3], size_t *input_offset, int *n_octaves);

/* Dims (nx, ny, nz) of octave o of volume v. */
int sift3d_plan_octave_dims(const sift3d_plan *plan, int volume, int octave, int dims[3]);

/*
 * Device pointer of one pyramid level inside a workspace: kind 0 = G_idx
 * (idx 0..S+2), kind 1 = D_idx (idx 0..S+1), kind 2 = B_idx, the BRIEF
 * pre-blur of G_idx (idx 1..S; only when the plan pre-blurs, i.e.
 * brief_blur > 0 and brief_n > 0). A view, no copy; the level is a
 * [nz][ny][nx] float32 array of the octave's dims.
 */
int sift3d_level(const sift3d_plan *plan, void *d_ws, int volume, int octave, int kind, int idx,
                 float **d_ptr);

/*
 * Gaussian scale space, DoG and sub-sampling (Section 3.2.2, Gaussian
 * Convolution, Sub-sampling, Difference-of-Gaussian):
 *   octave 0: G_0 = I blurred by sqrt(sigma0^2 - sigma_in^2);
 *   octave o > 0: G_0 = mean of each 2x2x2 block of G_S of octave o-1;
 *   G_i = G_{i-1} blurred by sigma0 sqrt(kappa^(2i) - kappa^(2i-2)),
 *         kappa = 2^(1/S), i = 1..S+2 (separable x, y, z passes, taps a
 *         normalised sampled Gaussian, clamp-to-edge);
 *   D_i = G_i - G_{i+1}, i = 0..S+1;
 *   and, when brief_n > 0 and brief_blur > 0, the BRIEF patch pre-blur of
 *   G_s, s = 1..S (Section 3.2.3: the patch is Gaussian-blurred before the
 *   pair differences), as whole levels with the same clamp-to-edge rule.
 * Independent levels (the last levels of octave o, the first of octave o+1,
 * the pre-blurs) share launches.
 * d_vol: the input, [nz][ny][nx] float32 (the packed volumes of a batch
 * plan), read only. d_ws: workspace of at least the planned size (256-byte
 * aligned); all levels are written into it.
 */
int sift3d_build_pyramid(const sift3d_plan *plan, const float *d_vol, void *d_ws, size_t ws_bytes,
                         void *stream);

/*
 * The pyramid is built by sift3d_pyramid_pass_count() level passes, run in
 * index order; sift3d_build_pyramid() runs them all. Pass i reads one level
 * once and writes G_level of `octave`, D_{level-1} (level > 0) and, for
 * level S of a non-final octave, G_0 of the next octave. Exposed so that a
 * caller can time or re-run single passes; the workspace must hold the
 * passes' inputs (pass 0 reads d_vol). The passes do not write the BRIEF
 * pre-blurred levels; sift3d_build_pyramid does.
 *   info[0] = octave, info[1] = level, info[2] = tap radius, info[3] = 1 if
 *   the pass also writes the next octave's G_0, info[4] = how it runs: 1 =
 *   one fused streaming launch, 2 = one compact launch, 0 = an xy launch
 *   followed by a z launch; info[5] = volume;
 *   *bytes = algorithmic HBM bytes of the pass: 4 per voxel read, 4 per
 *   voxel written for G and D, 4 per sub-sampled voxel.
 */
int sift3d_pyramid_pass_count(const sift3d_plan *plan, int *n_passes);
int sift3d_pyramid_pass_info(const sift3d_plan *plan, int pass, int info[6], size_t *bytes);
int sift3d_pyramid_pass(const sift3d_plan *plan, int pass, const float *d_vol, void *d_ws, size_t ws_bytes,
                        void *stream);

/*
 * The launches of sift3d_build_pyramid, exposed so that a caller can time
 * each one on its stream (the same kernels, grids and order; running steps
 * 0 .. count-1 in order is sift3d_build_pyramid). A launch may hold the
 * passes of several levels, octaves and volumes that are ready together.
 *   info[0] = kind: 0 = fused streaming pass, 1 = xy half and 2 = z half of
 *             the two-launch pass, 3 = compact pass;
 *   info[1] = level passes in it; info[2] = stand-alone BRIEF pre-blurs in it;
 *   info[3] = largest tap radius; info[4], info[5] = lowest and highest
 *             octave; info[6], info[7] = lowest and highest level index i of
 *             the G_i it writes (-1 if none); info[8] = 1 if its level
 *             passes also write the BRIEF pre-blurred levels of their source.
 *   *bytes = algorithmic HBM bytes of the levels the launch completes (0
 *             for an xy half): 4 per voxel read and per voxel written (G,
 *             D, sub-sampled G_0 of the next octave, pre-blurred level).
 * SIFT3D_E_ARG for a bad step index or a null plan or output.
 */
int sift3d_pyramid_step_count(const sift3d_plan *plan, int *n_steps);
int sift3d_pyramid_step_info(const sift3d_plan *plan, int step, int info[9], size_t *bytes);
int sift3d_pyramid_step(const sift3d_plan *plan, int step, const float *d_vol, void *d_ws, size_t ws_bytes,
                        void *stream);

/*
 * Autotune the plan's fused streaming launches on this device: for every
 * fused launch of the schedule, time `reps` launches (after one untimed) of
 * each candidate tile height (16 or 32 rows) and number of z-slabs per job
 * (1, and 1/2 .. 4 times the rule that fills every resident workgroup slot
 * once), and keep the fastest; the plan's schedule and device tables are
 * rebuilt with the choices. The candidates compute every voxel's stencils
 * in the same order, so a tuned plan gives bit-identical results. Runs the
 * whole pyramid of d_vol into d_ws first (every launch's input must exist)
 * and synchronises `stream` between candidates: a plan-time call, not to be
 * made while other work uses the plan. On error the plan is restored to the
 * default rule. reps in 1..1000.
 */
int sift3d_plan_tune(sift3d_plan *plan, const float *d_vol, void *d_ws, size_t ws_bytes, int reps, void *stream);

/* Results of the last sift3d_plan_tune: one record per fused launch;
 * info = {schedule step, default tile height, default slabs, tuned tile
 * height, tuned slabs, candidates timed}, ms = {default, tuned} average
 * launch time in milliseconds. */
int sift3d_plan_tuning_count(const sift3d_plan *plan, int *n);
int sift3d_plan_tuning(const sift3d_plan *plan, int idx, int info[6], float ms[2]);

/*
 * 4D extremum detection (Section 3.2.2, 4D Peak Detection): for every
 * octave, scale s = 1..S and interior voxel v (1 <= x <= nx-2, same for y,
 * z) keep v if |D_s(v)| > dog_threshold and the sum over its 80 neighbours
 * in D_{s-1}, D_s, D_{s+1} of sign(D_s(v) - neighbour) is >= votes (peak)
 * or <= -votes (valley). Each volume's keypoints are written to its block
 * d_kp[v * kp_capacity ...] in (octave, scale, z, y, x) order, at most
 * kp_capacity of them; d_count[v] (device ints) receives the total number
 * found, which may exceed kp_capacity (then the list is the first
 * kp_capacity in that order). Uses the workspace's scratch area; the
 * pyramid must have been built in d_ws. Inputs must be finite.
 */
int sift3d_detect(const sift3d_plan *plan, void *d_ws, size_t ws_bytes, sift3d_keypoint *d_kp,
                  int kp_capacity, int *d_count, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * detection as sift3d_detect, with the same outputs, but its scratch (row
 * counts, block sums and offsets, keypoint bit masks) is a static device
 * array of SIFT3D_DETECT_STATIC_SCRATCH bytes that the library holds on
 * every GPU it runs on until the process ends, not the workspace's scratch
 * area. The workspace only needs to hold the pyramid (its first bytes, up
 * to where the plan's detection scratch would start); ws_bytes may be the
 * full planned size. The call allocates nothing and issues no memset: the
 * kernels write every scratch word they read. The array's address on each
 * device is taken by sift3d_create with that device current, so a context
 * must have been created on the current device before this call.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (two streams, two threads) race and give wrong results.
 * SIFT3D_E_SCRATCH if the plan's detection scratch (it grows with the
 * number of rows, about 12 bytes per 62 voxels of every octave and scale)
 * exceeds SIFT3D_DETECT_STATIC_SCRATCH (a 512x512x384 volume needs about
 * 50 MB); SIFT3D_E_ARG / SIFT3D_E_WORKSPACE as for sift3d_detect.
 */
#define SIFT3D_DETECT_STATIC_SCRATCH ((size_t)64 << 20)
int sift3d_detect_static(const sift3d_plan *plan, void *d_ws, size_t ws_bytes, sift3d_keypoint *d_kp,
                         int kp_capacity, int *d_count, void *stream);

/* Bytes of detection scratch a plan needs (for sift3d_detect_static). */
int sift3d_plan_detect_scratch(const sift3d_plan *plan, size_t *bytes);

/*
 * Descriptors of keypoints 0 .. min(d_count[v], kp_capacity) - 1 of every
 * volume v, each on G_s of its octave; row k of volume v is at
 * v * kp_capacity + k. Any of the three outputs may be NULL to skip it.
 *   d_siftrank [cap][64] uint8: upright SIFT-Rank (Section 2, 2x2x2
 *     spatial x 8 orientation bins, normalised by ranking): over the
 *     window d in [-R, R]^3, R = ceil(siftrank_factor * sigma_s), the
 *     central-difference gradient g at clamp(v + d) adds |g| to orientation
 *     bin [gx>0] + 2[gy>0] + 4[gz>0] of spatial bin (bx + 2 by + 4 bz),
 *     where per axis d < 0 -> 0, d > 0 -> 1 and d = 0 splits half/half;
 *     element e = 8 * spatial + orientation holds the rank of its sum
 *     among the 64 (ties broken by index).
 *   d_brief [cap][brief_n/64] uint64: bit i (least significant first) is
 *     [B(p1_i) - B(p2_i) > 0] with p = clamp(v + offset) and B the
 *     sigma_b Gaussian pre-blur of G_s evaluated at p (Section 3.2.3),
 *     read from the pre-blurred level sift3d_build_pyramid wrote.
 *   d_rrief [cap][brief_n] uint8: rank of d_i = B(p1_i) - B(p2_i) among
 *     the brief_n differences (Section 3.2.3, RRIEF; ties by index).
 */
int sift3d_describe(const sift3d_plan *plan, const void *d_ws, size_t ws_bytes,
                    const sift3d_keypoint *d_kp, const int *d_count, int kp_capacity,
                    uint8_t *d_siftrank, uint64_t *d_brief, uint8_t *d_rrief, void *stream);

/*
 * Dominant orientations and SIFT-Rank after reorientation (Related Work,
 * 3D SIFT-Rank: dominant peaks of a discrete spherical histogram of
 * gradient directions give one or more 3x3 rotations per keypoint, and the
 * descriptor is computed in each rotated frame). For keypoint k of volume v
 * (row v * kp_capacity + k, k < min(d_count[v], kp_capacity)), on G_s of
 * its octave, over the SIFT-Rank window d in [-R, R]^3:
 *   - every sample's gradient g (central differences at clamp(v + d)) with
 *     |g| > 0 goes to the nearest of the 26 directions n/|n|,
 *     n in {-1,0,1}^3 \ {0}; a bin sums |g| and g;
 *   - peaks: bins whose sum is >= peak_ratio times the largest and above
 *     every bin within 60 degrees (equal sums: the lower bin number, with
 *     bins numbered in (z, y, x) order of n, wins), in decreasing order;
 *     each gives a primary axis e1 = the bin's mean gradient, normalised;
 *   - per primary axis, the same histogram of g - (g.e1) e1; each of its
 *     peaks gives e2 (its mean, orthogonal part, normalised), e3 = e1 x e2;
 *   - frames are listed primary by primary, at most SIFT3D_MAX_ORIENTATIONS;
 *   - per frame, SIFT-Rank with each sample's offset and gradient in frame
 *     coordinates (R^T d, R^T g) and the upright binning rules.
 * Outputs: d_nframes [cap] int (0..SIFT3D_MAX_ORIENTATIONS); d_frames
 * [cap][SIFT3D_MAX_ORIENTATIONS][9] float32, R[3 i + j] = component i of
 * axis j (unused frames zero); d_siftrank [cap][SIFT3D_MAX_ORIENTATIONS][64]
 * uint8 ranks (unused frames zero). Sums are fixed-point integers, so the
 * results are bit-reproducible. 0 < peak_ratio <= 1 (0.8 is the usual
 * value), else SIFT3D_E_ARG. The pyramid must have been built in d_ws.
 */
#define SIFT3D_MAX_ORIENTATIONS 4
int sift3d_orient(const sift3d_plan *plan, const void *d_ws, size_t ws_bytes,
                  const sift3d_keypoint *d_kp, const int *d_count, int kp_capacity, double peak_ratio,
                  int *d_nframes, float *d_frames, uint8_t *d_siftrank, void *stream);

/* build_pyramid + detect + describe on one stream. */
int sift3d_extract(const sift3d_plan *plan, const float *d_vol, void *d_ws, size_t ws_bytes,
                   sift3d_keypoint *d_kp, int kp_capacity, int *d_count, uint8_t *d_siftrank,
                   uint64_t *d_brief, uint8_t *d_rrief, void *stream);

/*
 * Request server: continuous batching of independent extractions on one GPU
 * (the per-volume work of sift3d_extract, for volumes that arrive over
 * time). A scheduler thread owned by the server admits requests in arrival
 * order. The request at the head of the queue is admitted together with up
 * to max_batch - 1 later waiting requests of the same shape (the group size
 * rounded down to a power of two), as one batch extraction: each launch
 * covers every volume of the group. A group is admitted while (a) fewer than
 * max_inflight groups are on the device and (b) a slot of its (shape, size)
 * is idle or can be allocated within hbm_budget bytes (idle slots of other
 * kinds are freed, least recently used first, to make room; a group that
 * still does not fit is halved before it waits). A slot is one device
 * allocation holding the packed input, the batch workspace and the keypoint
 * and descriptor buffers of the group; slots and plans are cached per
 * (shape, size). Groups are spread over n_streams non-blocking streams
 * (default priority) so that several run on the device at once. A batch
 * plan gives each volume the same results as a one-volume plan, so every
 * result is the same alone and among others. The server owns its slots,
 * plans, streams and thread; the context must outlive it.
 */
typedef struct sift3d_server sift3d_server;

typedef struct sift3d_server_config {
    size_t hbm_budget;  /* device bytes that slots may occupy in total (> 0)  */
    int n_streams;      /* 1..8                                             */
    int max_inflight;   /* groups on the device at once, 1..256             */
    int kp_capacity;    /* keypoint and descriptor rows per request, >= 1    */
    int max_batch;      /* requests per group, 1..64 (1 = no grouping)        */
    double admit_timeout_s; /* 0 = a request waits for admission without limit;
                               > 0: a request not admitted within this many
                               seconds of its submission ends with status
                               SIFT3D_E_TIMEOUT (it must still be released)  */
} sift3d_server_config;

/* Result of one request; device pointers stay valid until its release. */
typedef struct sift3d_result {
    int status;                  /* SIFT3D_OK, or the error that ended the request */
    int hip_error;               /* hipError_t when status == SIFT3D_E_HIP           */
    int count;                   /* keypoints found (rows held: min(count, capacity)) */
    int capacity;
    const sift3d_keypoint *d_kp; /* [capacity], canonical order                       */
    const uint8_t *d_siftrank;   /* [capacity][64]                                    */
    const uint64_t *d_brief;     /* [capacity][brief_n/64] (NULL if brief_n == 0)     */
    const uint8_t *d_rrief;      /* [capacity][brief_n]    (NULL if brief_n == 0)     */
    int stream;                  /* index of the server stream it ran on              */
    double t_submit, t_start, t_done; /* seconds on sift3d_server_clock: submitted,
                                        launched, completion seen by the scheduler   */
} sift3d_result;

typedef struct sift3d_server_counters {
    int64_t submitted, completed, failed;
    int in_flight, pending;                          /* requests */
    size_t allocated, peak_allocated, hbm_budget;   /* slot bytes */
    int64_t slot_allocations, slot_evictions;
    int64_t groups, grouped_requests;               /* groups launched, requests in them */
} sift3d_server_counters;

/* Create a server on the current HIP device and start its scheduler thread. */
int sift3d_server_create(sift3d_ctx *ctx, const sift3d_server_config *cfg, sift3d_server **out);

/* Device bytes of the slot a lone request of this shape occupies (plans it). */
int sift3d_server_footprint(sift3d_server *srv, int nx, int ny, int nz, size_t *bytes);

/*
 * Queue the extraction of one volume d_vol ([nz][ny][nx] float32 device
 * memory, owned by the caller, complete before the call and left untouched
 * until the request finishes). Returns at once with a ticket.
 * SIFT3D_E_WORKSPACE if the slot alone exceeds hbm_budget; SIFT3D_E_TOO_SMALL
 * if the shape gives no octave.
 */
int sift3d_server_submit(sift3d_server *srv, const float *d_vol, int nx, int ny, int nz, int64_t *ticket);

/*
 * Result of a ticket. wait != 0 blocks until it is finished; wait == 0
 * returns SIFT3D_PENDING if it is not. The request keeps its slot (and the
 * device pointers in *out stay valid) until sift3d_server_release.
 */
int sift3d_server_result(sift3d_server *srv, int64_t ticket, int wait, sift3d_result *out);

/*
 * Copy the first min(count, capacity) rows of a finished request's results
 * to host memory (any pointer may be NULL to skip that output). The copies
 * run on a stream of the server's own and the call waits for them only.
 */
int sift3d_server_fetch(sift3d_server *srv, int64_t ticket, sift3d_keypoint *h_kp, uint8_t *h_siftrank,
                        uint64_t *h_brief, uint8_t *h_rrief);

/* Give a finished request's slot back to the server; the ticket becomes invalid. */
int sift3d_server_release(sift3d_server *srv, int64_t ticket);

int sift3d_server_stats(sift3d_server *srv, sift3d_server_counters *out);

/* Seconds on the server's monotonic clock (the t_* fields of sift3d_result). */
double sift3d_server_clock(void);

/*
 * Stop the server: requests not yet admitted are cancelled (status
 * SIFT3D_E_ARG), those on the device finish; then all slots, plans and
 * streams are freed. Tickets and result pointers become invalid.
 */
int sift3d_server_destroy(sift3d_server *srv);

/*
 * Nearest-neighbour matching of descriptors (keypoints are matched by their
 * descriptors, Section 3.3). For every row i of A: d_idx[i] = the index of
 * the nearest row of B (the lowest index among equal distances), d_d1[i] =
 * its distance, d_d2[i] = the smallest distance over the other rows of B
 * (for a ratio test). Exact integer distances:
 *   kind SIFT3D_MATCH_BRIEF: rows of row_elems (1..4) uint64 words, the
 *     Hamming distance;
 *   kind SIFT3D_MATCH_RANKS: rows of row_elems (64, 128, 192 or 256) uint8
 *     ranks (SIFT-Rank, RRIEF), the squared Euclidean distance. Rank vectors
 *     of one length all have the same norm, so this orders neighbours as the
 *     distance of the unit-length normalised vectors does.
 * d_a [n_a][row], d_b [n_b][row] (4-byte aligned) and the int32 outputs
 * [n_a] are device memory owned by the caller. n_b == 0 gives d_idx = -1 and
 * d_d1 = d_d2 = INT32_MAX; n_b == 1 gives d_d2 = INT32_MAX. Stream-ordered,
 * allocates nothing. SIFT3D_E_ARG for a bad kind, size or pointer.
 */
#define SIFT3D_MATCH_BRIEF 0
#define SIFT3D_MATCH_RANKS 1
int sift3d_match(int kind, const void *d_a, int n_a, const void *d_b, int n_b, int row_elems, int32_t *d_idx,
                 int32_t *d_d1, int32_t *d_d2, void *stream);

/*
 * Unit-length normalisation of descriptors (Section 3.1, step e: descriptors
 * are scaled to unit length and stored, so that the nearest neighbour under
 * the Euclidean distance is also the largest scalar product). Row i of d_in
 * becomes row i of d_out, float32:
 *   kind SIFT3D_MATCH_BRIEF: rows of row_elems (1..4) uint64 words; entry
 *     b (b < 64 row_elems, bit b % 64 of word b / 64, least significant
 *     first) is +1/sqrt(64 row_elems) if the bit is set, else its negative.
 *     Squared distances of the results are 4 Hamming / (64 row_elems);
 *   kind SIFT3D_MATCH_RANKS: rows of row_elems (64..256, multiple of 64)
 *     uint8 ranks r; entry r_j / |r|, computed in double and rounded once;
 *     an all-zero row stays zero.
 * d_in [n][row] (4-byte aligned) and d_out [n][64 row_elems or row_elems]
 * are device memory owned by the caller. Stream-ordered, allocates nothing.
 * SIFT3D_E_ARG for a bad kind, size or pointer.
 */
int sift3d_normalize(int kind, const void *d_in, int n, int row_elems, float *d_out, void *stream);

/*
 * Matching units of one volume's keypoints: the rows the Hough vote
 * (sift3d_hough) and the matcher read, listed in keypoint order. K =
 * min(*d_count, kp_capacity) keypoints of d_kp are read.
 *   d_nframes != NULL (oriented descriptors, sift3d_orient's outputs): a
 *     unit per frame f < d_nframes[k] of keypoint k, in (k, f) order; its
 *     frame is d_frames[k][f] and its descriptor row k * 4 + f of d_desc;
 *   d_nframes == NULL (upright descriptors): a unit per keypoint, frame the
 *     identity, descriptor row k of d_desc (d_frames unused).
 * Unit u gets: d_unit[u] = k * SIFT3D_MAX_ORIENTATIONS + f (f = 0 upright);
 * d_geo[u][13] float32 = (xf, yf, zf, sigma, R[9]) with R[3 i + j] =
 * component i of axis j; d_desc_out[u] = a copy of the descriptor row
 * (desc_row_bytes bytes, a multiple of 4 up to 1024). d_desc and d_desc_out
 * may both be NULL to skip the copy. *d_n_units = the number of units (at
 * most kp_capacity * SIFT3D_MAX_ORIENTATIONS, or kp_capacity upright; the
 * outputs must hold that many rows). Device memory owned by the caller;
 * stream-ordered, allocates nothing. SIFT3D_E_ARG for a bad size or pointer.
 */
int sift3d_units(const sift3d_keypoint *d_kp, const int *d_count, int kp_capacity, const int *d_nframes,
                 const float *d_frames, const void *d_desc, int desc_row_bytes, int32_t *d_unit, float *d_geo,
                 void *d_desc_out, int *d_n_units, void *stream);

/*
 * Global 7-DoF similarity between two volumes by a Hough vote over matched
 * oriented keypoints, and its inliers (Section 3.3: matches count when they
 * are inliers to a global rotation + translation + isotropic scale found by
 * a Hough transform; the vote layout below is this library's reading).
 *   - A match i (A row i, B row d_match[i]) is valid when 0 <= d_match[i] <
 *     n_b and both rows have sigma > 0. It implies s = sigma_b / sigma_a,
 *     R = R_b R_a^T and p = x_b + s R (c - x_a), the image of A's reference
 *     point c. Its vote vector (log2 s, rotation vector of R, p) is divided
 *     by the bin widths (scale_bin, angle_bin x3, trans_bin x3); per
 *     coordinate q the bin floor(q) and its neighbour on the nearer side
 *     (+1 if q - floor(q) >= 1/2, else -1) are taken, and the match votes
 *     once for each of the 2^7 bins so formed. A bin key packs coordinate d
 *     (0 scale, 1..3 rotation, 4..6 p) as (c_d + 256) in bits 9d..9d+8; a
 *     match whose bins leave -256..255 (or whose vote is not finite) does
 *     not vote. The rotation vector is theta a with cos theta =
 *     clamp((tr R - 1)/2, -1, 1): from the antisymmetric part of R when cos
 *     theta >= -0.99, else from its symmetric part (the column of the
 *     largest diagonal of (R + R^T)/2 - cos theta I, signed to agree with
 *     the antisymmetric part).
 *   - The winning bin has the most votes; ties go to the smallest key.
 *   - Fit set: the matches voting for it. Each of `iterations` rounds, if
 *     the fit set has >= 3 matches, fits the least-squares similarity
 *     x_b ~ s R x_a + t of their positions (Horn's quaternion form) and
 *     marks as inliers the valid matches with |s R x_a + t - x_b| <=
 *     inlier_sigmas * sigma_b and |log2(s sigma_a / sigma_b)| <=
 *     inlier_log2s; they are the next round's fit set. Fewer than 3 stops
 *     the rounds (in the first: no transform, status 0).
 * d_geo_a [n_a][13], d_geo_b [n_b][13]: rows as sift3d_units writes them;
 * d_match [n_a] int32 (e.g. sift3d_match's d_idx). Arithmetic in double.
 * Outputs: *d_out (device memory) and d_inlier [n_a] uint8 (1 = inlier).
 * d_ws: workspace of sift3d_hough_workspace(n_a) bytes. Vote counts are
 * order-independent integers and every sum has a fixed order, so results
 * are reproducible. 0 <= n_a <= 2^21, n_b >= 0, widths > 0, inlier limits
 * >= 0, 1 <= iterations <= 16, else SIFT3D_E_ARG; SIFT3D_E_WORKSPACE for a
 * short workspace. Stream-ordered, allocates nothing.
 */
typedef struct sift3d_hough_params {
    double scale_bin;      /* [1.0] log2(scale) bin width                        */
    double angle_bin;      /* [pi/6] rotation-vector component bin width, rad    */
    double trans_bin;      /* [max(nx,ny,nz)/4] bin width of p, input voxels      */
    double centre[3];      /* [((nx-1)/2, (ny-1)/2, (nz-1)/2)] reference point c  */
    double inlier_sigmas;  /* [2.0] position tolerance in units of sigma_b       */
    double inlier_log2s;   /* [0.5] scale-ratio tolerance, log2 units             */
    int iterations;        /* [2] fit / inlier rounds                            */
} sift3d_hough_params;

typedef struct sift3d_similarity {
    int32_t status;        /* 1 = transform found, 0 = none                      */
    int32_t votes;         /* votes of the winning bin (0: no valid vote)        */
    int64_t bin;           /* packed key of the winning bin, -1 if none          */
    int32_t n_fit;         /* matches in the last fit                            */
    int32_t n_inliers;
    double scale;          /* x_b = scale * rot * x_a + trans                    */
    double rot[9];         /* row-major                                          */
    double trans[3];
} sift3d_similarity;

/* Defaults above for a volume A of dims (nx, ny, nz). Host only. */
int sift3d_hough_default_params(int nx, int ny, int nz, sift3d_hough_params *hp);
/* Workspace bytes sift3d_hough needs for n_a matches. Host only. */
int sift3d_hough_workspace(int n_a, size_t *bytes);
int sift3d_hough(const float *d_geo_a, int n_a, const float *d_geo_b, int n_b, const int32_t *d_match,
                 const sift3d_hough_params *hp, void *d_ws, size_t ws_bytes, sift3d_similarity *d_out,
                 uint8_t *d_inlier, void *stream);

/*
 * Uniform-filter approximation of a Gaussian blur (Related Work: the
 * Gaussian scale space can also be generated with separable uniform 1D
 * filters). Along x, then y, then z, `passes` uniform passes of width
 * 2*half_width+1 are applied; an output is the mean of the 2*half_width+1
 * samples centred on it, indices outside the volume clamped to the nearest
 * edge (each pass sees the volume's edges). FP32, each sum taken in index
 * order. d_in, d_out and d_tmp are distinct device buffers of nx*ny*nz
 * floats ([z][y][x], x fastest) owned by the caller; d_out receives the
 * result and d_tmp is overwritten. nx*ny <= 2^30, nz <= 2^30,
 * 1 <= passes <= 4, 0 <= half_width <= 8, passes * half_width <= 28. Stream-ordered, allocates nothing.
 * SIFT3D_E_ARG for a bad size, count or pointer.
 */
int sift3d_box_blur(const float *d_in, float *d_out, float *d_tmp, int nx, int ny, int nz, int half_width,
                    int passes, void *stream);

/*
 * Half-width of the uniform filter whose `passes`-fold repetition stands in
 * for a Gaussian of standard deviation sigma: a width-w uniform filter has
 * variance (w*w - 1)/12, so one of m equal passes ideally has width
 * sqrt(12 sigma^2 / m + 1); *half_width is the integer nearest to
 * (that width - 1) / 2 (halves round up). Host only. SIFT3D_E_ARG for
 * sigma < 0, passes < 1 or a null pointer.
 */
int sift3d_box_half_width(double sigma, int passes, int *half_width);

/* Static description of an error code. */
const char *sift3d_error_string(int code);

/* hipError_t of the last failing HIP call made by the library on this thread. */
int sift3d_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SIFT3D_H */
