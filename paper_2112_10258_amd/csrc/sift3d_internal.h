// Internal declarations of the gfx950 3D SIFT-Rank library: plan geometry,
// the device-side job tables and the launch argument blocks of the kernels.
//
// A plan covers one or several volumes. Everything a kernel needs to know
// about its work (which level of which octave of which volume, its dims,
// where its inputs and outputs live) sits in small tables that the plan
// uploads once to device memory. Table entries hold offsets, not pointers:
// workspace byte offsets, or element offsets into the packed input. Each
// launch passes the call's base pointers and the kernels add them, so the
// tables stay valid for any workspace and input buffer, and a launch can
// cover any number of volumes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "sift3d.h"

namespace s3d {

constexpr int kMaxOctaves = 12;
constexpr int kMaxScales = 5;               // S; S+3 Gaussian levels per octave
constexpr int kMaxR = 16;                   // largest blur tap radius
constexpr int kMaxTaps = 2 * kMaxR + 1;
constexpr int kMaxSiftR = 7;                // SIFT-Rank window half-width
constexpr int kMaxBriefR = 10;              // pre-blur tap radius (runs on the level kernels)
constexpr int kMaxPairs = 256;
constexpr int kMaxVolumes = 4096;

// Fused blur pass geometry (shared by host planning and the kernel).
constexpr int kBlurTX = 32;                 // tile width in x (one output column per lane)
constexpr int kBlurNY = 2;                  // consecutive y outputs per thread
// Tile height: 32 rows for launches over >= kBlurTallVoxels voxels (less
// halo staging and x-pass work per output), 16 rows below (more blocks).
constexpr int kBlurTYSmall = 16, kBlurTYTall = 32;
constexpr long long kBlurTallVoxels = 24LL << 20;
constexpr int blur_threads(int ty) { return kBlurTX * ty / kBlurNY; }

// Two-launch (xy, then z) level geometry.
constexpr int kXYTX = 64;                   // xy tile width (one wavefront per row)
constexpr int kXYTY = 16;                   // xy tile height
constexpr int kXYThreads = 256;
constexpr int kZPlanes = 16;                // z outputs per thread
constexpr int kZThreads = 256;              // 32 (x) x 8 (y) columns
// Octaves with at least this many voxels use the fused streaming pass; from
// kFusedMidVoxels on, so do the levels with radius <= kFusedMidMaxR (there
// the fused pass beats the xy + z pair even while the octave sits in the
// last-level cache).
constexpr long long kFusedMinVoxels = 24LL << 20;
constexpr long long kFusedMidVoxels = 2LL << 20;
constexpr int kFusedMidMaxR = 8;
constexpr int kMaxFusedR = 10;              // largest tap radius of the fused pass
constexpr int kMinSlabPlanes = 12;          // shortest slab of a fused launch (output planes)
// Pre-blur radius that the fused pass can write alongside a level: pass
// G_{s+1} stages G_s with a halo of R >= kFusedPreR, so it also writes B_s.
constexpr int kFusedPreR = 3;
// One-launch pass for small octaves: 32 x 8 x 4 output tiles computed from
// their whole source footprint; used below kFusedMidVoxels, except for radii
// above kFusedMidMaxR from kCompactWideVoxels on (there the footprint
// re-reads make the xy + z pair faster).
constexpr int kCTX = 32, kCTY = 8, kCTZ = 4;
constexpr long long kCompactWideVoxels = 1LL << 20;
constexpr int kCompactThreads = 256;
constexpr int kCompactMaxR = 10;

// Detection geometry.
constexpr int kDetThreads = 256;            // 4 waves
constexpr int kDetRowsPerWave = 4;
constexpr int kDetRowsPerBlock = (kDetThreads / 64) * kDetRowsPerWave;
constexpr int kScanThreads = 1024;
// Strict-extremum path (votes == 80): one wavefront per (62 output x plus
// a halo lane on each side, kDTWY consecutive y rows, kDTZ planes); 4
// wavefronts (kDTY = 4 kDTWY consecutive rows) per block. Mask word t of a
// row covers x = 62 t + bit. kDTZ + 2 planes per wavefront is a multiple of
// the plane loop's unroll (6); 28 re-reads fewer halo planes than 16 and
// still leaves thousands of blocks on the large octaves.
constexpr int kDTXOut = 62, kDTWY = 2, kDTY = 4 * kDTWY, kDTZ = 28;
constexpr int kRowBlock = 256;              // rows per count / emit block; volumes start on a block

// ---------------------------------------------------------------- device tables

// One job of an xy launch: the xy blur of one level of one octave.
struct DXYJob {
    long long src;        // workspace byte offset, or input element offset if src_input
    long long dst;        // workspace byte offset
    int src_input;
    int nx, ny, nz;
    int tiles_x, tiles_y;
    int block0;           // first block of the job within its launch
    int r, taps;          // tap radius, tap-set index
    int planes;           // consecutive planes per block
    int pad_[2];
};

// One job of a z launch: the z blur of one level plus its DoG and sub-sample.
struct DZJob {
    long long t;          // xy-blurred input (workspace byte offset)
    long long center;     // level the DoG subtracts from (see center_input), < 0: no DoG
    long long dst;
    long long dog;        // < 0: none
    long long sub;        // < 0: none
    int center_input;
    int nx, ny, nz;
    int mx, my, mz;
    int gx, gy, gz;       // blocks per axis
    int block0;
    int r, taps;
    int pad_[2];
};

// One octave of one volume, for detection and description.
struct DUnit {
    long long g0;         // workspace byte offset of G_0 (levels G, D, B follow at lstride)
    long long b1;         // workspace byte offset of the BRIEF level of s = 1 (B_s at (s-1) lstride)
    long long masks;      // byte offset of the keypoint bit masks [rows][words] in the detection scratch
    long long row_base;   // first global detection row of the unit
    long long rows;       // S * (nz-2) * (ny-2)
    long long lstride;    // floats between consecutive levels
    int nx, ny, nz, octave;
    int vol, words;       // volume index; 64-bit mask words per row
    int tiles_x, tiles_y, tiles_z;
    int tile_block0;      // first block of the unit in the strict-detection launch
    float sigma[kMaxScales + 1];  // input-space sigma per scale (index s)
    int pad_[2];
};

// One volume of the plan.
struct DVol {
    long long row_base;   // first global detection row (a multiple of kRowBlock)
    int unit0, n_units;   // its octaves in the unit table
};

// ---------------------------------------------------------------- launch arguments

// One job of a fused blur -> DoG -> sub-sample launch: one level of one
// octave of one volume, streamed as tiles x slabs workgroups.
struct DFJob {
    long long src;        // workspace byte offset, or input element offset if src_input
    long long dst;        // workspace byte offset of G_i
    long long dog;        // D_{i-1} (< 0: none)
    long long sub;        // next octave's G_0 (< 0: none)
    int src_input;
    int nx, ny, nz;
    int mx, my, mz;       // dims of `sub`
    int L;                // output planes per slab (even)
    int tiles_x, tiles_y, slabs;
    int block0;           // first block of the job within its launch
    int taps;             // tap-set index
    int pb_taps;          // tap set of the BRIEF pre-blur written alongside (pb >= 0)
    long long pb;         // B_s = pre-blur of this job's source G_s (< 0: none)
};

// One job of a compact launch: one level (or BRIEF pre-blur) of one octave
// of one volume, as tiles_x * tiles_y * tiles_z workgroups.
struct DCJob {
    long long src;        // workspace byte offset, or input element offset if src_input
    long long dst;        // workspace byte offset of G_i
    long long dog;        // D_{i-1} = src - dst (< 0: none)
    long long sub;        // next octave's G_0 (< 0: none)
    int src_input;
    int nx, ny, nz;
    int mx, my, mz;       // dims of `sub`
    int tiles_x, tiles_y, tiles_z;
    int block0;
    int r, taps;          // tap radius, tap-set index
    int pad_[3];
};

// Launches with few jobs also carry them inline (read through the scalar
// cache from the argument segment instead of a dependent global load).
constexpr int kInlineJobs = 8;
constexpr int kInlineUnits = 12;

struct FusedLaunch {
    const DFJob *jobs;    // this launch's jobs, block0 ascending; all share R and the DoG flag
    int n_jobs, n_blocks;
    char *ws;
    const float *in;      // packed input volumes
    const float *taps;    // [n_tapsets][kMaxTaps]
    DFJob inl[kInlineJobs];
};

struct CompactLaunch {
    const DCJob *jobs;    // this launch's jobs, block0 ascending (radii may differ)
    int n_jobs, n_blocks;
    char *ws;
    const float *in;
    const float *taps;
    DCJob inl[kInlineJobs];
};

struct XYLaunch {
    const DXYJob *jobs;   // this launch's jobs, block0 ascending
    int n_jobs, n_blocks;
    char *ws;
    const float *in;      // packed input volumes
    const float *taps;    // [n_tapsets][kMaxTaps]
    DXYJob inl[kInlineJobs];  // copy of jobs[0..n_jobs) when n_jobs <= kInlineJobs
};

struct ZLaunch {
    const DZJob *jobs;
    int n_jobs, n_blocks;
    char *ws;
    const float *in;
    const float *taps;
    DZJob inl[kInlineJobs];
};

struct DetLaunch {
    const DUnit *units;
    const DVol *vols;
    int n_units, n_vol, S;
    long long total_rows;     // including the padding rows between volumes
    int tile_blocks;          // blocks of the strict tile launch
    int n_blocks;             // count / scan / emit blocks (rows_per_block rows each)
    int rows_per_block;
    float thr;
    int votes;
    char *ws;                 // pyramid workspace (the D levels are read from it)
    char *scr;                // detection scratch: row counts, block sums and offsets, masks
    int *row_count;           // [total_rows]
    int *block_sum;           // [n_blocks]
    int *block_off;           // [n_blocks]
    int *counts;              // [n_vol] keypoints found per volume (device)
    sift3d_keypoint *kp;      // [n_vol][cap]
    int cap;
    DUnit inl[kInlineUnits];  // copy of units[0..n_units) when n_units <= kInlineUnits
};

struct DescLaunch {
    const DUnit *units;
    const DVol *vols;
    int n_vol, S;
    int sift_R[kMaxScales + 1];
    char *ws;
    const sift3d_keypoint *kp;    // [n_vol][cap]
    const int *counts;            // [n_vol]
    int cap;
    uint8_t *siftrank;            // [n_vol][cap][64]
    uint64_t *brief;              // [n_vol][cap][n/64]
    uint8_t *rrief;               // [n_vol][cap][n]
    int brief_n;
    const int32_t *pairs;         // [S][brief_n][2][3] (scale s at index s-1)
    int n_units;
    int sr_blocks;                // workgroups [0, sr_blocks) compute SIFT-Rank, the rest BRIEF / RRIEF
    DUnit inl[kInlineUnits];      // copy of units when n_units <= kInlineUnits
};

// Dominant orientations and oriented SIFT-Rank (orient.hip).
constexpr int kMaxOrient = SIFT3D_MAX_ORIENTATIONS;   // frames kept per keypoint

struct OrientLaunch {
    const DUnit *units;
    const DVol *vols;
    int n_vol, S, n_units;
    int sift_R[kMaxScales + 1];
    char *ws;
    const sift3d_keypoint *kp;    // [n_vol][cap]
    const int *counts;            // [n_vol]
    int cap;
    double tau;                   // peak threshold relative to the histogram maximum
    int *nframes;                 // [n_vol][cap]
    float *frames;                // [n_vol][cap][kMaxOrient][9]
    uint8_t *siftrank;            // [n_vol][cap][kMaxOrient][64]
    DUnit inl[kInlineUnits];      // copy of units when n_units <= kInlineUnits
};

// ---------------------------------------------------------------- host plan

// Matching units of one volume (sift3d_units).
struct UnitsArgs {
    const sift3d_keypoint *kp;
    const int *count;
    int cap;
    const int *nframes;     // NULL: upright, one unit per keypoint
    const float *frames;    // [cap][kMaxOrient][9]
    const uint8_t *desc;    // rows of row_bytes (NULL: no copy)
    int row_bytes;
    int32_t *unit;
    float *geo;             // [units][13]
    uint8_t *desc_out;
    int *n_units;
};

// The 7-DoF similarity Hough vote (sift3d_hough).
struct HoughArgs {
    const float *geo_a, *geo_b;        // [n][13]: x, y, z, sigma, R[9]
    const int32_t *match;
    int n_a, n_b;
    double width[7];                   // bin widths: log2 s, rotation vector x3, centre image x3
    double centre[3];
    double inl_sig, inl_log2s;
    int iterations;
    unsigned long long *keys;          // hash table [2^log2_slots]
    unsigned *counts;
    int log2_slots;
    unsigned long long *lo;            // [n_a] low corner of each match's bins (all ones: no vote)
    unsigned *best_count;
    unsigned long long *best_key;
    sift3d_similarity *out;
    uint8_t *inlier;                   // [n_a]
};

struct OctaveGeom {
    int nx, ny, nz;
    size_t n;             // voxels
    size_t level_bytes;   // one level, padded to 256 bytes
    size_t base;          // workspace byte offset of G_0
};

// How a level (or pre-blur) runs: an xy launch then a z launch, the fused
// streaming pass, or the compact pass.
constexpr int kPathSplit = 0, kPathFused = 1, kPathCompact = 2;

// One pyramid level: G_dst of `octave` of volume `vol` from G_src (or the input).
struct BlurLaunch {
    int vol;
    int r;
    bool dog;
    int path;             // kPathSplit, kPathFused or kPathCompact
    int tapset;           // index into sift3d_plan::tapsets
    int src_kind;         // -1 = input volume, 0 = G level of the octave
    int src_idx, dst_idx, dog_idx;
    int octave;
    int sub_octave;       // -1 = no sub-sample output
};

// A unit of work of the pyramid schedule: a level pass (index into
// sift3d_plan::blur) or the BRIEF pre-blur of G_s of one octave of one volume.
struct Task {
    int kind;             // 0 = level pass, 1 = pre-blur
    int pass;             // level pass index (kind 0)
    int vol, octave, s;   // pre-blur target (kind 1)
};

// One launch of the schedule: a fused pass, or the xy / z half of a set of
// split tasks (their jobs are entries [first, first + count) of the device
// job table of that kind).
struct Step {
    int type;             // 0 = fused launch, 1 = xy launch, 2 = z launch, 3 = compact launch
    std::vector<int> tasks;
    int first, count, n_blocks, max_r;
    bool dog;             // fused launches: jobs write a DoG level
    int ty;               // fused launches: tile height
    bool pb;              // fused launches: jobs also write a BRIEF pre-blurred level
};

struct VolPlan {
    int nx, ny, nz;
    size_t in_off;        // element offset in the packed input
    std::vector<OctaveGeom> oct;
    int unit0;
};

}  // namespace s3d

struct sift3d_ctx {
    sift3d_params p;
    int device;
    int n_cu;                           // compute units of the device
    std::vector<double> draws;          // [brief_n][2][3]
    std::vector<int32_t> offsets;       // [S][brief_n][2][3]
    int32_t *d_offsets;                 // device copy
};

struct sift3d_plan {
    sift3d_ctx *ctx;
    int n_vol, cap, S;
    std::vector<s3d::VolPlan> vols;
    size_t in_elems;                    // floats of the packed input
    size_t row_count_off, block_sum_off, block_off_off;   // workspace byte offsets
    size_t det_scratch_off, det_scratch_bytes;            // detection scratch area of the workspace
    size_t ws_bytes;
    long long total_rows;
    int tile_blocks;
    std::vector<s3d::BlurLaunch> blur;  // level passes of all volumes in dependency order
    int brief_rb;                       // pre-blur radius (-1: none, B_s = G_s)
    int brief_tapset;
    double base_sigma;
    std::vector<double> inc_sigma;      // G_1..G_{S+2}
    std::vector<std::vector<float>> tapsets;  // kMaxTaps floats each
    std::vector<int> tapset_r;
    std::vector<s3d::Task> tasks;
    std::vector<s3d::Step> sched;       // launches of sift3d_build_pyramid
    std::vector<int> solo_xy, solo_z;   // per task: index of its single-job entry (-1: fused)
    std::vector<int> solo_f;            // per task: index of its single-job fused entry (-1: none)
    std::vector<int> solo_c;            // per task: index of its single-job compact entry (-1: none)
    // host copies of the device tables
    std::vector<s3d::DUnit> units;
    std::vector<s3d::DVol> dvols;
    std::vector<s3d::DXYJob> xyjobs;
    std::vector<s3d::DZJob> zjobs;
    std::vector<s3d::DFJob> fjobs;
    std::vector<s3d::DCJob> cjobs;
    // device tables (one allocation, owned by the plan)
    void *d_tables;
    // autotuned fused launches: schedule step -> (tile height, slabs per job)
    std::vector<std::pair<int, int>> fused_tune;       // (0, 0): default rule
    struct TuneRecord {
        int step, def_ty, def_slabs, ty, slabs, candidates;
        float def_ms, ms;
    };
    std::vector<TuneRecord> tuning;
    s3d::DUnit *d_units;
    s3d::DVol *d_vols;
    s3d::DXYJob *d_xy;
    s3d::DZJob *d_z;
    s3d::DFJob *d_f;
    s3d::DCJob *d_c;
    float *d_taps;
};

namespace s3d {
// Launchers (return hipError_t of the launch).
hipError_t launch_blur(const FusedLaunch &a, int r, bool dog, bool pb, int ty, hipStream_t st);
int fused_blocks_per_cu(int r, bool dog, bool pb, int ty);
hipError_t launch_blur_xy(const XYLaunch &a, int max_r, hipStream_t st);
hipError_t launch_blur_z(const ZLaunch &a, int max_r, hipStream_t st);
hipError_t launch_blur_compact(const CompactLaunch &a, int max_r, hipStream_t st);
hipError_t launch_detect(const DetLaunch &a, hipStream_t st);
hipError_t launch_describe(const DescLaunch &a, long long kp_slots, int n_cu, hipStream_t st);
hipError_t launch_orient(const OrientLaunch &a, long long kp_slots, int n_cu, hipStream_t st);
hipError_t launch_normalize(int kind, const void *in, int n, int row_elems, float *out, hipStream_t st);
hipError_t launch_units(const UnitsArgs &a, hipStream_t st);
int hough_log2_slots(int n_a);   // hash-table size: 2^l >= 2 * 2^7 * n_a, l >= 8
hipError_t launch_hough(const HoughArgs &a, hipStream_t st);

// Workspace levels of an octave, in units of one padded level.
inline int lev_G(int i) { return i; }
inline int lev_D(int S, int i) { return S + 3 + i; }
inline int lev_B(int S, int s) { return 2 * S + 5 + (s - 1); }   // s = 1..S
inline int lev_T(int S) { return 3 * S + 5; }
inline int lev_Tb(int S, int s) { return 3 * S + 6 + (s - 1); }
inline int levels_per_octave(int S) { return 4 * S + 6; }
}  // namespace s3d
