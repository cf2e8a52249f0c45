// Internal declarations of the gfx950 3D SIFT-Rank library: plan geometry,
// kernel argument blocks and the launchers implemented in the .hip files.
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
constexpr int kMaxBriefR = 6;               // pre-blur tap radius
constexpr int kMaxPairs = 256;

// Fused blur pass geometry (shared by host planning and the kernel).
constexpr int kBlurTX = 32;                 // tile width in x (one output column per lane)
constexpr int kBlurTY = 16;                 // tile height in y
constexpr int kBlurNY = 2;                  // consecutive y outputs per thread
constexpr int kBlurThreads = kBlurTX * kBlurTY / kBlurNY;

// Two-launch (xy, then z) level geometry.
constexpr int kXYTX = 64;                   // xy tile width (one wavefront per row)
constexpr int kXYTY = 16;                   // xy tile height
constexpr int kXYThreads = 256;
constexpr int kZPlanes = 16;                // z outputs per thread
constexpr int kZThreads = 256;              // 32 (x) x 8 (y) columns
constexpr int kMaxJobs = 16;                // jobs per xy / z launch
// Octaves with at least this many voxels use the fused streaming pass.
constexpr long long kFusedMinVoxels = 24LL << 20;

// Detection geometry.
constexpr int kDetThreads = 256;            // 4 waves
constexpr int kDetRowsPerWave = 4;
constexpr int kDetRowsPerBlock = (kDetThreads / 64) * kDetRowsPerWave;
constexpr int kScanThreads = 1024;
// Strict-extremum path (votes == 80): one wavefront per (64 x, one y row,
// kDTZ planes); 4 wavefronts (4 consecutive y rows) per block.
constexpr int kDTX = 64, kDTY = 4, kDTZ = 16;
constexpr int kRowBlock = 256;              // rows per count / emit block

// One launch of the fused blur -> DoG -> sub-sample pass.
struct BlurArgs {
    const float *src;     // G_{i-1} (or the input volume)
    float *dst;           // G_i
    float *dog;           // D_{i-1} = src - dst, or nullptr
    float *sub;           // 2x2x2 mean of dst into the next octave's G_0, or nullptr
    int nx, ny, nz;
    int mx, my, mz;       // dims of `sub`
    int L;                // output planes per slab (even)
    int tiles_x, tiles_y, slabs;
    int n_blocks;         // tiles_x * tiles_y * slabs
    float w[kMaxTaps];    // taps w[t + r], t = -r..r
};

constexpr int kMaxTapSets = 8;              // distinct tap sets per xy / z launch

// One job of an xy or z launch: one level of one volume. Jobs of one launch
// may have different tap radii; each block dispatches on its job's radius.
struct XYJob {
    const float *src;
    float *dst;
    int nx, ny, nz;
    int tiles_x, tiles_y;
    int block0;           // first block of this job in the launch
    int r;                // tap radius
    int taps;             // index into XYArgs::w
};

struct XYArgs {
    XYJob job[kMaxJobs];
    int n_jobs;
    int n_blocks;
    float w[kMaxTapSets][kMaxTaps];
};

struct ZJob {
    const float *t;       // xy-blurred input
    const float *center;  // level the DoG subtracts from (when dog != nullptr)
    float *dst;
    float *dog;           // or nullptr
    float *sub;           // or nullptr
    int nx, ny, nz;
    int mx, my, mz;
    int gx, gy, gz;       // blocks per axis
    int block0;
    int r;
    int taps;
};

struct ZArgs {
    ZJob job[kMaxJobs];
    int n_jobs;
    int n_blocks;
    float w[kMaxTapSets][kMaxTaps];
};

struct DetOctave {
    const float *D;       // D_0 of the octave
    long long lstride;    // floats between consecutive levels
    int nx, ny, nz;
    int pad_;
    long long row_base;   // first global row of the octave
    long long rows;       // S * (nz-2) * (ny-2)
    float sigma[kMaxScales + 1];  // input-space sigma per scale (index s)
    unsigned long long *masks;    // [rows][words] keypoint bits, x = 64 w + bit
    int words;            // ceil(nx / 64)
    int tiles_x, tiles_y, tiles_z;
    int block0;           // first tile block of the octave
};

struct DetectArgs {
    DetOctave oc[kMaxOctaves];
    int n_oct;
    int S;
    long long total_rows;
    int n_blocks;
    float thr;
    int votes;
    int *row_count;       // [total_rows]
    int *block_sum;       // [n_blocks]
    int *block_off;       // [n_blocks]
    int *d_count;         // total keypoints (device)
    sift3d_keypoint *kp;
    int cap;
    int tile_blocks;      // blocks of the tile launch (all octaves)
    int row_blocks;       // blocks of kRowBlock rows
};

struct DescOctave {
    const float *G;       // G_0 of the octave
    const float *B;       // pre-blurred B_1 (B_s = B + (s-1) * lstride)
    long long lstride;    // floats between consecutive levels
    int nx, ny, nz, pad_;
};

struct DescribeArgs {
    DescOctave oc[kMaxOctaves];
    int n_oct;
    int S;
    int sift_R[kMaxScales + 1];        // per scale
    const sift3d_keypoint *kp;
    const int *d_count;
    int cap;
    uint8_t *siftrank;
    uint64_t *brief;
    uint8_t *rrief;
    int brief_n;
    const int32_t *pairs;              // [S][brief_n][2][3] (scale s at index s-1)
};

struct OctaveGeom {
    int nx, ny, nz;
    size_t n;             // voxels
    size_t level_bytes;   // one level, padded to 256 bytes
    size_t base;          // byte offset of G_0 in the workspace
};

// One pyramid level: G_dst of `octave` from G_src (or the input volume).
struct BlurLaunch {
    int r;
    bool dog;
    bool fused;           // fused streaming pass, else xy + z jobs
    BlurArgs a;           // fused geometry (pointers bound per call)
    int tapset;           // index into sift3d_plan::tapsets
    int src_kind;         // -1 = input volume, 0 = G level of the octave
    int src_idx, dst_idx, dog_idx;
    int octave;
    int sub_octave;       // -1 = no sub-sample output
};

// A unit of work of the pyramid schedule: a level pass (index into
// sift3d_plan::blur) or the BRIEF pre-blur of G_s of one octave.
struct Task {
    int kind;             // 0 = level pass, 1 = pre-blur
    int pass;             // level pass index (kind 0)
    int octave, s;        // pre-blur target (kind 1)
};

// One launch of the schedule: a fused pass, or the xy / z half of a set of
// split tasks.
struct Step {
    int type;             // 0 = fused pass, 1 = xy launch, 2 = z launch
    std::vector<int> tasks;
};

}  // namespace s3d

struct sift3d_ctx {
    sift3d_params p;
    int device;
    std::vector<double> draws;          // [brief_n][2][3]
    std::vector<int32_t> offsets;       // [S][brief_n][2][3]
    int32_t *d_offsets;                 // device copy
};

struct sift3d_plan {
    sift3d_ctx *ctx;
    int nx, ny, nz, cap;
    int n_oct;
    int S;
    std::vector<s3d::OctaveGeom> oct;
    size_t pyramid_bytes;
    size_t row_count_off, block_sum_off, block_off_off, masks_off;
    size_t ws_bytes;
    long long total_rows;
    int det_blocks;
    std::vector<s3d::BlurLaunch> blur;  // level passes in dependency order
    int brief_rb;                       // pre-blur radius (-1: none, B_s = G_s)
    int brief_tapset;
    std::vector<std::vector<float>> tapsets;  // kMaxTaps floats each
    std::vector<int> tapset_r;
    std::vector<s3d::Task> tasks;
    std::vector<s3d::Step> sched;       // launches of sift3d_build_pyramid
    double base_sigma;
    std::vector<double> inc_sigma;      // G_1..G_{S+2}
};

namespace s3d {
// Launchers (return hipError_t of the launch).
hipError_t launch_blur(const BlurArgs &a, int r, bool dog, hipStream_t st);
hipError_t launch_detect(const DetectArgs &a, hipStream_t st);
hipError_t launch_describe(const DescribeArgs &a, int grid, hipStream_t st);
hipError_t launch_blur_xy(const XYArgs &a, hipStream_t st);
hipError_t launch_blur_z(const ZArgs &a, hipStream_t st);

// Workspace levels of an octave, in units of one padded level.
inline int lev_G(int i) { return i; }
inline int lev_D(int S, int i) { return S + 3 + i; }
inline int lev_B(int S, int s) { return 2 * S + 5 + (s - 1); }   // s = 1..S
inline int lev_T(int S) { return 3 * S + 5; }
inline int lev_Tb(int S, int s) { return 3 * S + 6 + (s - 1); }
inline int levels_per_octave(int S) { return 4 * S + 6; }
}  // namespace s3d
