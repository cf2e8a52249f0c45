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

// Detection geometry.
constexpr int kDetThreads = 256;            // 4 waves
constexpr int kDetRowsPerWave = 4;
constexpr int kDetRowsPerBlock = (kDetThreads / 64) * kDetRowsPerWave;
constexpr int kScanThreads = 1024;

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

struct DetOctave {
    const float *D;       // D_0 of the octave
    long long lstride;    // floats between consecutive levels
    int nx, ny, nz;
    int pad_;
    long long row_base;   // first global row of the octave
    long long rows;       // S * (nz-2) * (ny-2)
    float sigma[kMaxScales + 1];  // input-space sigma per scale (index s)
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
};

struct DescOctave {
    const float *G;       // G_0 of the octave
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
    int brief_rb;
    const int32_t *pairs;              // [S][brief_n][2][3] (scale s at index s-1)
    double wb[2 * kMaxBriefR + 1];
};

struct OctaveGeom {
    int nx, ny, nz;
    size_t n;             // voxels
    size_t level_bytes;   // one level, padded to 256 bytes
    size_t base;          // byte offset of G_0 in the workspace
};

struct BlurLaunch {
    int r;
    bool dog;
    BlurArgs a;           // pointers are workspace-relative until bound
    int src_kind;         // -1 = input volume, 0 = G level of the octave
    int src_idx, dst_idx, dog_idx;
    int octave;
    int sub_octave;       // -1 = no sub-sample output
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
    size_t row_count_off, block_sum_off, block_off_off;
    size_t ws_bytes;
    long long total_rows;
    int det_blocks;
    std::vector<s3d::BlurLaunch> blur;  // in launch order
    double base_sigma;
    std::vector<double> inc_sigma;      // G_1..G_{S+2}
};

namespace s3d {
// Launchers (return hipError_t of the launch).
hipError_t launch_blur(const BlurArgs &a, int r, bool dog, hipStream_t st);
hipError_t launch_detect(const DetectArgs &a, hipStream_t st);
hipError_t launch_describe(const DescribeArgs &a, int grid, hipStream_t st);
}  // namespace s3d
