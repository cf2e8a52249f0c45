// Host side of the C ABI: parameter checks, contexts, plans (octave
// geometry, workspace layout, launch shapes) and the stream-ordered entry
// points. Nothing here synchronises the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "sift3d_internal.h"

using namespace s3d;

namespace {

thread_local int g_last_hip = 0;

int hip_fail(hipError_t e)
{
    g_last_hip = (int)e;
    return SIFT3D_E_HIP;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Blur of level s of an octave in that octave's voxels: sigma0 * 2^(s/S).
double scale_sigma(const sift3d_params &p, double s) { return p.sigma0 * std::pow(2.0, s / p.scales); }

int tap_radius(double sigma, double trunc) { return sigma > 0.0 ? (int)std::ceil(trunc * sigma) : 0; }

// Normalised sampled Gaussian, w[t + r] for t = -r..r, computed in double.
std::vector<double> gaussian(double sigma, double trunc)
{
    const int r = tap_radius(sigma, trunc);
    std::vector<double> w(2 * r + 1, 1.0);
    if (r == 0) return w;
    double sum = 0.0;
    for (int t = -r; t <= r; ++t) {
        w[t + r] = std::exp(-(double)t * t / (2.0 * sigma * sigma));
        sum += w[t + r];
    }
    for (double &v : w) v /= sum;
    return w;
}

int check_params(const sift3d_params *p)
{
    if (p == nullptr) return SIFT3D_E_ARG;
    if (p->n_octaves < 0 || p->min_dim < 4 || p->scales < 1 || p->scales > kMaxScales) return SIFT3D_E_ARG;
    if (!(p->sigma0 > 0.0) || p->sigma_in < 0.0 || p->sigma_in > p->sigma0 || !(p->trunc > 0.0)) return SIFT3D_E_ARG;
    if (!(p->dog_threshold >= 0.0f) || p->votes < 1 || p->votes > 80) return SIFT3D_E_ARG;
    if (p->brief_n < 0 || p->brief_n > kMaxPairs || p->brief_n % 64 != 0) return SIFT3D_E_ARG;
    if (p->brief_blur < 0.0 || !(p->siftrank_factor > 0.0)) return SIFT3D_E_ARG;
    if (p->pyramid_mode < 0 || p->pyramid_mode > 2) return SIFT3D_E_ARG;
    // kernel limits
    const double top = scale_sigma(*p, p->scales + 2);
    const double prev = scale_sigma(*p, p->scales + 1);
    if (tap_radius(std::sqrt(top * top - prev * prev), p->trunc) > kMaxR) return SIFT3D_E_UNSUPPORTED;
    if (tap_radius(std::sqrt(p->sigma0 * p->sigma0 - p->sigma_in * p->sigma_in), p->trunc) > kMaxR)
        return SIFT3D_E_UNSUPPORTED;
    if ((int)std::ceil(p->siftrank_factor * scale_sigma(*p, p->scales)) > kMaxSiftR) return SIFT3D_E_UNSUPPORTED;
    if (tap_radius(p->brief_blur, p->trunc) > kMaxBriefR) return SIFT3D_E_UNSUPPORTED;
    return SIFT3D_OK;
}

// Output planes per slab: few enough slabs that the z halo (2R planes per
// slab) stays cheap, enough blocks to occupy the 256 compute units.
int choose_slab(int nz, int tiles, int r)
{
    const int target_blocks = 1024;
    const int min_l = std::max(8, 2 * r);
    int slabs = std::max(1, (target_blocks + tiles - 1) / tiles);
    int L = (nz + slabs - 1) / slabs;
    L = std::max(L, min_l);
    L = (L + 1) & ~1;
    return std::min(L, (nz + 1) & ~1);
}

// Method 3 point pairs (Section 3.2.3): p1 ~ N(0, sigma), p2 ~ N(p1, sigma)
// with sigma the keypoint scale in octave voxels. From draws (z1, z2):
// u1 = z1, u2 = z1 + z2, offset = floor(sigma_s * u + 0.5). out: [n][2][3].
void pair_offsets(const sift3d_params &p, const double *draws, int s, int32_t *out)
{
    const double sig = scale_sigma(p, s);
    for (int i = 0; i < p.brief_n; ++i)
        for (int d = 0; d < 3; ++d) {
            const double z1 = draws[(size_t)i * 6 + d], z2 = draws[(size_t)i * 6 + 3 + d];
            const double u1 = z1, u2 = z1 + z2;
            out[(size_t)i * 6 + d] = (int32_t)std::floor(sig * u1 + 0.5);
            out[(size_t)i * 6 + 3 + d] = (int32_t)std::floor(sig * u2 + 0.5);
        }
}

int xy_blocks(const OctaveGeom &g)
{
    return ((g.nx + kXYTX - 1) / kXYTX) * ((g.ny + kXYTY - 1) / kXYTY) * g.nz;
}

int z_blocks(const OctaveGeom &g)
{
    return ((g.nx + 31) / 32) * ((g.ny + 7) / 8) * ((g.nz + kZPlanes - 1) / kZPlanes);
}

// Geometry of job j of an xy launch; block0 continues after job j-1.
void set_xy_job(XYArgs &a, int j, const OctaveGeom &g)
{
    XYJob &jb = a.job[j];
    jb.nx = g.nx;
    jb.ny = g.ny;
    jb.nz = g.nz;
    jb.tiles_x = (g.nx + kXYTX - 1) / kXYTX;
    jb.tiles_y = (g.ny + kXYTY - 1) / kXYTY;
    jb.block0 = j == 0 ? 0 : a.job[j - 1].block0 + a.job[j - 1].tiles_x * a.job[j - 1].tiles_y * a.job[j - 1].nz;
}

void set_z_job(ZArgs &a, int j, const OctaveGeom &g, const OctaveGeom *sub)
{
    ZJob &jb = a.job[j];
    jb.nx = g.nx;
    jb.ny = g.ny;
    jb.nz = g.nz;
    jb.mx = sub ? sub->nx : 0;
    jb.my = sub ? sub->ny : 0;
    jb.mz = sub ? sub->nz : 0;
    jb.gx = (g.nx + 31) / 32;
    jb.gy = (g.ny + 7) / 8;
    jb.gz = (g.nz + kZPlanes - 1) / kZPlanes;
    jb.block0 = j == 0 ? 0 : a.job[j - 1].block0 + a.job[j - 1].gx * a.job[j - 1].gy * a.job[j - 1].gz;
}

int pass_index(const sift3d_plan *pl, int o, int level)
{
    for (size_t b = 0; b < pl->blur.size(); ++b)
        if (pl->blur[b].octave == o && pl->blur[b].dst_idx == level) return (int)b;
    return -1;
}

// List scheduler: alternating xy and z launches, each holding every split
// task whose inputs are ready (at most kMaxJobs jobs and kMaxTapSets tap
// sets per launch); fused passes are launches of their own.
void build_schedule(sift3d_plan *pl)
{
    const int S = pl->S;
    pl->tasks.clear();
    pl->sched.clear();
    for (size_t b = 0; b < pl->blur.size(); ++b) pl->tasks.push_back(Task{0, (int)b, pl->blur[b].octave, 0});
    if (pl->brief_rb >= 0)
        for (int o = 0; o < pl->n_oct; ++o)
            for (int s = 1; s <= S; ++s) pl->tasks.push_back(Task{1, -1, o, s});
    const int nt = (int)pl->tasks.size();
    std::vector<char> xy_done(nt, 0), done(nt, 0);
    std::vector<int> task_of_pass(pl->blur.size(), -1);
    for (int t = 0; t < nt; ++t)
        if (pl->tasks[t].kind == 0) task_of_pass[pl->tasks[t].pass] = t;
    auto pass_done = [&](int o, int level) {
        const int b = pass_index(pl, o, level);
        return b >= 0 && done[task_of_pass[b]];
    };
    auto ready = [&](int t) {
        const Task &k = pl->tasks[t];
        if (k.kind == 1) return pass_done(k.octave, k.s);
        const BlurLaunch &L = pl->blur[k.pass];
        if (L.src_kind < 0) return true;
        if (L.src_idx == 0 && L.octave > 0) return pass_done(L.octave - 1, S);  // G_0 from the sub-sample
        return pass_done(L.octave, L.src_idx);
    };
    auto is_fused = [&](int t) { return pl->tasks[t].kind == 0 && pl->blur[pl->tasks[t].pass].fused; };
    auto tapset_of = [&](int t) {
        return pl->tasks[t].kind == 0 ? pl->blur[pl->tasks[t].pass].tapset : pl->brief_tapset;
    };
    auto emit = [&](int type, const std::vector<int> &ts) {
        Step st{type, {}};
        std::vector<int> sets;
        for (int t : ts) {
            const int id = tapset_of(t);
            const bool known = std::find(sets.begin(), sets.end(), id) != sets.end();
            if ((int)st.tasks.size() == kMaxJobs || (!known && (int)sets.size() == kMaxTapSets)) {
                pl->sched.push_back(st);
                st.tasks.clear();
                sets.clear();
            }
            if (std::find(sets.begin(), sets.end(), id) == sets.end()) sets.push_back(id);
            st.tasks.push_back(t);
        }
        if (!st.tasks.empty()) pl->sched.push_back(st);
    };
    int remaining = nt;
    while (remaining > 0) {
        bool progress = false;
        for (int t = 0; t < nt; ++t)
            if (!done[t] && is_fused(t) && ready(t)) {
                pl->sched.push_back(Step{0, {t}});
                done[t] = 1;
                --remaining;
                progress = true;
            }
        std::vector<int> xs;
        for (int t = 0; t < nt; ++t)
            if (!done[t] && !xy_done[t] && !is_fused(t) && ready(t)) xs.push_back(t);
        emit(1, xs);
        for (int t : xs) xy_done[t] = 1;
        std::vector<int> zs;
        for (int t = 0; t < nt; ++t)
            if (!done[t] && xy_done[t]) zs.push_back(t);
        emit(2, zs);
        for (int t : zs) {
            done[t] = 1;
            --remaining;
        }
        if (!zs.empty()) progress = true;
        if (!progress) break;  // not reachable for a well-formed pyramid
    }
}

}  // namespace

extern "C" {

int sift3d_default_params(sift3d_params *p)
{
    if (p == nullptr) return SIFT3D_E_ARG;
    p->n_octaves = 0;
    p->min_dim = 16;
    p->scales = 3;
    p->sigma0 = 1.6;
    p->sigma_in = 0.0;
    p->trunc = 3.0;
    p->dog_threshold = 0.01f;
    p->votes = 80;
    p->brief_n = 256;
    p->brief_blur = 0.95;
    p->siftrank_factor = 2.0;
    p->pyramid_mode = 0;
    return SIFT3D_OK;
}

int sift3d_create(const sift3d_params *p, const double *pair_draws, int n_draws, sift3d_ctx **out)
{
    if (out == nullptr) return SIFT3D_E_ARG;
    *out = nullptr;
    int rc = check_params(p);
    if (rc != SIFT3D_OK) return rc;
    if (p->brief_n > 0 && (pair_draws == nullptr || n_draws < p->brief_n)) return SIFT3D_E_ARG;
    sift3d_ctx *c = new (std::nothrow) sift3d_ctx();
    if (c == nullptr) return SIFT3D_E_ARG;
    c->p = *p;
    c->d_offsets = nullptr;
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e);
    }
    const int n = p->brief_n, S = p->scales;
    c->draws.assign(pair_draws, pair_draws + (size_t)n * 6);
    c->offsets.resize((size_t)S * n * 6);
    for (int s = 1; s <= S; ++s) pair_offsets(*p, c->draws.data(), s, &c->offsets[(size_t)(s - 1) * n * 6]);
    if (n > 0) {
        const size_t bytes = c->offsets.size() * sizeof(int32_t);
        e = hipMalloc((void **)&c->d_offsets, bytes);
        if (e != hipSuccess) {
            delete c;
            return hip_fail(e);
        }
        e = hipMemcpy(c->d_offsets, c->offsets.data(), bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(c->d_offsets);
            delete c;
            return hip_fail(e);
        }
    }
    *out = c;
    return SIFT3D_OK;
}

int sift3d_destroy(sift3d_ctx *ctx)
{
    if (ctx == nullptr) return SIFT3D_E_ARG;
    if (ctx->d_offsets != nullptr) (void)hipFree(ctx->d_offsets);
    delete ctx;
    return SIFT3D_OK;
}

int sift3d_pair_offsets(const sift3d_params *p, const double *pair_draws, int n_draws, int scale, int32_t *out)
{
    const int rc = check_params(p);
    if (rc != SIFT3D_OK) return rc;
    if (out == nullptr || scale < 1 || scale > p->scales) return SIFT3D_E_ARG;
    if (p->brief_n > 0 && (pair_draws == nullptr || n_draws < p->brief_n)) return SIFT3D_E_ARG;
    pair_offsets(*p, pair_draws, scale, out);
    return SIFT3D_OK;
}

int sift3d_plan_create(sift3d_ctx *ctx, int nx, int ny, int nz, int kp_capacity, sift3d_plan **out)
{
    if (out == nullptr) return SIFT3D_E_ARG;
    *out = nullptr;
    if (ctx == nullptr || nx < 1 || ny < 1 || nz < 1 || kp_capacity < 0) return SIFT3D_E_ARG;
    if ((long long)nx * ny > (1LL << 30) || (long long)nx * ny * nz > (1LL << 40)) return SIFT3D_E_ARG;
    const sift3d_params &p = ctx->p;
    sift3d_plan *pl = new (std::nothrow) sift3d_plan();
    if (pl == nullptr) return SIFT3D_E_ARG;
    pl->ctx = ctx;
    pl->nx = nx;
    pl->ny = ny;
    pl->nz = nz;
    pl->cap = kp_capacity;
    pl->S = p.scales;
    const int S = p.scales, nlev = levels_per_octave(S);
    // octave geometry: halve (floor) while the smallest dim stays >= min_dim
    int cx = nx, cy = ny, cz = nz;
    size_t off = 0;
    while (std::min(cx, std::min(cy, cz)) >= p.min_dim) {
        if (p.n_octaves > 0 && (int)pl->oct.size() == p.n_octaves) break;
        if ((int)pl->oct.size() == kMaxOctaves) break;
        OctaveGeom g;
        g.nx = cx;
        g.ny = cy;
        g.nz = cz;
        g.n = (size_t)cx * cy * cz;
        g.level_bytes = align256(g.n * sizeof(float));
        g.base = off;
        off += g.level_bytes * nlev;
        pl->oct.push_back(g);
        cx /= 2;
        cy /= 2;
        cz /= 2;
    }
    pl->n_oct = (int)pl->oct.size();
    if (pl->n_oct == 0) {
        delete pl;
        return SIFT3D_E_TOO_SMALL;
    }
    pl->pyramid_bytes = off;
    // detection scratch
    long long rows = 0;
    for (const auto &g : pl->oct) rows += (long long)S * (g.nz - 2) * (g.ny - 2);
    pl->total_rows = rows;
    pl->det_blocks = (int)((rows + kDetRowsPerBlock - 1) / kDetRowsPerBlock);
    pl->row_count_off = off;
    off += align256((size_t)rows * sizeof(int));
    pl->block_sum_off = off;
    off += align256((size_t)pl->det_blocks * sizeof(int));
    pl->block_off_off = off;
    off += align256((size_t)pl->det_blocks * sizeof(int));
    pl->masks_off = off;
    for (const auto &g : pl->oct)
        off += align256((size_t)S * (g.nz - 2) * (g.ny - 2) * ((g.nx + 63) / 64) * sizeof(unsigned long long));
    pl->ws_bytes = off;

    // blur schedule: G_0 of octave 0 from the input, then G_1..G_{S+2} per
    // octave, the pass writing G_S also writing the next octave's G_0
    pl->base_sigma = std::sqrt(p.sigma0 * p.sigma0 - p.sigma_in * p.sigma_in);
    for (int i = 1; i <= S + 2; ++i) {
        const double a = scale_sigma(p, i), b = scale_sigma(p, i - 1);
        pl->inc_sigma.push_back(std::sqrt(a * a - b * b));
    }
    // tap sets: 0 = base blur, i = increment of G_i, S+3 = BRIEF pre-blur
    auto add_taps = [&](double sigma) {
        const std::vector<double> w = gaussian(sigma, p.trunc);
        std::vector<float> f(kMaxTaps, 0.0f);
        for (size_t t = 0; t < w.size(); ++t) f[t] = (float)w[t];
        pl->tapsets.push_back(f);
        pl->tapset_r.push_back((int)(w.size() - 1) / 2);
    };
    add_taps(pl->base_sigma);
    for (int i = 1; i <= S + 2; ++i) add_taps(pl->inc_sigma[i - 1]);
    add_taps(p.brief_blur);
    pl->brief_tapset = S + 3;
    pl->brief_rb = (p.brief_blur > 0.0 && p.brief_n > 0) ? pl->tapset_r[S + 3] : -1;

    for (int o = 0; o < pl->n_oct; ++o) {
        const OctaveGeom &g = pl->oct[o];
        for (int i = (o == 0 ? 0 : 1); i <= S + 2; ++i) {
            BlurLaunch L{};
            L.tapset = i;
            L.r = pl->tapset_r[i];
            L.dog = i > 0;
            L.octave = o;
            L.src_kind = i == 0 ? -1 : 0;
            L.src_idx = i - 1;
            L.dst_idx = i;
            L.dog_idx = i - 1;
            L.sub_octave = (i == S && o + 1 < pl->n_oct) ? o + 1 : -1;
            L.fused = p.pyramid_mode == 1 || (p.pyramid_mode == 0 && (long long)g.n >= kFusedMinVoxels);
            if (L.fused) {
                BlurArgs &a = L.a;
                a.nx = g.nx;
                a.ny = g.ny;
                a.nz = g.nz;
                if (L.sub_octave >= 0) {
                    a.mx = pl->oct[o + 1].nx;
                    a.my = pl->oct[o + 1].ny;
                    a.mz = pl->oct[o + 1].nz;
                }
                a.tiles_x = (g.nx + kBlurTX - 1) / kBlurTX;
                a.tiles_y = (g.ny + kBlurTY - 1) / kBlurTY;
                a.L = choose_slab(g.nz, a.tiles_x * a.tiles_y, L.r);
                a.slabs = (g.nz + a.L - 1) / a.L;
                a.n_blocks = a.tiles_x * a.tiles_y * a.slabs;
                for (int t = 0; t < kMaxTaps; ++t) a.w[t] = pl->tapsets[i][t];
            }
            pl->blur.push_back(L);
        }
    }
    build_schedule(pl);
    *out = pl;
    return SIFT3D_OK;
}

int sift3d_plan_destroy(sift3d_plan *plan)
{
    if (plan == nullptr) return SIFT3D_E_ARG;
    delete plan;
    return SIFT3D_OK;
}

int sift3d_plan_info(const sift3d_plan *plan, size_t *workspace_bytes, int *n_octaves)
{
    if (plan == nullptr) return SIFT3D_E_ARG;
    if (workspace_bytes) *workspace_bytes = plan->ws_bytes;
    if (n_octaves) *n_octaves = plan->n_oct;
    return SIFT3D_OK;
}

int sift3d_plan_octave_dims(const sift3d_plan *plan, int octave, int dims[3])
{
    if (plan == nullptr || dims == nullptr || octave < 0 || octave >= plan->n_oct) return SIFT3D_E_ARG;
    dims[0] = plan->oct[octave].nx;
    dims[1] = plan->oct[octave].ny;
    dims[2] = plan->oct[octave].nz;
    return SIFT3D_OK;
}

static float *raw_level(const sift3d_plan *pl, const void *ws, int o, int lev)
{
    const OctaveGeom &g = pl->oct[o];
    return reinterpret_cast<float *>(const_cast<char *>(static_cast<const char *>(ws)) + g.base +
                                     (size_t)lev * g.level_bytes);
}

static float *level_ptr(const sift3d_plan *pl, const void *ws, int o, int kind, int idx)
{
    return raw_level(pl, ws, o, kind == 0 ? lev_G(idx) : lev_D(pl->S, idx));
}

int sift3d_level(const sift3d_plan *plan, void *d_ws, int octave, int kind, int idx, float **d_ptr)
{
    if (plan == nullptr || d_ws == nullptr || d_ptr == nullptr) return SIFT3D_E_ARG;
    if (octave < 0 || octave >= plan->n_oct || kind < 0 || kind > 1) return SIFT3D_E_ARG;
    if (idx < 0 || idx >= (kind == 0 ? plan->S + 3 : plan->S + 2)) return SIFT3D_E_ARG;
    *d_ptr = level_ptr(plan, d_ws, octave, kind, idx);
    return SIFT3D_OK;
}

static int check_ws(const sift3d_plan *plan, const void *ws, size_t bytes)
{
    if (plan == nullptr || ws == nullptr) return SIFT3D_E_ARG;
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return SIFT3D_E_ARG;
    if (bytes < plan->ws_bytes) return SIFT3D_E_WORKSPACE;
    return SIFT3D_OK;
}

// Device pointers of a task's xy and z halves for one call.
struct TaskPtrs {
    const float *src;
    float *t, *dst, *dog, *sub;
    const OctaveGeom *g, *sub_g;
    int r, tapset;
};

static TaskPtrs task_ptrs(const sift3d_plan *plan, const Task &k, const float *d_vol, const void *d_ws)
{
    TaskPtrs q{};
    const int S = plan->S;
    if (k.kind == 0) {
        const BlurLaunch &L = plan->blur[k.pass];
        q.src = L.src_kind < 0 ? d_vol : level_ptr(plan, d_ws, L.octave, 0, L.src_idx);
        q.t = raw_level(plan, d_ws, L.octave, lev_T(S));
        q.dst = level_ptr(plan, d_ws, L.octave, 0, L.dst_idx);
        q.dog = L.dog ? level_ptr(plan, d_ws, L.octave, 1, L.dog_idx) : nullptr;
        q.sub = L.sub_octave >= 0 ? level_ptr(plan, d_ws, L.sub_octave, 0, 0) : nullptr;
        q.g = &plan->oct[L.octave];
        q.sub_g = L.sub_octave >= 0 ? &plan->oct[L.sub_octave] : nullptr;
        q.r = L.r;
        q.tapset = L.tapset;
    } else {
        q.src = raw_level(plan, d_ws, k.octave, lev_G(k.s));
        q.t = raw_level(plan, d_ws, k.octave, lev_Tb(S, k.s));
        q.dst = raw_level(plan, d_ws, k.octave, lev_B(S, k.s));
        q.dog = nullptr;
        q.sub = nullptr;
        q.g = &plan->oct[k.octave];
        q.sub_g = nullptr;
        q.r = plan->brief_rb;
        q.tapset = plan->brief_tapset;
    }
    return q;
}

extern "C++" {
// Tap-set slot of a launch (deduplicated, at most kMaxTapSets per launch).
template <typename Args>
static int tap_slot(const sift3d_plan *plan, Args &a, std::vector<int> &sets, int tapset)
{
    for (size_t i = 0; i < sets.size(); ++i)
        if (sets[i] == tapset) return (int)i;
    const int slot = (int)sets.size();
    sets.push_back(tapset);
    for (int t = 0; t < kMaxTaps; ++t) a.w[slot][t] = plan->tapsets[tapset][t];
    return slot;
}
}  // extern "C++"

static int run_step(const sift3d_plan *plan, int type, const std::vector<int> &tasks, const float *d_vol,
                    void *d_ws, hipStream_t st)
{
    hipError_t e = hipSuccess;
    if (type == 0) {
        const BlurLaunch &L = plan->blur[plan->tasks[tasks[0]].pass];
        BlurArgs a = L.a;
        a.src = L.src_kind < 0 ? d_vol : level_ptr(plan, d_ws, L.octave, 0, L.src_idx);
        a.dst = level_ptr(plan, d_ws, L.octave, 0, L.dst_idx);
        a.dog = L.dog ? level_ptr(plan, d_ws, L.octave, 1, L.dog_idx) : nullptr;
        a.sub = L.sub_octave >= 0 ? level_ptr(plan, d_ws, L.sub_octave, 0, 0) : nullptr;
        e = launch_blur(a, L.r, L.dog, st);
    } else if (type == 1) {
        XYArgs a{};
        std::vector<int> sets;
        int j = 0;
        for (int t : tasks) {
            const TaskPtrs q = task_ptrs(plan, plan->tasks[t], d_vol, d_ws);
            set_xy_job(a, j, *q.g);
            a.job[j].src = q.src;
            a.job[j].dst = q.t;
            a.job[j].r = q.r;
            a.job[j].taps = tap_slot(plan, a, sets, q.tapset);
            ++j;
        }
        a.n_jobs = j;
        a.n_blocks = a.job[j - 1].block0 + a.job[j - 1].tiles_x * a.job[j - 1].tiles_y * a.job[j - 1].nz;
        e = launch_blur_xy(a, st);
    } else {
        ZArgs a{};
        std::vector<int> sets;
        int j = 0;
        for (int t : tasks) {
            const TaskPtrs q = task_ptrs(plan, plan->tasks[t], d_vol, d_ws);
            set_z_job(a, j, *q.g, q.sub_g);
            a.job[j].t = q.t;
            a.job[j].center = q.src;
            a.job[j].dst = q.dst;
            a.job[j].dog = q.dog;
            a.job[j].sub = q.sub;
            a.job[j].r = q.r;
            a.job[j].taps = tap_slot(plan, a, sets, q.tapset);
            ++j;
        }
        a.n_jobs = j;
        a.n_blocks = a.job[j - 1].block0 + a.job[j - 1].gx * a.job[j - 1].gy * a.job[j - 1].gz;
        e = launch_blur_z(a, st);
    }
    return e == hipSuccess ? SIFT3D_OK : hip_fail(e);
}

int sift3d_build_pyramid(const sift3d_plan *plan, const float *d_vol, void *d_ws, size_t ws_bytes, void *stream)
{
    int rc = check_ws(plan, d_ws, ws_bytes);
    if (rc != SIFT3D_OK) return rc;
    if (d_vol == nullptr) return SIFT3D_E_ARG;
    for (const Step &stp : plan->sched) {
        rc = run_step(plan, stp.type, stp.tasks, d_vol, d_ws, static_cast<hipStream_t>(stream));
        if (rc != SIFT3D_OK) return rc;
    }
    return SIFT3D_OK;
}

int sift3d_pyramid_pass_count(const sift3d_plan *plan, int *n_passes)
{
    if (plan == nullptr || n_passes == nullptr) return SIFT3D_E_ARG;
    *n_passes = (int)plan->blur.size();
    return SIFT3D_OK;
}

int sift3d_pyramid_pass_info(const sift3d_plan *plan, int pass, int info[5], size_t *bytes)
{
    if (plan == nullptr || pass < 0 || pass >= (int)plan->blur.size()) return SIFT3D_E_ARG;
    const BlurLaunch &L = plan->blur[pass];
    if (info != nullptr) {
        info[0] = L.octave;
        info[1] = L.dst_idx;
        info[2] = L.r;
        info[3] = L.sub_octave >= 0 ? 1 : 0;
        info[4] = L.fused ? 1 : 0;
    }
    if (bytes != nullptr) {
        const size_t n = plan->oct[L.octave].n;
        size_t b = 8 * n + (L.dog ? 4 * n : 0);
        if (L.sub_octave >= 0) b += 4 * plan->oct[L.sub_octave].n;
        *bytes = b;
    }
    return SIFT3D_OK;
}

int sift3d_pyramid_pass(const sift3d_plan *plan, int pass, const float *d_vol, void *d_ws, size_t ws_bytes,
                        void *stream)
{
    int rc = check_ws(plan, d_ws, ws_bytes);
    if (rc != SIFT3D_OK) return rc;
    if (pass < 0 || pass >= (int)plan->blur.size()) return SIFT3D_E_ARG;
    const BlurLaunch &L = plan->blur[pass];
    if (L.src_kind < 0 && d_vol == nullptr) return SIFT3D_E_ARG;
    int t = -1;
    for (size_t k = 0; k < plan->tasks.size(); ++k)
        if (plan->tasks[k].kind == 0 && plan->tasks[k].pass == pass) t = (int)k;
    const std::vector<int> one{t};
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (L.fused) return run_step(plan, 0, one, d_vol, d_ws, st);
    rc = run_step(plan, 1, one, d_vol, d_ws, st);
    if (rc != SIFT3D_OK) return rc;
    return run_step(plan, 2, one, d_vol, d_ws, st);
}

int sift3d_detect(const sift3d_plan *plan, void *d_ws, size_t ws_bytes, sift3d_keypoint *d_kp, int kp_capacity,
                  int *d_count, void *stream)
{
    int rc = check_ws(plan, d_ws, ws_bytes);
    if (rc != SIFT3D_OK) return rc;
    if (d_count == nullptr || kp_capacity < 0 || (kp_capacity > 0 && d_kp == nullptr)) return SIFT3D_E_ARG;
    const sift3d_params &p = plan->ctx->p;
    DetectArgs a{};
    for (int o = 0; o < plan->n_oct; ++o) {
        const OctaveGeom &g = plan->oct[o];
        DetOctave &d = a.oc[o];
        d.D = level_ptr(plan, d_ws, o, 1, 0);
        d.lstride = (long long)(g.level_bytes / sizeof(float));
        d.nx = g.nx;
        d.ny = g.ny;
        d.nz = g.nz;
        d.row_base = 0;
        for (int q = 0; q < o; ++q)
            d.row_base += (long long)plan->S * (plan->oct[q].nz - 2) * (plan->oct[q].ny - 2);
        d.rows = (long long)plan->S * (g.nz - 2) * (g.ny - 2);
        for (int s = 0; s <= plan->S; ++s) d.sigma[s] = (float)(scale_sigma(p, s) * std::ldexp(1.0, o));
        d.words = (g.nx + 63) / 64;
        d.tiles_x = d.words;
        d.tiles_y = (g.ny - 2 + kDTY - 1) / kDTY;   // interior rows 1..ny-2
        d.tiles_z = (g.nz - 2 + kDTZ - 1) / kDTZ;   // interior planes 1..nz-2
        d.block0 = a.tile_blocks;
        a.tile_blocks += d.tiles_x * d.tiles_y * d.tiles_z;
    }
    {
        size_t moff = plan->masks_off;
        for (int o = 0; o < plan->n_oct; ++o) {
            a.oc[o].masks = reinterpret_cast<unsigned long long *>(static_cast<char *>(d_ws) + moff);
            moff += align256((size_t)a.oc[o].rows * a.oc[o].words * sizeof(unsigned long long));
        }
    }
    a.row_blocks = (int)((plan->total_rows + kRowBlock - 1) / kRowBlock);
    a.n_oct = plan->n_oct;
    a.S = plan->S;
    a.total_rows = plan->total_rows;
    a.n_blocks = plan->det_blocks;
    a.thr = p.dog_threshold;
    a.votes = p.votes;
    char *ws = static_cast<char *>(d_ws);
    a.row_count = reinterpret_cast<int *>(ws + plan->row_count_off);
    a.block_sum = reinterpret_cast<int *>(ws + plan->block_sum_off);
    a.block_off = reinterpret_cast<int *>(ws + plan->block_off_off);
    a.d_count = d_count;
    a.kp = d_kp;
    a.cap = kp_capacity;
    const hipError_t e = launch_detect(a, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SIFT3D_OK : hip_fail(e);
}

int sift3d_describe(const sift3d_plan *plan, const void *d_ws, size_t ws_bytes, const sift3d_keypoint *d_kp,
                    const int *d_count, int kp_capacity, uint8_t *d_siftrank, uint64_t *d_brief, uint8_t *d_rrief,
                    void *stream)
{
    int rc = check_ws(plan, d_ws, ws_bytes);
    if (rc != SIFT3D_OK) return rc;
    if (d_count == nullptr || kp_capacity < 0 || (kp_capacity > 0 && d_kp == nullptr)) return SIFT3D_E_ARG;
    const sift3d_params &p = plan->ctx->p;
    if (p.brief_n == 0) d_brief = nullptr, d_rrief = nullptr;
    DescribeArgs a{};
    for (int o = 0; o < plan->n_oct; ++o) {
        const OctaveGeom &g = plan->oct[o];
        a.oc[o].G = level_ptr(plan, d_ws, o, 0, 0);
        a.oc[o].B = plan->brief_rb >= 0 ? raw_level(plan, d_ws, o, lev_B(plan->S, 1)) : level_ptr(plan, d_ws, o, 0, 1);
        a.oc[o].lstride = (long long)(g.level_bytes / sizeof(float));
        a.oc[o].nx = g.nx;
        a.oc[o].ny = g.ny;
        a.oc[o].nz = g.nz;
    }
    a.n_oct = plan->n_oct;
    a.S = plan->S;
    for (int s = 0; s <= plan->S; ++s) a.sift_R[s] = (int)std::ceil(p.siftrank_factor * scale_sigma(p, s));
    a.kp = d_kp;
    a.d_count = d_count;
    a.cap = kp_capacity;
    a.siftrank = d_siftrank;
    a.brief = d_brief;
    a.rrief = d_rrief;
    a.brief_n = p.brief_n;
    a.pairs = plan->ctx->d_offsets;
    const int grid = std::min(kp_capacity, 4096);
    const hipError_t e = launch_describe(a, grid, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SIFT3D_OK : hip_fail(e);
}

int sift3d_extract(const sift3d_plan *plan, const float *d_vol, void *d_ws, size_t ws_bytes, sift3d_keypoint *d_kp,
                   int kp_capacity, int *d_count, uint8_t *d_siftrank, uint64_t *d_brief, uint8_t *d_rrief,
                   void *stream)
{
    int rc = sift3d_build_pyramid(plan, d_vol, d_ws, ws_bytes, stream);
    if (rc != SIFT3D_OK) return rc;
    rc = sift3d_detect(plan, d_ws, ws_bytes, d_kp, kp_capacity, d_count, stream);
    if (rc != SIFT3D_OK) return rc;
    return sift3d_describe(plan, d_ws, ws_bytes, d_kp, d_count, kp_capacity, d_siftrank, d_brief, d_rrief,
                           stream);
}

const char *sift3d_error_string(int code)
{
    switch (code) {
    case SIFT3D_OK: return "ok";
    case SIFT3D_E_ARG: return "invalid argument";
    case SIFT3D_E_TOO_SMALL: return "volume too small: no octave";
    case SIFT3D_E_WORKSPACE: return "workspace too small";
    case SIFT3D_E_HIP: return "HIP runtime error";
    case SIFT3D_E_UNSUPPORTED: return "parameter outside the supported range";
    default: return "unknown error";
    }
}

int sift3d_last_hip_error(void) { return g_last_hip; }

}  // extern "C"
