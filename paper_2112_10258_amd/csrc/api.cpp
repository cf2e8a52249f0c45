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
    for (int o = 0; o < pl->n_oct; ++o) {
        const OctaveGeom &g = pl->oct[o];
        for (int i = (o == 0 ? 0 : 1); i <= S + 2; ++i) {
            const double sig = i == 0 ? pl->base_sigma : pl->inc_sigma[i - 1];
            const std::vector<double> w = gaussian(sig, p.trunc);
            BlurLaunch L{};
            L.r = (int)(w.size() - 1) / 2;
            L.dog = i > 0;
            L.octave = o;
            L.src_kind = i == 0 ? -1 : 0;
            L.src_idx = i - 1;
            L.dst_idx = i;
            L.dog_idx = i - 1;
            L.sub_octave = (i == S && o + 1 < pl->n_oct) ? o + 1 : -1;
            L.fused = (long long)g.n >= kFusedMinVoxels;
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
                for (int t = 0; t < kMaxTaps; ++t) a.w[t] = t < (int)w.size() ? (float)w[t] : 0.0f;
            } else {
                const OctaveGeom *sub = L.sub_octave >= 0 ? &pl->oct[o + 1] : nullptr;
                set_xy_job(L.xy, 0, g);
                L.xy.n_jobs = 1;
                L.xy.n_blocks = L.xy.job[0].block0 + xy_blocks(g);
                set_z_job(L.z, 0, g, sub);
                L.z.n_jobs = 1;
                L.z.n_blocks = z_blocks(g);
                for (int t = 0; t < kMaxTaps; ++t) L.xy.w[t] = L.z.w[t] = t < (int)w.size() ? (float)w[t] : 0.0f;
            }
            pl->blur.push_back(L);
        }
    }
    // BRIEF pre-blur: B_s = G_s blurred by sigma_b (none when sigma_b == 0)
    {
        const std::vector<double> wb = gaussian(p.brief_blur, p.trunc);
        pl->brief_rb = p.brief_blur > 0.0 ? (int)(wb.size() - 1) / 2 : -1;
        pl->wb.assign(kMaxTaps, 0.0f);
        for (size_t t = 0; t < wb.size(); ++t) pl->wb[t] = (float)wb[t];
    }
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

static int run_pass(const sift3d_plan *plan, const BlurLaunch &L, const float *d_vol, void *d_ws, hipStream_t st)
{
    const float *src = L.src_kind < 0 ? d_vol : level_ptr(plan, d_ws, L.octave, 0, L.src_idx);
    float *dst = level_ptr(plan, d_ws, L.octave, 0, L.dst_idx);
    float *dog = L.dog ? level_ptr(plan, d_ws, L.octave, 1, L.dog_idx) : nullptr;
    float *sub = L.sub_octave >= 0 ? level_ptr(plan, d_ws, L.sub_octave, 0, 0) : nullptr;
    hipError_t e;
    if (L.fused) {
        BlurArgs a = L.a;
        a.src = src;
        a.dst = dst;
        a.dog = dog;
        a.sub = sub;
        e = launch_blur(a, L.r, L.dog, st);
    } else {
        float *t = raw_level(plan, d_ws, L.octave, lev_T(plan->S));
        XYArgs xy = L.xy;
        xy.job[0].src = src;
        xy.job[0].dst = t;
        e = launch_blur_xy(xy, L.r, st);
        if (e == hipSuccess) {
            ZArgs z = L.z;
            z.job[0].t = t;
            z.job[0].center = src;
            z.job[0].dst = dst;
            z.job[0].dog = dog;
            z.job[0].sub = sub;
            e = launch_blur_z(z, L.r, L.dog, st);
        }
    }
    return e == hipSuccess ? SIFT3D_OK : hip_fail(e);
}

// B_s = G_s blurred by the BRIEF pre-blur, for every octave and s = 1..S,
// as job lists of at most kMaxJobs (octave, s) levels per launch pair.
static int run_preblur(const sift3d_plan *plan, const void *d_ws, hipStream_t st)
{
    if (plan->brief_rb < 0) return SIFT3D_OK;
    const int S = plan->S;
    std::vector<std::pair<int, int>> jobs;
    for (int o = 0; o < plan->n_oct; ++o)
        for (int s = 1; s <= S; ++s) jobs.emplace_back(o, s);
    for (size_t j0 = 0; j0 < jobs.size(); j0 += kMaxJobs) {
        XYArgs xy{};
        ZArgs z{};
        const int nj = (int)std::min<size_t>(kMaxJobs, jobs.size() - j0);
        for (int j = 0; j < nj; ++j) {
            const int o = jobs[j0 + j].first, s = jobs[j0 + j].second;
            const OctaveGeom &g = plan->oct[o];
            set_xy_job(xy, j, g);
            xy.job[j].src = raw_level(plan, d_ws, o, lev_G(s));
            xy.job[j].dst = raw_level(plan, d_ws, o, lev_Tb(S, s));
            set_z_job(z, j, g, nullptr);
            z.job[j].t = xy.job[j].dst;
            z.job[j].center = nullptr;
            z.job[j].dst = raw_level(plan, d_ws, o, lev_B(S, s));
            z.job[j].dog = nullptr;
            z.job[j].sub = nullptr;
        }
        xy.n_jobs = z.n_jobs = nj;
        xy.n_blocks = xy.job[nj - 1].block0 + xy_blocks(plan->oct[jobs[j0 + nj - 1].first]);
        z.n_blocks = z.job[nj - 1].block0 + z_blocks(plan->oct[jobs[j0 + nj - 1].first]);
        for (int t = 0; t < kMaxTaps; ++t) xy.w[t] = z.w[t] = plan->wb[t];
        hipError_t e = launch_blur_xy(xy, plan->brief_rb, st);
        if (e == hipSuccess) e = launch_blur_z(z, plan->brief_rb, false, st);
        if (e != hipSuccess) return hip_fail(e);
    }
    return SIFT3D_OK;
}

int sift3d_build_pyramid(const sift3d_plan *plan, const float *d_vol, void *d_ws, size_t ws_bytes, void *stream)
{
    int rc = check_ws(plan, d_ws, ws_bytes);
    if (rc != SIFT3D_OK) return rc;
    if (d_vol == nullptr) return SIFT3D_E_ARG;
    for (const BlurLaunch &L : plan->blur) {
        rc = run_pass(plan, L, d_vol, d_ws, static_cast<hipStream_t>(stream));
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

int sift3d_pyramid_pass_info(const sift3d_plan *plan, int pass, int info[4], size_t *bytes)
{
    if (plan == nullptr || pass < 0 || pass >= (int)plan->blur.size()) return SIFT3D_E_ARG;
    const BlurLaunch &L = plan->blur[pass];
    if (info != nullptr) {
        info[0] = L.octave;
        info[1] = L.dst_idx;
        info[2] = L.r;
        info[3] = L.sub_octave >= 0 ? 1 : 0;
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
    return run_pass(plan, L, d_vol, d_ws, static_cast<hipStream_t>(stream));
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
    if (d_brief != nullptr || d_rrief != nullptr) {
        rc = run_preblur(plan, d_ws, static_cast<hipStream_t>(stream));
        if (rc != SIFT3D_OK) return rc;
    }
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
