// Host side of the C ABI: parameter checks, contexts, plans (octave
// geometry, workspace layout, launch shapes) and the stream-ordered entry
// points. Nothing here synchronises the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "sift3d_internal.h"

using namespace s3d;

namespace {

thread_local int g_last_hip = 0;

// Detection scratch of the allocation-free entry point (sift3d_detect_static):
// row counts, block sums and offsets and keypoint bit masks. Every GPU holds
// its own copy of this array from module load until the process ends. In
// host code its name is not a device address: the address on each device
// comes from hipGetSymbolAddress, taken once per device (with that device
// current) by sift3d_create, and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[SIFT3D_DETECT_STATIC_SCRATCH];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (the current device).
hipError_t static_scratch(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (p == nullptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

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
    if (p->pyramid_mode < 0 || p->pyramid_mode > 3) return SIFT3D_E_ARG;
    if (p->brief_method < 1 || p->brief_method > 5) return SIFT3D_E_ARG;
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

// Output planes per slab when a fused launch splits each job's depth into
// `slabs` slabs, even, and at least kMinSlabPlanes: shorter slabs add more
// blocks but pay 2R halo planes each, and on a 145x174x145 octave 12 planes
// beat both 8 (every resident slot filled, 2.25x the planes at R = 5) and
// 2R (16 at R = 8: G_4 35 -> 31.5 us).
//
// The fused pass runs its plane loop in rounds of 2R + 2 steps (the length
// of its register ring), and a slab of L planes takes L + 2R steps, so
// steps past the end of a slab in its last round still cost their loads
// and barriers. When a slab has more than one round, L is raised (by less
// than one round) until L + 2R fills whole rounds; the last slab of a job
// keeps the remainder.
int slab_planes(int nz, int slabs, int r)
{
    int L = (nz + slabs - 1) / slabs;
    L = std::max(L, kMinSlabPlanes);
    L = (L + 1) & ~1;
    const int round = 2 * r + 2;
    if (L + 2 * r > round) L = ((L + 2 * r + round - 1) / round) * round - 2 * r;   // even: round and 2r are
    return std::min(L, (nz + 1) & ~1);
}

// P(|z|^2 <= x) for a standard-normal 3-vector z (chi-square CDF, 3 dof).
static double chi3_cdf(double x)
{
    return std::erf(std::sqrt(x / 2.0)) - std::sqrt(2.0 * x / M_PI) * std::exp(-x / 2.0);
}

// Point pairs of the five selection methods (Section 3.2.3), sigma = the
// keypoint scale in octave voxels, each point rounded to the nearest voxel
// (floor(c + 0.5)). The randomness is the draws (z1, z2), two standard-normal
// 3-vectors per pair. out: [n][2][3].
//   1: p1, p2 uniform in the ball of radius 2 sigma: direction z/|z|, radius
//      2 sigma F(|w|^2)^(1/3) with F the chi-square(3) CDF (so F(|w|^2) is
//      uniform); p1 = (direction of z1, norm of z2), p2 the reverse.
//   2: p1 = sigma z1, p2 = sigma z2.
//   3: p1 = sigma z1, p2 = sigma (z1 + z2), i.e. p2 ~ N(p1, sigma).
//   4: p1 = 0, p2 = sigma z2.
//   5: p1 = 0, p2 on a regular spherical grid: n/64 radii 2 sigma (k+1)/(n/64),
//      polar angles pi (j + 1/2)/8, azimuths 2 pi (i + (j mod 2)/2)/8, pair
//      64 k + 8 j + i.
void pair_offsets(const sift3d_params &p, const double *draws, int s, int32_t *out)
{
    const double sig = scale_sigma(p, s);
    const int n = p.brief_n;
    auto put = [&](int i, int which, const double c[3]) {
        for (int d = 0; d < 3; ++d) out[(size_t)i * 6 + which * 3 + d] = (int32_t)std::floor(c[d] + 0.5);
    };
    for (int i = 0; i < n; ++i) {
        const double *z1 = draws + (size_t)i * 6, *z2 = z1 + 3;
        double a[3] = {0.0, 0.0, 0.0}, b[3] = {0.0, 0.0, 0.0};
        switch (p.brief_method) {
        case 1: {
            const double n1 = std::sqrt(z1[0] * z1[0] + z1[1] * z1[1] + z1[2] * z1[2]);
            const double n2 = std::sqrt(z2[0] * z2[0] + z2[1] * z2[1] + z2[2] * z2[2]);
            const double ra = 2.0 * sig * std::cbrt(chi3_cdf(n2 * n2));
            const double rb = 2.0 * sig * std::cbrt(chi3_cdf(n1 * n1));
            for (int d = 0; d < 3; ++d) {
                a[d] = n1 > 0.0 ? z1[d] / n1 * ra : 0.0;
                b[d] = n2 > 0.0 ? z2[d] / n2 * rb : 0.0;
            }
            break;
        }
        case 2:
            for (int d = 0; d < 3; ++d) {
                a[d] = sig * z1[d];
                b[d] = sig * z2[d];
            }
            break;
        case 4:
            for (int d = 0; d < 3; ++d) b[d] = sig * z2[d];
            break;
        case 5: {
            const int nr = std::max(1, n / 64);
            const int k = i / 64, j = (i / 8) % 8, q = i % 8;
            const double r = 2.0 * sig * (k + 1) / nr;
            const double th = M_PI * (j + 0.5) / 8.0, ph = 2.0 * M_PI * (q + 0.5 * (j % 2)) / 8.0;
            b[0] = r * std::sin(th) * std::cos(ph);
            b[1] = r * std::sin(th) * std::sin(ph);
            b[2] = r * std::cos(th);
            break;
        }
        default:   // 3
            for (int d = 0; d < 3; ++d) {
                a[d] = sig * z1[d];
                b[d] = sig * (z1[d] + z2[d]);
            }
            break;
        }
        put(i, 0, a);
        put(i, 1, b);
    }
}

// Planes per xy block: 4 while that still leaves >= 1024 blocks for the
// octave (4 per CU), fewer on small octaves.
int xy_planes(const OctaveGeom &g)
{
    const int tiles = ((g.nx + kXYTX - 1) / kXYTX) * ((g.ny + kXYTY - 1) / kXYTY);
    int P = 4;
    while (P > 1 && tiles * ((g.nz + P - 1) / P) < 1024) P /= 2;
    return P;
}

int xy_blocks(const OctaveGeom &g)
{
    const int P = xy_planes(g);
    return ((g.nx + kXYTX - 1) / kXYTX) * ((g.ny + kXYTY - 1) / kXYTY) * ((g.nz + P - 1) / P);
}

int z_blocks(const OctaveGeom &g)
{
    return ((g.nx + 31) / 32) * ((g.ny + 7) / 8) * ((g.nz + kZPlanes - 1) / kZPlanes);
}

int compact_blocks(const OctaveGeom &g)
{
    return ((g.nx + kCTX - 1) / kCTX) * ((g.ny + kCTY - 1) / kCTY) * ((g.nz + kCTZ - 1) / kCTZ);
}

size_t level_off(const OctaveGeom &g, int lev) { return g.base + (size_t)lev * g.level_bytes; }

// The xy and z jobs of a split task (block0 left for the caller).
void task_jobs(const sift3d_plan *pl, const Task &k, DXYJob &xy, DZJob &z)
{
    const int S = pl->S;
    xy = DXYJob{};
    z = DZJob{};
    const VolPlan &vp = pl->vols[k.vol];
    const OctaveGeom *g, *sub = nullptr;
    if (k.kind == 0) {
        const BlurLaunch &L = pl->blur[k.pass];
        g = &vp.oct[L.octave];
        if (L.src_kind < 0) {
            xy.src = (long long)vp.in_off;
            xy.src_input = 1;
        } else {
            xy.src = (long long)level_off(*g, lev_G(L.src_idx));
        }
        xy.dst = z.t = (long long)level_off(*g, lev_T(S));
        z.center = L.dog ? xy.src : -1;
        z.center_input = xy.src_input;
        z.dst = (long long)level_off(*g, lev_G(L.dst_idx));
        z.dog = L.dog ? (long long)level_off(*g, lev_D(S, L.dog_idx)) : -1;
        if (L.sub_octave >= 0) {
            sub = &vp.oct[L.sub_octave];
            z.sub = (long long)level_off(*sub, lev_G(0));
        } else {
            z.sub = -1;
        }
        xy.r = z.r = L.r;
        xy.taps = z.taps = L.tapset;
    } else {
        g = &vp.oct[k.octave];
        xy.src = (long long)level_off(*g, lev_G(k.s));
        xy.dst = z.t = (long long)level_off(*g, lev_Tb(S, k.s));
        z.center = -1;
        z.dst = (long long)level_off(*g, lev_B(S, k.s));
        z.dog = -1;
        z.sub = -1;
        xy.r = z.r = pl->brief_rb;
        xy.taps = z.taps = pl->brief_tapset;
    }
    xy.nx = z.nx = g->nx;
    xy.ny = z.ny = g->ny;
    xy.nz = z.nz = g->nz;
    xy.tiles_x = (g->nx + kXYTX - 1) / kXYTX;
    xy.tiles_y = (g->ny + kXYTY - 1) / kXYTY;
    xy.planes = xy_planes(*g);
    z.mx = sub ? sub->nx : 0;
    z.my = sub ? sub->ny : 0;
    z.mz = sub ? sub->nz : 0;
    z.gx = (g->nx + 31) / 32;
    z.gy = (g->ny + 7) / 8;
    z.gz = (g->nz + kZPlanes - 1) / kZPlanes;
}

// How a level of an octave of n voxels blurred with radius r runs. The
// fused and compact passes are compiled for radii up to 10; larger radii
// always run split.
int level_path(const sift3d_params &p, long long n, int r)
{
    switch (p.pyramid_mode) {
    case 1: return r <= kMaxFusedR ? kPathFused : kPathSplit;
    case 2: return kPathSplit;
    case 3: return r <= kCompactMaxR ? kPathCompact : kPathSplit;
    default: break;
    }
    if (n >= kFusedMinVoxels) return r <= kMaxFusedR ? kPathFused : kPathSplit;
    if (n >= kFusedMidVoxels) return r <= kFusedMidMaxR ? kPathFused : kPathSplit;
    if (n >= kCompactWideVoxels && r > kFusedMidMaxR) return kPathSplit;
    return r <= kCompactMaxR ? kPathCompact : kPathSplit;
}

// The compact job of a task (block0 left for the caller).
DCJob compact_job(const sift3d_plan *pl, const Task &k)
{
    const int S = pl->S;
    DCJob c{};
    const OctaveGeom *g;
    if (k.kind == 1) {
        // BRIEF pre-blur: G_s -> B_s, no DoG, no sub-sample
        g = &pl->vols[k.vol].oct[k.octave];
        c.src = (long long)level_off(*g, lev_G(k.s));
        c.dst = (long long)level_off(*g, lev_B(S, k.s));
        c.dog = -1;
        c.sub = -1;
        c.r = pl->brief_rb;
        c.taps = pl->brief_tapset;
    } else {
        const BlurLaunch &L = pl->blur[k.pass];
        const VolPlan &vp = pl->vols[L.vol];
        g = &vp.oct[L.octave];
        if (L.src_kind < 0) {
            c.src = (long long)vp.in_off;
            c.src_input = 1;
        } else {
            c.src = (long long)level_off(*g, lev_G(L.src_idx));
        }
        c.dst = (long long)level_off(*g, lev_G(L.dst_idx));
        c.dog = L.dog ? (long long)level_off(*g, lev_D(S, L.dog_idx)) : -1;
        if (L.sub_octave >= 0) {
            const OctaveGeom &m = vp.oct[L.sub_octave];
            c.sub = (long long)level_off(m, lev_G(0));
            c.mx = m.nx;
            c.my = m.ny;
            c.mz = m.nz;
        } else {
            c.sub = -1;
        }
        c.r = L.r;
        c.taps = L.tapset;
    }
    c.nx = g->nx;
    c.ny = g->ny;
    c.nz = g->nz;
    c.tiles_x = (g->nx + kCTX - 1) / kCTX;
    c.tiles_y = (g->ny + kCTY - 1) / kCTY;
    c.tiles_z = (g->nz + kCTZ - 1) / kCTZ;
    return c;
}

// The fused job of a level-pass task, its depth split into `slabs` slabs
// (block0 left for the caller).
DFJob fused_job(const sift3d_plan *pl, const Task &k, int slabs, int ty, bool with_pb = false)
{
    const int S = pl->S;
    DFJob f{};
    if (k.kind == 1) {
        // BRIEF pre-blur: G_s -> B_s, no DoG, no sub-sample
        const OctaveGeom &g = pl->vols[k.vol].oct[k.octave];
        f.src = (long long)level_off(g, lev_G(k.s));
        f.dst = (long long)level_off(g, lev_B(S, k.s));
        f.dog = -1;
        f.sub = -1;
        f.nx = g.nx;
        f.ny = g.ny;
        f.nz = g.nz;
        f.tiles_x = (g.nx + kBlurTX - 1) / kBlurTX;
        f.tiles_y = (g.ny + ty - 1) / ty;
        f.L = slab_planes(g.nz, slabs, pl->brief_rb);
        f.slabs = (g.nz + f.L - 1) / f.L;
        f.taps = pl->brief_tapset;
        f.pb = -1;
        return f;
    }
    const BlurLaunch &L = pl->blur[k.pass];
    const VolPlan &vp = pl->vols[L.vol];
    const OctaveGeom &g = vp.oct[L.octave];
    if (L.src_kind < 0) {
        f.src = (long long)vp.in_off;
        f.src_input = 1;
    } else {
        f.src = (long long)level_off(g, lev_G(L.src_idx));
    }
    f.dst = (long long)level_off(g, lev_G(L.dst_idx));
    f.dog = L.dog ? (long long)level_off(g, lev_D(S, L.dog_idx)) : -1;
    if (L.sub_octave >= 0) {
        const OctaveGeom &m = vp.oct[L.sub_octave];
        f.sub = (long long)level_off(m, lev_G(0));
        f.mx = m.nx;
        f.my = m.ny;
        f.mz = m.nz;
    } else {
        f.sub = -1;
    }
    f.nx = g.nx;
    f.ny = g.ny;
    f.nz = g.nz;
    f.tiles_x = (g.nx + kBlurTX - 1) / kBlurTX;
    f.tiles_y = (g.ny + ty - 1) / ty;
    f.L = slab_planes(g.nz, slabs, L.r);
    f.slabs = (g.nz + f.L - 1) / f.L;
    f.taps = L.tapset;
    if (with_pb) {
        // B_s of the source level G_s (s = src_idx)
        f.pb = (long long)level_off(g, lev_B(S, L.src_idx));
        f.pb_taps = pl->brief_tapset;
    } else {
        f.pb = -1;
    }
    return f;
}

// Tile height of a fused pass launched alone over one octave.
int solo_ty(const OctaveGeom &g) { return (long long)g.n >= kBlurTallVoxels ? kBlurTYTall : kBlurTYSmall; }

// Slabs per job for a fused launch over jobs with `tiles` (x, y) tiles in
// total: enough blocks to fill every resident slot of the device once (CUs x
// the fused pass's workgroups per CU at this radius, from its registers and
// LDS), no more.
int fused_slabs(const sift3d_plan *pl, long long tiles, int r, bool dog, bool pb, int ty)
{
    const int per_cu = std::max(1, fused_blocks_per_cu(r, dog, pb, ty));
    const long long slots = (long long)pl->ctx->n_cu * per_cu;
    return (int)std::max<long long>(1, (slots + tiles - 1) / tiles);
}

// List scheduler over all volumes: alternating xy and z launches, each
// holding every split task whose inputs are ready; fused passes are
// launches of their own. Fills the job tables (schedule entries first, then
// one single-job entry per task for sift3d_pyramid_pass).
void build_schedule(sift3d_plan *pl)
{
    const int S = pl->S;
    pl->tasks.clear();
    pl->sched.clear();
    pl->xyjobs.clear();
    pl->zjobs.clear();
    pl->fjobs.clear();
    pl->cjobs.clear();
    for (size_t b = 0; b < pl->blur.size(); ++b)
        pl->tasks.push_back(Task{0, (int)b, pl->blur[b].vol, pl->blur[b].octave, 0});
    if (pl->brief_rb >= 0)
        for (int v = 0; v < pl->n_vol; ++v)
            for (int o = 0; o < (int)pl->vols[v].oct.size(); ++o)
                for (int s = 1; s <= S; ++s) pl->tasks.push_back(Task{1, -1, v, o, s});
    const int nt = (int)pl->tasks.size();
    std::vector<char> xy_done(nt, 0), done(nt, 0);
    // task of the level pass writing G_level of (volume, octave), and of each
    // pre-blur task, in dense tables (linear in the number of tasks)
    const int nlev = S + 3;
    auto key = [&](int v, int o, int level) { return ((size_t)v * kMaxOctaves + o) * nlev + level; };
    std::vector<int> level_task((size_t)pl->n_vol * kMaxOctaves * nlev, -1);
    std::vector<int> preblur_task((size_t)pl->n_vol * kMaxOctaves * nlev, -1);
    for (int t = 0; t < nt; ++t) {
        const Task &k = pl->tasks[t];
        if (k.kind == 0) {
            const BlurLaunch &L = pl->blur[k.pass];
            level_task[key(L.vol, L.octave, L.dst_idx)] = t;
        } else {
            preblur_task[key(k.vol, k.octave, k.s)] = t;
        }
    }
    // the task whose completion makes task t ready (-1: ready from the start)
    std::vector<int> dep(nt, -1);
    for (int t = 0; t < nt; ++t) {
        const Task &k = pl->tasks[t];
        if (k.kind == 1) {
            dep[t] = level_task[key(k.vol, k.octave, k.s)];
            continue;
        }
        const BlurLaunch &L = pl->blur[k.pass];
        if (L.src_kind < 0) continue;
        if (L.src_idx == 0 && L.octave > 0)
            dep[t] = level_task[key(L.vol, L.octave - 1, S)];  // G_0 from the sub-sample
        else
            dep[t] = level_task[key(L.vol, L.octave, L.src_idx)];
    }
    auto ready = [&](int t) { return dep[t] < 0 || done[dep[t]]; };
    auto task_r = [&](int t) { return pl->tasks[t].kind == 0 ? pl->blur[pl->tasks[t].pass].r : pl->brief_rb; };
    auto task_dog = [&](int t) { return pl->tasks[t].kind == 0 && pl->blur[pl->tasks[t].pass].dog; };
    auto task_geom = [&](int t) -> const OctaveGeom & {
        const Task &k = pl->tasks[t];
        return pl->vols[k.vol].oct[k.kind == 0 ? pl->blur[k.pass].octave : k.octave];
    };
    // pre-blurs take their path by the same rule as the level passes
    const sift3d_params &pp = pl->ctx->p;
    auto path_of = [&](int t) {
        const Task &k = pl->tasks[t];
        if (k.kind == 0) return pl->blur[k.pass].path;
        return level_path(pp, (long long)task_geom(t).n, pl->brief_rb);
    };
    auto is_fused = [&](int t) { return path_of(t) == kPathFused; };
    auto is_split = [&](int t) { return path_of(t) == kPathSplit; };
    // A fused level pass G_{s+1} (s = 1..S) also writes B_s when the
    // pre-blur radius is kFusedPreR: that pre-blur task is then done by it.
    std::vector<char> with_pb(nt, 0);
    int absorbed = 0;
    if (pl->brief_rb == kFusedPreR)
        for (int t = 0; t < nt; ++t) {
            const Task &k = pl->tasks[t];
            if (k.kind != 0 || !is_fused(t)) continue;
            const BlurLaunch &L = pl->blur[k.pass];
            if (!L.dog || L.src_kind != 0 || L.src_idx < 1 || L.src_idx > S || L.r < kFusedPreR) continue;
            const int u = preblur_task[key(L.vol, L.octave, L.src_idx)];
            if (u >= 0 && !done[u]) {
                done[u] = 1;
                with_pb[t] = 1;
                ++absorbed;
            }
        }
    // one compact launch for all ready compact tasks (any radii)
    auto emit_compact = [&](const std::vector<int> &ts) {
        if (ts.empty()) return;
        Step st{3, ts, (int)pl->cjobs.size(), (int)ts.size(), 0, 0, false, 0};
        for (int t : ts) {
            DCJob c = compact_job(pl, pl->tasks[t]);
            c.block0 = st.n_blocks;
            st.n_blocks += c.tiles_x * c.tiles_y * c.tiles_z;
            st.max_r = std::max(st.max_r, c.r);
            pl->cjobs.push_back(c);
        }
        pl->sched.push_back(st);
    };
    auto emit = [&](int type, const std::vector<int> &ts) {
        if (ts.empty()) return;
        Step st{type, ts, 0, (int)ts.size(), 0, 0, false, 0};
        st.first = type == 1 ? (int)pl->xyjobs.size() : (int)pl->zjobs.size();
        int blocks = 0;
        for (int t : ts) {
            DXYJob xy;
            DZJob z;
            task_jobs(pl, pl->tasks[t], xy, z);
            const VolPlan &vp = pl->vols[pl->tasks[t].vol];
            const int o = pl->tasks[t].kind == 0 ? pl->blur[pl->tasks[t].pass].octave : pl->tasks[t].octave;
            st.max_r = std::max(st.max_r, xy.r);
            if (type == 1) {
                xy.block0 = blocks;
                blocks += xy_blocks(vp.oct[o]);
                pl->xyjobs.push_back(xy);
            } else {
                z.block0 = blocks;
                blocks += z_blocks(vp.oct[o]);
                pl->zjobs.push_back(z);
            }
        }
        st.n_blocks = blocks;
        pl->sched.push_back(st);
    };
    // one fused launch per (radius, DoG, pre-blur) group of ready fused tasks
    auto emit_fused = [&](const std::vector<int> &ts) {
        std::vector<int> left = ts;
        while (!left.empty()) {
            const int r0 = task_r(left[0]);
            const bool dog0 = task_dog(left[0]);
            const bool pb0 = with_pb[left[0]] != 0;
            std::vector<int> grp, rest;
            for (int t : left)
                (task_r(t) == r0 && task_dog(t) == dog0 && (with_pb[t] != 0) == pb0 ? grp : rest).push_back(t);
            long long voxels = 0;
            for (int t : grp) voxels += (long long)task_geom(t).n;
            // tile height and slabs: the default rule, or the tuned pair of this step
            const size_t si = pl->sched.size();
            const bool tuned = si < pl->fused_tune.size() && pl->fused_tune[si].first > 0;
            const int ty = tuned ? pl->fused_tune[si].first : (voxels >= kBlurTallVoxels ? kBlurTYTall : kBlurTYSmall);
            long long tiles = 0;
            for (int t : grp) {
                const OctaveGeom &g = task_geom(t);
                tiles += (long long)((g.nx + kBlurTX - 1) / kBlurTX) * ((g.ny + ty - 1) / ty);
            }
            const int slabs = tuned ? pl->fused_tune[si].second : fused_slabs(pl, tiles, r0, dog0, pb0, ty);
            Step st{0, grp, (int)pl->fjobs.size(), (int)grp.size(), 0, r0, dog0, ty, pb0};
            for (int t : grp) {
                DFJob f = fused_job(pl, pl->tasks[t], slabs, ty, pb0);
                f.block0 = st.n_blocks;
                st.n_blocks += f.tiles_x * f.tiles_y * f.slabs;
                pl->fjobs.push_back(f);
            }
            pl->sched.push_back(st);
            left.swap(rest);
        }
    };
    int remaining = nt - absorbed;
    while (remaining > 0) {
        bool progress = false;
        std::vector<int> fs;
        for (int t = 0; t < nt; ++t)
            if (!done[t] && is_fused(t) && ready(t)) fs.push_back(t);
        std::vector<int> cs;
        for (int t = 0; t < nt; ++t)
            if (!done[t] && path_of(t) == kPathCompact && ready(t)) cs.push_back(t);
        emit_fused(fs);
        emit_compact(cs);
        for (const std::vector<int> *v : {&fs, &cs})
            for (int t : *v) {
                done[t] = 1;
                --remaining;
                progress = true;
            }
        std::vector<int> xs;
        for (int t = 0; t < nt; ++t)
            if (!done[t] && !xy_done[t] && is_split(t) && ready(t)) xs.push_back(t);
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
    // single-job entries
    pl->solo_xy.assign(nt, -1);
    pl->solo_z.assign(nt, -1);
    pl->solo_f.assign(nt, -1);
    pl->solo_c.assign(nt, -1);
    for (int t = 0; t < nt; ++t) {
        if (pl->tasks[t].kind == 1 && !is_split(t)) continue;  // pre-blurs have no single-pass entry
        if (path_of(t) == kPathCompact) {
            DCJob c = compact_job(pl, pl->tasks[t]);
            c.block0 = 0;
            pl->solo_c[t] = (int)pl->cjobs.size();
            pl->cjobs.push_back(c);
            continue;
        }
        if (is_fused(t)) {
            const BlurLaunch &L = pl->blur[pl->tasks[t].pass];
            const OctaveGeom &g = pl->vols[L.vol].oct[L.octave];
            const int ty = solo_ty(g);
            const long long tiles = (long long)((g.nx + kBlurTX - 1) / kBlurTX) * ((g.ny + ty - 1) / ty);
            DFJob f = fused_job(pl, pl->tasks[t], fused_slabs(pl, tiles, L.r, L.dog, false, ty), ty);
            f.block0 = 0;
            pl->solo_f[t] = (int)pl->fjobs.size();
            pl->fjobs.push_back(f);
            continue;
        }
        DXYJob xy;
        DZJob z;
        task_jobs(pl, pl->tasks[t], xy, z);
        xy.block0 = z.block0 = 0;
        pl->solo_xy[t] = (int)pl->xyjobs.size();
        pl->xyjobs.push_back(xy);
        pl->solo_z[t] = (int)pl->zjobs.size();
        pl->zjobs.push_back(z);
    }
}

// Upload the plan's device tables (one allocation; a previous one is freed).
int upload_tables(sift3d_plan *pl)
{
    if (pl->d_tables != nullptr) {
        (void)hipFree(pl->d_tables);
        pl->d_tables = nullptr;
    }
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t b_units = al(pl->units.size() * sizeof(DUnit));
    const size_t b_vols = al(pl->dvols.size() * sizeof(DVol));
    const size_t b_xy = al(std::max<size_t>(1, pl->xyjobs.size()) * sizeof(DXYJob));
    const size_t b_z = al(std::max<size_t>(1, pl->zjobs.size()) * sizeof(DZJob));
    const size_t b_f = al(std::max<size_t>(1, pl->fjobs.size()) * sizeof(DFJob));
    const size_t b_c = al(std::max<size_t>(1, pl->cjobs.size()) * sizeof(DCJob));
    const size_t b_taps = al(pl->tapsets.size() * kMaxTaps * sizeof(float));
    const size_t total = b_units + b_vols + b_xy + b_z + b_f + b_c + b_taps;
    std::vector<char> host(total, 0);
    size_t off = 0;
    std::memcpy(host.data() + off, pl->units.data(), pl->units.size() * sizeof(DUnit));
    off += b_units;
    std::memcpy(host.data() + off, pl->dvols.data(), pl->dvols.size() * sizeof(DVol));
    off += b_vols;
    std::memcpy(host.data() + off, pl->xyjobs.data(), pl->xyjobs.size() * sizeof(DXYJob));
    off += b_xy;
    std::memcpy(host.data() + off, pl->zjobs.data(), pl->zjobs.size() * sizeof(DZJob));
    off += b_z;
    std::memcpy(host.data() + off, pl->fjobs.data(), pl->fjobs.size() * sizeof(DFJob));
    off += b_f;
    std::memcpy(host.data() + off, pl->cjobs.data(), pl->cjobs.size() * sizeof(DCJob));
    off += b_c;
    for (size_t i = 0; i < pl->tapsets.size(); ++i)
        std::memcpy(host.data() + off + i * kMaxTaps * sizeof(float), pl->tapsets[i].data(), kMaxTaps * sizeof(float));
    hipError_t e = hipMalloc(&pl->d_tables, total);
    if (e != hipSuccess) {
        pl->d_tables = nullptr;
        return hip_fail(e);
    }
    e = hipMemcpy(pl->d_tables, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e);
    char *d = static_cast<char *>(pl->d_tables);
    pl->d_units = reinterpret_cast<DUnit *>(d);
    pl->d_vols = reinterpret_cast<DVol *>(d + b_units);
    pl->d_xy = reinterpret_cast<DXYJob *>(d + b_units + b_vols);
    pl->d_z = reinterpret_cast<DZJob *>(d + b_units + b_vols + b_xy);
    pl->d_f = reinterpret_cast<DFJob *>(d + b_units + b_vols + b_xy + b_z);
    pl->d_c = reinterpret_cast<DCJob *>(d + b_units + b_vols + b_xy + b_z + b_f);
    pl->d_taps = reinterpret_cast<float *>(d + b_units + b_vols + b_xy + b_z + b_f + b_c);
    return SIFT3D_OK;
}

// Octave, level, detection and schedule geometry of a plan over n volumes.
int make_plan(sift3d_ctx *ctx, int n, const int *dims, int kp_capacity, sift3d_plan **out)
{
    if (out == nullptr) return SIFT3D_E_ARG;
    *out = nullptr;
    if (ctx == nullptr || dims == nullptr || n < 1 || n > kMaxVolumes || kp_capacity < 0) return SIFT3D_E_ARG;
    const sift3d_params &p = ctx->p;
    const int S = p.scales, nlev = levels_per_octave(S);
    sift3d_plan *pl = new (std::nothrow) sift3d_plan();
    if (pl == nullptr) return SIFT3D_E_ARG;
    pl->ctx = ctx;
    pl->n_vol = n;
    pl->cap = kp_capacity;
    pl->S = S;
    pl->d_tables = nullptr;
    size_t off = 0, in_off = 0;
    for (int v = 0; v < n; ++v) {
        const int nx = dims[3 * v], ny = dims[3 * v + 1], nz = dims[3 * v + 2];
        // a plane at most 1 GiB: the fused pass and detection address planes
        // with 32-bit byte offsets, and the fused pass discards stores at 2^31
        if (nx < 1 || ny < 1 || nz < 1 || (long long)nx * ny > (1LL << 28) ||
            (long long)nx * ny * nz > (1LL << 40)) {
            delete pl;
            return SIFT3D_E_ARG;
        }
        VolPlan vp;
        vp.nx = nx;
        vp.ny = ny;
        vp.nz = nz;
        vp.in_off = in_off;
        in_off += (size_t)nx * ny * nz;
        in_off = (in_off + 63) & ~(size_t)63;  // each volume 256-byte aligned in the packed input
        // octave geometry: halve (floor) while the smallest dim stays >= min_dim
        int cx = nx, cy = ny, cz = nz;
        while (std::min(cx, std::min(cy, cz)) >= p.min_dim) {
            if (p.n_octaves > 0 && (int)vp.oct.size() == p.n_octaves) break;
            if ((int)vp.oct.size() == kMaxOctaves) break;
            OctaveGeom g;
            g.nx = cx;
            g.ny = cy;
            g.nz = cz;
            g.n = (size_t)cx * cy * cz;
            g.level_bytes = align256(g.n * sizeof(float));
            g.base = off;
            off += g.level_bytes * nlev;
            vp.oct.push_back(g);
            cx /= 2;
            cy /= 2;
            cz /= 2;
        }
        if (vp.oct.empty()) {
            delete pl;
            return SIFT3D_E_TOO_SMALL;
        }
        pl->vols.push_back(vp);
    }
    pl->in_elems = in_off;

    // tap sets: 0 = base blur, i = increment of G_i, S+3 = BRIEF pre-blur
    pl->base_sigma = std::sqrt(p.sigma0 * p.sigma0 - p.sigma_in * p.sigma_in);
    for (int i = 1; i <= S + 2; ++i) {
        const double a = scale_sigma(p, i), b = scale_sigma(p, i - 1);
        pl->inc_sigma.push_back(std::sqrt(a * a - b * b));
    }
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

    // detection units and rows (each volume starts on a kRowBlock boundary)
    long long rows = 0;
    int tile_blocks = 0;
    for (int v = 0; v < n; ++v) {
        VolPlan &vp = pl->vols[v];
        rows = (rows + kRowBlock - 1) / kRowBlock * kRowBlock;
        vp.unit0 = (int)pl->units.size();
        pl->dvols.push_back(DVol{rows, vp.unit0, (int)vp.oct.size()});
        for (int o = 0; o < (int)vp.oct.size(); ++o) {
            const OctaveGeom &g = vp.oct[o];
            DUnit u{};
            u.g0 = (long long)g.base;
            u.b1 = (long long)level_off(g, pl->brief_rb >= 0 ? lev_B(S, 1) : lev_G(1));
            u.row_base = rows;
            u.rows = (long long)S * (g.nz - 2) * (g.ny - 2);
            u.lstride = (long long)(g.level_bytes / sizeof(float));
            u.nx = g.nx;
            u.ny = g.ny;
            u.nz = g.nz;
            u.octave = o;
            u.vol = v;
            u.words = (g.nx - 2 + kDTXOut - 1) / kDTXOut;   // interior x 1..nx-2, 62 per word
            u.tiles_x = u.words;
            u.tiles_y = (g.ny - 2 + kDTY - 1) / kDTY;  // interior rows 1..ny-2
            u.tiles_z = (g.nz - 2 + kDTZ - 1) / kDTZ;  // interior planes 1..nz-2
            u.tile_block0 = tile_blocks;
            tile_blocks += u.tiles_x * u.tiles_y * u.tiles_z;
            for (int s = 0; s <= S; ++s) u.sigma[s] = (float)(scale_sigma(p, s) * std::ldexp(1.0, o));
            rows += u.rows;
            pl->units.push_back(u);
        }
    }
    rows = (rows + kRowBlock - 1) / kRowBlock * kRowBlock;
    pl->total_rows = rows;
    pl->tile_blocks = tile_blocks;
    const long long nblk = (rows + kDetRowsPerBlock - 1) / kDetRowsPerBlock;
    pl->row_count_off = off;
    off += align256((size_t)rows * sizeof(int));
    pl->block_sum_off = off;
    off += align256((size_t)nblk * sizeof(int));
    pl->block_off_off = off;
    off += align256((size_t)nblk * sizeof(int));
    for (DUnit &u : pl->units) {
        u.masks = (long long)(off - pl->row_count_off);
        off += align256((size_t)u.rows * u.words * sizeof(unsigned long long));
    }
    pl->det_scratch_off = pl->row_count_off;
    pl->det_scratch_bytes = off - pl->row_count_off;
    pl->ws_bytes = off;

    // level passes
    for (int v = 0; v < n; ++v) {
        const VolPlan &vp = pl->vols[v];
        const int no = (int)vp.oct.size();
        for (int o = 0; o < no; ++o) {
            const OctaveGeom &g = vp.oct[o];
            for (int i = (o == 0 ? 0 : 1); i <= S + 2; ++i) {
                BlurLaunch L{};
                L.vol = v;
                L.tapset = i;
                L.r = pl->tapset_r[i];
                L.dog = i > 0;
                L.octave = o;
                L.src_kind = i == 0 ? -1 : 0;
                L.src_idx = i - 1;
                L.dst_idx = i;
                L.dog_idx = i - 1;
                L.sub_octave = (i == S && o + 1 < no) ? o + 1 : -1;
                L.path = level_path(p, (long long)g.n, L.r);
                pl->blur.push_back(L);
            }
        }
    }
    build_schedule(pl);
    const int rc = upload_tables(pl);
    if (rc != SIFT3D_OK) {
        if (pl->d_tables) (void)hipFree(pl->d_tables);
        delete pl;
        return rc;
    }
    *out = pl;
    return SIFT3D_OK;
}

float *ws_float(const void *ws, size_t off)
{
    return reinterpret_cast<float *>(const_cast<char *>(static_cast<const char *>(ws)) + off);
}

int check_ws(const sift3d_plan *plan, const void *ws, size_t bytes)
{
    if (plan == nullptr || ws == nullptr) return SIFT3D_E_ARG;
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return SIFT3D_E_ARG;
    if (bytes < plan->ws_bytes) return SIFT3D_E_WORKSPACE;
    return SIFT3D_OK;
}

int run_step(const sift3d_plan *plan, const Step &stp, const float *d_in, void *d_ws, hipStream_t st)
{
    hipError_t e = hipSuccess;
    char *ws = static_cast<char *>(d_ws);
    if (stp.type == 0) {
        FusedLaunch a{};
        a.jobs = plan->d_f + stp.first;
        a.n_jobs = stp.count;
        a.n_blocks = stp.n_blocks;
        a.ws = ws;
        a.in = d_in;
        a.taps = plan->d_taps;
        if (stp.count <= kInlineJobs)
            for (int j = 0; j < stp.count; ++j) a.inl[j] = plan->fjobs[stp.first + j];
        e = launch_blur(a, stp.max_r, stp.dog, stp.pb, stp.ty, st);
    } else if (stp.type == 3) {
        CompactLaunch a{};
        a.jobs = plan->d_c + stp.first;
        a.n_jobs = stp.count;
        a.n_blocks = stp.n_blocks;
        a.ws = ws;
        a.in = d_in;
        a.taps = plan->d_taps;
        if (stp.count <= kInlineJobs)
            for (int j = 0; j < stp.count; ++j) a.inl[j] = plan->cjobs[stp.first + j];
        e = launch_blur_compact(a, stp.max_r, st);
    } else if (stp.type == 1) {
        XYLaunch a{};
        a.jobs = plan->d_xy + stp.first;
        a.n_jobs = stp.count;
        a.n_blocks = stp.n_blocks;
        a.ws = ws;
        a.in = d_in;
        a.taps = plan->d_taps;
        if (stp.count <= kInlineJobs)
            for (int j = 0; j < stp.count; ++j) a.inl[j] = plan->xyjobs[stp.first + j];
        e = launch_blur_xy(a, stp.max_r, st);
    } else {
        ZLaunch a{};
        a.jobs = plan->d_z + stp.first;
        a.n_jobs = stp.count;
        a.n_blocks = stp.n_blocks;
        a.ws = ws;
        a.in = d_in;
        a.taps = plan->d_taps;
        if (stp.count <= kInlineJobs)
            for (int j = 0; j < stp.count; ++j) a.inl[j] = plan->zjobs[stp.first + j];
        e = launch_blur_z(a, stp.max_r, st);
    }
    return e == hipSuccess ? SIFT3D_OK : hip_fail(e);
}

}  // namespace

namespace {
int run_detect(const sift3d_plan *plan, char *ws, char *scr, sift3d_keypoint *d_kp, int kp_capacity, int *d_count,
               hipStream_t stream);
}  // namespace

namespace s3d {
// Nearest-neighbour matching launcher (match.hip).
hipError_t launch_match(int kind, const void *a, int n_a, const void *b, int n_b, int row_elems, int32_t *idx,
                        int32_t *d1, int32_t *d2, hipStream_t st);
// Uniform-filter blur launcher (box.hip).
hipError_t launch_box(const float *in, float *out, float *tmp, int nx, int ny, int nz, int h, int passes,
                      hipStream_t st);
}  // namespace s3d

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
    p->brief_method = 3;
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
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device);
    void *scr = nullptr;
    if (e == hipSuccess) e = static_scratch(c->device, &scr);   // once per device: the static detection scratch
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

int sift3d_ctx_params(const sift3d_ctx *ctx, sift3d_params *out)
{
    if (ctx == nullptr || out == nullptr) return SIFT3D_E_ARG;
    *out = ctx->p;
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
    const int dims[3] = {nx, ny, nz};
    return make_plan(ctx, 1, dims, kp_capacity, out);
}

int sift3d_plan_create_batch(sift3d_ctx *ctx, int n_volumes, const int *dims, int kp_capacity, sift3d_plan **out)
{
    return make_plan(ctx, n_volumes, dims, kp_capacity, out);
}

int sift3d_plan_destroy(sift3d_plan *plan)
{
    if (plan == nullptr) return SIFT3D_E_ARG;
    if (plan->d_tables != nullptr) (void)hipFree(plan->d_tables);
    delete plan;
    return SIFT3D_OK;
}

int sift3d_plan_info(const sift3d_plan *plan, size_t *workspace_bytes, int *n_volumes, size_t *input_elems)
{
    if (plan == nullptr) return SIFT3D_E_ARG;
    if (workspace_bytes) *workspace_bytes = plan->ws_bytes;
    if (n_volumes) *n_volumes = plan->n_vol;
    if (input_elems) *input_elems = plan->in_elems;
    return SIFT3D_OK;
}

int sift3d_plan_volume(const sift3d_plan *plan, int volume, int dims[3], size_t *input_offset, int *n_octaves)
{
    if (plan == nullptr || volume < 0 || volume >= plan->n_vol) return SIFT3D_E_ARG;
    const VolPlan &vp = plan->vols[volume];
    if (dims) {
        dims[0] = vp.nx;
        dims[1] = vp.ny;
        dims[2] = vp.nz;
    }
    if (input_offset) *input_offset = vp.in_off;
    if (n_octaves) *n_octaves = (int)vp.oct.size();
    return SIFT3D_OK;
}

int sift3d_plan_octave_dims(const sift3d_plan *plan, int volume, int octave, int dims[3])
{
    if (plan == nullptr || dims == nullptr || volume < 0 || volume >= plan->n_vol) return SIFT3D_E_ARG;
    const VolPlan &vp = plan->vols[volume];
    if (octave < 0 || octave >= (int)vp.oct.size()) return SIFT3D_E_ARG;
    dims[0] = vp.oct[octave].nx;
    dims[1] = vp.oct[octave].ny;
    dims[2] = vp.oct[octave].nz;
    return SIFT3D_OK;
}

int sift3d_level(const sift3d_plan *plan, void *d_ws, int volume, int octave, int kind, int idx, float **d_ptr)
{
    if (plan == nullptr || d_ws == nullptr || d_ptr == nullptr || volume < 0 || volume >= plan->n_vol)
        return SIFT3D_E_ARG;
    const VolPlan &vp = plan->vols[volume];
    if (octave < 0 || octave >= (int)vp.oct.size() || kind < 0 || kind > 2) return SIFT3D_E_ARG;
    if (kind == 2) {
        if (plan->brief_rb < 0 || idx < 1 || idx > plan->S) return SIFT3D_E_ARG;
        *d_ptr = ws_float(d_ws, level_off(vp.oct[octave], lev_B(plan->S, idx)));
        return SIFT3D_OK;
    }
    if (idx < 0 || idx >= (kind == 0 ? plan->S + 3 : plan->S + 2)) return SIFT3D_E_ARG;
    *d_ptr = ws_float(d_ws, level_off(vp.oct[octave], kind == 0 ? lev_G(idx) : lev_D(plan->S, idx)));
    return SIFT3D_OK;
}

int sift3d_build_pyramid(const sift3d_plan *plan, const float *d_vol, void *d_ws, size_t ws_bytes, void *stream)
{
    int rc = check_ws(plan, d_ws, ws_bytes);
    if (rc != SIFT3D_OK) return rc;
    if (d_vol == nullptr) return SIFT3D_E_ARG;
    for (const Step &stp : plan->sched) {
        rc = run_step(plan, stp, d_vol, d_ws, static_cast<hipStream_t>(stream));
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

int sift3d_pyramid_pass_info(const sift3d_plan *plan, int pass, int info[6], size_t *bytes)
{
    if (plan == nullptr || pass < 0 || pass >= (int)plan->blur.size()) return SIFT3D_E_ARG;
    const BlurLaunch &L = plan->blur[pass];
    const VolPlan &vp = plan->vols[L.vol];
    if (info != nullptr) {
        info[0] = L.octave;
        info[1] = L.dst_idx;
        info[2] = L.r;
        info[3] = L.sub_octave >= 0 ? 1 : 0;
        info[4] = L.path;
        info[5] = L.vol;
    }
    if (bytes != nullptr) {
        const size_t n = vp.oct[L.octave].n;
        size_t b = 8 * n + (L.dog ? 4 * n : 0);
        if (L.sub_octave >= 0) b += 4 * vp.oct[L.sub_octave].n;
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
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (L.path == kPathCompact) {
        const DCJob &c = plan->cjobs[plan->solo_c[t]];
        return run_step(plan, Step{3, {t}, plan->solo_c[t], 1, c.tiles_x * c.tiles_y * c.tiles_z, L.r, false, 0},
                        d_vol, d_ws, st);
    }
    if (L.path == kPathFused) {
        const DFJob &f = plan->fjobs[plan->solo_f[t]];
        const int ty = solo_ty(plan->vols[L.vol].oct[L.octave]);
        return run_step(plan, Step{0, {t}, plan->solo_f[t], 1, f.tiles_x * f.tiles_y * f.slabs, L.r, L.dog, ty},
                        d_vol, d_ws, st);
    }
    const VolPlan &vp = plan->vols[L.vol];
    const OctaveGeom &g = vp.oct[L.octave];
    rc = run_step(plan, Step{1, {t}, plan->solo_xy[t], 1, xy_blocks(g), L.r, false, 0}, d_vol, d_ws, st);
    if (rc != SIFT3D_OK) return rc;
    return run_step(plan, Step{2, {t}, plan->solo_z[t], 1, z_blocks(g), L.r, false, 0}, d_vol, d_ws, st);
}

int sift3d_pyramid_step_count(const sift3d_plan *plan, int *n_steps)
{
    if (plan == nullptr || n_steps == nullptr) return SIFT3D_E_ARG;
    *n_steps = (int)plan->sched.size();
    return SIFT3D_OK;
}

int sift3d_pyramid_step_info(const sift3d_plan *plan, int step, int info[9], size_t *bytes)
{
    if (plan == nullptr || step < 0 || step >= (int)plan->sched.size()) return SIFT3D_E_ARG;
    const Step &stp = plan->sched[step];
    int n_level = 0, n_pre = 0, omin = 1 << 30, omax = -1, lmin = 1 << 30, lmax = -1, rmax = 0;
    size_t b = 0;
    for (int t : stp.tasks) {
        const Task &k = plan->tasks[t];
        const bool completes = stp.type != 1;   // an xy launch completes no level
        if (k.kind == 0) {
            const BlurLaunch &L = plan->blur[k.pass];
            const VolPlan &vp = plan->vols[L.vol];
            const size_t n = vp.oct[L.octave].n;
            ++n_level;
            omin = std::min(omin, L.octave);
            omax = std::max(omax, L.octave);
            lmin = std::min(lmin, L.dst_idx);
            lmax = std::max(lmax, L.dst_idx);
            rmax = std::max(rmax, L.r);
            if (completes) {
                b += 8 * n + (L.dog ? 4 * n : 0);
                if (L.sub_octave >= 0) b += 4 * vp.oct[L.sub_octave].n;
                if (stp.type == 0 && stp.pb) b += 4 * n;   // the BRIEF pre-blurred level written alongside
            }
        } else {
            ++n_pre;
            omin = std::min(omin, k.octave);
            omax = std::max(omax, k.octave);
            rmax = std::max(rmax, plan->brief_rb);
            if (completes) b += 8 * plan->vols[k.vol].oct[k.octave].n;
        }
    }
    if (info != nullptr) {
        info[0] = stp.type;
        info[1] = n_level;
        info[2] = n_pre;
        info[3] = rmax;
        info[4] = omax >= 0 ? omin : -1;
        info[5] = omax;
        info[6] = lmax >= 0 ? lmin : -1;
        info[7] = lmax;
        info[8] = stp.type == 0 && stp.pb ? 1 : 0;
    }
    if (bytes != nullptr) *bytes = b;
    return SIFT3D_OK;
}

int sift3d_pyramid_step(const sift3d_plan *plan, int step, const float *d_vol, void *d_ws, size_t ws_bytes,
                        void *stream)
{
    int rc = check_ws(plan, d_ws, ws_bytes);
    if (rc != SIFT3D_OK) return rc;
    if (d_vol == nullptr || step < 0 || step >= (int)plan->sched.size()) return SIFT3D_E_ARG;
    return run_step(plan, plan->sched[step], d_vol, d_ws, static_cast<hipStream_t>(stream));
}

int sift3d_detect(const sift3d_plan *plan, void *d_ws, size_t ws_bytes, sift3d_keypoint *d_kp, int kp_capacity,
                  int *d_count, void *stream)
{
    int rc = check_ws(plan, d_ws, ws_bytes);
    if (rc != SIFT3D_OK) return rc;
    if (d_count == nullptr || kp_capacity < 0 || (kp_capacity > 0 && d_kp == nullptr)) return SIFT3D_E_ARG;
    char *ws = static_cast<char *>(d_ws);
    return run_detect(plan, ws, ws + plan->det_scratch_off, d_kp, kp_capacity, d_count, static_cast<hipStream_t>(stream));
}

int sift3d_plan_tune(sift3d_plan *plan, const float *d_vol, void *d_ws, size_t ws_bytes, int reps, void *stream)
{
    int rc = check_ws(plan, d_ws, ws_bytes);
    if (rc != SIFT3D_OK) return rc;
    if (d_vol == nullptr || reps < 1 || reps > 1000) return SIFT3D_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // start from the default rule
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e);
    plan->tuning.clear();
    plan->fused_tune.clear();
    build_schedule(plan);
    if ((rc = upload_tables(plan)) != SIFT3D_OK) return rc;
    // every level the launches read
    for (const Step &stp : plan->sched)
        if ((rc = run_step(plan, stp, d_vol, d_ws, st)) != SIFT3D_OK) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(e);
    }
    // average ms of `reps` launches of step i, after one untimed launch
    auto time_step = [&](int i, float &ms) -> int {
        int r = run_step(plan, plan->sched[i], d_vol, d_ws, st);
        hipError_t ee = hipEventRecord(e0, st);
        for (int k = 0; r == SIFT3D_OK && ee == hipSuccess && k < reps; ++k) r = run_step(plan, plan->sched[i], d_vol, d_ws, st);
        if (ee == hipSuccess) ee = hipEventRecord(e1, st);
        if (ee == hipSuccess) ee = hipEventSynchronize(e1);
        if (ee == hipSuccess) ee = hipEventElapsedTime(&ms, e0, e1);
        if (r != SIFT3D_OK) return r;
        if (ee != hipSuccess) return hip_fail(ee);
        ms /= (float)reps;
        return SIFT3D_OK;
    };
    // re-plan with the current overrides (the stream is idle: every timing synchronised)
    auto replan = [&]() -> int {
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e);
        build_schedule(plan);
        return upload_tables(plan);
    };
    plan->fused_tune.assign(plan->sched.size(), {0, 0});
    const size_t n = plan->sched.size();
    for (size_t i = 0; i < n && rc == SIFT3D_OK; ++i) {
        const Step def = plan->sched[i];
        if (def.type != 0) continue;
        const int def_slabs = plan->fjobs[def.first].slabs;
        sift3d_plan::TuneRecord tr{(int)i, def.ty, def_slabs, def.ty, def_slabs, 0, 0.f, 0.f};
        if ((rc = time_step((int)i, tr.def_ms)) != SIFT3D_OK) break;
        tr.ms = tr.def_ms;
        int best_req = 0;                       // requested slabs of the best candidate (0: default rule)
        std::vector<std::pair<int, int>> tried{{def.ty, def_slabs}};
        // candidates: both tile heights, slabs around the default fill rule
        // (tile heights and slab splits change no result: every voxel's
        // stencils run in the same order)
        for (int ty : {kBlurTYSmall, kBlurTYTall}) {
            long long tiles = 0;
            for (int t : def.tasks) {
                const Task &k = plan->tasks[t];
                const OctaveGeom &g = plan->vols[k.vol].oct[k.kind == 0 ? plan->blur[k.pass].octave : k.octave];
                tiles += (long long)((g.nx + kBlurTX - 1) / kBlurTX) * ((g.ny + ty - 1) / ty);
            }
            const int s0 = fused_slabs(plan, tiles, def.max_r, def.dog, def.pb, ty);
            std::vector<int> cands;
            for (int sl : {1, (s0 + 1) / 2, s0, (3 * s0 + 1) / 2, 2 * s0, 3 * s0, 4 * s0})
                if (sl >= 1 && std::find(cands.begin(), cands.end(), sl) == cands.end()) cands.push_back(sl);
            for (int sl : cands) {
                plan->fused_tune[i] = {ty, sl};
                if ((rc = replan()) != SIFT3D_OK) break;
                // the slab length rules can merge requests: time each layout once
                const std::pair<int, int> got{ty, plan->fjobs[plan->sched[i].first].slabs};
                if (std::find(tried.begin(), tried.end(), got) != tried.end()) continue;
                tried.push_back(got);
                float ms = 0.f;
                if ((rc = time_step((int)i, ms)) != SIFT3D_OK) break;
                ++tr.candidates;
                if (ms < tr.ms) {
                    tr.ms = ms;
                    tr.ty = got.first;
                    tr.slabs = got.second;
                    best_req = sl;
                }
            }
            if (rc != SIFT3D_OK) break;
        }
        plan->fused_tune[i] = best_req > 0 ? std::make_pair(tr.ty, best_req) : std::make_pair(0, 0);
        plan->tuning.push_back(tr);
    }
    if (rc == SIFT3D_OK) rc = replan();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SIFT3D_OK) {
        // back to the default rule
        plan->fused_tune.clear();
        plan->tuning.clear();
        (void)hipStreamSynchronize(st);
        build_schedule(plan);
        (void)upload_tables(plan);
    }
    return rc;
}

int sift3d_plan_tuning_count(const sift3d_plan *plan, int *n)
{
    if (plan == nullptr || n == nullptr) return SIFT3D_E_ARG;
    *n = (int)plan->tuning.size();
    return SIFT3D_OK;
}

int sift3d_plan_tuning(const sift3d_plan *plan, int idx, int info[6], float ms[2])
{
    if (plan == nullptr || idx < 0 || idx >= (int)plan->tuning.size() || info == nullptr || ms == nullptr)
        return SIFT3D_E_ARG;
    const auto &t = plan->tuning[idx];
    info[0] = t.step;
    info[1] = t.def_ty;
    info[2] = t.def_slabs;
    info[3] = t.ty;
    info[4] = t.slabs;
    info[5] = t.candidates;
    ms[0] = t.def_ms;
    ms[1] = t.ms;
    return SIFT3D_OK;
}

int sift3d_plan_detect_scratch(const sift3d_plan *plan, size_t *bytes)
{
    if (plan == nullptr || bytes == nullptr) return SIFT3D_E_ARG;
    *bytes = plan->det_scratch_bytes;
    return SIFT3D_OK;
}

int sift3d_detect_static(const sift3d_plan *plan, void *d_ws, size_t ws_bytes, sift3d_keypoint *d_kp,
                         int kp_capacity, int *d_count, void *stream)
{
    if (plan == nullptr || d_ws == nullptr || reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) return SIFT3D_E_ARG;
    if (d_count == nullptr || kp_capacity < 0 || (kp_capacity > 0 && d_kp == nullptr)) return SIFT3D_E_ARG;
    if (plan->det_scratch_bytes > SIFT3D_DETECT_STATIC_SCRATCH) return SIFT3D_E_SCRATCH;
    if (ws_bytes < plan->det_scratch_off) return SIFT3D_E_WORKSPACE;     // the pyramid part only
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    void *scr = nullptr;
    if (e == hipSuccess) e = static_scratch(dev, &scr);
    if (e != hipSuccess) return hip_fail(e);
    return run_detect(plan, static_cast<char *>(d_ws), static_cast<char *>(scr), d_kp, kp_capacity, d_count,
                      static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace {

int run_detect(const sift3d_plan *plan, char *ws, char *scr, sift3d_keypoint *d_kp, int kp_capacity, int *d_count,
               hipStream_t stream)
{
    const sift3d_params &p = plan->ctx->p;
    DetLaunch a{};
    a.units = plan->d_units;
    a.vols = plan->d_vols;
    a.n_units = (int)plan->units.size();
    a.n_vol = plan->n_vol;
    a.S = plan->S;
    a.total_rows = plan->total_rows;
    a.tile_blocks = plan->tile_blocks;
    a.thr = p.dog_threshold;
    a.votes = p.votes;
    a.ws = ws;
    a.scr = scr;
    a.row_count = reinterpret_cast<int *>(scr + (plan->row_count_off - plan->det_scratch_off));
    a.block_sum = reinterpret_cast<int *>(scr + (plan->block_sum_off - plan->det_scratch_off));
    a.block_off = reinterpret_cast<int *>(scr + (plan->block_off_off - plan->det_scratch_off));
    a.counts = d_count;
    a.kp = d_kp;
    a.cap = kp_capacity;
    if (a.n_units <= kInlineUnits)
        for (int u = 0; u < a.n_units; ++u) a.inl[u] = plan->units[u];
    const hipError_t e = launch_detect(a, stream);
    return e == hipSuccess ? SIFT3D_OK : hip_fail(e);
}

}  // namespace

extern "C" {

int sift3d_describe(const sift3d_plan *plan, const void *d_ws, size_t ws_bytes, const sift3d_keypoint *d_kp,
                    const int *d_count, int kp_capacity, uint8_t *d_siftrank, uint64_t *d_brief, uint8_t *d_rrief,
                    void *stream)
{
    int rc = check_ws(plan, d_ws, ws_bytes);
    if (rc != SIFT3D_OK) return rc;
    if (d_count == nullptr || kp_capacity < 0 || (kp_capacity > 0 && d_kp == nullptr)) return SIFT3D_E_ARG;
    const sift3d_params &p = plan->ctx->p;
    if (p.brief_n == 0) d_brief = nullptr, d_rrief = nullptr;
    DescLaunch a{};
    a.units = plan->d_units;
    a.vols = plan->d_vols;
    a.n_vol = plan->n_vol;
    a.S = plan->S;
    for (int s = 0; s <= plan->S; ++s) a.sift_R[s] = (int)std::ceil(p.siftrank_factor * scale_sigma(p, s));
    a.ws = const_cast<char *>(static_cast<const char *>(d_ws));
    a.kp = d_kp;
    a.counts = d_count;
    a.cap = kp_capacity;
    a.siftrank = d_siftrank;
    a.brief = d_brief;
    a.rrief = d_rrief;
    a.brief_n = p.brief_n;
    a.pairs = plan->ctx->d_offsets;
    a.n_units = (int)plan->units.size();
    if (a.n_units <= kInlineUnits)
        for (int u = 0; u < a.n_units; ++u) a.inl[u] = plan->units[u];
    const hipError_t e = launch_describe(a, (long long)kp_capacity * plan->n_vol, plan->ctx->n_cu,
                                         static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SIFT3D_OK : hip_fail(e);
}

int sift3d_orient(const sift3d_plan *plan, const void *d_ws, size_t ws_bytes, const sift3d_keypoint *d_kp,
                  const int *d_count, int kp_capacity, double peak_ratio, int *d_nframes, float *d_frames,
                  uint8_t *d_siftrank, void *stream)
{
    int rc = check_ws(plan, d_ws, ws_bytes);
    if (rc != SIFT3D_OK) return rc;
    if (d_count == nullptr || kp_capacity < 0 || (kp_capacity > 0 && d_kp == nullptr)) return SIFT3D_E_ARG;
    if (!(peak_ratio > 0.0 && peak_ratio <= 1.0)) return SIFT3D_E_ARG;
    if (kp_capacity > 0 && (d_nframes == nullptr || d_frames == nullptr || d_siftrank == nullptr)) return SIFT3D_E_ARG;
    const sift3d_params &p = plan->ctx->p;
    OrientLaunch a{};
    a.units = plan->d_units;
    a.vols = plan->d_vols;
    a.n_vol = plan->n_vol;
    a.S = plan->S;
    for (int s = 0; s <= plan->S; ++s) a.sift_R[s] = (int)std::ceil(p.siftrank_factor * scale_sigma(p, s));
    a.ws = const_cast<char *>(static_cast<const char *>(d_ws));
    a.kp = d_kp;
    a.counts = d_count;
    a.cap = kp_capacity;
    a.tau = peak_ratio;
    a.nframes = d_nframes;
    a.frames = d_frames;
    a.siftrank = d_siftrank;
    a.n_units = (int)plan->units.size();
    if (a.n_units <= kInlineUnits)
        for (int u = 0; u < a.n_units; ++u) a.inl[u] = plan->units[u];
    const hipError_t e = launch_orient(a, (long long)kp_capacity * plan->n_vol, plan->ctx->n_cu,
                                       static_cast<hipStream_t>(stream));
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

int sift3d_match(int kind, const void *d_a, int n_a, const void *d_b, int n_b, int row_elems, int32_t *d_idx,
                 int32_t *d_d1, int32_t *d_d2, void *stream)
{
    if (n_a < 0 || n_b < 0) return SIFT3D_E_ARG;
    if (kind == SIFT3D_MATCH_BRIEF) {
        if (row_elems < 1 || row_elems > kMaxPairs / 64) return SIFT3D_E_ARG;
    } else if (kind == SIFT3D_MATCH_RANKS) {
        if (row_elems < 64 || row_elems > kMaxPairs || row_elems % 64 != 0) return SIFT3D_E_ARG;
    } else {
        return SIFT3D_E_ARG;
    }
    if (n_a == 0) return SIFT3D_OK;
    if (d_a == nullptr || d_idx == nullptr || d_d1 == nullptr || d_d2 == nullptr || (n_b > 0 && d_b == nullptr))
        return SIFT3D_E_ARG;
    if (reinterpret_cast<uintptr_t>(d_a) % 4 != 0 || reinterpret_cast<uintptr_t>(d_b) % 4 != 0) return SIFT3D_E_ARG;
    const hipError_t e = launch_match(kind, d_a, n_a, d_b, n_b, row_elems, d_idx, d_d1, d_d2,
                                      static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SIFT3D_OK : hip_fail(e);
}

int sift3d_normalize(int kind, const void *d_in, int n, int row_elems, float *d_out, void *stream)
{
    if (n < 0) return SIFT3D_E_ARG;
    size_t align;
    if (kind == SIFT3D_MATCH_BRIEF) {
        if (row_elems < 1 || row_elems > kMaxPairs / 64) return SIFT3D_E_ARG;
        align = 8;
    } else if (kind == SIFT3D_MATCH_RANKS) {
        if (row_elems < 64 || row_elems > kMaxPairs || row_elems % 64 != 0) return SIFT3D_E_ARG;
        align = 4;
    } else {
        return SIFT3D_E_ARG;
    }
    if (n == 0) return SIFT3D_OK;
    if (d_in == nullptr || d_out == nullptr) return SIFT3D_E_ARG;
    if (reinterpret_cast<uintptr_t>(d_in) % align != 0 || reinterpret_cast<uintptr_t>(d_out) % 4 != 0)
        return SIFT3D_E_ARG;
    const hipError_t e = launch_normalize(kind, d_in, n, row_elems, d_out, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SIFT3D_OK : hip_fail(e);
}

int sift3d_units(const sift3d_keypoint *d_kp, const int *d_count, int kp_capacity, const int *d_nframes,
                 const float *d_frames, const void *d_desc, int desc_row_bytes, int32_t *d_unit, float *d_geo,
                 void *d_desc_out, int *d_n_units, void *stream)
{
    if (d_kp == nullptr || d_count == nullptr || d_unit == nullptr || d_geo == nullptr || d_n_units == nullptr)
        return SIFT3D_E_ARG;
    if (kp_capacity < 0 || kp_capacity > (1 << 26)) return SIFT3D_E_ARG;
    if (d_nframes != nullptr && d_frames == nullptr) return SIFT3D_E_ARG;
    if ((d_desc == nullptr) != (d_desc_out == nullptr)) return SIFT3D_E_ARG;
    if (d_desc != nullptr) {
        if (desc_row_bytes < 4 || desc_row_bytes > 1024 || desc_row_bytes % 4 != 0) return SIFT3D_E_ARG;
        if (reinterpret_cast<uintptr_t>(d_desc) % 4 != 0 || reinterpret_cast<uintptr_t>(d_desc_out) % 4 != 0)
            return SIFT3D_E_ARG;
    }
    UnitsArgs a{};
    a.kp = d_kp;
    a.count = d_count;
    a.cap = kp_capacity;
    a.nframes = d_nframes;
    a.frames = d_frames;
    a.desc = static_cast<const uint8_t *>(d_desc);
    a.row_bytes = desc_row_bytes;
    a.unit = d_unit;
    a.geo = d_geo;
    a.desc_out = static_cast<uint8_t *>(d_desc_out);
    a.n_units = d_n_units;
    const hipError_t e = launch_units(a, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SIFT3D_OK : hip_fail(e);
}

int sift3d_hough_default_params(int nx, int ny, int nz, sift3d_hough_params *hp)
{
    if (hp == nullptr || nx < 1 || ny < 1 || nz < 1) return SIFT3D_E_ARG;
    hp->scale_bin = 1.0;
    hp->angle_bin = M_PI / 6.0;
    hp->trans_bin = 0.25 * std::max(nx, std::max(ny, nz));
    hp->centre[0] = (nx - 1) / 2.0;
    hp->centre[1] = (ny - 1) / 2.0;
    hp->centre[2] = (nz - 1) / 2.0;
    hp->inlier_sigmas = 2.0;
    hp->inlier_log2s = 0.5;
    hp->iterations = 2;
    return SIFT3D_OK;
}

namespace {
constexpr int kHoughMaxMatches = 1 << 21;

// Workspace of the Hough vote: table keys, table counts, per-match low
// corners, the two winner scalars; each part 256-byte aligned.
struct HoughLayout {
    size_t keys, counts, lo, best, total;
    int log2_slots;
};

HoughLayout hough_layout(int n_a)
{
    HoughLayout L{};
    L.log2_slots = hough_log2_slots(n_a);
    const size_t slots = (size_t)1 << L.log2_slots;
    L.keys = 0;
    L.counts = align256(L.keys + slots * sizeof(unsigned long long));
    L.lo = align256(L.counts + slots * sizeof(unsigned));
    L.best = align256(L.lo + (size_t)std::max(n_a, 1) * sizeof(unsigned long long));
    L.total = align256(L.best + 16);
    return L;
}

bool finite_positive(double v) { return std::isfinite(v) && v > 0.0; }
}  // namespace

int sift3d_hough_workspace(int n_a, size_t *bytes)
{
    if (bytes == nullptr || n_a < 0 || n_a > kHoughMaxMatches) return SIFT3D_E_ARG;
    *bytes = hough_layout(n_a).total;
    return SIFT3D_OK;
}

int sift3d_hough(const float *d_geo_a, int n_a, const float *d_geo_b, int n_b, const int32_t *d_match,
                 const sift3d_hough_params *hp, void *d_ws, size_t ws_bytes, sift3d_similarity *d_out,
                 uint8_t *d_inlier, void *stream)
{
    if (hp == nullptr || d_out == nullptr || d_ws == nullptr) return SIFT3D_E_ARG;
    if (n_a < 0 || n_a > kHoughMaxMatches || n_b < 0) return SIFT3D_E_ARG;
    if (n_a > 0 && (d_geo_a == nullptr || d_match == nullptr || d_inlier == nullptr)) return SIFT3D_E_ARG;
    if (n_b > 0 && d_geo_b == nullptr) return SIFT3D_E_ARG;
    if (!finite_positive(hp->scale_bin) || !finite_positive(hp->angle_bin) || !finite_positive(hp->trans_bin))
        return SIFT3D_E_ARG;
    if (!(hp->inlier_sigmas >= 0.0) || !(hp->inlier_log2s >= 0.0) || !std::isfinite(hp->inlier_sigmas) ||
        !std::isfinite(hp->inlier_log2s))
        return SIFT3D_E_ARG;
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(hp->centre[k])) return SIFT3D_E_ARG;
    if (hp->iterations < 1 || hp->iterations > 16) return SIFT3D_E_ARG;
    if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0 || reinterpret_cast<uintptr_t>(d_out) % 8 != 0)
        return SIFT3D_E_ARG;
    const HoughLayout L = hough_layout(n_a);
    if (ws_bytes < L.total) return SIFT3D_E_WORKSPACE;
    char *ws = static_cast<char *>(d_ws);
    HoughArgs a{};
    a.geo_a = d_geo_a;
    a.geo_b = d_geo_b;
    a.match = d_match;
    a.n_a = n_a;
    a.n_b = n_b;
    a.width[0] = hp->scale_bin;
    for (int k = 1; k < 4; ++k) a.width[k] = hp->angle_bin;
    for (int k = 4; k < 7; ++k) a.width[k] = hp->trans_bin;
    for (int k = 0; k < 3; ++k) a.centre[k] = hp->centre[k];
    a.inl_sig = hp->inlier_sigmas;
    a.inl_log2s = hp->inlier_log2s;
    a.iterations = hp->iterations;
    a.keys = reinterpret_cast<unsigned long long *>(ws + L.keys);
    a.counts = reinterpret_cast<unsigned *>(ws + L.counts);
    a.log2_slots = L.log2_slots;
    a.lo = reinterpret_cast<unsigned long long *>(ws + L.lo);
    a.best_count = reinterpret_cast<unsigned *>(ws + L.best);
    a.best_key = reinterpret_cast<unsigned long long *>(ws + L.best + 8);
    a.out = d_out;
    a.inlier = d_inlier;
    const hipError_t e = launch_hough(a, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SIFT3D_OK : hip_fail(e);
}

int sift3d_box_blur(const float *d_in, float *d_out, float *d_tmp, int nx, int ny, int nz, int half_width,
                    int passes, void *stream)
{
    if (d_in == nullptr || d_out == nullptr || d_tmp == nullptr) return SIFT3D_E_ARG;
    if (d_in == d_out || d_in == d_tmp || d_out == d_tmp) return SIFT3D_E_ARG;
    // positions along an axis stay far from int overflow (tile start + 120)
    if (nx < 1 || ny < 1 || nz < 1 || nz > (1 << 30) || (long long)nx * ny > (1LL << 30)) return SIFT3D_E_ARG;
    if (passes < 1 || passes > 4 || half_width < 0 || half_width > 8 || passes * half_width > 28) return SIFT3D_E_ARG;
    const hipError_t e = launch_box(d_in, d_out, d_tmp, nx, ny, nz, half_width, passes,
                                    static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SIFT3D_OK : hip_fail(e);
}

int sift3d_box_half_width(double sigma, int passes, int *half_width)
{
    if (half_width == nullptr || !(sigma >= 0.0) || passes < 1) return SIFT3D_E_ARG;
    const double w = std::sqrt(12.0 * sigma * sigma / passes + 1.0);
    const double h = std::floor((w - 1.0) / 2.0 + 0.5);
    if (h > 1e9) return SIFT3D_E_ARG;
    *half_width = (int)h;
    return SIFT3D_OK;
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
    case SIFT3D_E_SCRATCH: return "detection scratch larger than the static maximum";
    case SIFT3D_E_TIMEOUT: return "request not admitted within the server's admission timeout";
    case SIFT3D_PENDING: return "request not finished";
    default: return "unknown error";
    }
}

int sift3d_last_hip_error(void) { return g_last_hip; }

}  // extern "C"
