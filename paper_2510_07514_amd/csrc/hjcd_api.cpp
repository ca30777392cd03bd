// Host side of libhjcd: argument checks, robot / scene tables, the
// per-call plan (robot-grouped seed layout) and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hjcd.h"
#include "hjcd_internal.hpp"
#include "hjcd_launch.hpp"
#include "hjcd_tables.hpp"

using namespace hjcd;

namespace hjcd {

namespace {
thread_local std::string g_err;
}  // namespace

hjcd_status fail(hjcd_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

}  // namespace hjcd

namespace {

hjcd_status ensure(hjcd_ctx c, DevBuf& b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (b.cap >= bytes) return HJCD_OK;
    if (b.p) {
        // scratch is reused across calls; make sure nothing still reads it
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipFree(b.p));
        b.p = nullptr;
        b.cap = 0;
    }
    size_t want = bytes + bytes / 4;
    if (hipMalloc(&b.p, want) != hipSuccess) {
        b.p = nullptr;
        return fail(HJCD_E_NOMEM, "device allocation of %zu bytes failed", want);
    }
    b.cap = want;
    (void)c;
    return HJCD_OK;
}

// Host metadata of one call goes through one pinned staging region.
struct Staging {
    hjcd_ctx c;
    hipStream_t st;
    bool may_grow = true;  // false: the buffer the context was created with must do
    hjcd_status begin(size_t total) {
        HIP_TRY(hipEventSynchronize(c->staging_ev));
        if (c->pinned_cap < total && !may_grow)
            return fail(HJCD_E_INVALID, "%zu bytes of layout exceed the context's %zu-byte staging buffer", total,
                        c->pinned_cap);
        if (c->pinned_cap < total) {
            if (c->pinned) HIP_TRY(hipHostFree(c->pinned));
            c->pinned = nullptr;
            c->pinned_cap = 0;
            size_t want = std::max<size_t>(total + total / 4, 1 << 16);
            if (hipHostMalloc(&c->pinned, want, hipHostMallocDefault) != hipSuccess)
                return fail(HJCD_E_NOMEM, "pinned host allocation of %zu bytes failed", want);
            c->pinned_cap = want;
        }
        c->pinned_used = 0;
        return HJCD_OK;
    }
    hjcd_status put(void* dst, const void* src, size_t bytes) {
        if (bytes == 0) return HJCD_OK;
        size_t off = (c->pinned_used + 255) & ~size_t(255);
        char* p = (char*)c->pinned + off;
        std::memcpy(p, src, bytes);
        c->pinned_used = off + bytes;
        HIP_TRY(hipMemcpyAsync(dst, p, bytes, hipMemcpyHostToDevice, st));
        return HJCD_OK;
    }
    hjcd_status end() {
        HIP_TRY(hipEventRecord(c->staging_ev, st));
        return HJCD_OK;
    }
};

size_t staging_bytes(std::initializer_list<size_t> parts) {
    size_t s = 0;
    for (size_t p : parts) s += ((p + 255) & ~size_t(255)) + 256;
    return s;
}

bool finite_f(float x) { return std::isfinite(x); }

// Obstacle grid of a scene (see ObstacleGrid): margin 0.3 m (coarse link
// spheres up to that radius use it), at most 32 cells per axis and cells of
// at least 0.1 m over the obstacles' bounding boxes grown by the margin.
constexpr double kGridMargin = 0.3;

bool build_grid(hjcd_scene sc, int32_t n_sph, const float* sph, int32_t n_box, const float* box) {
    const int32_t no = n_sph + n_box;
    std::vector<double> lo((size_t)3 * no), hi((size_t)3 * no);
    double glo[3] = {1e300, 1e300, 1e300}, ghi[3] = {-1e300, -1e300, -1e300};
    for (int32_t o = 0; o < no; ++o)
        for (int k = 0; k < 3; ++k) {
            double c, h;
            if (o < n_sph) {
                c = sph[4 * o + k];
                h = sph[4 * o + 3];
            } else {
                c = box[6 * (o - n_sph) + k];
                h = box[6 * (o - n_sph) + 3 + k];
            }
            lo[3 * o + k] = c - h - kGridMargin;
            hi[3 * o + k] = c + h + kGridMargin;
            glo[k] = std::min(glo[k], lo[3 * o + k]);
            ghi[k] = std::max(ghi[k], hi[3 * o + k]);
        }
    double cell = 0.1;
    for (int k = 0; k < 3; ++k) cell = std::max(cell, (ghi[k] - glo[k]) / 32.0);
    int32_t n[3];
    for (int k = 0; k < 3; ++k) n[k] = std::max(1, (int32_t)std::ceil((ghi[k] - glo[k]) / cell));
    const int64_t nc = (int64_t)n[0] * n[1] * n[2];
    std::vector<std::vector<int32_t>> lists((size_t)nc);
    for (int32_t o = 0; o < no; ++o) {
        int32_t a[3], b[3];
        for (int k = 0; k < 3; ++k) {
            a[k] = std::max(0, (int32_t)std::floor((lo[3 * o + k] - glo[k]) / cell) - 1);
            b[k] = std::min(n[k] - 1, (int32_t)std::floor((hi[3 * o + k] - glo[k]) / cell) + 1);
        }
        // one cell more on each side than the grown box touches: a centre
        // rounded into a neighbouring cell still finds the obstacle
        for (int32_t i = a[0]; i <= b[0]; ++i)
            for (int32_t j = a[1]; j <= b[1]; ++j)
                for (int32_t k = a[2]; k <= b[2]; ++k) lists[((int64_t)i * n[1] + j) * n[2] + k].push_back(o);
    }
    std::vector<int32_t> start((size_t)nc + 1, 0), items;
    for (int64_t c = 0; c < nc; ++c) {
        start[c] = (int32_t)items.size();
        items.insert(items.end(), lists[c].begin(), lists[c].end());
    }
    start[nc] = (int32_t)items.size();
    if (hipMalloc(&sc->g_start, sizeof(int32_t) * start.size()) != hipSuccess ||
        hipMalloc(&sc->g_items, sizeof(int32_t) * std::max<size_t>(items.size(), 1)) != hipSuccess ||
        hipMemcpy(sc->g_start, start.data(), sizeof(int32_t) * start.size(), hipMemcpyHostToDevice) != hipSuccess ||
        (!items.empty() &&
         hipMemcpy(sc->g_items, items.data(), sizeof(int32_t) * items.size(), hipMemcpyHostToDevice) != hipSuccess))
        return false;
    for (int k = 0; k < 3; ++k) {
        sc->g_lo[k] = (float)glo[k];
        sc->g_n[k] = n[k];
    }
    sc->g_h = (float)cell;
    sc->g_margin = (float)kGridMargin;
    return true;
}

// Static workspace of hjcd_solve_noalloc: one copy per device, held from
// module load to process end.  Host code never uses the symbol's name as an
// address: hjcd_ctx_create looks up this device's copy once
// (hipGetSymbolAddress, with the device current) and the solve passes that
// address to its kernels.
static __device__ __align__(256) unsigned char scratch[HJCD_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Records this device's copy of `scratch` (the device must be current).
hjcd_status init_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(HJCD_E_DEVICE, "device %d beyond the scratch table", device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return HJCD_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(HJCD_E_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
    return HJCD_OK;
}

void* scratch_of(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
}

// Pinned staging bytes every context starts with: enough for the layout
// upload of hjcd_solve_noalloc at HJCD_NOALLOC_MAX_TARGETS targets.
size_t layout_staging_bytes(int32_t T) {
    return staging_bytes({sizeof(int64_t) * (T + 1), sizeof(int64_t) * (T + 1), sizeof(int32_t) * (size_t)T,
                          sizeof(int64_t) * (T + 1)});
}

}  // namespace

ObstacleGrid hjcd::scene_grid(const hjcd_scene_s* sc, const hjcd_robot_s* r) {
    ObstacleGrid g{};
    if (!sc || !sc->g_start || !r) return g;
    float rmax = 0.f;
    for (int l = 0; l <= r->n; ++l) rmax = std::max(rmax, r->host.coarse[l][3]);
    // the cell a centre rounds into is at most a cell away from the true one
    // (covered by the extra ring of cells); the radius must fit the margin
    if (rmax > sc->g_margin - 1e-4f) return g;
    g.start = sc->g_start;
    g.items = sc->g_items;
    for (int k = 0; k < 3; ++k) {
        g.lo[k] = sc->g_lo[k];
        g.n[k] = sc->g_n[k];
    }
    g.inv_h = 1.f / sc->g_h;
    return g;
}

hjcd_status hjcd::check_params(const hjcd_params* p) {
    if (!p) return fail(HJCD_E_INVALID, "params is NULL");
    if (p->cd_sweeps < 0 || p->cd_sweeps > (1 << 20) || p->polish_iters < 0 || p->polish_iters > (1 << 20))
        return fail(HJCD_E_INVALID, "iteration counts must be in [0, 2^20]");
    const float f[] = {p->eps_cd, p->nu_cd, p->gamma, p->delta0, p->delta_decay, p->delta_min,
                       p->proj_eps, p->tie_eps, p->lambda_, p->lambda_gn, p->trust_R, p->ls_beta, p->eps_pol,
                       p->ups_pol, p->sigma, p->mu, p->succ_pos, p->succ_ori};
    for (float x : f)
        if (!finite_f(x)) return fail(HJCD_E_INVALID, "parameters must be finite");
    if (!(p->lambda_ > 0.f)) return fail(HJCD_E_INVALID, "lambda must be > 0");
    if (p->lambda_gn < 0.f) return fail(HJCD_E_INVALID, "lambda_gn must be >= 0");
    if (!(p->trust_R > 0.f)) return fail(HJCD_E_INVALID, "trust_R must be > 0");
    if (!(p->ls_beta > 1.f)) return fail(HJCD_E_INVALID, "ls_beta must be > 1");
    if (p->ls_A < 0 || p->ls_A > 64) return fail(HJCD_E_INVALID, "ls_A must be in [0, 64]");
    if (p->weight_mode != 0 && p->weight_mode != 1) return fail(HJCD_E_INVALID, "weight_mode must be 0 or 1");
    if (p->sigma < 0.f || p->proj_eps < 0.f || p->tie_eps < 0.f)
        return fail(HJCD_E_INVALID, "sigma, proj_eps and tie_eps must be >= 0");
    if (p->top_k < 1 || p->top_k > HJCD_MAX_TOPK)
        return fail(HJCD_E_INVALID, "top_k must be in [1, %d]", HJCD_MAX_TOPK);
    if (p->resample_K < 0 || (p->resample_K > 0 && p->resample_B < p->resample_K))
        return fail(HJCD_E_INVALID, "resample needs K >= 0 and B >= K");
    if (p->polish_variant != 0 && p->polish_variant != 1) return fail(HJCD_E_INVALID, "polish_variant must be 0 or 1");
    if (p->collect_stats < 0 || p->collect_stats > 2) return fail(HJCD_E_INVALID, "collect_stats must be 0, 1 or 2");
    if (p->cd_lanes_per_seed < 0 || p->cd_lanes_per_seed > 2)
        return fail(HJCD_E_INVALID, "cd_lanes_per_seed must be 0, 1 or 2");
    return HJCD_OK;
}

KernelParams hjcd::kparams(const hjcd_params& p) {
    KernelParams k;
    k.cd_sweeps = p.cd_sweeps;
    k.polish_iters = p.polish_iters;
    k.ls_A = p.ls_A;
    k.weight_mode = p.weight_mode;
    k.eps_cd2 = p.eps_cd * p.eps_cd;
    k.nu_cd = p.nu_cd;
    k.gamma = p.gamma;
    k.delta0 = p.delta0;
    k.delta_decay = p.delta_decay;
    k.delta_min = p.delta_min;
    k.proj_eps2 = p.proj_eps * p.proj_eps;
    k.tie_eps = p.tie_eps;
    k.lam = p.lambda_;
    k.lambda_gn = p.lambda_gn;
    k.trust_R = p.trust_R;
    k.inv_beta = 1.f / p.ls_beta;
    k.eps_pol2 = p.eps_pol * p.eps_pol;
    k.ups_pol = p.ups_pol;
    k.sigma = p.sigma;
    k.mu = p.mu;
    k.seed = p.rng_seed;
    return k;
}

namespace hjcd {

hjcd_status check_offsets(int32_t T, const int64_t* offs) {
    if (T < 0) return fail(HJCD_E_INVALID, "T must be >= 0");
    if (!offs) return fail(HJCD_E_INVALID, "seed_offsets is NULL");
    if (offs[0] != 0) return fail(HJCD_E_INVALID, "seed_offsets[0] must be 0");
    for (int32_t t = 0; t < T; ++t)
        if (offs[t + 1] < offs[t]) return fail(HJCD_E_INVALID, "seed_offsets must be non-decreasing (at %d)", t);
    if (offs[T] > ((int64_t)1 << 40)) return fail(HJCD_E_INVALID, "too many seeds");
    return HJCD_OK;
}

// Pure argument checks come first in every entry point; the context is
// checked and its device bound only after them, right before device work.
hjcd_status check_ctx(hjcd_ctx c) {
    if (!c) return fail(HJCD_E_INVALID, "ctx is NULL");
    return HJCD_OK;
}

hjcd_status bind(hjcd_ctx c) {
    HIP_TRY(hipSetDevice(c->device));
    return HJCD_OK;
}

hjcd_status check_robot(hjcd_ctx c, hjcd_robot r) {
    if (!r) return fail(HJCD_E_INVALID, "robot is NULL");
    if (r->ctx != c) return fail(HJCD_E_INVALID, "robot belongs to another context");
    return HJCD_OK;
}

void group_targets(int32_t n_robots, int32_t T, const int32_t* robot_of_target, const int64_t* offs,
                   TargetGroups& g) {
    g.rb_tb.assign(n_robots + 1, 0);
    g.perm.clear();
    g.identity = true;
    if (robot_of_target && n_robots > 1) {
        std::vector<int32_t> cnt(n_robots, 0);
        for (int32_t t = 0; t < T; ++t) cnt[robot_of_target[t]]++;
        for (int i = 0; i < n_robots; ++i) g.rb_tb[i + 1] = g.rb_tb[i] + cnt[i];
        g.perm.resize(T);
        std::vector<int32_t> pos(g.rb_tb.begin(), g.rb_tb.end() - 1);
        for (int32_t t = 0; t < T; ++t) g.perm[pos[robot_of_target[t]]++] = t;
        for (int32_t b = 0; b < T; ++b)
            if (g.perm[b] != b) g.identity = false;
    } else {
        const int r0 = robot_of_target ? robot_of_target[0] : 0;
        for (int i = 0; i <= n_robots; ++i) g.rb_tb[i] = (i <= r0) ? 0 : T;
    }
    g.voffs.assign(T + 1, 0);
    if (g.identity) {
        std::memcpy(g.voffs.data(), offs, sizeof(int64_t) * (T + 1));
    } else {
        for (int32_t b = 0; b < T; ++b) g.voffs[b + 1] = g.voffs[b] + (offs[g.perm[b] + 1] - offs[g.perm[b]]);
    }
}

}  // namespace hjcd

namespace {

// ---- stats ------------------------------------------------------------------
enum StatStage { SS_INIT = 0, SS_CD, SS_RESAMPLE, SS_POLISH, SS_COLLIDE, SS_SELECT };

struct StatScope {
    hjcd_ctx c;
    hipStream_t st;
    bool on;     // stage times
    bool count;  // executed-work counters (the kernels built with them)
    hjcd_status begin(int32_t mode, int64_t seeds) {
        on = mode != 0;
        count = mode == 1;
        if (!on) return HJCD_OK;
        c->ev_used = 0;
        c->stats = hjcd_stats{};
        c->stats.seeds = (uint64_t)seeds;
        c->stats_stream = st;
        hjcd_status s = ensure(c, c->counters, 16 * sizeof(unsigned long long));
        if (s != HJCD_OK) return s;
        HIP_TRY(hipMemsetAsync(c->counters.p, 0, 16 * sizeof(unsigned long long), st));
        return mark(-1);
    }
    hjcd_status mark(int stage) {
        if (!on) return HJCD_OK;
        if (c->ev_used >= hjcd_ctx_s::kEv) return HJCD_OK;
        c->ev_stage[c->ev_used] = stage;
        HIP_TRY(hipEventRecord(c->ev[c->ev_used++], st));
        return HJCD_OK;
    }
    unsigned long long* counters() const { return count ? (unsigned long long*)c->counters.p : nullptr; }
    void end() {
        if (on) c->stats_pending = true;
    }
};

}  // namespace

// =============================================================================
// C ABI
// =============================================================================
extern "C" {

const char* hjcd_last_error(void) { return g_err.c_str(); }

const char* hjcd_version(void) { return "hjcd 0.1 (gfx950)"; }

void hjcd_params_default(hjcd_params* p) {
    if (!p) return;
    *p = hjcd_params{};
    p->cd_sweeps = 20;
    p->polish_iters = 20;
    p->eps_cd = 5e-3f;
    p->nu_cd = 5e-2f;
    p->gamma = 1e-7f;
    p->delta0 = 1.0f;
    p->delta_decay = 0.9f;
    p->delta_min = 0.1f;
    p->proj_eps = 1e-5f;
    p->tie_eps = 1e-5f;
    p->lambda_ = 1e-3f;
    p->lambda_gn = 1e-4f;
    p->trust_R = 0.2f;
    p->ls_beta = 2.0f;
    p->ls_A = 4;
    p->weight_mode = 0;
    p->eps_pol = 1e-5f;
    p->ups_pol = 1e-5f;
    p->sigma = 0.05f;
    p->mu = 0.0f;
    p->resample_K = 0;
    p->resample_B = 0;
    p->top_k = 1;
    p->succ_pos = 1e-3f;
    p->succ_ori = (float)(3.14159265358979323846 / 180.0);
    p->rng_seed = 0;
    p->collect_stats = 0;
    p->polish_variant = 0;
    p->cd_lanes_per_seed = 1;
}

hjcd_status hjcd_ctx_create(int device, hjcd_ctx* out) {
    if (!out) return fail(HJCD_E_INVALID, "out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
        return fail(HJCD_E_DEVICE, "no HIP device available");
    if (device < 0 || device >= count) return fail(HJCD_E_DEVICE, "device %d out of range (%d devices)", device, count);
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(HJCD_E_DEVICE, "device %d is %s, libhjcd is built for gfx950", device, prop.gcnArchName);
    HIP_TRY(hipSetDevice(device));
    hjcd_ctx c = new hjcd_ctx_s();
    c->device = device;
    if (hipEventCreateWithFlags(&c->staging_ev, hipEventDisableTiming) != hipSuccess) {
        delete c;
        return fail(HJCD_E_DEVICE, "event creation failed");
    }
    for (int i = 0; i < hjcd_ctx_s::kEv; ++i) {
        if (hipEventCreate(&c->ev[i]) != hipSuccess) {
            hjcd_ctx_destroy(c);
            return fail(HJCD_E_DEVICE, "event creation failed");
        }
    }
    hjcd_status s = init_scratch(device);
    if (s != HJCD_OK) {
        hjcd_ctx_destroy(c);
        return s;
    }
    const size_t pin = layout_staging_bytes(HJCD_NOALLOC_MAX_TARGETS);
    if (hipHostMalloc(&c->pinned, pin, hipHostMallocDefault) != hipSuccess) {
        c->pinned = nullptr;
        hjcd_ctx_destroy(c);
        return fail(HJCD_E_NOMEM, "pinned host allocation of %zu bytes failed", pin);
    }
    c->pinned_cap = pin;
    *out = c;
    return HJCD_OK;
}

void hjcd_ctx_destroy(hjcd_ctx c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    DevBuf* bufs[] = {&c->voffs, &c->voffs2, &c->coffs, &c->tperm, &c->tkeys_dummy, &c->q_work, &c->q_work2, &c->ep,
                      &c->eo, &c->cost, &c->flag, &c->rank, &c->counters};
    for (DevBuf* b : bufs)
        if (b->p) (void)hipFree(b->p);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->staging_ev) (void)hipEventDestroy(c->staging_ev);
    for (int i = 0; i < hjcd_ctx_s::kEv; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    delete c;
}

hjcd_status hjcd_load_robot(hjcd_ctx c, const hjcd_robot_desc* d, hjcd_robot* out) {
    if (!out) return fail(HJCD_E_INVALID, "out is NULL");
    *out = nullptr;
    hjcd_status s;
    if (!d) return fail(HJCD_E_INVALID, "robot description is NULL");
    if (d->dof < 1) return fail(HJCD_E_INVALID, "dof must be >= 1");
    if (d->dof > HJCD_MAX_DOF) return fail(HJCD_E_UNSUPPORTED, "dof %d > %d", d->dof, HJCD_MAX_DOF);
    if (d->convention != HJCD_DH_MODIFIED && d->convention != HJCD_DH_STANDARD)
        return fail(HJCD_E_INVALID, "unknown DH convention %d", d->convention);
    if (!d->a || !d->d || !d->alpha || !d->offset || !d->q_min || !d->q_max)
        return fail(HJCD_E_INVALID, "DH arrays and limits are required");
    if (d->n_spheres < 0 || d->n_spheres > HJCD_MAX_SPHERES)
        return fail(HJCD_E_UNSUPPORTED, "n_spheres must be in [0, %d]", HJCD_MAX_SPHERES);
    if (d->n_spheres > 0 && (!d->sphere_link || !d->sphere_xyzr))
        return fail(HJCD_E_INVALID, "sphere arrays are NULL");
    if (d->min_link_gap < 0) return fail(HJCD_E_INVALID, "min_link_gap must be >= 0");
    const int n = d->dof;
    for (int i = 0; i < n; ++i) {
        const double v[] = {d->a[i], d->d[i], d->alpha[i], d->offset[i], d->q_min[i], d->q_max[i]};
        for (double x : v)
            if (!std::isfinite(x)) return fail(HJCD_E_INVALID, "joint %d has a non-finite parameter", i);
        if (!(d->q_min[i] <= d->q_max[i])) return fail(HJCD_E_INVALID, "joint %d: q_min > q_max", i);
        if (std::fabs(d->q_min[i]) > HJCD_MAX_ANGLE || std::fabs(d->q_max[i]) > HJCD_MAX_ANGLE ||
            std::fabs(d->offset[i]) > HJCD_MAX_ANGLE)
            return fail(HJCD_E_UNSUPPORTED, "joint %d: limits and offset must lie within +-%g rad", i,
                        (double)HJCD_MAX_ANGLE);
    }
    double tool[16];
    for (int i = 0; i < 16; ++i) tool[i] = d->tool ? d->tool[i] : (i % 5 == 0 ? 1.0 : 0.0);
    for (double x : tool)
        if (!std::isfinite(x)) return fail(HJCD_E_INVALID, "tool transform is not finite");
    // rigid: R^T R = I, bottom row (0 0 0 1)
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s2 = 0;
            for (int k = 0; k < 3; ++k) s2 += tool[4 * k + a] * tool[4 * k + b];
            if (std::fabs(s2 - (a == b ? 1.0 : 0.0)) > 1e-6) return fail(HJCD_E_INVALID, "tool rotation is not orthonormal");
        }
    if (std::fabs(tool[12]) + std::fabs(tool[13]) + std::fabs(tool[14]) + std::fabs(tool[15] - 1.0) > 1e-9)
        return fail(HJCD_E_INVALID, "tool bottom row must be (0 0 0 1)");
    for (int i = 0; i < d->n_spheres; ++i) {
        if (d->sphere_link[i] < 0 || d->sphere_link[i] > n)
            return fail(HJCD_E_INVALID, "sphere %d: link %d outside 0..%d", i, d->sphere_link[i], n);
        for (int k = 0; k < 4; ++k)
            if (!std::isfinite(d->sphere_xyzr[4 * i + k])) return fail(HJCD_E_INVALID, "sphere %d not finite", i);
        if (d->sphere_xyzr[4 * i + 3] < 0) return fail(HJCD_E_INVALID, "sphere %d has a negative radius", i);
    }
    if ((s = check_ctx(c)) != HJCD_OK) return s;
    if ((s = bind(c)) != HJCD_OK) return s;

    hjcd_robot r = new hjcd_robot_s();
    r->ctx = c;
    r->device = c->device;
    r->n = n;
    DevRobot& h = r->host;
    std::memset(&h, 0, sizeof(h));
    h.n = n;
    h.conv = d->convention;
    for (int i = 0; i < n; ++i) {
        h.off[i] = (float)d->offset[i];
        h.lo[i] = (float)d->q_min[i];
        h.hi[i] = (float)d->q_max[i];
        h.ca[i] = (float)std::cos(d->alpha[i]);
        h.sa[i] = (float)std::sin(d->alpha[i]);
        h.a[i] = (float)d->a[i];
        h.d[i] = (float)d->d[i];
        h.px[i] = (float)d->a[i];
        h.py[i] = (float)(-d->d[i] * std::sin(d->alpha[i]));
        h.pz[i] = (float)(d->d[i] * std::cos(d->alpha[i]));
    }
    bool rot = false;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 4; ++j) {
            h.tool[4 * i + j] = (float)tool[4 * i + j];
            if (j < 3 && std::fabs(tool[4 * i + j] - (i == j ? 1.0 : 0.0)) > 0) rot = true;
        }
    h.tool_rot = rot ? 1 : 0;
    // spheres grouped by link (stable), coarse enclosing sphere per link
    std::vector<int> order(d->n_spheres);
    for (int i = 0; i < d->n_spheres; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return d->sphere_link[x] < d->sphere_link[y]; });
    h.n_sph = d->n_spheres;
    for (int l = 0; l <= n; ++l) {
        h.link_first[l] = 0;
        h.link_count[l] = 0;
        h.coarse[l][3] = -1.f;
    }
    for (int k = 0; k < d->n_spheres; ++k) {
        const int i = order[k];
        for (int q = 0; q < 4; ++q) h.sph[k][q] = (float)d->sphere_xyzr[4 * i + q];
        const int l = d->sphere_link[i];
        if (h.link_count[l] == 0) h.link_first[l] = k;
        h.link_count[l]++;
    }
    for (int l = 0; l <= n; ++l) {
        const int cnt = h.link_count[l];
        if (cnt == 0) continue;
        double cx = 0, cy = 0, cz = 0;
        for (int k = 0; k < cnt; ++k) {
            const int i = order[h.link_first[l] + k];
            cx += d->sphere_xyzr[4 * i];
            cy += d->sphere_xyzr[4 * i + 1];
            cz += d->sphere_xyzr[4 * i + 2];
        }
        cx /= cnt;
        cy /= cnt;
        cz /= cnt;
        double R = 0;
        for (int k = 0; k < cnt; ++k) {
            const int i = order[h.link_first[l] + k];
            const double dx = d->sphere_xyzr[4 * i] - cx, dy = d->sphere_xyzr[4 * i + 1] - cy,
                         dz = d->sphere_xyzr[4 * i + 2] - cz;
            R = std::max(R, std::sqrt(dx * dx + dy * dy + dz * dz) + d->sphere_xyzr[4 * i + 3]);
        }
        // conservative against single-precision rounding of the link frames
        h.coarse[l][0] = (float)cx;
        h.coarse[l][1] = (float)cy;
        h.coarse[l][2] = (float)cz;
        h.coarse[l][3] = (float)(R + 1e-4);
    }
    h.n_pairs = 0;
    if (d->min_link_gap > 0) {
        for (int la = 0; la <= n; ++la)
            for (int lb = la + d->min_link_gap; lb <= n; ++lb)
                if (h.link_count[la] > 0 && h.link_count[lb] > 0) {
                    h.pair_a[h.n_pairs] = (uint8_t)la;
                    h.pair_b[h.n_pairs] = (uint8_t)lb;
                    h.n_pairs++;
                }
    }
    if (hipMalloc(&r->dev, sizeof(DevRobot)) != hipSuccess) {
        delete r;
        return fail(HJCD_E_NOMEM, "robot table allocation failed");
    }
    if (hipMemcpy(r->dev, &h, sizeof(DevRobot), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(r->dev);
        delete r;
        return fail(HJCD_E_DEVICE, "robot table upload failed");
    }
    *out = r;
    return HJCD_OK;
}

void hjcd_robot_destroy(hjcd_robot r) {
    if (!r) return;
    (void)hipSetDevice(r->device);
    (void)hipDeviceSynchronize();
    if (r->dev) (void)hipFree(r->dev);
    delete r;
}

int32_t hjcd_robot_dof(hjcd_robot r) { return r ? r->n : -1; }

hjcd_status hjcd_load_scene(hjcd_ctx c, int32_t n_sph, const float* sph, int32_t n_box, const float* box,
                            hjcd_scene* out) {
    if (!out) return fail(HJCD_E_INVALID, "out is NULL");
    *out = nullptr;
    hjcd_status s;
    if (n_sph < 0 || n_box < 0 || n_sph + n_box > HJCD_MAX_OBSTACLES)
        return fail(HJCD_E_INVALID, "obstacle counts must be in [0, %d]", HJCD_MAX_OBSTACLES);
    if ((n_sph > 0 && !sph) || (n_box > 0 && !box)) return fail(HJCD_E_INVALID, "obstacle arrays are NULL");
    for (int i = 0; i < 4 * n_sph; ++i)
        if (!std::isfinite(sph[i])) return fail(HJCD_E_INVALID, "obstacle spheres must be finite");
    for (int i = 0; i < n_sph; ++i)
        if (sph[4 * i + 3] < 0) return fail(HJCD_E_INVALID, "obstacle sphere %d has a negative radius", i);
    for (int i = 0; i < 6 * n_box; ++i)
        if (!std::isfinite(box[i])) return fail(HJCD_E_INVALID, "boxes must be finite");
    for (int i = 0; i < n_box; ++i)
        for (int k = 3; k < 6; ++k)
            if (box[6 * i + k] < 0) return fail(HJCD_E_INVALID, "box %d has a negative half-extent", i);
    if ((s = check_ctx(c)) != HJCD_OK) return s;
    if ((s = bind(c)) != HJCD_OK) return s;
    hjcd_scene sc = new hjcd_scene_s();
    sc->ctx = c;
    sc->device = c->device;
    sc->n_sph = n_sph;
    sc->n_box = n_box;
    std::vector<float> bx((size_t)8 * n_box, 0.f);
    for (int i = 0; i < n_box; ++i) {
        for (int k = 0; k < 3; ++k) {
            bx[8 * i + k] = box[6 * i + k];
            bx[8 * i + 4 + k] = box[6 * i + 3 + k];
        }
    }
    bool ok = true;
    if (n_sph > 0) ok = ok && hipMalloc(&sc->sph, sizeof(float) * 4 * n_sph) == hipSuccess;
    if (ok && n_box > 0) ok = ok && hipMalloc(&sc->box, sizeof(float) * 8 * n_box) == hipSuccess;
    if (ok && n_sph > 0) ok = hipMemcpy(sc->sph, sph, sizeof(float) * 4 * n_sph, hipMemcpyHostToDevice) == hipSuccess;
    if (ok && n_box > 0) ok = hipMemcpy(sc->box, bx.data(), sizeof(float) * 8 * n_box, hipMemcpyHostToDevice) == hipSuccess;
    if (ok && n_sph + n_box >= kGridMinObstacles) ok = build_grid(sc, n_sph, sph, n_box, box);
    if (!ok) {
        hjcd_scene_destroy(sc);
        return fail(HJCD_E_NOMEM, "scene upload failed");
    }
    *out = sc;
    return HJCD_OK;
}

void hjcd_scene_destroy(hjcd_scene sc) {
    if (!sc) return;
    (void)hipSetDevice(sc->device);
    (void)hipDeviceSynchronize();
    if (sc->sph) (void)hipFree(sc->sph);
    if (sc->box) (void)hipFree(sc->box);
    if (sc->g_start) (void)hipFree(sc->g_start);
    if (sc->g_items) (void)hipFree(sc->g_items);
    delete sc;
}

// ---- stages -----------------------------------------------------------------

hjcd_status hjcd_fk(hjcd_ctx c, hjcd_robot r, int64_t S, const float* q, float* pose, float* jac, void* stream) {
    hjcd_status s;
    if (S < 0) return fail(HJCD_E_INVALID, "S must be >= 0");
    if (S > 0 && (!q || !pose)) return fail(HJCD_E_INVALID, "q and pose are required");
    if ((s = check_ctx(c)) != HJCD_OK) return s;
    if ((s = check_robot(c, r)) != HJCD_OK) return s;
    if ((s = bind(c)) != HJCD_OK) return s;
    HIP_TRY(launch_fk(r->dev, r->n, S, q, pose, jac, (hipStream_t)stream));
    return HJCD_OK;
}

static hjcd_status upload_offsets(hjcd_ctx c, int32_t T, const int64_t* offs, hipStream_t st) {
    hjcd_status s = ensure(c, c->voffs, sizeof(int64_t) * (T + 1));
    if (s != HJCD_OK) return s;
    Staging sg{c, st};
    if ((s = sg.begin(staging_bytes({sizeof(int64_t) * (T + 1)}))) != HJCD_OK) return s;
    if ((s = sg.put(c->voffs.p, offs, sizeof(int64_t) * (T + 1))) != HJCD_OK) return s;
    return sg.end();
}

static SeedMap identity_map(hjcd_ctx c, int32_t T, int64_t S, const uint32_t* tkeys) {
    SeedMap m;
    m.voffs = (const int64_t*)c->voffs.p;
    m.tperm = nullptr;
    m.T = T;
    m.tb = 0;
    m.te = T;
    m.base = 0;
    m.Sv = S;
    m.tkeys = tkeys;
    return m;
}

hjcd_status hjcd_init_seeds(hjcd_ctx c, hjcd_robot r, int32_t T, const int64_t* offs, const uint32_t* tkeys,
                            uint64_t rng_seed, float* q, void* stream) {
    hjcd_status s;
    if ((s = check_offsets(T, offs)) != HJCD_OK) return s;
    const int64_t S = offs[T];
    if (S > 0 && !q) return fail(HJCD_E_INVALID, "q is NULL");
    if ((s = check_ctx(c)) != HJCD_OK) return s;
    if ((s = check_robot(c, r)) != HJCD_OK) return s;
    if (S == 0) return HJCD_OK;
    if ((s = bind(c)) != HJCD_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = upload_offsets(c, T, offs, st)) != HJCD_OK) return s;
    // seed init only: a solve pass with no CD and no polish writes the seeds
    hjcd_params p;
    hjcd_params_default(&p);
    p.rng_seed = rng_seed;
    SolveArgs a{};
    a.rb = r->dev;
    a.n = r->n;
    a.map = identity_map(c, T, S, tkeys);
    a.S = S;
    a.targets = nullptr;  // no residual is computed without targets
    a.q_out = q;
    a.init_mode = INIT_UNIFORM;
    a.do_cd = 0;
    a.do_polish = 0;
    a.kp = kparams(p);
    a.counters = nullptr;
    HIP_TRY(launch_solve(a, st));
    return HJCD_OK;
}

static hjcd_status stage_common(hjcd_ctx c, hjcd_robot r, int32_t T, const float* targets, const int64_t* offs,
                                const uint32_t* tkeys, const hjcd_params* p, float* q, float* ep, float* eo,
                                float* cost, float* traj, void* stream, bool cd) {
    hjcd_status s;
    if ((s = check_params(p)) != HJCD_OK) return s;
    if ((s = check_offsets(T, offs)) != HJCD_OK) return s;
    const int64_t S = offs[T];
    if (S > 0 && (!q || !targets)) return fail(HJCD_E_INVALID, "q and targets are required");
    if ((s = check_ctx(c)) != HJCD_OK) return s;
    if ((s = check_robot(c, r)) != HJCD_OK) return s;
    if (S == 0) return HJCD_OK;
    if ((s = bind(c)) != HJCD_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    StatScope ss{c, st, false};
    if ((s = ss.begin(p->collect_stats, S)) != HJCD_OK) return s;
    if ((s = upload_offsets(c, T, offs, st)) != HJCD_OK) return s;
    SolveArgs a{};
    a.rb = r->dev;
    a.n = r->n;
    a.map = identity_map(c, T, S, tkeys);
    a.S = S;
    a.targets = targets;
    a.q_in = q;
    a.q_in_stride = S;
    a.q_out = q;
    a.err_p = ep;
    a.err_o = eo;
    a.cost = cost;
    a.traj = traj;
    a.init_mode = INIT_LOAD;
    a.do_cd = cd ? 1 : 0;
    a.do_polish = cd ? 0 : 1;
    a.kp = kparams(*p);
    a.counters = ss.counters();
    a.variant = p->polish_variant;
    a.cd_lanes = p->cd_lanes_per_seed == 2 ? 2 : 1;
    HIP_TRY(launch_solve(a, st));
    if ((s = ss.mark(cd ? SS_CD : SS_POLISH)) != HJCD_OK) return s;
    ss.end();
    return HJCD_OK;
}

hjcd_status hjcd_cd(hjcd_ctx c, hjcd_robot r, int32_t T, const float* targets, const int64_t* offs,
                    const uint32_t* tkeys, const hjcd_params* p, float* q, float* ep, float* eo, float* cost,
                    float* traj, void* stream) {
    return stage_common(c, r, T, targets, offs, tkeys, p, q, ep, eo, cost, traj, stream, true);
}

hjcd_status hjcd_polish(hjcd_ctx c, hjcd_robot r, int32_t T, const float* targets, const int64_t* offs,
                        const uint32_t* tkeys, const hjcd_params* p, float* q, float* ep, float* eo,
                        float* cost, float* traj, void* stream) {
    return stage_common(c, r, T, targets, offs, tkeys, p, q, ep, eo, cost, traj, stream, false);
}

hjcd_status hjcd_collide(hjcd_ctx c, hjcd_robot r, hjcd_scene sc, int64_t S, const float* q, uint8_t* flag,
                         void* stream) {
    hjcd_status s;
    if (S < 0) return fail(HJCD_E_INVALID, "S must be >= 0");
    if (S > 0 && (!q || !flag)) return fail(HJCD_E_INVALID, "q and flag are required");
    if ((s = check_ctx(c)) != HJCD_OK) return s;
    if ((s = check_robot(c, r)) != HJCD_OK) return s;
    if (sc && sc->ctx != c) return fail(HJCD_E_INVALID, "scene belongs to another context");
    if (S == 0) return HJCD_OK;
    if ((s = bind(c)) != HJCD_OK) return s;
    CollideArgs a{};
    a.rb = r->dev;
    a.n = r->n;
    a.S = S;
    a.q = q;
    a.q_stride = S;
    a.osph = sc ? sc->sph : nullptr;
    a.n_osph = sc ? sc->n_sph : 0;
    a.obox = sc ? sc->box : nullptr;
    a.n_obox = sc ? sc->n_box : 0;
    a.grid = scene_grid(sc, r);
    a.flag = flag;
    a.counters = nullptr;
    a.n_pairs = r->host.n_pairs;
    HIP_TRY(launch_collide(a, (hipStream_t)stream));
    return HJCD_OK;
}

hjcd_status hjcd_resample(hjcd_ctx c, hjcd_robot r, int32_t T, const int64_t* offs, const uint32_t* tkeys,
                          const hjcd_params* p, const float* q_in, const float* cost_in, float* q_out,
                          void* stream) {
    hjcd_status s;
    if ((s = check_params(p)) != HJCD_OK) return s;
    if ((s = check_offsets(T, offs)) != HJCD_OK) return s;
    if (p->resample_K < 1) return fail(HJCD_E_INVALID, "resample_K must be >= 1");
    for (int32_t t = 0; t < T; ++t)
        if (offs[t + 1] == offs[t]) return fail(HJCD_E_INVALID, "target %d has no seeds to resample", t);
    const int32_t K = p->resample_K;
    const int32_t Bp = (p->resample_B / K) * K;
    if (T > 0 && (!q_in || !cost_in || !q_out)) return fail(HJCD_E_INVALID, "q_in, cost_in and q_out are required");
    if ((s = check_ctx(c)) != HJCD_OK) return s;
    if ((s = check_robot(c, r)) != HJCD_OK) return s;
    if (T == 0 || Bp == 0) return HJCD_OK;
    if ((s = bind(c)) != HJCD_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = upload_offsets(c, T, offs, st)) != HJCD_OK) return s;
    if ((s = ensure(c, c->rank, sizeof(int32_t) * (size_t)T * K)) != HJCD_OK) return s;
    HIP_TRY(launch_rank(T, (const int64_t*)c->voffs.p, cost_in, K, (int32_t*)c->rank.p, st));
    HIP_TRY(launch_replicate(r->dev, r->n, 0, T, T, (const int64_t*)c->voffs.p, nullptr, offs[T], q_in,
                             (const int32_t*)c->rank.p, K, Bp, tkeys, p->rng_seed, p->mu, p->sigma, q_out, st));
    return HJCD_OK;
}

static hjcd_status select_common(hjcd_ctx c, int32_t T, const int64_t* offs, int32_t n, int32_t n_stride,
                                 const hjcd_params* p, const float* q, const float* cost, const float* ep,
                                 const float* eo, const uint8_t* flag, const float* q_ref, float* q_out,
                                 float* ep_out, float* eo_out, uint8_t* fl_out, int32_t* n_free, uint8_t* solved,
                                 void* stream) {
    hjcd_status s;
    if ((s = check_params(p)) != HJCD_OK) return s;
    if ((s = check_offsets(T, offs)) != HJCD_OK) return s;
    if (n < 1 || n > HJCD_MAX_DOF || n_stride < n || n_stride > HJCD_MAX_DOF)
        return fail(HJCD_E_INVALID, "need 1 <= n <= n_stride <= %d", HJCD_MAX_DOF);
    const int64_t S = offs[T];
    if (T == 0) return check_ctx(c);
    if ((S > 0 && (!q || !cost || !ep || !eo || !flag)) || !q_out || !ep_out || !eo_out || !fl_out || !n_free ||
        !solved)
        return fail(HJCD_E_INVALID, "select arrays are required");
    if ((s = check_ctx(c)) != HJCD_OK) return s;
    if ((s = bind(c)) != HJCD_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = upload_offsets(c, T, offs, st)) != HJCD_OK) return s;
    SelectArgs a{};
    a.T = T;
    a.offsets = (const int64_t*)c->voffs.p;
    a.tperm = nullptr;
    a.n = n;
    a.n_stride = n_stride;
    a.S = S;
    a.q = q;
    a.cost = cost;
    a.err_p = ep;
    a.err_o = eo;
    a.flag = flag;
    a.k = p->top_k;
    a.succ_pos = p->succ_pos;
    a.succ_ori = p->succ_ori;
    a.q_out = q_out;
    a.ep_out = ep_out;
    a.eo_out = eo_out;
    a.fl_out = fl_out;
    a.n_free = n_free;
    a.solved = solved;
    a.q_ref = q_ref;
    HIP_TRY(launch_select(a, st));
    return HJCD_OK;
}

hjcd_status hjcd_select(hjcd_ctx c, int32_t T, const int64_t* offs, int32_t n, int32_t n_stride,
                        const hjcd_params* p, const float* q, const float* cost, const float* ep, const float* eo,
                        const uint8_t* flag, float* q_out, float* ep_out, float* eo_out, uint8_t* fl_out,
                        int32_t* n_free, uint8_t* solved, void* stream) {
    return select_common(c, T, offs, n, n_stride, p, q, cost, ep, eo, flag, nullptr, q_out, ep_out, eo_out, fl_out,
                         n_free, solved, stream);
}

hjcd_status hjcd_select_near(hjcd_ctx c, int32_t T, const int64_t* offs, int32_t n, int32_t n_stride,
                             const hjcd_params* p, const float* q, const float* cost, const float* ep,
                             const float* eo, const uint8_t* flag, const float* q_ref, float* q_out, float* ep_out,
                             float* eo_out, uint8_t* fl_out, int32_t* n_free, uint8_t* solved, void* stream) {
    if (T > 0 && !q_ref) return fail(HJCD_E_INVALID, "q_ref is required");
    return select_common(c, T, offs, n, n_stride, p, q, cost, ep, eo, flag, q_ref, q_out, ep_out, eo_out, fl_out,
                         n_free, solved, stream);
}

hjcd_status hjcd_warm_seeds(hjcd_ctx c, hjcd_robot r, int32_t T, int32_t k, int32_t n_stride, const float* q_prev,
                            int32_t M, const uint32_t* tkeys, const hjcd_params* p, float* q_out, void* stream) {
    hjcd_status s;
    if ((s = check_params(p)) != HJCD_OK) return s;
    if (T < 0 || k < 1 || M < 0) return fail(HJCD_E_INVALID, "need T >= 0, k >= 1, M >= 0");
    if ((s = check_ctx(c)) != HJCD_OK) return s;
    if ((s = check_robot(c, r)) != HJCD_OK) return s;
    if (n_stride < r->n || n_stride > HJCD_MAX_DOF)
        return fail(HJCD_E_INVALID, "n_stride must be in [dof, %d]", HJCD_MAX_DOF);
    if ((int64_t)T * M == 0) return HJCD_OK;
    if (!q_prev || !q_out) return fail(HJCD_E_INVALID, "q_prev and q_out are required");
    if ((s = bind(c)) != HJCD_OK) return s;
    HIP_TRY(launch_warm(r->dev, r->n, T, k, n_stride, q_prev, M, tkeys, p->rng_seed, p->mu, p->sigma, q_out,
                        (hipStream_t)stream));
    return HJCD_OK;
}

// ---- the whole solve --------------------------------------------------------

// The whole solve.  Work arrays come from the context (grown on demand) or,
// with `noalloc`, from this device's static workspace (nothing allocated).
static hjcd_status solve_impl(hjcd_ctx c, int32_t n_robots, const hjcd_robot* robots, hjcd_scene sc, int32_t T,
                              const int32_t* robot_of_target, const float* targets, const int64_t* offs,
                              const uint32_t* tkeys, const float* seeds, const hjcd_params* p, float* q_out,
                              float* ep, float* eo, uint8_t* flag, int32_t* n_free, uint8_t* solved, void* stream,
                              bool noalloc, const float* q_ref = nullptr) {
    hjcd_status s;
    if (n_robots < 1 || n_robots > HJCD_MAX_ROBOTS || !robots)
        return fail(HJCD_E_INVALID, "need 1..%d robots", HJCD_MAX_ROBOTS);
    if ((s = check_params(p)) != HJCD_OK) return s;
    if ((s = check_offsets(T, offs)) != HJCD_OK) return s;
    if (robot_of_target)
        for (int32_t t = 0; t < T; ++t)
            if (robot_of_target[t] < 0 || robot_of_target[t] >= n_robots)
                return fail(HJCD_E_INVALID, "robot_of_target[%d] = %d out of range", t, robot_of_target[t]);
    if (T > 0 && (!targets || !q_out || !ep || !eo || !flag || !n_free || !solved))
        return fail(HJCD_E_INVALID, "targets and outputs are required");
    const bool resample = p->resample_K > 0;
    if (resample)
        for (int32_t t = 0; t < T; ++t)
            if (offs[t + 1] == offs[t]) return fail(HJCD_E_INVALID, "target %d has no seeds to resample", t);
    if ((s = check_ctx(c)) != HJCD_OK) return s;
    for (int i = 0; i < n_robots; ++i)
        if ((s = check_robot(c, robots[i])) != HJCD_OK) return s;
    if (sc && sc->ctx != c) return fail(HJCD_E_INVALID, "scene belongs to another context");
    if (noalloc && p->collect_stats)
        return fail(HJCD_E_UNSUPPORTED, "hjcd_solve_noalloc collects no statistics (collect_stats must be 0)");
    if (noalloc && T > HJCD_NOALLOC_MAX_TARGETS)
        return fail(HJCD_E_INVALID, "T = %d exceeds HJCD_NOALLOC_MAX_TARGETS (%d)", T, HJCD_NOALLOC_MAX_TARGETS);
    if (T == 0) return HJCD_OK;
    if ((s = bind(c)) != HJCD_OK) return s;
    int n_max = 0;
    for (int i = 0; i < n_robots; ++i) n_max = std::max(n_max, robots[i]->n);
    const int64_t S = offs[T];
    hipStream_t st = (hipStream_t)stream;

    // plan: permuted target order grouped by robot, CSR over it
    TargetGroups grp;
    group_targets(n_robots, T, robot_of_target, offs, grp);
    const std::vector<int32_t>& perm = grp.perm;
    const std::vector<int32_t>& rb_tb = grp.rb_tb;
    const std::vector<int64_t>& voffs = grp.voffs;
    const bool identity = grp.identity;
    const int32_t K = p->resample_K;
    const int32_t Bp = resample ? (p->resample_B / K) * K : 0;
    const int64_t S2 = resample ? (int64_t)T * Bp : S;
    std::vector<int64_t> voffs2;
    if (resample) {
        voffs2.resize(T + 1);
        for (int32_t b = 0; b <= T; ++b) voffs2[b] = (int64_t)b * Bp;
    }

    // work arrays
    const int64_t Sf = resample ? S2 : S;  // slots of the final stage
    const size_t sz_voffs = sizeof(int64_t) * (T + 1), sz_perm = sizeof(int32_t) * (size_t)T;
    const size_t sz_qw = sizeof(float) * (size_t)n_max * std::max<int64_t>(S, 1);
    const size_t sz_qw2 = resample ? sizeof(float) * (size_t)n_max * std::max<int64_t>(S2, 1) : 0;
    const size_t sz_f = sizeof(float) * std::max<int64_t>(Sf, 1);
    const size_t sz_cost = sizeof(float) * std::max<int64_t>(std::max(S, Sf), 1);
    const size_t sz_flag = std::max<int64_t>(Sf, 1);
    const size_t sz_rank = resample ? sizeof(int32_t) * (size_t)T * K : 0;
    void *w_voffs, *w_voffs2, *w_perm, *w_coffs, *w_qw, *w_qw2, *w_ep, *w_eo, *w_cost, *w_flag, *w_rank;
    if (!noalloc) {
        if ((s = ensure(c, c->voffs, sz_voffs)) != HJCD_OK || (s = ensure(c, c->voffs2, sz_voffs)) != HJCD_OK ||
            (s = ensure(c, c->tperm, sz_perm)) != HJCD_OK || (s = ensure(c, c->coffs, sz_voffs)) != HJCD_OK ||
            (s = ensure(c, c->q_work, sz_qw)) != HJCD_OK ||
            (resample && (s = ensure(c, c->q_work2, sz_qw2)) != HJCD_OK) ||
            (s = ensure(c, c->ep, sz_f)) != HJCD_OK || (s = ensure(c, c->eo, sz_f)) != HJCD_OK ||
            (s = ensure(c, c->cost, sz_cost)) != HJCD_OK || (s = ensure(c, c->flag, sz_flag)) != HJCD_OK ||
            (resample && (s = ensure(c, c->rank, sz_rank)) != HJCD_OK))
            return s;
        w_voffs = c->voffs.p;
        w_voffs2 = c->voffs2.p;
        w_perm = c->tperm.p;
        w_coffs = c->coffs.p;
        w_qw = c->q_work.p;
        w_qw2 = c->q_work2.p;
        w_ep = c->ep.p;
        w_eo = c->eo.p;
        w_cost = c->cost.p;
        w_flag = c->flag.p;
        w_rank = c->rank.p;
    } else {
        // carve this device's static workspace into 256-byte aligned pieces;
        // every piece is written before it is read, so nothing needs clearing
        char* base = (char*)scratch_of(c->device);
        if (!base) return fail(HJCD_E_DEVICE, "no static workspace address for device %d", c->device);
        size_t off = 0;
        auto take = [&](size_t bytes) -> void* {
            void* q = base + off;
            off += (bytes + 255) & ~size_t(255);
            return q;
        };
        w_voffs = take(sz_voffs);
        w_voffs2 = take(sz_voffs);
        w_perm = take(sz_perm);
        w_coffs = take(sz_voffs);
        w_rank = take(sz_rank);
        w_qw = take(sz_qw);
        w_qw2 = take(sz_qw2);
        w_ep = take(sz_f);
        w_eo = take(sz_f);
        w_cost = take(sz_cost);
        w_flag = take(sz_flag);
        if (off > (size_t)HJCD_NOALLOC_SCRATCH_BYTES)
            return fail(HJCD_E_INVALID, "the solve needs %zu bytes of workspace; HJCD_NOALLOC_SCRATCH_BYTES is %zu",
                        off, (size_t)HJCD_NOALLOC_SCRATCH_BYTES);
    }
    StatScope ss{c, st, false};
    if ((s = ss.begin(p->collect_stats, S)) != HJCD_OK) return s;
    {
        Staging sg{c, st, !noalloc};
        if ((s = sg.begin(layout_staging_bytes(T))) != HJCD_OK) return s;
        if ((s = sg.put(w_voffs, voffs.data(), sz_voffs)) != HJCD_OK) return s;
        if (resample && (s = sg.put(w_voffs2, voffs2.data(), sz_voffs)) != HJCD_OK) return s;
        if (!identity && (s = sg.put(w_perm, perm.data(), sz_perm)) != HJCD_OK) return s;
        // caller offsets, for gathering the caller's seeds into the grouped layout
        if (!identity && seeds && (s = sg.put(w_coffs, offs, sz_voffs)) != HJCD_OK) return s;
        if ((s = sg.end()) != HJCD_OK) return s;
    }
    const int64_t* d_voffs = (const int64_t*)w_voffs;
    const int64_t* d_voffs2 = (const int64_t*)w_voffs2;
    const int32_t* d_perm = identity ? nullptr : (const int32_t*)w_perm;
    float* qw = (float*)w_qw;
    const float* q_src = seeds;
    int64_t q_src_stride = S;
    if (seeds && !identity) {
        // grouped copy of the caller's seeds
        HIP_TRY(launch_gather(n_max, T, (const int64_t*)w_coffs, d_voffs, d_perm, S, S, seeds, qw, st));
        q_src = qw;
    }
    const KernelParams kp = kparams(*p);

    auto make_map = [&](int ri, const int64_t* vo, int64_t per_target_base_mul) {
        SeedMap m;
        m.voffs = vo;
        m.tperm = d_perm;
        m.T = T;
        m.tb = rb_tb[ri];
        m.te = rb_tb[ri + 1];
        if (per_target_base_mul >= 0) {
            m.base = (int64_t)m.tb * per_target_base_mul;
            m.Sv = (int64_t)(m.te - m.tb) * per_target_base_mul;
        } else {
            m.base = voffs[m.tb];
            m.Sv = voffs[m.te] - voffs[m.tb];
        }
        m.tkeys = tkeys;
        return m;
    };

    if (!resample) {
        // PO-CCD per robot, then PJ-IK per robot: two kernels, each compiled
        // for its stage alone (fewer live registers than one fused kernel)
        auto stage_args = [&](int ri, bool cd) {
            SolveArgs a{};
            a.rb = robots[ri]->dev;
            a.n = robots[ri]->n;
            a.n_rows = n_max;
            a.map = make_map(ri, d_voffs, -1);
            a.S = S;
            a.targets = targets;
            a.q_in = cd ? q_src : qw;
            a.q_in_stride = cd ? q_src_stride : S;
            a.q_out = qw;
            a.err_p = (float*)w_ep;
            a.err_o = (float*)w_eo;
            a.cost = (float*)w_cost;
            a.traj = nullptr;
            a.init_mode = cd ? (seeds ? INIT_LOAD : INIT_UNIFORM) : INIT_LOAD;
            a.do_cd = cd ? 1 : 0;
            a.do_polish = cd ? 0 : 1;
            a.kp = kp;
            a.counters = ss.counters();
            a.variant = p->polish_variant;
            a.cd_lanes = p->cd_lanes_per_seed == 2 ? 2 : 1;
            return a;
        };
        for (int ri = 0; ri < n_robots; ++ri) {
            const SolveArgs a = stage_args(ri, true);
            if (a.map.Sv > 0) HIP_TRY(launch_solve(a, st));
        }
        if ((s = ss.mark(SS_CD)) != HJCD_OK) return s;
        for (int ri = 0; ri < n_robots; ++ri) {
            const SolveArgs a = stage_args(ri, false);
            if (a.map.Sv > 0) HIP_TRY(launch_solve(a, st));
        }
        if ((s = ss.mark(SS_POLISH)) != HJCD_OK) return s;
    } else {
        for (int ri = 0; ri < n_robots; ++ri) {
            SolveArgs a{};
            a.rb = robots[ri]->dev;
            a.n = robots[ri]->n;
            a.n_rows = n_max;
            a.map = make_map(ri, d_voffs, -1);
            if (a.map.Sv == 0) continue;
            a.S = S;
            a.targets = targets;
            a.q_in = q_src;
            a.q_in_stride = q_src_stride;
            a.q_out = qw;
            a.cost = (float*)w_cost;
            a.init_mode = seeds ? INIT_LOAD : INIT_UNIFORM;
            a.do_cd = 1;
            a.do_polish = 0;
            a.kp = kp;
            a.counters = ss.counters();
            a.cd_lanes = p->cd_lanes_per_seed == 2 ? 2 : 1;
            HIP_TRY(launch_solve(a, st));
        }
        if ((s = ss.mark(SS_CD)) != HJCD_OK) return s;
        HIP_TRY(launch_rank(T, d_voffs, (const float*)w_cost, K, (int32_t*)w_rank, st));
        float* qw2 = (float*)w_qw2;
        for (int ri = 0; ri < n_robots; ++ri) {
            HIP_TRY(launch_replicate(robots[ri]->dev, robots[ri]->n, rb_tb[ri], rb_tb[ri + 1], T, d_voffs, d_perm, S,
                                     qw, (const int32_t*)w_rank, K, Bp, tkeys, p->rng_seed, p->mu, p->sigma,
                                     qw2, st));
        }
        if ((s = ss.mark(SS_RESAMPLE)) != HJCD_OK) return s;
        for (int ri = 0; ri < n_robots; ++ri) {
            SolveArgs a{};
            a.rb = robots[ri]->dev;
            a.n = robots[ri]->n;
            a.n_rows = n_max;
            a.map = make_map(ri, d_voffs2, Bp);
            if (a.map.Sv == 0) continue;
            a.S = S2;
            a.targets = targets;
            a.q_in = qw2;
            a.q_in_stride = S2;
            a.q_out = qw2;
            a.err_p = (float*)w_ep;
            a.err_o = (float*)w_eo;
            a.cost = (float*)w_cost;
            a.init_mode = INIT_LOAD;
            a.do_cd = 0;
            a.do_polish = 1;
            a.kp = kp;
            a.counters = ss.counters();
            a.variant = p->polish_variant;
            a.cd_lanes = p->cd_lanes_per_seed == 2 ? 2 : 1;
            HIP_TRY(launch_solve(a, st));
        }
        if ((s = ss.mark(SS_POLISH)) != HJCD_OK) return s;
    }
    const float* qf = resample ? (const float*)w_qw2 : qw;
    const int64_t* d_vf = resample ? d_voffs2 : d_voffs;
    for (int ri = 0; ri < n_robots; ++ri) {
        const int32_t tb = rb_tb[ri], te = rb_tb[ri + 1];
        const int64_t base = resample ? (int64_t)tb * Bp : voffs[tb];
        const int64_t cnt = resample ? (int64_t)(te - tb) * Bp : voffs[te] - voffs[tb];
        if (cnt == 0) continue;
        CollideArgs a{};
        a.rb = robots[ri]->dev;
        a.n = robots[ri]->n;
        a.S = cnt;
        a.q = qf + base;
        a.q_stride = Sf;
        a.osph = sc ? sc->sph : nullptr;
        a.n_osph = sc ? sc->n_sph : 0;
        a.obox = sc ? sc->box : nullptr;
        a.n_obox = sc ? sc->n_box : 0;
        a.grid = scene_grid(sc, robots[ri]);
        a.flag = (uint8_t*)w_flag + base;
        a.counters = ss.counters();
        a.n_pairs = robots[ri]->host.n_pairs;
        HIP_TRY(launch_collide(a, st));
    }
    if ((s = ss.mark(SS_COLLIDE)) != HJCD_OK) return s;
    SelectArgs a{};
    a.T = T;
    a.offsets = d_vf;
    a.tperm = d_perm;
    a.n = n_max;
    a.n_stride = n_max;
    a.S = Sf;
    a.q = qf;
    a.cost = (const float*)w_cost;
    a.err_p = (const float*)w_ep;
    a.err_o = (const float*)w_eo;
    a.flag = (const uint8_t*)w_flag;
    a.k = p->top_k;
    a.succ_pos = p->succ_pos;
    a.succ_ori = p->succ_ori;
    a.q_out = q_out;
    a.ep_out = ep;
    a.eo_out = eo;
    a.fl_out = flag;
    a.n_free = n_free;
    a.solved = solved;
    a.q_ref = q_ref;
    HIP_TRY(launch_select(a, st));
    if ((s = ss.mark(SS_SELECT)) != HJCD_OK) return s;
    ss.end();
    return HJCD_OK;
}

hjcd_status hjcd_solve(hjcd_ctx c, int32_t n_robots, const hjcd_robot* robots, hjcd_scene sc, int32_t T,
                       const int32_t* robot_of_target, const float* targets, const int64_t* offs,
                       const uint32_t* tkeys, const float* seeds, const hjcd_params* p, float* q_out, float* ep,
                       float* eo, uint8_t* flag, int32_t* n_free, uint8_t* solved, void* stream) {
    return solve_impl(c, n_robots, robots, sc, T, robot_of_target, targets, offs, tkeys, seeds, p, q_out, ep, eo, flag,
                      n_free, solved, stream, false);
}

hjcd_status hjcd_solve_near(hjcd_ctx c, int32_t n_robots, const hjcd_robot* robots, hjcd_scene sc, int32_t T,
                            const int32_t* robot_of_target, const float* targets, const int64_t* offs,
                            const uint32_t* tkeys, const float* seeds, const hjcd_params* p, const float* q_ref,
                            float* q_out, float* ep, float* eo, uint8_t* flag, int32_t* n_free, uint8_t* solved,
                            void* stream) {
    if (T > 0 && !q_ref) return fail(HJCD_E_INVALID, "q_ref is required");
    return solve_impl(c, n_robots, robots, sc, T, robot_of_target, targets, offs, tkeys, seeds, p, q_out, ep, eo, flag,
                      n_free, solved, stream, false, q_ref);
}

hjcd_status hjcd_solve_noalloc(hjcd_ctx c, int32_t n_robots, const hjcd_robot* robots, hjcd_scene sc, int32_t T,
                               const int32_t* robot_of_target, const float* targets, const int64_t* offs,
                               const uint32_t* tkeys, const float* seeds, const hjcd_params* p, float* q_out,
                               float* ep, float* eo, uint8_t* flag, int32_t* n_free, uint8_t* solved, void* stream) {
    return solve_impl(c, n_robots, robots, sc, T, robot_of_target, targets, offs, tkeys, seeds, p, q_out, ep, eo, flag,
                      n_free, solved, stream, true);
}

hjcd_status hjcd_get_stats(hjcd_ctx c, hjcd_stats* out) {
    hjcd_status s;
    if (!out) return fail(HJCD_E_INVALID, "out is NULL");
    if ((s = check_ctx(c)) != HJCD_OK) return s;
    if ((s = bind(c)) != HJCD_OK) return s;
    if (c->stats_pending) {
        if (c->ev_used > 0) HIP_TRY(hipEventSynchronize(c->ev[c->ev_used - 1]));
        for (int i = 1; i < c->ev_used; ++i) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, c->ev[i - 1], c->ev[i]));
            switch (c->ev_stage[i]) {
                case SS_INIT: c->stats.ms_init += ms; break;
                case SS_CD: c->stats.ms_cd += ms; break;
                case SS_RESAMPLE: c->stats.ms_resample += ms; break;
                case SS_POLISH: c->stats.ms_polish += ms; break;
                case SS_COLLIDE: c->stats.ms_collide += ms; break;
                case SS_SELECT: c->stats.ms_select += ms; break;
                default: break;
            }
        }
        if (c->ev_used > 1) HIP_TRY(hipEventElapsedTime(&c->stats.ms_total, c->ev[0], c->ev[c->ev_used - 1]));
        unsigned long long h[16] = {};
        HIP_TRY(hipMemcpy(h, c->counters.p, sizeof(h), hipMemcpyDeviceToHost));
        c->stats.cd_iters = h[0];
        c->stats.cd_perturb = h[1];
        c->stats.pol_iters = h[2];
        c->stats.pol_trials = h[3];
        c->stats.pol_dogleg = h[4];
        c->stats.pol_single = h[5];
        c->stats.pol_perturb = h[6];
        c->stats.coll_coarse = h[7];
        c->stats.coll_fine = h[8];
        c->stats_pending = false;
    }
    *out = c->stats;
    return HJCD_OK;
}

hjcd_status hjcd_philox(hjcd_ctx c, const uint32_t ctr[4], const uint32_t key[2], int64_t count, uint32_t* out,
                        void* stream) {
    hjcd_status s;
    if (!ctr || !key) return fail(HJCD_E_INVALID, "ctr and key are required");
    if (count < 0) return fail(HJCD_E_INVALID, "count must be >= 0");
    if (count > 0 && !out) return fail(HJCD_E_INVALID, "out is NULL");
    if ((s = check_ctx(c)) != HJCD_OK) return s;
    if ((s = bind(c)) != HJCD_OK) return s;
    HIP_TRY(launch_philox(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1], count, out, (hipStream_t)stream));
    return HJCD_OK;
}

}  // extern "C"
