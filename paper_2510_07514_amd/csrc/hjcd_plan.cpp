// Reusable plans of libhjcd: one uneven batch captured into a hipGraph, with
// the per-seed kernel's launch shape autotuned per robot.  See the plans
// section of include/hjcd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/hjcd.h"
#include "hjcd_internal.hpp"
#include "hjcd_launch.hpp"

using namespace hjcd;

struct hjcd_plan_s {
    hjcd_ctx ctx = nullptr;
    int device = 0;
    int32_t n_robots = 0;
    hjcd_robot robots[HJCD_MAX_ROBOTS] = {};
    hjcd_scene scene = nullptr;
    int32_t T = 0;
    int n_max = 0;
    int64_t S = 0;
    TargetGroups grp;
    hjcd_params params{};
    KernelParams kp{};
    // caller buffers
    const float* targets = nullptr;
    const uint32_t* tkeys = nullptr;
    const float* seeds = nullptr;
    float *q_out = nullptr, *ep_out = nullptr, *eo_out = nullptr;
    uint8_t* fl_out = nullptr;
    int32_t* n_free = nullptr;
    uint8_t* solved = nullptr;
    // plan-owned device buffers
    int64_t* d_voffs = nullptr;
    int64_t* d_coffs = nullptr;
    int32_t* d_perm = nullptr;
    float* qw = nullptr;
    float* ep = nullptr;
    float* eo = nullptr;
    float* cost = nullptr;
    uint8_t* fl = nullptr;
    // top-K and replication between the stages (resample_K > 0): per target
    // B' = floor(B/K) K polished slots at t B' (grouped order), their own
    // joint, cost and offset arrays (a robot's branch ranks its CD costs
    // while another branch polishes, so the two stages never share one)
    bool resample = false;
    int32_t K = 0, Bp = 0;
    int64_t S2 = 0;
    int64_t* d_voffs2 = nullptr;
    int32_t* rank = nullptr;
    float* qw2 = nullptr;
    float* cost2 = nullptr;
    hjcd_tune_choice choice[HJCD_MAX_ROBOTS] = {};
    hipStream_t main = nullptr;
    hipStream_t side[HJCD_MAX_ROBOTS] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[HJCD_MAX_ROBOTS] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

template <typename T>
hjcd_status dalloc(T** p, size_t count) {
    if (hipMalloc((void**)p, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess)
        return fail(HJCD_E_NOMEM, "plan device allocation of %zu bytes failed", sizeof(T) * count);
    return HJCD_OK;
}

void plan_free(hjcd_plan p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    void* bufs[] = {p->d_voffs, p->d_coffs, p->d_perm, p->qw, p->ep, p->eo, p->cost, p->fl,
                    p->d_voffs2, p->rank, p->qw2, p->cost2};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    for (int i = 0; i < HJCD_MAX_ROBOTS; ++i) {
        if (p->side[i]) (void)hipStreamDestroy(p->side[i]);
        if (p->join[i]) (void)hipEventDestroy(p->join[i]);
    }
    if (p->fork) (void)hipEventDestroy(p->fork);
    if (p->main) (void)hipStreamDestroy(p->main);
}

SolveArgs solve_args(hjcd_plan p, int ri, int stage) {
    SolveArgs a{};
    a.rb = p->robots[ri]->dev;
    a.n = p->robots[ri]->n;
    a.n_rows = p->n_max;
    SeedMap m{};
    m.voffs = p->d_voffs;
    m.tperm = p->grp.identity ? nullptr : p->d_perm;
    m.T = p->T;
    m.tb = p->grp.rb_tb[ri];
    m.te = p->grp.rb_tb[ri + 1];
    m.base = p->grp.voffs[m.tb];
    m.Sv = p->grp.voffs[m.te] - p->grp.voffs[m.tb];
    m.tkeys = p->tkeys;
    a.map = m;
    a.S = p->S;
    a.targets = p->targets;
    // stage 0: PO-CCD, 1: PJ-IK on the CD results
    const bool gathered = p->seeds && !p->grp.identity;
    a.q_in = stage == 1 || gathered ? p->qw : p->seeds;
    a.q_in_stride = p->S;
    a.q_out = p->qw;
    a.err_p = p->ep;
    a.err_o = p->eo;
    a.cost = p->cost;
    if (stage == 0 && p->resample) {
        // only the CD costs are read (by the ranking); the error arrays hold
        // the polished slots, which another robot's branch may be writing
        a.err_p = nullptr;
        a.err_o = nullptr;
    }
    if (stage == 1 && p->resample) {
        // PJ-IK on the replicated slots of this robot's targets
        a.map.voffs = p->d_voffs2;
        a.map.base = (int64_t)m.tb * p->Bp;
        a.map.Sv = (int64_t)(m.te - m.tb) * p->Bp;
        a.S = p->S2;
        a.q_in = p->qw2;
        a.q_in_stride = p->S2;
        a.q_out = p->qw2;
        a.cost = p->cost2;
    }
    a.traj = nullptr;
    a.init_mode = (stage == 1 || p->seeds) ? INIT_LOAD : INIT_UNIFORM;
    a.do_cd = stage == 0;
    a.do_polish = stage == 1;
    a.kp = p->kp;
    a.counters = nullptr;
    a.variant = p->choice[ri].variant;
    a.block_threads = stage == 1 ? p->choice[ri].block_threads : 256;
    a.cd_lanes = p->choice[ri].cd_lanes;
    return a;
}

CollideArgs collide_args(hjcd_plan p, int ri) {
    const int32_t tb = p->grp.rb_tb[ri], te = p->grp.rb_tb[ri + 1];
    const int64_t base = p->resample ? (int64_t)tb * p->Bp : p->grp.voffs[tb];
    CollideArgs a{};
    a.rb = p->robots[ri]->dev;
    a.n = p->robots[ri]->n;
    a.S = p->resample ? (int64_t)(te - tb) * p->Bp : p->grp.voffs[te] - base;
    a.q = (p->resample ? p->qw2 : p->qw) + base;
    a.q_stride = p->resample ? p->S2 : p->S;
    a.osph = p->scene ? p->scene->sph : nullptr;
    a.n_osph = p->scene ? p->scene->n_sph : 0;
    a.obox = p->scene ? p->scene->box : nullptr;
    a.n_obox = p->scene ? p->scene->n_box : 0;
    a.grid = scene_grid(p->scene, p->robots[ri]);
    a.flag = p->fl + base;
    a.counters = nullptr;
    a.n_pairs = p->robots[ri]->host.n_pairs;
    return a;
}

// Top-K ranking of robot ri's targets by their CD costs and the noisy
// replication of the K best into the polished slots (Alg. HJCD-IK).
hipError_t launch_between(hjcd_plan p, int ri, hipStream_t st) {
    const int32_t tb = p->grp.rb_tb[ri], te = p->grp.rb_tb[ri + 1];
    hipError_t e = launch_rank(te - tb, p->d_voffs + tb, p->cost, p->K, p->rank + (int64_t)tb * p->K, st);
    if (e != hipSuccess) return e;
    return launch_replicate(p->robots[ri]->dev, p->robots[ri]->n, tb, te, p->T, p->d_voffs,
                            p->grp.identity ? nullptr : p->d_perm, p->S, p->qw, p->rank, p->K, p->Bp, p->tkeys,
                            p->params.rng_seed, p->params.mu, p->params.sigma, p->qw2, st);
}

// The whole solve on `st`: per robot, solve then collision on a branch of
// its own; the selection after every branch has joined.
hjcd_status enqueue(hjcd_plan p, hipStream_t st) {
    if (p->seeds && !p->grp.identity)
        HIP_TRY(launch_gather(p->n_max, p->T, p->d_coffs, p->d_voffs, p->d_perm, p->S, p->S, p->seeds, p->qw, st));
    HIP_TRY(hipEventRecord(p->fork, st));
    for (int ri = 0; ri < p->n_robots; ++ri) {
        if (p->choice[ri].seeds == 0) continue;
        HIP_TRY(hipStreamWaitEvent(p->side[ri], p->fork, 0));
        HIP_TRY(launch_solve(solve_args(p, ri, 0), p->side[ri]));
        if (p->resample) HIP_TRY(launch_between(p, ri, p->side[ri]));
        HIP_TRY(launch_solve(solve_args(p, ri, 1), p->side[ri]));
        HIP_TRY(launch_collide(collide_args(p, ri), p->side[ri]));
        HIP_TRY(hipEventRecord(p->join[ri], p->side[ri]));
        HIP_TRY(hipStreamWaitEvent(st, p->join[ri], 0));
    }
    SelectArgs a{};
    a.T = p->T;
    a.offsets = p->resample ? p->d_voffs2 : p->d_voffs;
    a.tperm = p->grp.identity ? nullptr : p->d_perm;
    a.n = p->n_max;
    a.n_stride = p->n_max;
    a.S = p->resample ? p->S2 : p->S;
    a.q = p->resample ? p->qw2 : p->qw;
    a.cost = p->resample ? p->cost2 : p->cost;
    a.err_p = p->ep;
    a.err_o = p->eo;
    a.flag = p->fl;
    a.k = p->params.top_k;
    a.succ_pos = p->params.succ_pos;
    a.succ_ori = p->params.succ_ori;
    a.q_out = p->q_out;
    a.ep_out = p->ep_out;
    a.eo_out = p->eo_out;
    a.fl_out = p->fl_out;
    a.n_free = p->n_free;
    a.solved = p->solved;
    HIP_TRY(launch_select(a, st));
    return HJCD_OK;
}

// Time each candidate launch shape of robot ri's PJ-IK kernel (the variant
// and workgroup size apply to it; PO-CCD keeps the default shape) on the
// plan's buffers, one warm-up and two timed launches, and keep the fastest.
hjcd_status autotune(hjcd_plan p, int ri, float* qs) {
    static const int kBlocks[] = {64, 128, 256};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    // PO-CCD lanes per seed (robots of 9 joints or more): one warm-up and two
    // timed launches each; both write the same results into qw
    {
        const int nl = p->robots[ri]->n >= 9 ? 2 : 1;
        float best_cd = 3.4e38f;
        int best_lanes = 1;
        // caller seeds regrouped into qw are updated in place by PO-CCD: they
        // are gathered again before every launch (the gathers are timed too)
        const bool gathered = p->seeds && !p->grp.identity;
        auto cd_once = [&]() -> hipError_t {
            if (gathered) {
                const hipError_t g = launch_gather(p->n_max, p->T, p->d_coffs, p->d_voffs, p->d_perm, p->S, p->S,
                                                   p->seeds, p->qw, p->main);
                if (g != hipSuccess) return g;
            }
            return launch_solve(solve_args(p, ri, 0), p->main);
        };
        for (int l = 1; l <= nl; ++l) {
            p->choice[ri].cd_lanes = l;
            HIP_TRY(cd_once());
            HIP_TRY(hipEventRecord(e0, p->main));
            for (int r = 0; r < 2; ++r) HIP_TRY(cd_once());
            HIP_TRY(hipEventRecord(e1, p->main));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            ms *= 0.5f;
            if (ms < best_cd) {
                best_cd = ms;
                best_lanes = l;
            }
        }
        p->choice[ri].cd_lanes = best_lanes;
        p->choice[ri].cd_ms = best_cd;
    }
    hjcd_tune_choice best = p->choice[ri];
    best.ms = 3.4e38f;
    // PO-CCD once more from the original seeds; every timed PJ-IK launch then
    // polishes the same CD results (read from qw) into the scratch rows `qs`
    if (p->seeds && !p->grp.identity)
        HIP_TRY(launch_gather(p->n_max, p->T, p->d_coffs, p->d_voffs, p->d_perm, p->S, p->S, p->seeds, p->qw,
                              p->main));
    HIP_TRY(launch_solve(solve_args(p, ri, 0), p->main));
    if (p->resample) HIP_TRY(launch_between(p, ri, p->main));
    for (int v = 0; v < 2; ++v) {
        for (int bt : kBlocks) {
            p->choice[ri].variant = v;
            p->choice[ri].block_threads = bt;
            SolveArgs a = solve_args(p, ri, 1);
            a.q_out = qs;
            HIP_TRY(launch_solve(a, p->main));
            HIP_TRY(hipEventRecord(e0, p->main));
            for (int r = 0; r < 2; ++r) HIP_TRY(launch_solve(a, p->main));
            HIP_TRY(hipEventRecord(e1, p->main));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            ms *= 0.5f;
            if (ms < best.ms) {
                best = p->choice[ri];
                best.ms = ms;
            }
        }
    }
    p->choice[ri] = best;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return HJCD_OK;
}

}  // namespace

extern "C" {

hjcd_status hjcd_plan_create(hjcd_ctx c, int32_t n_robots, const hjcd_robot* robots, hjcd_scene sc, int32_t T,
                             const int32_t* robot_of_target, const float* targets, const int64_t* offs,
                             const uint32_t* tkeys, const float* seeds, const hjcd_params* params, float* q_out,
                             float* err_p, float* err_o, uint8_t* flag, int32_t* n_free, uint8_t* solved,
                             int32_t tune, void* stream, hjcd_plan* out) {
    if (!out) return fail(HJCD_E_INVALID, "out is NULL");
    *out = nullptr;
    hjcd_status s;
    if (n_robots < 1 || n_robots > HJCD_MAX_ROBOTS || !robots)
        return fail(HJCD_E_INVALID, "need 1..%d robots", HJCD_MAX_ROBOTS);
    if ((s = check_params(params)) != HJCD_OK) return s;
    if ((s = check_offsets(T, offs)) != HJCD_OK) return s;
    if (T < 1) return fail(HJCD_E_INVALID, "a plan needs T >= 1");
    if (params->resample_K > 0)
        for (int32_t t = 0; t < T; ++t)
            if (offs[t + 1] == offs[t]) return fail(HJCD_E_INVALID, "target %d has no seeds to resample", t);
    if (robot_of_target)
        for (int32_t t = 0; t < T; ++t)
            if (robot_of_target[t] < 0 || robot_of_target[t] >= n_robots)
                return fail(HJCD_E_INVALID, "robot_of_target[%d] = %d out of range", t, robot_of_target[t]);
    if (!targets || !q_out || !err_p || !err_o || !flag || !n_free || !solved)
        return fail(HJCD_E_INVALID, "targets and outputs are required");
    if (!c) return fail(HJCD_E_INVALID, "ctx is NULL");
    for (int i = 0; i < n_robots; ++i)
        if ((s = check_robot(c, robots[i])) != HJCD_OK) return s;
    if (sc && sc->ctx != c) return fail(HJCD_E_INVALID, "scene belongs to another context");
    HIP_TRY(hipSetDevice(c->device));

    auto* p = new hjcd_plan_s();
    auto bail = [&](hjcd_status st) {
        plan_free(p);
        delete p;
        return st;
    };
    p->ctx = c;
    p->device = c->device;
    p->n_robots = n_robots;
    for (int i = 0; i < n_robots; ++i) p->robots[i] = robots[i];
    p->scene = sc;
    p->T = T;
    for (int i = 0; i < n_robots; ++i) p->n_max = std::max(p->n_max, robots[i]->n);
    p->S = offs[T];
    p->params = *params;
    p->params.collect_stats = 0;
    p->kp = kparams(p->params);
    p->targets = targets;
    p->tkeys = tkeys;
    p->seeds = seeds;
    p->q_out = q_out;
    p->ep_out = err_p;
    p->eo_out = err_o;
    p->fl_out = flag;
    p->n_free = n_free;
    p->solved = solved;
    group_targets(n_robots, T, robot_of_target, offs, p->grp);
    for (int ri = 0; ri < n_robots; ++ri) {
        p->choice[ri].variant = params->polish_variant;
        p->choice[ri].block_threads = 64;  // hjcd_solve's PJ-IK default
        p->choice[ri].cd_lanes = robots[ri]->n >= 9 && params->cd_lanes_per_seed == 2 ? 2 : 1;
        p->choice[ri].cd_ms = 0.f;
        p->choice[ri].ms = 0.f;
        p->choice[ri].seeds = p->grp.voffs[p->grp.rb_tb[ri + 1]] - p->grp.voffs[p->grp.rb_tb[ri]];
    }
    p->resample = params->resample_K > 0;
    p->K = p->resample ? params->resample_K : 0;
    p->Bp = p->resample ? (params->resample_B / p->K) * p->K : 0;
    p->S2 = (int64_t)T * p->Bp;
    const size_t S1 = (size_t)std::max<int64_t>(p->S, 1);
    const size_t Sf = (size_t)std::max<int64_t>(p->resample ? p->S2 : p->S, 1);  // slots of the final stage
    if ((s = dalloc(&p->d_voffs, T + 1)) != HJCD_OK || (s = dalloc(&p->d_coffs, T + 1)) != HJCD_OK ||
        (s = dalloc(&p->d_perm, T)) != HJCD_OK || (s = dalloc(&p->qw, (size_t)p->n_max * S1)) != HJCD_OK ||
        (s = dalloc(&p->ep, std::max(S1, Sf))) != HJCD_OK || (s = dalloc(&p->eo, std::max(S1, Sf))) != HJCD_OK ||
        (s = dalloc(&p->cost, S1)) != HJCD_OK || (s = dalloc(&p->fl, Sf)) != HJCD_OK)
        return bail(s);
    std::vector<int64_t> voffs2;
    if (p->resample) {
        if ((s = dalloc(&p->d_voffs2, T + 1)) != HJCD_OK || (s = dalloc(&p->rank, (size_t)T * p->K)) != HJCD_OK ||
            (s = dalloc(&p->qw2, (size_t)p->n_max * Sf)) != HJCD_OK || (s = dalloc(&p->cost2, Sf)) != HJCD_OK)
            return bail(s);
        voffs2.resize(T + 1);
        for (int32_t b = 0; b <= T; ++b) voffs2[b] = (int64_t)b * p->Bp;
    }
    if (hipStreamCreateWithFlags(&p->main, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) != hipSuccess)
        return bail(fail(HJCD_E_DEVICE, "plan stream / event creation failed"));
    for (int ri = 0; ri < n_robots; ++ri)
        if (hipStreamCreateWithFlags(&p->side[ri], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&p->join[ri], hipEventDisableTiming) != hipSuccess)
            return bail(fail(HJCD_E_DEVICE, "plan stream / event creation failed"));
    // the batch layout, uploaded once
    hipStream_t ust = p->main;
    if (hipMemcpyAsync(p->d_voffs, p->grp.voffs.data(), sizeof(int64_t) * (T + 1), hipMemcpyHostToDevice, ust) !=
            hipSuccess ||
        hipMemcpyAsync(p->d_coffs, offs, sizeof(int64_t) * (T + 1), hipMemcpyHostToDevice, ust) != hipSuccess ||
        (!p->grp.identity &&
         hipMemcpyAsync(p->d_perm, p->grp.perm.data(), sizeof(int32_t) * T, hipMemcpyHostToDevice, ust) !=
             hipSuccess) ||
        (p->resample &&
         hipMemcpyAsync(p->d_voffs2, voffs2.data(), sizeof(int64_t) * (T + 1), hipMemcpyHostToDevice, ust) !=
             hipSuccess) ||
        hipStreamSynchronize(ust) != hipSuccess)
        return bail(fail(HJCD_E_DEVICE, "plan upload failed"));
    // the caller's stream (NULL: the default stream) may still be producing
    // the inputs the autotuner reads
    {
        hipEvent_t ready;
        if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess)
            return bail(fail(HJCD_E_DEVICE, "plan event creation failed"));
        const bool ok = hipEventRecord(ready, (hipStream_t)stream) == hipSuccess &&
                        hipStreamWaitEvent(p->main, ready, 0) == hipSuccess;
        (void)hipEventDestroy(ready);
        if (!ok) return bail(fail(HJCD_E_DEVICE, "plan stream ordering failed"));
    }
    if (tune) {
        if (p->seeds && !p->grp.identity &&
            launch_gather(p->n_max, T, p->d_coffs, p->d_voffs, p->d_perm, p->S, p->S, p->seeds, p->qw, p->main) !=
                hipSuccess)
            return bail(fail(HJCD_E_DEVICE, "seed gather failed"));
        float* qs = nullptr;
        if ((s = dalloc(&qs, (size_t)p->n_max * Sf)) != HJCD_OK) return bail(s);
        for (int ri = 0; ri < n_robots && s == HJCD_OK; ++ri)
            if (p->choice[ri].seeds > 0) s = autotune(p, ri, qs);
        (void)hipStreamSynchronize(p->main);
        (void)hipFree(qs);
        if (s != HJCD_OK) return bail(s);
    }
    // capture
    if (hipStreamBeginCapture(p->main, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return bail(fail(HJCD_E_DEVICE, "graph capture could not start"));
    s = enqueue(p, p->main);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(p->main, &g);
    if (s != HJCD_OK) {
        if (g) (void)hipGraphDestroy(g);
        return bail(s);
    }
    if (ec != hipSuccess) return bail(fail(HJCD_E_DEVICE, "graph capture failed: %s", hipGetErrorString(ec)));
    p->graph = g;
    if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
        return bail(fail(HJCD_E_DEVICE, "graph instantiation failed"));
    *out = p;
    return HJCD_OK;
}

hjcd_status hjcd_plan_execute(hjcd_plan p, void* stream) {
    if (!p) return fail(HJCD_E_INVALID, "plan is NULL");
    HIP_TRY(hipSetDevice(p->device));
    HIP_TRY(hipGraphLaunch(p->exec, (hipStream_t)stream));
    return HJCD_OK;
}

hjcd_status hjcd_plan_choice(hjcd_plan p, int32_t robot, hjcd_tune_choice* out) {
    if (!p || !out) return fail(HJCD_E_INVALID, "plan and out are required");
    if (robot < 0 || robot >= p->n_robots) return fail(HJCD_E_INVALID, "robot %d out of range", robot);
    *out = p->choice[robot];
    return HJCD_OK;
}

void hjcd_plan_destroy(hjcd_plan p) {
    if (!p) return;
    (void)hipSetDevice(p->device);
    if (p->main) (void)hipStreamSynchronize(p->main);
    (void)hipDeviceSynchronize();
    plan_free(p);
    delete p;
}

}  // extern "C"
