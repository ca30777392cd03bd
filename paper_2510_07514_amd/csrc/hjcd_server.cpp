// Serving loop of libhjcd: continuous batching of IK requests over resident
// seed slots (HJCD_SERVE_BATCHED) and the one-request-at-a-time comparison
// form (HJCD_SERVE_PLAIN).  See the serving section of include/hjcd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/hjcd.h"
#include "hjcd_internal.hpp"
#include "hjcd_launch.hpp"

using namespace hjcd;

namespace {

using Clock = std::chrono::steady_clock;

// Philox target key of target i of a request: tag + i, request-local, so a
// request draws the same numbers alone and in any mix, and a request with
// tag t0 draws what targets t0 .. t0 + n - 1 of an hjcd_solve batch draw.
uint32_t target_key(uint64_t tag, int i) { return (uint32_t)(tag + (uint64_t)i); }

struct Request {
    int64_t id = 0;
    uint64_t tag = 0;
    int32_t n_targets = 0, M = 0;
    double arrival = 0, admitted = -1, done = -1;
    std::vector<float> poses;  // [n_targets][7]
    // placement (batched mode)
    int64_t base = -1;
    int32_t nblocks = 0;
    int32_t tbl0 = -1;
    int stage = SERVE_CD;
    int iter = 0;
    bool fuse = false;  // this step ends its PO-CCD and runs its first PJ-IK chunk
    // results
    std::vector<int32_t> status;  // per target: 0 running, 1 solved, 2 finished
    std::vector<float> res;       // [n_targets][n + 3]
    int32_t n_done = 0, n_solved = 0;
};

// First-fit allocator of contiguous runs over a fixed number of units.
struct RunAllocator {
    std::vector<uint8_t> used;
    int64_t free_units = 0;
    void init(int64_t n) {
        used.assign((size_t)n, 0);
        free_units = n;
    }
    int64_t alloc(int64_t k) {
        if (k <= 0 || k > free_units) return -1;
        int64_t run = 0;
        for (int64_t i = 0; i < (int64_t)used.size(); ++i) {
            run = used[(size_t)i] ? 0 : run + 1;
            if (run == k) {
                const int64_t b = i - k + 1;
                for (int64_t j = b; j <= i; ++j) used[(size_t)j] = 1;
                free_units -= k;
                return b;
            }
        }
        return -1;
    }
    void release(int64_t b, int64_t k) {
        for (int64_t j = b; j < b + k; ++j) used[(size_t)j] = 0;
        free_units += k;
    }
};

template <typename T>
T* dev_alloc(size_t count, bool& ok) {
    void* p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc(&p, sizeof(T) * count) != hipSuccess) {
        ok = false;
        return nullptr;
    }
    return (T*)p;
}

}  // namespace

struct hjcd_server_s {
    hjcd_ctx ctx = nullptr;
    int device = 0;
    hjcd_robot robot = nullptr;
    hjcd_scene scene = nullptr;
    hjcd_params params{};
    hjcd_server_config cfg{};
    int n = 0;
    hipStream_t stream = nullptr;
    // resident state (batched)
    int64_t C = 0;     // slots
    int32_t Tc = 0;    // target table entries
    ServeState st{};
    float* d_pose = nullptr;
    uint32_t* d_tkey = nullptr;
    // step pipelines: each has its stream, its per-step transfers (one
    // host-to-device upload of every list the step's kernels read, one
    // device-to-host readback of the decisions), its requests and the event
    // of its step in flight.  A request stays with the pipeline that admitted
    // it; pipelines run their steps concurrently, so a request that arrives
    // while one step runs starts on a free pipeline instead of waiting.
    struct Pipe {
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        char* d_up = nullptr;
        char* h_up = nullptr;
        char* d_down = nullptr;
        char* h_down = nullptr;
        bool busy = false;
        std::vector<std::unique_ptr<Request>> active;
    };
    std::vector<Pipe> pipes;  // hjcd_server_config::pipelines of them (batched mode)
    size_t up_cap = 0;
    size_t down_cap = 0;
    // plain mode staging
    float* h_pose = nullptr;
    uint32_t* h_tkey = nullptr;
    // plain mode buffers
    int64_t plain_cap_seeds = 0;
    int32_t plain_cap_targets = 0;
    float *p_targets = nullptr, *p_q = nullptr, *p_ep = nullptr, *p_eo = nullptr;
    uint8_t *p_fl = nullptr, *p_sv = nullptr;
    int32_t* p_nf = nullptr;
    uint32_t* p_keys = nullptr;
    // scheduling
    RunAllocator blocks, tslots;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::unique_ptr<Request>> pending;  // by arrival
    std::map<int64_t, std::unique_ptr<Request>> finished;
    std::deque<int64_t> unpolled;
    std::vector<double> latencies;
    int64_t next_id = 1;
    std::thread worker;
    std::atomic<bool> stop{false};
    bool started = false;
    Clock::time_point epoch;
    // stats
    hjcd_server_stats stats{};
    double resident_sum = 0;
    std::string worker_error;

    double now() const { return std::chrono::duration<double>(Clock::now() - epoch).count(); }
};

namespace {

size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

hjcd_status server_alloc_batched(hjcd_server s) {
    bool ok = true;
    const int64_t C = s->C;
    const int32_t Tc = s->Tc;
    const int64_t nb_max = C / 64;
    s->st.q = dev_alloc<float>((size_t)s->n * C, ok);
    s->st.sstate = dev_alloc<uint8_t>(C, ok);
    s->st.slot_target = dev_alloc<int32_t>(C, ok);
    s->st.slot_m = dev_alloc<uint32_t>(C, ok);
    s->st.err_p = dev_alloc<float>(C, ok);
    s->st.err_o = dev_alloc<float>(C, ok);
    s->st.cost = dev_alloc<float>(C, ok);
    s->st.C = C;
    s->d_pose = dev_alloc<float>((size_t)7 * Tc, ok);
    s->d_tkey = dev_alloc<uint32_t>(Tc, ok);
    s->st.tgt_pose = s->d_pose;
    s->st.tgt_key = s->d_tkey;
    s->st.Tc = Tc;
    s->up_cap = align16(sizeof(ServeAdmit) * Tc) + align16(sizeof(float) * 7 * Tc) +
                3 * align16(sizeof(ServeBlock) * nb_max) + align16(sizeof(int32_t) * nb_max) +
                3 * align16(sizeof(int32_t) * Tc) + align16(sizeof(int64_t) * Tc);
    s->down_cap = align16(sizeof(int32_t) * Tc) + align16(sizeof(float) * Tc * (s->n + 3));
    s->pipes.resize(s->cfg.pipelines);
    for (auto& P : s->pipes) {
        P.d_up = dev_alloc<char>(s->up_cap, ok);
        P.d_down = dev_alloc<char>(s->down_cap, ok);
    }
    if (!ok) return fail(HJCD_E_NOMEM, "server device allocation failed (%lld slots)", (long long)C);
    for (auto& P : s->pipes) {
        if (hipHostMalloc((void**)&P.h_up, s->up_cap, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&P.h_down, s->down_cap, hipHostMallocDefault) != hipSuccess)
            return fail(HJCD_E_NOMEM, "server pinned host allocation failed");
        if (hipStreamCreateWithFlags(&P.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&P.done, hipEventDisableTiming) != hipSuccess)
            return fail(HJCD_E_DEVICE, "server stream creation failed");
    }
    // every slot starts dead
    HIP_TRY(hipMemsetAsync(s->st.sstate, 0, C, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->blocks.init(nb_max);
    s->tslots.init(Tc);
    return HJCD_OK;
}

void server_free(hjcd_server s) {
    for (auto& P : s->pipes) {
        if (P.stream) (void)hipStreamSynchronize(P.stream);
        if (P.d_up) (void)hipFree(P.d_up);
        if (P.d_down) (void)hipFree(P.d_down);
        if (P.h_up) (void)hipHostFree(P.h_up);
        if (P.h_down) (void)hipHostFree(P.h_down);
        if (P.done) (void)hipEventDestroy(P.done);
        if (P.stream) (void)hipStreamDestroy(P.stream);
    }
    void* dptr[] = {s->st.q,    s->st.sstate, s->st.slot_target, s->st.slot_m, s->st.err_p, s->st.err_o,
                    s->st.cost, s->d_pose,    s->d_tkey,         s->p_targets, s->p_q,     s->p_ep,
                    s->p_eo,    s->p_fl,      s->p_sv,           s->p_nf,      s->p_keys};
    for (void* p : dptr)
        if (p) (void)hipFree(p);
    void* hptr[] = {s->h_pose, s->h_tkey};
    for (void* p : hptr)
        if (p) (void)hipHostFree(p);
    if (s->stream) (void)hipStreamDestroy(s->stream);
}

void finish_request(hjcd_server s, std::unique_ptr<Request> r) {
    // caller holds s->mu
    s->stats.completed++;
    s->stats.targets_done += r->n_targets;
    s->stats.targets_solved += r->n_solved;
    s->stats.last_done_s = std::max(s->stats.last_done_s, r->done);
    s->latencies.push_back((r->done - r->arrival) * 1e3);
    s->unpolled.push_back(r->id);
    s->finished[r->id] = std::move(r);
    s->cv.notify_all();
}

// ---------------------------------------------------------------------------
// batched worker
// ---------------------------------------------------------------------------
// Bump allocator over the pinned upload arena; device address = same offset
// in d_up.
struct Arena {
    char* h;
    char* d;
    size_t off = 0;
    template <typename T>
    T* take(size_t count, T** dev) {
        T* p = (T*)(h + off);
        *dev = (T*)(d + off);
        off += align16(sizeof(T) * count);
        return p;
    }
};

// Launches one step of pipeline P: admits the arrived requests that fit
// (they join P), uploads the step's lists and enqueues its kernels and the
// decision readback on P's stream, then records P's event.  Nothing waits.
hjcd_status launch_step(hjcd_server s, hjcd_server_s::Pipe& P) {
    const int n = s->n;
    const hjcd_params& p = s->params;
    const int c = s->cfg.chunk_iters;
    const int64_t nb_max = s->C / 64;
    const int32_t Tc = s->Tc;
    Arena ar{P.h_up, P.d_up};
    ServeAdmit* d_adm;
    float* d_upose;
    ServeAdmit* h_adm = ar.take<ServeAdmit>(Tc, &d_adm);
    float* h_upose = ar.take<float>((size_t)7 * Tc, &d_upose);
    // 1. admission of arrived requests that fit, in arrival order
    int32_t n_adm = 0, n_up = 0;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        const double t = s->now();
        while (!s->pending.empty() && s->pending.front()->arrival <= t) {
            Request* r = s->pending.front().get();
            const int64_t seeds = (int64_t)r->n_targets * r->M;
            const int64_t nb = (seeds + 63) / 64;
            const int64_t b = s->blocks.alloc(nb);
            if (b < 0) break;
            const int64_t tb = s->tslots.alloc(r->n_targets);
            if (tb < 0) {
                s->blocks.release(b, nb);
                break;
            }
            r->base = b * 64;
            r->nblocks = (int32_t)nb;
            r->tbl0 = (int32_t)tb;
            r->admitted = t;
            r->status.assign(r->n_targets, 0);
            r->res.assign((size_t)r->n_targets * (n + 3), 0.f);
            std::memcpy(h_upose + (size_t)n_up * 7, r->poses.data(), sizeof(float) * 7 * r->n_targets);
            h_adm[n_adm++] = ServeAdmit{r->base, r->n_targets, r->M, r->nblocks * 64, r->tbl0, n_up,
                                        target_key(r->tag, 0)};
            n_up += r->n_targets;
            s->stats.admitted++;
            P.active.push_back(std::move(s->pending.front()));
            s->pending.pop_front();
        }
    }
    if (P.active.empty()) return HJCD_OK;

    // 2. the chunk's lists: every resident block at its stage's next
    //    iterations; the blocks whose PO-CCD ends in this chunk again, for
    //    their first PJ-IK chunk in a second launch of the same step; the
    //    PJ-IK blocks for the collision check (every lane at the stage's end);
    //    PJ-IK targets still running for the decision.  A request's PJ-IK
    //    chunks span the same request-local iterations either way, so running
    //    its first one in the step that ends its PO-CCD leaves every decision
    //    unchanged and saves a round trip.
    const auto cd_ends = [&](const Request* r) {
        return r->stage == SERVE_CD && std::min(r->iter + c, p.cd_sweeps) >= p.cd_sweeps;
    };
    int32_t nb = 0, nb2 = 0, nchk = 0, nt = 0;
    int64_t resident = 0;
    for (auto& Q : s->pipes)
        if (&Q != &P && Q.busy)
            for (auto& up : Q.active) resident += (int64_t)up->nblocks * 64;
    for (auto& up : P.active) {
        resident += (int64_t)up->nblocks * 64;
        nb += up->nblocks;
        const bool fuse = cd_ends(up.get());
        up->fuse = fuse;
        if (fuse) nb2 += up->nblocks;
        if (up->stage == SERVE_POLISH || fuse) {
            nchk += up->nblocks;
            for (int k = 0; k < up->n_targets; ++k) nt += up->status[k] == 0;
        }
    }
    (void)nb_max;
    ServeBlock *d_blk, *d_blk2, *d_chk;
    int32_t *d_all, *d_rt, *d_rn, *d_rfinal;
    int64_t* d_rfirst;
    ServeBlock* h_blk = ar.take<ServeBlock>(nb, &d_blk);
    ServeBlock* h_blk2 = ar.take<ServeBlock>(nb2, &d_blk2);
    ServeBlock* h_chk = ar.take<ServeBlock>(nchk, &d_chk);
    int32_t* h_all = ar.take<int32_t>(nchk, &d_all);
    int32_t* h_rt = ar.take<int32_t>(nt, &d_rt);
    int64_t* h_rfirst = ar.take<int64_t>(nt, &d_rfirst);
    int32_t* h_rn = ar.take<int32_t>(nt, &d_rn);
    int32_t* h_rfinal = ar.take<int32_t>(nt, &d_rfinal);
    if (ar.off > s->up_cap) return fail(HJCD_E_INTERNAL, "serving upload arena overflow");
    int32_t ib = 0, ib2 = 0, ic = 0, it = 0;
    for (auto& up : P.active) {
        Request* r = up.get();
        const bool cd = r->stage == SERVE_CD;
        const bool fuse = r->fuse;
        const int len = cd ? p.cd_sweeps : p.polish_iters;
        const int k0 = r->iter, k1 = std::min(r->iter + c, len);
        // this step's PJ-IK iterations: the stage's next chunk, or its first
        const int q0 = cd ? 0 : k0, q1 = cd ? std::min(c, p.polish_iters) : k1;
        const bool pol = !cd || fuse;
        const bool last = pol && q1 >= p.polish_iters;
        for (int b = 0; b < r->nblocks; ++b) {
            const int32_t blk_id = (int32_t)(r->base / 64) + b;
            h_blk[ib++] = ServeBlock{blk_id, r->stage, k0, k1};
            if (fuse) h_blk2[ib2++] = ServeBlock{blk_id, SERVE_POLISH, q0, q1};
            if (pol) {
                h_chk[ic] = ServeBlock{blk_id, SERVE_POLISH, q0, q1};
                h_all[ic++] = last ? 1 : 0;
            }
        }
        if (!pol) continue;
        for (int k = 0; k < r->n_targets; ++k) {
            if (r->status[k] != 0) continue;
            h_rt[it] = r->tbl0 + k;
            h_rfirst[it] = r->base + (int64_t)k * r->M;
            h_rn[it] = r->M;
            h_rfinal[it] = last ? 1 : 0;
            it++;
        }
    }
    HIP_TRY(hipMemcpyAsync(P.d_up, P.h_up, ar.off, hipMemcpyHostToDevice, P.stream));
    if (n_adm > 0) HIP_TRY(launch_serve_admit(d_adm, n_adm, d_upose, s->d_pose, s->d_tkey, s->st, P.stream));

    ServeChunkArgs ca{};
    ca.rb = s->robot->dev;
    ca.n = n;
    ca.st = s->st;
    ca.blocks = d_blk;
    ca.nb = nb;
    ca.kp = kparams(p);
    HIP_TRY(launch_serve_chunk(ca, P.stream));
    if (nb2 > 0) {  // first PJ-IK chunk of the requests whose PO-CCD just ended
        ServeChunkArgs c2 = ca;
        c2.blocks = d_blk2;
        c2.nb = nb2;
        HIP_TRY(launch_serve_chunk(c2, P.stream));
    }
    if (nchk > 0) {
        ServeCheckArgs ck{};
        ck.rb = s->robot->dev;
        ck.n = n;
        ck.st = s->st;
        ck.blocks = d_chk;
        ck.nb = nchk;
        ck.all_lanes = d_all;
        ck.osph = s->scene ? s->scene->sph : nullptr;
        ck.n_osph = s->scene ? s->scene->n_sph : 0;
        ck.obox = s->scene ? s->scene->box : nullptr;
        ck.n_obox = s->scene ? s->scene->n_box : 0;
        ck.grid = scene_grid(s->scene, s->robot);
        HIP_TRY(launch_serve_check(ck, P.stream));
    }
    int32_t* h_status = (int32_t*)P.h_down;
    float* h_res = (float*)(P.h_down + align16(sizeof(int32_t) * Tc));
    if (nt > 0) {
        ServeReduceArgs ra{};
        ra.st = s->st;
        ra.n = n;
        ra.targets = d_rt;
        ra.first_slot = d_rfirst;
        ra.n_seeds = d_rn;
        ra.final_ = d_rfinal;
        ra.nt = nt;
        ra.succ_pos = p.succ_pos;
        ra.succ_ori = p.succ_ori;
        ra.status = (int32_t*)P.d_down;
        ra.res = (float*)(P.d_down + align16(sizeof(int32_t) * Tc));
        HIP_TRY(launch_serve_reduce(ra, P.stream));
        // status rows, then result rows (contiguous from the arena start up to nt rows)
        HIP_TRY(hipMemcpyAsync(h_status, P.d_down, sizeof(int32_t) * nt, hipMemcpyDeviceToHost, P.stream));
        HIP_TRY(hipMemcpyAsync(h_res, ra.res, sizeof(float) * nt * (n + 3), hipMemcpyDeviceToHost, P.stream));
    }
    HIP_TRY(hipEventRecord(P.done, P.stream));
    bool overlapped = false;  // another pipeline's step is in flight
    for (const auto& Q : s->pipes) overlapped = overlapped || (&Q != &P && Q.busy);
    P.busy = true;
    {
        // the statistics are read under the same mutex by hjcd_server_get_stats
        std::unique_lock<std::mutex> lk(s->mu);
        s->stats.chunks++;
        if (overlapped) s->stats.overlapped_steps++;
        s->resident_sum += (double)resident;
        s->stats.resident_slots_peak = std::max<int64_t>(s->stats.resident_slots_peak, resident);
    }
    return HJCD_OK;
}

// Completes pipeline P's step once its event has passed: records finished
// targets (from the readback), advances stages, completes requests whose
// targets are all finished (their slots return to the pool).
hjcd_status finish_step(hjcd_server s, hjcd_server_s::Pipe& P) {
    const int n = s->n;
    const hjcd_params& p = s->params;
    const int c = s->cfg.chunk_iters;
    const int32_t Tc = s->Tc;
    const int32_t* h_status = (const int32_t*)P.h_down;
    const float* h_res = (const float*)(P.h_down + align16(sizeof(int32_t) * Tc));
    P.busy = false;
    const double t_done = s->now();
    int32_t it = 0;

    // 3. bookkeeping: results, stage transitions, completions
    std::vector<std::unique_ptr<Request>> keep;
    std::vector<std::unique_ptr<Request>> done;
    for (auto& up : P.active) {
        Request* r = up.get();
        const bool fuse = r->fuse;
        if (r->stage == SERVE_POLISH || fuse) {
            for (int k = 0; k < r->n_targets; ++k) {
                if (r->status[k] != 0) continue;
                const int32_t stt = h_status[it];
                if (stt != 0) {
                    r->status[k] = stt;
                    std::memcpy(&r->res[(size_t)k * (n + 3)], h_res + (size_t)it * (n + 3), sizeof(float) * (n + 3));
                    r->n_done++;
                    if (stt == 1) r->n_solved++;
                }
                it++;
            }
        }
        if (fuse) {
            r->stage = SERVE_POLISH;
            r->iter = std::min(c, p.polish_iters);
        } else {
            const int len = r->stage == SERVE_CD ? p.cd_sweeps : p.polish_iters;
            r->iter = std::min(r->iter + c, len);
        }
        if (r->n_done == r->n_targets) {
            r->done = t_done;
            s->blocks.release(r->base / 64, r->nblocks);
            s->tslots.release(r->tbl0, r->n_targets);
            done.push_back(std::move(up));
        } else {
            keep.push_back(std::move(up));
        }
    }
    P.active.swap(keep);
    {
        std::unique_lock<std::mutex> lk(s->mu);
        for (auto& r : done) finish_request(s, std::move(r));
    }
    return HJCD_OK;
}

// ---------------------------------------------------------------------------
// plain worker: one request at a time through hjcd_solve
// ---------------------------------------------------------------------------
hjcd_status plain_step(hjcd_server s) {
    std::unique_ptr<Request> r;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->pending.empty() || s->pending.front()->arrival > s->now()) return HJCD_OK;
        r = std::move(s->pending.front());
        s->pending.pop_front();
        r->admitted = s->now();
        s->stats.admitted++;
    }
    const int n = s->n;
    const int32_t T = r->n_targets;
    const int64_t S = (int64_t)T * r->M;
    if (S > s->plain_cap_seeds || T > s->plain_cap_targets) {
        return fail(HJCD_E_INTERNAL, "plain request larger than the buffers sized at create");
    }
    // targets SoA and keys
    for (int k = 0; k < T; ++k) {
        s->h_tkey[k] = target_key(r->tag, k);
        for (int d = 0; d < 7; ++d) s->h_pose[d * T + k] = r->poses[(size_t)k * 7 + d];
    }
    HIP_TRY(hipMemcpyAsync(s->p_targets, s->h_pose, sizeof(float) * 7 * T, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->p_keys, s->h_tkey, sizeof(uint32_t) * T, hipMemcpyHostToDevice, s->stream));
    std::vector<int64_t> offs(T + 1);
    for (int k = 0; k <= T; ++k) offs[k] = (int64_t)k * r->M;
    hjcd_params p = s->params;
    p.top_k = 1;
    p.collect_stats = 0;
    hjcd_robot rb = s->robot;
    hjcd_status st = hjcd_solve(s->ctx, 1, &rb, s->scene, T, nullptr, s->p_targets, offs.data(), s->p_keys,
                                nullptr, &p, s->p_q, s->p_ep, s->p_eo, s->p_fl, s->p_nf, s->p_sv, s->stream);
    if (st != HJCD_OK) return st;
    std::vector<float> q((size_t)T * n), ep(T), eo(T);
    std::vector<uint8_t> fl(T), sv(T);
    HIP_TRY(hipMemcpyAsync(q.data(), s->p_q, sizeof(float) * T * n, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(ep.data(), s->p_ep, sizeof(float) * T, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(eo.data(), s->p_eo, sizeof(float) * T, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(fl.data(), s->p_fl, T, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(sv.data(), s->p_sv, T, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    r->done = s->now();
    r->status.assign(T, 2);
    r->res.assign((size_t)T * (n + 3), 0.f);
    for (int k = 0; k < T; ++k) {
        float* row = &r->res[(size_t)k * (n + 3)];
        std::memcpy(row, &q[(size_t)k * n], sizeof(float) * n);
        row[n] = ep[k];
        row[n + 1] = eo[k];
        row[n + 2] = (float)fl[k];
        if (sv[k]) {
            r->status[k] = 1;
            r->n_solved++;
        }
    }
    r->n_done = T;
    std::unique_lock<std::mutex> lk(s->mu);
    s->stats.chunks++;
    finish_request(s, std::move(r));
    return HJCD_OK;
}

// One scheduler pass of the batched server: completes the steps whose events
// have passed, then launches a step on a free pipeline that has requests or
// can admit arrived ones.  Sets `progressed` when it did either.
hjcd_status batched_pass(hjcd_server s, bool& progressed, bool& any_busy) {
    progressed = false;
    for (auto& P : s->pipes) {
        if (!P.busy) continue;
        const hipError_t e = hipEventQuery(P.done);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return fail(HJCD_E_DEVICE, "serving step failed: %s", hipGetErrorString(e));
        hjcd_status st = finish_step(s, P);
        if (st != HJCD_OK) return st;
        progressed = true;
    }
    bool arrived;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        arrived = !s->pending.empty() && s->pending.front()->arrival <= s->now();
    }
    for (auto& P : s->pipes) {
        if (P.busy || (P.active.empty() && !arrived)) continue;
        hjcd_status st = launch_step(s, P);
        if (st != HJCD_OK) return st;
        if (P.busy) {
            progressed = true;
            break;  // one launch per pass; the next pass sees the new arrivals
        }
    }
    any_busy = false;
    for (auto& P : s->pipes) any_busy = any_busy || P.busy;
    return HJCD_OK;
}

void worker_main(hjcd_server s) {
    (void)hipSetDevice(s->device);
    const bool plain = s->cfg.mode == HJCD_SERVE_PLAIN;
    while (!s->stop.load()) {
        hjcd_status st = HJCD_OK;
        if (!plain) {
            bool progressed = false, any_busy = false;
            st = batched_pass(s, progressed, any_busy);
            if (st == HJCD_OK && !progressed) {
                if (any_busy) {
                    // a step is in flight: poll its event again shortly
                    std::this_thread::sleep_for(std::chrono::microseconds(10));
                } else {
                    std::unique_lock<std::mutex> lk(s->mu);
                    bool resident = false;
                    for (auto& P : s->pipes) resident = resident || !P.active.empty();
                    if (!resident) {
                        if (s->pending.empty()) {
                            s->cv.wait_for(lk, std::chrono::milliseconds(50));
                        } else {
                            const double dt = s->pending.front()->arrival - s->now();
                            if (dt > 0)
                                s->cv.wait_for(lk, std::chrono::microseconds((int64_t)std::min(dt * 1e6, 5e4)));
                        }
                    }
                }
            }
        } else {
            {
                std::unique_lock<std::mutex> lk(s->mu);
                const bool idle = s->pending.empty() || s->pending.front()->arrival > s->now();
                if (idle) {
                    if (s->pending.empty()) {
                        s->cv.wait_for(lk, std::chrono::milliseconds(50));
                    } else {
                        const double dt = s->pending.front()->arrival - s->now();
                        if (dt > 0)
                            s->cv.wait_for(lk, std::chrono::microseconds((int64_t)std::min(dt * 1e6, 5e4)));
                    }
                    continue;
                }
            }
            st = plain_step(s);
        }
        if (st != HJCD_OK) {
            std::unique_lock<std::mutex> lk(s->mu);
            s->worker_error = hjcd_last_error();
            s->stop.store(true);
            s->cv.notify_all();
            return;
        }
    }
}

}  // namespace

extern "C" {

hjcd_status hjcd_server_create(hjcd_ctx ctx, hjcd_robot robot, hjcd_scene scene, const hjcd_params* params,
                               const hjcd_server_config* config, hjcd_server* out) {
    if (!out) return fail(HJCD_E_INVALID, "out is NULL");
    *out = nullptr;
    hjcd_status s;
    if ((s = check_params(params)) != HJCD_OK) return s;
    if (!config) return fail(HJCD_E_INVALID, "config is NULL");
    if (config->mode != HJCD_SERVE_BATCHED && config->mode != HJCD_SERVE_PLAIN)
        return fail(HJCD_E_INVALID, "unknown serve mode %d", config->mode);
    if (config->chunk_iters < 1) return fail(HJCD_E_INVALID, "chunk_iters must be >= 1");
    if (config->max_slots < 0 || config->max_targets < 0 || config->max_queue < 0)
        return fail(HJCD_E_INVALID, "server sizes must be >= 0");
    if (config->pipelines < 0 || config->pipelines > HJCD_SERVE_MAX_PIPELINES)
        return fail(HJCD_E_INVALID, "pipelines must be in 0..%d", HJCD_SERVE_MAX_PIPELINES);
    if (params->polish_iters < 1) return fail(HJCD_E_UNSUPPORTED, "serving needs polish_iters >= 1");
    if (params->resample_K > 0) return fail(HJCD_E_UNSUPPORTED, "serving does not resample between stages");
    if (!ctx) return fail(HJCD_E_INVALID, "ctx is NULL");
    if (!robot || robot->ctx != ctx) return fail(HJCD_E_INVALID, "robot is NULL or from another context");
    if (scene && scene->ctx != ctx) return fail(HJCD_E_INVALID, "scene belongs to another context");
    HIP_TRY(hipSetDevice(ctx->device));
    const size_t per_slot = sizeof(float) * (robot->n + 3) + 1 + 8;
    int64_t C = config->max_slots;
    if (C == 0) {
        size_t budget = config->hbm_budget;
        if (budget == 0) {
            size_t fr = 0, tot = 0;
            HIP_TRY(hipMemGetInfo(&fr, &tot));
            budget = std::min<size_t>(fr / 4, (size_t)8 << 30);
        }
        C = (int64_t)(budget / per_slot) / 64 * 64;  // the budget is a cap: whole blocks within it
    } else {
        C = ((C + 63) / 64) * 64;
    }
    if (C < 64) return fail(HJCD_E_NOMEM, "memory budget holds less than one 64-slot block");
    auto* srv = new hjcd_server_s();
    srv->ctx = ctx;
    srv->device = ctx->device;
    srv->robot = robot;
    srv->scene = scene;
    srv->params = *params;
    srv->cfg = *config;
    if (srv->cfg.max_queue == 0) srv->cfg.max_queue = 1 << 22;
    if (srv->cfg.pipelines == 0) srv->cfg.pipelines = 2;
    srv->n = robot->n;
    if (hipStreamCreateWithFlags(&srv->stream, hipStreamNonBlocking) != hipSuccess) {
        delete srv;
        return fail(HJCD_E_DEVICE, "stream creation failed");
    }
    srv->C = C;
    srv->Tc = config->max_targets > 0 ? config->max_targets
                                      : (int32_t)std::min<int64_t>(1 << 20, std::max<int64_t>(64, C / 32));
    srv->stats.max_slots = C;
    if (config->mode == HJCD_SERVE_BATCHED) {
        if ((s = server_alloc_batched(srv)) != HJCD_OK) {
            server_free(srv);
            delete srv;
            return s;
        }
    } else {
        bool ok = true;
        srv->plain_cap_seeds = C;
        srv->plain_cap_targets = srv->Tc;
        srv->p_targets = dev_alloc<float>((size_t)7 * srv->Tc, ok);
        srv->p_keys = dev_alloc<uint32_t>(srv->Tc, ok);
        srv->p_q = dev_alloc<float>((size_t)srv->Tc * srv->n, ok);
        srv->p_ep = dev_alloc<float>(srv->Tc, ok);
        srv->p_eo = dev_alloc<float>(srv->Tc, ok);
        srv->p_fl = dev_alloc<uint8_t>(srv->Tc, ok);
        srv->p_sv = dev_alloc<uint8_t>(srv->Tc, ok);
        srv->p_nf = dev_alloc<int32_t>(srv->Tc, ok);
        if (hipHostMalloc((void**)&srv->h_pose, sizeof(float) * 7 * srv->Tc, hipHostMallocDefault) != hipSuccess)
            ok = false;
        if (hipHostMalloc((void**)&srv->h_tkey, sizeof(uint32_t) * srv->Tc, hipHostMallocDefault) != hipSuccess)
            ok = false;
        if (!ok) {
            server_free(srv);
            delete srv;
            return fail(HJCD_E_NOMEM, "server allocation failed");
        }
    }
    srv->epoch = Clock::now();
    *out = srv;
    return HJCD_OK;
}

hjcd_status hjcd_server_start(hjcd_server srv) {
    if (!srv) return fail(HJCD_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->started) return fail(HJCD_E_INVALID, "server already started");
    srv->started = true;
    srv->epoch = Clock::now();
    srv->worker = std::thread(worker_main, srv);
    return HJCD_OK;
}

hjcd_status hjcd_server_submit(hjcd_server srv, int32_t n_targets, const float* targets, int32_t seeds_per_target,
                               uint64_t tag, double arrival_s, int64_t* request_id) {
    if (!srv) return fail(HJCD_E_INVALID, "server is NULL");
    if (n_targets < 1 || !targets) return fail(HJCD_E_INVALID, "need n_targets >= 1 and targets");
    if (seeds_per_target < 1) return fail(HJCD_E_INVALID, "seeds_per_target must be >= 1");
    if (!std::isfinite(arrival_s)) return fail(HJCD_E_INVALID, "arrival time must be finite");
    for (int i = 0; i < 7 * n_targets; ++i)
        if (!std::isfinite(targets[i])) return fail(HJCD_E_INVALID, "targets must be finite");
    for (int k = 0; k < n_targets; ++k) {
        const float* q = targets + 7 * k + 3;
        if (!(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3] > 1e-12f))
            return fail(HJCD_E_INVALID, "target %d has a zero quaternion", k);
    }
    const int64_t seeds = (int64_t)n_targets * seeds_per_target;
    if (seeds > srv->C || n_targets > srv->Tc)
        return fail(HJCD_E_NOMEM, "request of %lld seeds / %d targets can never fit (%lld slots, %d targets)",
                    (long long)seeds, n_targets, (long long)srv->C, srv->Tc);
    auto r = std::make_unique<Request>();
    r->tag = tag;
    r->n_targets = n_targets;
    r->M = seeds_per_target;
    r->poses.assign(targets, targets + 7 * (size_t)n_targets);
    std::unique_lock<std::mutex> lk(srv->mu);
    if ((int64_t)srv->pending.size() >= srv->cfg.max_queue) return fail(HJCD_E_BUSY, "request queue is full");
    r->arrival = std::max(arrival_s, 0.0);
    r->id = srv->next_id++;
    if (request_id) *request_id = r->id;
    if (srv->stats.submitted == 0 || r->arrival < srv->stats.first_arrival_s) srv->stats.first_arrival_s = r->arrival;
    srv->stats.submitted++;
    // keep pending ordered by arrival (stable for equal times)
    auto it = srv->pending.end();
    while (it != srv->pending.begin() && (*(it - 1))->arrival > r->arrival) --it;
    srv->pending.insert(it, std::move(r));
    srv->cv.notify_all();
    return HJCD_OK;
}

hjcd_status hjcd_server_poll(hjcd_server srv, int32_t max, hjcd_request_info* out, int32_t* n_out) {
    if (!srv || !n_out || (max > 0 && !out)) return fail(HJCD_E_INVALID, "bad poll arguments");
    std::unique_lock<std::mutex> lk(srv->mu);
    int32_t k = 0;
    while (k < max && !srv->unpolled.empty()) {
        const int64_t id = srv->unpolled.front();
        srv->unpolled.pop_front();
        auto f = srv->finished.find(id);
        if (f == srv->finished.end()) continue;
        const Request& r = *f->second;
        out[k++] = hjcd_request_info{r.id, r.tag, r.n_targets, r.n_solved, r.arrival, r.admitted, r.done};
    }
    *n_out = k;
    return HJCD_OK;
}

hjcd_status hjcd_server_result(hjcd_server srv, int64_t request_id, float* q, float* err_p, float* err_o,
                               uint8_t* flag) {
    if (!srv) return fail(HJCD_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto f = srv->finished.find(request_id);
    if (f == srv->finished.end()) return fail(HJCD_E_INVALID, "request %lld is not a completed request", (long long)request_id);
    const Request& r = *f->second;
    const int n = srv->n;
    for (int k = 0; k < r.n_targets; ++k) {
        const float* row = &r.res[(size_t)k * (n + 3)];
        if (q) std::memcpy(q + (size_t)k * n, row, sizeof(float) * n);
        if (err_p) err_p[k] = row[n];
        if (err_o) err_o[k] = row[n + 1];
        if (flag) flag[k] = (uint8_t)row[n + 2];
    }
    srv->finished.erase(f);
    return HJCD_OK;
}

hjcd_status hjcd_server_wait(hjcd_server srv, double timeout_s) {
    if (!srv) return fail(HJCD_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    const auto deadline = Clock::now() + std::chrono::duration<double>(timeout_s);
    while (srv->stats.completed < srv->stats.submitted) {
        if (!srv->worker_error.empty()) return fail(HJCD_E_DEVICE, "server worker failed: %s", srv->worker_error.c_str());
        if (srv->cv.wait_until(lk, deadline) == std::cv_status::timeout &&
            srv->stats.completed < srv->stats.submitted)
            return fail(HJCD_E_BUSY, "timed out with %lld of %lld requests completed",
                        (long long)srv->stats.completed, (long long)srv->stats.submitted);
    }
    return HJCD_OK;
}

hjcd_status hjcd_server_get_stats(hjcd_server srv, hjcd_server_stats* out) {
    if (!srv || !out) return fail(HJCD_E_INVALID, "bad stats arguments");
    std::unique_lock<std::mutex> lk(srv->mu);
    hjcd_server_stats st = srv->stats;
    st.mean_resident_slots = st.chunks ? srv->resident_sum / (double)st.chunks : 0.0;
    if (!srv->latencies.empty()) {
        std::vector<double> l = srv->latencies;
        std::sort(l.begin(), l.end());
        auto pct = [&](double q) {
            const double pos = q * (double)(l.size() - 1);
            const size_t i = (size_t)pos;
            const double f = pos - (double)i;
            return i + 1 < l.size() ? l[i] * (1 - f) + l[i + 1] * f : l[i];
        };
        st.p50_latency_ms = pct(0.50);
        st.p99_latency_ms = pct(0.99);
    }
    const double span = st.last_done_s - st.first_arrival_s;
    st.solves_per_s = span > 0 ? (double)st.targets_solved / span : 0.0;
    *out = st;
    return HJCD_OK;
}

void hjcd_server_destroy(hjcd_server srv) {
    if (!srv) return;
    srv->stop.store(true);
    srv->cv.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    (void)hipSetDevice(srv->device);
    if (srv->stream) (void)hipStreamSynchronize(srv->stream);
    for (auto& P : srv->pipes)
        if (P.stream) (void)hipStreamSynchronize(P.stream);
    server_free(srv);
    delete srv;
}

}  // extern "C"
