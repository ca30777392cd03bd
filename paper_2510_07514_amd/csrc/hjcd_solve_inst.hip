// One instantiation of the per-seed solve kernel (PO-CCD and / or PJ-IK) for
// the joint-count bucket HJCD_NM; the build compiles this file once per
// bucket so the buckets compile in parallel.
#include <hip/hip_runtime.h>

#include "hjcd_device.hpp"
#include "hjcd_launch.hpp"

#ifndef HJCD_NM
#error "HJCD_NM must be defined"
#endif

namespace hjcd {

// Buckets below 8 are exact joint counts (the host dispatches a 6- or 7-joint
// chain to them): the joint loops then have no runtime bound and the chain
// takes exactly n registers per joint array.
constexpr bool kExactN = HJCD_NM < 8;

// Occupancy variants of the per-seed solve kernels (a launch-shape choice of
// the autotuner and of hjcd_params.polish_variant; both variants compile the
// same device code, so their results are bit-identical).  Minimum waves per
// SIMD:
//   NM <= 8:       variant 0: 3 (at most 168 VGPRs, a few spills; faster than
//                  the two waves of the unconstrained ~200), variant 1: 2
//   8 < NM <= 16:  variant 0: 2 (at most 256 VGPRs), variant 1: 1 (as allocated)
//   NM > 16:       variant 0: 1 (as allocated), variant 1: 2 (with spills)
template <int NM, int V>
struct SolveOcc {
    static constexpr int waves = NM <= 8 ? (V == 0 ? 3 : 2) : NM <= 16 ? (V == 0 ? 2 : 1) : (V == 0 ? 1 : 2);
    // line-search form (same results): the shuffle form needs ~50 more live
    // registers, which spill at three waves per SIMD up to 8 joints and at two
    // above, so up to 24 joints the searching lanes' records go through LDS
    // (24-joint chain, 2,000 x 256: 5.11 -> 3.81 ms, spills 188 -> 99
    // registers; 20-joint streaming launch, 20,000 x 256: 69.1 -> 64.8 ms;
    // 12 joints 2-3% faster; 16 joints at one wave per SIMD 4.93 -> 3.03 ms).
    // At 32 joints (one wave, no spills) the shuffles measured faster (3.93 vs
    // 4.09 ms).
    static constexpr int ls = NM <= 24 ? kLsLds : kLsShfl;
};

// LDS of the line-search records of a workgroup of `threads` threads.
template <int NM, int LS>
constexpr size_t ls_lds_bytes(int threads) {
    return LS == kLsLds ? (size_t)(threads / 64) * ls_wave_floats<NM>() * sizeof(float) : 0;
}

// This wave's records in the workgroup's dynamic LDS (LDS line-search form).
template <int NM, int LS>
__device__ __forceinline__ float* ls_records() {
    if constexpr (LS == kLsLds) {
        extern __shared__ float ls_dyn[];
        return ls_dyn + (threadIdx.x >> 6) * ls_wave_floats<NM>();
    } else {
        return nullptr;
    }
}

// PO-CCD's perturbation rows of this wave in the workgroup's dynamic LDS.
template <int NM>
__device__ __forceinline__ float* cd_records() {
    extern __shared__ float ls_dyn[];
    return ls_dyn + (threadIdx.x >> 6) * perturb_wave_floats<NM>();
}

// PO-CCD perturbations spread through LDS (same results) in the buckets
// where it measured faster: 7 joints (k_cd 1.38 -> 1.32 ms on 1,000 x 1,024)
// and 24 (4.45 -> 4.29 ms on 2,000 x 256); at 12, 20 and 32 joints it was
// 2-5% slower (there more lanes perturb per wave and the passes add up).
constexpr bool kCdPerturbSpread = HJCD_NM <= 8 || HJCD_NM == 24;

template <int NM>
constexpr size_t cd_lds_bytes(int threads) {
    return kCdPerturbSpread ? (size_t)(threads / 64) * perturb_wave_floats<NM>() * sizeof(float) : 0;
}

// ----------------------------------------------------------------------------
// Per-seed solve: seed init, PO-CCD and/or PJ-IK, results to HBM.
// ----------------------------------------------------------------------------
// Initial joint values of seed sl: uniform draws in the limits, or the
// caller's values (live lanes) clamped to the limits.
template <int NM>
__device__ __forceinline__ void init_seed(const SolveArgs& a, int n, const Slot& sl, bool live, float* th) {
#pragma unroll
    for (int j = 0; j < NM; ++j) th[j] = 0.f;
    if (a.init_mode == INIT_UNIFORM) {
        uniform_seed<NM>(a.rb, n, th, a.kp.seed, sl.m, sl.tkey);
    } else if (live) {
#pragma unroll
        for (int j = 0; j < NM; ++j)
            if (j < n) th[j] = clampf(a.q_in[(int64_t)j * a.q_in_stride + sl.s], a.rb->lo[j], a.rb->hi[j]);
    }
}

// Result of the seed in slot s: joint values (rows n .. n_rows - 1 zero for
// mixed-dof batches), |r_p|, phi and cost.
template <int NM>
__device__ __forceinline__ void write_seed(const SolveArgs& a, int n, const float* th, const Err& e, int64_t s) {
#pragma unroll
    for (int j = 0; j < NM; ++j)
        if (j < n) a.q_out[(int64_t)j * a.S + s] = th[j];
    for (int j = n; j < a.n_rows; ++j) a.q_out[(int64_t)j * a.S + s] = 0.f;
    if (a.err_p) a.err_p[s] = sqrtf(e.ep2);
    if (a.err_o) a.err_o[s] = e.phi;
    if (a.cost) a.cost[s] = cost_of(e);
}

// STATS: the kernel counts executed work into a.counters; without it the
// counters are dead code and hold no registers (launches with no counters).
template <int NM, int LS, bool STATS>
__device__ __forceinline__ void solve_body(const SolveArgs& a, bool do_cd, bool do_polish) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = v < a.map.Sv;
    const int n = kExactN ? HJCD_NM : a.n;
    Slot sl;
    if (live) {
        sl = map_lane(a.map, v);
    } else {
        sl.s = 0;
        sl.t = 0;
        sl.m = 0;
        sl.tkey = 0;
    }
    Target tg{};
    if (a.targets) tg = load_target(a.targets, a.map.T, sl.t);
    float th[NM];
    init_seed<NM>(a, n, sl, live, th);
    Counters cnt;
    Err e{};
    if (do_cd) {
        bool frozen = !live;
        po_ccd<NM, kCdPerturbSpread>(a.rb, n, tg, a.kp, sl.m, sl.tkey, th, live, frozen, cnt, a.traj, a.S, sl.s,
                                     0, a.kp.cd_sweeps, e, kCdPerturbSpread ? cd_records<NM>() : nullptr);
    }
    if (do_polish) {
        bool frozen = !live;
        pj_ik<NM, LS>(robot_ref(a.rb), n, tg, a.kp, sl.m, sl.tkey, th, live, frozen, cnt,
                      do_cd ? nullptr : a.traj, a.S, sl.s, 0, a.kp.polish_iters, e, true, ls_records<NM, LS>());
    }
    if (!do_cd && !do_polish && a.targets) {
        Frame ee;
        V3 Pd[1], Zd[1];
        fk_chain<NM, false>(a.rb, n, th, Pd, Zd, ee);
        e = residual(ee, tg);
    }
    if (live) write_seed<NM>(a, n, th, e, sl.s);
    flush_counters(cnt, a.counters, STATS && a.counters != nullptr);
}

// PJ-IK with seed streaming.  Wave w owns the seeds [w P, (w + 1) P) of the
// launch (P = seeds_per_wave, a multiple of 64) and starts on the first 64;
// a lane whose seed has converged or run all its iterations writes that
// seed's result and takes the wave's next seed.  Lanes stay busy while the
// range lasts instead of idling once their seed has converged.  A seed's
// iterations, keys and arithmetic do not depend on its lane or on when it
// starts, so the results equal those of one seed per lane.
template <int NM, int LS, bool STATS>
__device__ __forceinline__ void polish_stream(const SolveArgs& a) {
    const int lane = (int)(threadIdx.x & 63u);
    const int64_t P = a.seeds_per_wave;
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    int64_t next = w * P;
    const int64_t end = next + P < a.map.Sv ? next + P : a.map.Sv;
    const int n = kExactN ? HJCD_NM : a.n;
    const RobotRef rb = robot_ref(a.rb);
    const int K = a.kp.polish_iters;
    Counters cnt;
    Slot sl;
    sl.s = 0;
    sl.t = 0;
    sl.m = 0;
    sl.tkey = 0;
    Target tg{};
    float th[NM];
#pragma unroll
    for (int j = 0; j < NM; ++j) th[j] = 0.f;
    bool has = false, frozen = true;
    int it = 0;
    float last_ep = 0.f, last_phi = 0.f;
    for (;;) {
        // free lanes take the wave's next seeds, in lane order
        const uint64_t fr = __ballot(!has);
        if (next < end && fr != 0ull) {
            const int64_t v = next + __popcll(fr & ((1ull << lane) - 1ull));
            if (!has && v < end) {
                sl = map_lane(a.map, v);
                if (a.targets) tg = load_target(a.targets, a.map.T, sl.t);
                init_seed<NM>(a, n, sl, true, th);
                has = true;
                frozen = false;
                it = 0;
            }
            next += __popcll(fr);
        }
        if (!wave_any(has)) break;
        const bool run = has && !frozen && it < K;
        if (wave_any(run)) {
            bool fz = !run;
            pj_ik_iter<NM, LS>(rb, n, tg, a.kp, sl.m, sl.tkey, th, false, fz, cnt, nullptr, a.S, sl.s, it,
                               last_ep, last_phi, ls_records<NM, LS>());
            if (run) {
                frozen = fz;
                ++it;
            }
        }
        // converged, or all iterations run: the seed's result
        if (has && (frozen || it >= K)) {
            Frame ee;
            V3 Pd[1], Zd[1];
            fk_chain<NM, false>(rb, n, th, Pd, Zd, ee);
            write_seed<NM>(a, n, th, residual(ee, tg), sl.s);
            has = false;
            frozen = true;
        }
    }
    flush_counters(cnt, a.counters, STATS && a.counters != nullptr);
}

// Occupancy of the single-stage kernels.  In the 20- and 24-joint buckets two
// waves per SIMD, although the kernels then spill (at 20 joints PJ-IK about 60
// registers, PO-CCD about 210): at one wave per SIMD nothing hides the latency
// of a wave's own dependent instructions, and two waves measured faster (20
// joints, 20,000 x 256: PJ-IK 104 -> 71 ms, PO-CCD 76 -> 49 ms; 24 joints,
// 8,000 x 256: PO-CCD 37.3 -> 34.1 ms, PJ-IK 34.8 -> 34.3 ms).  At 32 joints
// the spills outweigh it (PO-CCD 49 -> 62 ms, PJ-IK 33 -> 38 ms): one wave.
// PJ-IK keeps the other occupancy as the alternative variant.
template <int NM, int V>
struct PolishOcc {
    static constexpr int waves = (NM > 16 && NM <= 24) ? (V == 0 ? 2 : 1) : SolveOcc<NM, V>::waves;
    static constexpr int ls = SolveOcc<NM, V>::ls;
};
template <int NM>
struct CdOcc {
    static constexpr int waves = (NM > 16 && NM <= 24) ? 2 : SolveOcc<NM, 0>::waves;
    // two lanes per seed hold half the per-joint state; allocation without a
    // bound (device assembly of this build): ~270 VGPRs at 20 joints, ~310 at
    // 24 (one lane: ~470 and more), so two waves per SIMD spill 8 and 47
    // registers there (one lane: 214 and 481); 3 waves up to 16 joints
    static constexpr int pair_waves = NM <= 16 ? 3 : (NM <= 24 ? 2 : 1);
};

// PO-CCD with two lanes per seed (po_ccd_pair), buckets of 12 joints and more:
// lane 2v and 2v + 1 share seed v; the even lane writes the result.
constexpr bool kPairCd = HJCD_NM >= 12;

template <int NM, bool STATS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CdOcc<NM>::pair_waves))) void k_cd_pair(
    SolveArgs a) {
    const int64_t v = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 1;
    const bool live = v < a.map.Sv;
    const bool even = (threadIdx.x & 1u) == 0;
    const int n = a.n;
    Slot sl;
    if (live) {
        sl = map_lane(a.map, v);
    } else {
        sl.s = 0;
        sl.t = 0;
        sl.m = 0;
        sl.tkey = 0;
    }
    Target tg{};
    if (a.targets) tg = load_target(a.targets, a.map.T, sl.t);
    float th[NM];
    init_seed<NM>(a, n, sl, live, th);
    Counters cnt;
    Err e{};
    bool frozen = !live;
    po_ccd_pair<NM>(a.rb, n, tg, a.kp, sl.m, sl.tkey, th, live, frozen, cnt, a.traj, a.S, sl.s, 0,
                    a.kp.cd_sweeps, e);
    if (live && even) write_seed<NM>(a, n, th, e, sl.s);
    flush_counters(cnt, a.counters, STATS && a.counters != nullptr);
}

// Seed initialisation only (hjcd_init_seeds): uniform draws written out.
template <int NM>
__global__ __launch_bounds__(256) void k_seed(SolveArgs a) {
    solve_body<NM, kLsSeq, false>(a, false, false);
}

// PO-CCD only, and PJ-IK only: the whole solve runs them as two launches, each
// kernel compiled for its stage alone.
template <int NM, bool STATS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CdOcc<NM>::waves))) void k_cd(SolveArgs a) {
    solve_body<NM, kLsSeq, STATS>(a, true, false);
}

template <int NM, int V, bool STATS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PolishOcc<NM, V>::waves))) void k_polish(
    SolveArgs a) {
    solve_body<NM, PolishOcc<NM, V>::ls, STATS>(a, false, true);
}

// PJ-IK only, streaming seeds through the waves (large launches).
template <int NM, int V, bool STATS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PolishOcc<NM, V>::waves))) void k_polish_stream(
    SolveArgs a) {
    polish_stream<NM, PolishOcc<NM, V>::ls, STATS>(a);
}

// ----------------------------------------------------------------------------
// Serving chunk: wave w of the workgroup advances block entry 4 blockIdx + w
// by iterations [k0, k1) of its stage; slot state persists in HBM.
// ----------------------------------------------------------------------------
template <int NM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SolveOcc<NM, 0>::waves))) void k_serve_chunk(
    ServeChunkArgs a) {
    const int e = (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (e >= a.nb) return;  // whole wave leaves together
    const ServeBlock blk = a.blocks[e];
    const int lane = threadIdx.x & 63;
    const int64_t s = (int64_t)blk.block * 64 + lane;
    const int n = kExactN ? HJCD_NM : a.n;
    uint8_t st = a.st.sstate[s];
    const bool live = (st & SLOT_LIVE) && !(st & SLOT_RETIRED);
    const int32_t t = live ? a.st.slot_target[s] : 0;
    const uint32_t m = live ? a.st.slot_m[s] : 0u;
    const uint32_t tkey = live ? a.st.tgt_key[t] : 0u;
    Target tg = load_target(a.st.tgt_pose, a.st.Tc, t);
    float th[NM];
#pragma unroll
    for (int j = 0; j < NM; ++j) th[j] = 0.f;
    if (blk.stage == SERVE_CD && blk.k0 == 0) {
        uniform_seed<NM>(a.rb, n, th, a.kp.seed, m, tkey);
    } else if (live) {
#pragma unroll
        for (int j = 0; j < NM; ++j)
            if (j < n) th[j] = a.st.q[(int64_t)j * a.st.C + s];
    }
    Counters cnt;
    Err er{};
    // the wave's LDS rows of the spread line search, single-coordinate trials
    // and perturbations (both stages), in the buckets that use them
    constexpr int LS = SolveOcc<NM, 0>::ls;
    static_assert(!kCdPerturbSpread || LS == kLsLds, "PO-CCD's perturbation rows live in the line-search rows");
    static_assert(perturb_wave_floats<NM>() <= ls_wave_floats<NM>(), "rows too small");
    __shared__ float rows[LS == kLsLds ? 4 * ls_wave_floats<NM>() : 1];
    float* const wrows = LS == kLsLds ? rows + (threadIdx.x >> 6) * ls_wave_floats<NM>() : nullptr;
    if (blk.stage == SERVE_CD) {
        bool frozen = !live || (st & SLOT_CD_FROZEN);
        po_ccd<NM, kCdPerturbSpread>(a.rb, n, tg, a.kp, m, tkey, th, live, frozen, cnt, nullptr, 0, s, blk.k0, blk.k1,
                                     er, wrows);
        if (frozen) st |= SLOT_CD_FROZEN;
    } else {
        bool frozen = !live || (st & SLOT_POL_FROZEN);
        pj_ik<NM, LS>(robot_ref(a.rb), n, tg, a.kp, m, tkey, th, live, frozen, cnt, nullptr, 0, s, blk.k0, blk.k1, er,
                      true, wrows);
        // the exit test of iteration k1 (or the one after the last iteration)
        // on the state this chunk leaves: a seed converged by the chunk's last
        // step is eligible for the collision check at this chunk's end
        if (live && er.ep2 < a.kp.eps_pol2 && er.phi < a.kp.ups_pol) frozen = true;
        if (frozen) st |= SLOT_POL_FROZEN;
    }
    if (live) {
#pragma unroll
        for (int j = 0; j < NM; ++j)
            if (j < n) a.st.q[(int64_t)j * a.st.C + s] = th[j];
        a.st.err_p[s] = sqrtf(er.ep2);
        a.st.err_o[s] = er.phi;
        a.st.cost[s] = cost_of(er);
        a.st.sstate[s] = st;
    }
    // the serving loop counts no executed work: cnt is dead code here
}

template <int NM>
hipError_t launch_serve_chunk_nm(const ServeChunkArgs& a, hipStream_t st);

template <>
hipError_t launch_serve_chunk_nm<HJCD_NM>(const ServeChunkArgs& a, hipStream_t st) {
    if (a.nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_serve_chunk<HJCD_NM>, dim3((unsigned)((a.nb + 3) / 4)), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int NM>
hipError_t launch_solve_nm(const SolveArgs& a, hipStream_t st);

// Templated on the bucket and file-local: every bucket's translation unit
// defines its own (one shared name would let the linker keep a single body).
constexpr int kPolishThreads = 64;
constexpr int kOtherThreads = 256;

template <int NM, bool STATS>
static hipError_t launch_solve_stats(const SolveArgs& a, hipStream_t st) {
    // default workgroup: one wave for PJ-IK (a workgroup's slot frees as soon as
    // its one wave is done, so a long-running wave holds back no others:
    // measured 1-2% faster on the 7-joint workload and 8% on the 20-joint one
    // than 256 threads), 256 threads for the other stages (one wave: within
    // 0.5% for PO-CCD)
    const int bt = a.block_threads > 0 ? a.block_threads : (a.do_polish ? kPolishThreads : kOtherThreads);
    if (bt % 64 != 0 || bt > 256) return hipErrorInvalidValue;  // whole waves; launch bound 256
    const unsigned nb = (unsigned)((a.map.Sv + bt - 1) / bt);
    if (a.do_cd && a.do_polish) return hipErrorInvalidValue;  // the stages run as separate launches
    // PJ-IK streams seeds through its waves once the launch holds enough
    // seeds to keep every wave slot busy with several seeds per lane, in the
    // buckets that run one or two waves per SIMD (measured: with three waves
    // per SIMD the other waves already fill the issue slots an idle lane
    // leaves, and streaming only lengthens the tail).  A launch that records
    // trajectories keeps one seed per lane; its arithmetic is the same.
    const int64_t sf = HJCD_NM > 16 && !a.traj ? stream_factor(a.map.Sv) : 1;
    SolveArgs ps = a;
    ps.seeds_per_wave = 64 * sf;
    const int64_t seeds_per_block = ps.seeds_per_wave * (bt / 64);
    const unsigned nbp = (unsigned)((a.map.Sv + seeds_per_block - 1) / seeds_per_block);
    const size_t lds0 = ls_lds_bytes<HJCD_NM, PolishOcc<HJCD_NM, 0>::ls>(bt);  // line-search records
    const size_t lds1 = ls_lds_bytes<HJCD_NM, PolishOcc<HJCD_NM, 1>::ls>(bt);
    bool pair_cd = false;
    if constexpr (kPairCd) pair_cd = a.do_cd && a.cd_lanes == 2;  // smaller buckets keep one lane
    if (pair_cd) {
        if constexpr (kPairCd) {
            const unsigned nb2 = (unsigned)((2 * a.map.Sv + bt - 1) / bt);
            hipLaunchKernelGGL((k_cd_pair<HJCD_NM, STATS>), dim3(nb2), dim3(bt), 0, st, a);
        }
    } else if (a.do_cd)
        hipLaunchKernelGGL((k_cd<HJCD_NM, STATS>), dim3(nb), dim3(bt), cd_lds_bytes<HJCD_NM>(bt), st, a);
    else if (!a.do_polish)
        hipLaunchKernelGGL((k_seed<HJCD_NM>), dim3(nb), dim3(bt), 0, st, a);
    else if (sf > 1 && a.variant == 1)
        hipLaunchKernelGGL((k_polish_stream<HJCD_NM, 1, STATS>), dim3(nbp), dim3(bt), lds1, st, ps);
    else if (sf > 1)
        hipLaunchKernelGGL((k_polish_stream<HJCD_NM, 0, STATS>), dim3(nbp), dim3(bt), lds0, st, ps);
    else if (a.variant == 1)
        hipLaunchKernelGGL((k_polish<HJCD_NM, 1, STATS>), dim3(nb), dim3(bt), lds1, st, a);
    else
        hipLaunchKernelGGL((k_polish<HJCD_NM, 0, STATS>), dim3(nb), dim3(bt), lds0, st, a);
    return hipGetLastError();
}

// Launches that count executed work run the kernels compiled with counters;
// the others run the builds without them (7 joints: PJ-IK 3.13 -> 3.03 ms,
// spills 10 -> 2 registers; 24 joints 3.78 -> 3.60 ms), except at 20 joints,
// where the build without counters places its spills worse and measured
// 1-3% slower (both builds skip the counting when a.counters is null).
constexpr bool kCounterFreeBuild = HJCD_NM != 20;

template <>
hipError_t launch_solve_nm<HJCD_NM>(const SolveArgs& a, hipStream_t st) {
    if constexpr (kCounterFreeBuild) {
        if (!a.counters) return launch_solve_stats<HJCD_NM, false>(a, st);
    }
    return launch_solve_stats<HJCD_NM, true>(a, st);
}

}  // namespace hjcd
