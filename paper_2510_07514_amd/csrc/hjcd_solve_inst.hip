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

// ----------------------------------------------------------------------------
// Per-seed solve: seed init, PO-CCD and/or PJ-IK, results to HBM.
// ----------------------------------------------------------------------------
template <int NM>
__global__ __launch_bounds__(256) void k_solve(SolveArgs a) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = v < a.map.Sv;
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
#pragma unroll
    for (int j = 0; j < NM; ++j) th[j] = 0.f;
    if (a.init_mode == INIT_UNIFORM) {
        uniform_seed<NM>(a.rb, n, th, a.kp.seed, sl.m, sl.tkey);
    } else if (live) {
#pragma unroll
        for (int j = 0; j < NM; ++j)
            if (j < n) th[j] = clampf(a.q_in[(int64_t)j * a.q_in_stride + sl.s], a.rb->lo[j], a.rb->hi[j]);
    }
    Counters cnt;
    Err e{};
    if (a.do_cd) po_ccd<NM>(a.rb, n, tg, a.kp, sl.m, sl.tkey, th, live, cnt, a.traj, a.S, sl.s, e);
    if (a.do_polish) pj_ik<NM>(a.rb, n, tg, a.kp, sl.m, sl.tkey, th, live, cnt, a.do_cd ? nullptr : a.traj,
                               a.S, sl.s, e);
    if (!a.do_cd && !a.do_polish && a.targets) {
        Frame ee;
        V3 Pd[1], Zd[1];
        fk_chain<NM, false>(a.rb, n, th, Pd, Zd, ee);
        e = residual(ee, tg);
    }
    if (live) {
#pragma unroll
        for (int j = 0; j < NM; ++j)
            if (j < n) a.q_out[(int64_t)j * a.S + sl.s] = th[j];
        for (int j = n; j < a.n_rows; ++j) a.q_out[(int64_t)j * a.S + sl.s] = 0.f;
        if (a.err_p) a.err_p[sl.s] = sqrtf(e.ep2);
        if (a.err_o) a.err_o[sl.s] = e.phi;
        if (a.cost) a.cost[sl.s] = cost_of(e);
    }
    flush_counters(cnt, a.counters, a.counters != nullptr);
}

template <int NM>
hipError_t launch_solve_nm(const SolveArgs& a, hipStream_t st);

template <>
hipError_t launch_solve_nm<HJCD_NM>(const SolveArgs& a, hipStream_t st) {
    const unsigned nb = (unsigned)((a.map.Sv + 255) / 256);
    hipLaunchKernelGGL(k_solve<HJCD_NM>, dim3(nb), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace hjcd
