// Private declarations shared by the C ABI (hjcd_api.cpp) and the serving
// loop (hjcd_server.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/hjcd.h"
#include "hjcd_launch.hpp"
#include "hjcd_tables.hpp"

namespace hjcd {

// Thread-local error text behind hjcd_last_error(); returns s.
hjcd_status fail(hjcd_status s, const char* fmt, ...);

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::hjcd::fail(HJCD_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
};

hjcd_status check_params(const hjcd_params* p);
KernelParams kparams(const hjcd_params& p);
hjcd_status check_offsets(int32_t T, const int64_t* offs);
hjcd_status check_robot(hjcd_ctx c, hjcd_robot r);

// Targets of a multi-robot batch regrouped so that each robot's targets (and
// seeds) are contiguous: perm[b] = caller target of grouped position b,
// robot i owns grouped targets [rb_tb[i], rb_tb[i+1]), voffs = CSR seed
// offsets in grouped order; identity when no regrouping was needed.
struct TargetGroups {
    std::vector<int32_t> perm;
    std::vector<int32_t> rb_tb;
    std::vector<int64_t> voffs;
    bool identity = true;
};
void group_targets(int32_t n_robots, int32_t T, const int32_t* robot_of_target, const int64_t* offs,
                   TargetGroups& g);

}  // namespace hjcd

struct hjcd_ctx_s {
    int device = 0;
    hjcd::DevBuf voffs, voffs2, coffs, tperm, tkeys_dummy, q_work, q_work2, ep, eo, cost, flag, rank, counters;
    void* pinned = nullptr;
    size_t pinned_cap = 0;
    size_t pinned_used = 0;
    hipEvent_t staging_ev = nullptr;
    // stats
    static constexpr int kEv = 16;
    hipEvent_t ev[kEv] = {};
    int ev_used = 0;
    int ev_stage[kEv] = {};
    bool stats_pending = false;
    hjcd_stats stats{};
    hipStream_t stats_stream = nullptr;
};

// Robots, scenes, servers and plans keep their context's device id: they may
// be destroyed after the context (their memory is their own), so their
// destroy functions never read the context.
struct hjcd_robot_s {
    hjcd_ctx ctx = nullptr;
    int device = 0;
    hjcd::DevRobot host;
    hjcd::DevRobot* dev = nullptr;
    int n = 0;
};

struct hjcd_scene_s {
    hjcd_ctx ctx = nullptr;
    int device = 0;
    float* sph = nullptr;
    int32_t n_sph = 0;
    float* box = nullptr;
    int32_t n_box = 0;
    // obstacle grid (hjcd_launch.hpp ObstacleGrid), device arrays owned here
    int32_t* g_start = nullptr;
    int32_t* g_items = nullptr;
    float g_lo[3] = {0.f, 0.f, 0.f};
    float g_h = 0.f;
    int32_t g_n[3] = {0, 0, 0};
    float g_margin = 0.f;
};

namespace hjcd {
// The scene's obstacle grid for a robot whose coarse link spheres all fit its
// margin; an empty grid (flat obstacle loops) otherwise or without a scene.
ObstacleGrid scene_grid(const hjcd_scene_s* sc, const hjcd_robot_s* r);
}  // namespace hjcd
