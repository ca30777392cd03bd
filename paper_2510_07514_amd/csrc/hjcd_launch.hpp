// Internal launch interface between the C ABI (hjcd_api.cpp) and the kernels
// (hjcd_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hjcd_tables.hpp"

namespace hjcd {

// Seeds live in a robot-grouped slot layout: targets are permuted so that
// the targets of one robot are consecutive (tperm: permuted position ->
// target id, nullptr = identity) and voffs [T+1] is the CSR of seed slots
// over the permuted targets.  One launch covers the permuted targets
// [tb, te) of one robot, i.e. the slots [base, base + Sv).
struct SeedMap {
    const int64_t* voffs;    // [T+1] device
    const int32_t* tperm;    // [T] device or nullptr
    int32_t T;
    int32_t tb, te;
    int64_t base, Sv;
    const uint32_t* tkeys;   // [T] by target id, device or nullptr
};

struct KernelParams {
    int32_t cd_sweeps, polish_iters, ls_A, weight_mode;
    float eps_cd2, nu_cd, gamma, delta0, delta_decay, delta_min, proj_eps2, tie_eps;
    float lam, lambda_gn, trust_R, inv_beta;
    float eps_pol2, ups_pol, sigma, mu;
    uint64_t seed;
};

enum InitMode { INIT_LOAD = 0, INIT_UNIFORM = 1 };

// Per-seed CD and/or PJ-IK over the slots of `map`.  q_in [n][q_in_stride]
// (INIT_LOAD) or unused; q_out [n][S] (may alias q_in); err_p / err_o / cost
// [S] nullable; traj [rows][n+2][S] nullable.
struct SolveArgs {
    const DevRobot* rb;
    int32_t n;
    int32_t n_rows;          // q_out rows n..n_rows-1 are written as 0 (mixed-dof batches)
    SeedMap map;
    int64_t S;               // seed slots (row stride of q arrays)
    const float* targets;    // [7][T]
    const float* q_in;
    int64_t q_in_stride;     // row stride of q_in (usually S)
    float* q_out;
    float* err_p;
    float* err_o;
    float* cost;
    float* traj;
    int32_t init_mode;
    int32_t do_cd, do_polish;
    KernelParams kp;
    unsigned long long* counters;  // [9] or nullptr
    int32_t variant;         // occupancy variant of PJ-IK (0 default, 1 the alternative)
    int32_t block_threads;   // workgroup size: 64, 128 or 256 (0 = 256)
    int64_t seeds_per_wave;  // PJ-IK seed streaming: seeds per wave (set by the launch)
    int32_t cd_lanes;        // lanes per seed of PO-CCD: 1, or 2 (buckets of 12 joints and more)
};

// Seeds per lane of a PJ-IK launch over Sv seeds: Sv / (8192 x 64) between 1
// and 8, so a launch keeps at least about 8,192 waves (several per wave slot
// of the chip); above 1 the launch streams seeds through its waves.
inline int64_t stream_factor(int64_t Sv) {
    const int64_t r = Sv / (64 * 8192);
    return r < 1 ? 1 : (r > 8 ? 8 : r);
}

hipError_t launch_solve(const SolveArgs& a, hipStream_t st);

hipError_t launch_fk(const DevRobot* rb, int n, int64_t S, const float* q, float* pose, float* jac,
                     hipStream_t st);

// Uniform grid over a scene's obstacles (built by hjcd_load_scene for
// scenes of kGridMinObstacles obstacles or more): cell (i, j, k) of size h
// from corner lo lists, in [start[c], start[c + 1]) of items, every obstacle
// (sphere index, or n_osph + box index) whose bounding box grown by the
// grid's margin overlaps the cell.  A coarse sphere of radius <= margin whose
// centre lies in a cell can only touch the obstacles that cell lists, and
// none when its centre lies outside the grid.  start == nullptr: no grid
// (flat loops over every obstacle).
struct ObstacleGrid {
    const int32_t* start;
    const int32_t* items;
    float lo[3];
    float inv_h;
    int32_t n[3];
};
constexpr int kGridMinObstacles = 96;

struct CollideArgs {
    const DevRobot* rb;
    int32_t n;
    int64_t S;
    const float* q;          // [n][q_stride]
    int64_t q_stride;
    const float* osph;       // [n_osph][4]
    int32_t n_osph;
    const float* obox;       // [n_obox][8]: cx cy cz 0 hx hy hz 0
    int32_t n_obox;
    uint8_t* flag;
    unsigned long long* counters;
    ObstacleGrid grid;
    int32_t n_pairs;  // the robot's self-collision link pairs (0: no self pass)
};

hipError_t launch_collide(const CollideArgs& a, hipStream_t st);

struct SelectArgs {
    int32_t T;
    const int64_t* offsets;  // [T+1] device, CSR over permuted targets
    const int32_t* tperm;    // [T] permuted position -> target id, nullptr = identity
    int32_t n, n_stride;
    int64_t S;
    const float* q;          // [n][S]
    const float* cost;
    const float* err_p;
    const float* err_o;
    const uint8_t* flag;
    int32_t k;
    float succ_pos, succ_ori;
    float* q_out;
    float* ep_out;
    float* eo_out;
    uint8_t* fl_out;
    int32_t* n_free;
    uint8_t* solved;
    const float* q_ref;      // [T][n_stride] by target id, or nullptr (cost order)
};

hipError_t launch_select(const SelectArgs& a, hipStream_t st);

// Warm start for targets on a path: q_out [n][T*M] from q_prev [T*k][n_stride].
hipError_t launch_warm(const DevRobot* rb, int n, int32_t T, int32_t k, int32_t n_stride, const float* q_prev,
                       int32_t M, const uint32_t* tkeys, uint64_t seed, float mu, float sigma, float* q_out,
                       hipStream_t st);

// Mid top-K ranking over permuted targets: rank [T][K] = seed indices
// (within target) of the K smallest (cost, index); rank r >= M repeats rank
// r % M.
hipError_t launch_rank(int32_t T, const int64_t* offsets, const float* cost, int32_t K, int32_t* rank,
                       hipStream_t st);

// Noisy replication for the permuted targets [tb, te): slot b*Bp + i*K + kk
// of q_out [n][T*Bp] <- q_in [n][S_in] at offsets[b] + rank[b][kk].
hipError_t launch_replicate(const DevRobot* rb, int n, int32_t tb, int32_t te, int32_t T,
                            const int64_t* offsets, const int32_t* tperm, int64_t S_in,
                            const float* q_in, const int32_t* rank, int32_t K, int32_t Bp,
                            const uint32_t* tkeys, uint64_t seed, float mu, float sigma, float* q_out,
                            hipStream_t st);

// Gather caller-layout seeds [n][S] (CSR `offsets` by target id) into the
// robot-grouped layout q_out [n][S] (CSR `voffs` over permuted targets).
hipError_t launch_gather(int n, int32_t T, const int64_t* offsets, const int64_t* voffs,
                         const int32_t* tperm, int64_t S, int64_t in_stride, const float* q_in,
                         float* q_out, hipStream_t st);

// ---- serving -----------------------------------------------------------------
// Resident seed slots of the serving loop.  Slots come in blocks of 64 (one
// wave); every block belongs to one request, so all its lanes share the stage
// and the iteration range of a chunk.
enum SlotBits : uint8_t {
    SLOT_LIVE = 1,       // slot holds a seed
    SLOT_CD_FROZEN = 2,  // PO-CCD exit test passed
    SLOT_POL_FROZEN = 4, // PJ-IK exit test passed
    SLOT_CHECKED = 8,    // collision tested
    SLOT_COLLIDES = 16,  // collision test result
    SLOT_RETIRED = 32    // its target is finished: no more work
};
enum ServeStage { SERVE_CD = 0, SERVE_POLISH = 1 };

struct ServeBlock {
    int32_t block;  // slots [64 block, 64 block + 64)
    int32_t stage;  // ServeStage
    int32_t k0, k1; // iteration range of this chunk
};

struct ServeState {
    float* q;                  // [n][C]
    uint8_t* sstate;           // [C]
    int32_t* slot_target;      // [C] target table index
    uint32_t* slot_m;          // [C] seed index within the target
    float* err_p;              // [C]
    float* err_o;              // [C]
    float* cost;               // [C]
    int64_t C;
    const float* tgt_pose;     // [7][Tc]
    const uint32_t* tgt_key;   // [Tc]
    int32_t Tc;
};

struct ServeChunkArgs {
    const DevRobot* rb;
    int32_t n;
    ServeState st;
    const ServeBlock* blocks;  // [nb]
    int32_t nb;
    KernelParams kp;
};

hipError_t launch_serve_chunk(const ServeChunkArgs& a, hipStream_t stream);

// Collision test of the blocks' slots that are live, not retired, not yet
// tested and (all_lanes or PJ-IK-frozen).
struct ServeCheckArgs {
    const DevRobot* rb;
    int32_t n;
    ServeState st;
    const ServeBlock* blocks;
    int32_t nb;
    const int32_t* all_lanes;  // [nb] 1: test every live lane of the block (end of PJ-IK)
    const float* osph;
    int32_t n_osph;
    const float* obox;
    int32_t n_obox;
    ObstacleGrid grid;
};

hipError_t launch_serve_check(const ServeCheckArgs& a, hipStream_t stream);

// Per-target decision after a chunk: a target with a tested collision-free
// seed within (succ_pos, succ_ori) is solved (best such seed by (cost,
// index)); a target marked final takes its best seed by (flag, cost, index).
// Finished targets retire their slots.
struct ServeReduceArgs {
    ServeState st;
    int32_t n;
    const int32_t* targets;    // [nt] target table indices
    const int64_t* first_slot; // [nt]
    const int32_t* n_seeds;    // [nt]
    const int32_t* final_;     // [nt]
    int32_t nt;
    float succ_pos, succ_ori;
    int32_t* status;           // [nt] out: 0 running, 1 solved, 2 finished unsolved
    float* res;                // [nt][n + 3] out: q, err_p, err_o, flag
};

hipError_t launch_serve_reduce(const ServeReduceArgs& a, hipStream_t stream);

// Slot and target-table initialisation for admitted requests: slot base + i
// (i < n_targets * M) gets target tbl0 + i / M, seed index i % M; padding
// lanes up to `padded` are dead.  Target tbl0 + k takes pose row up0 + k of
// the upload (AoS [7] floats) and Philox key key0 + k.
struct ServeAdmit {
    int64_t base;
    int32_t n_targets;
    int32_t M;
    int32_t padded;  // slots allocated (multiple of 64)
    int32_t tbl0;    // first target table index (targets of a request are consecutive)
    int32_t up0;     // first pose row in the upload
    uint32_t key0;   // Philox key of the request's first target
};

hipError_t launch_serve_admit(const ServeAdmit* adm, int32_t n_adm, const float* up_pose, float* tgt_pose,
                              uint32_t* tgt_key, ServeState st, hipStream_t stream);

hipError_t launch_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                         int64_t count, uint32_t* out, hipStream_t st);

}  // namespace hjcd
