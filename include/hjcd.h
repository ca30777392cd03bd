/*
 * libhjcd: batched HJCD-IK on AMD Instinct MI355X (gfx950).
 *
 * HJCD-IK (arXiv 2510.07514) solves inverse kinematics (Sec. II, eq. ik /
 * eq. opt) by sampling many seeds per target pose, running an
 * orientation-aware greedy coordinate descent on each (PO-CCD, Sec. III,
 * Sec. IV-A, Alg. PO-CCD), polishing with a damped weighted Jacobian solver
 * (PJ-IK, Sec. IV-B, Alg. PJ-IK), filtering with sphere collision checks
 * (Sec. IV-C) and returning the best collision-free configurations
 * (Alg. HJCD-IK).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Status codes: HJCD_OK (0) or a negative hjcd_status.  No exception
 *    crosses the ABI.  On a non-OK status hjcd_last_error() returns a
 *    thread-local message.  Every argument check runs before any device
 *    work is queued, so a rejected call changes nothing.
 *  - Device pointers are HIP device allocations on the context's device
 *    (e.g. torch tensor data_ptr()); host pointers are marked "host".  The
 *    caller owns every array; the library never frees or keeps them past the
 *    call's stream work.
 *  - Work is queued on `stream` (a hipStream_t, NULL = legacy default
 *    stream) and is asynchronous: outputs are valid once the stream has
 *    synchronised.  Context-owned scratch is reused across calls, so calls
 *    on one context must be issued from one host thread at a time and must
 *    not overlap on different streams.
 *  - Layouts: per-seed joint arrays are structure-of-arrays float32
 *    [n][S] (joint-major, seed index fastest) so that one seed per lane
 *    reads coalesced rows.  Seeds are grouped per target in CSR order:
 *    target t owns seeds seed_offsets[t] .. seed_offsets[t+1]-1.
 *    Targets are SoA float32 [7][T]: px, py, pz (m), qw, qx, qy, qz (unit
 *    quaternion, renormalised by the library).
 *  - Random draws use Philox4x32-10 keyed by (rng_seed) with counter
 *    (seed index within its target, target key, stage << 24 | iteration,
 *    block); target_keys (device uint32 [T], NULL = target index) make the
 *    draws of a target independent of its position in a batch.
 */
#ifndef HJCD_H
#define HJCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HJCD_MAX_DOF 32
#define HJCD_MAX_ANGLE 1000.0  /* |q_min|, |q_max|, |offset| bound (rad) */
#define HJCD_MAX_SPHERES 1024
#define HJCD_MAX_OBSTACLES 65536
#define HJCD_MAX_TOPK 64
#define HJCD_MAX_ROBOTS 16

typedef enum {
    HJCD_OK = 0,
    HJCD_E_INVALID = -1,      /* bad argument: null, size, non-finite, out of range */
    HJCD_E_NOMEM = -2,        /* device allocation failed */
    HJCD_E_DEVICE = -3,       /* no usable gfx950 device / HIP runtime error */
    HJCD_E_UNSUPPORTED = -4,  /* valid but unsupported (e.g. dof > HJCD_MAX_DOF) */
    HJCD_E_BUSY = -5,         /* server queue full */
    HJCD_E_INTERNAL = -6
} hjcd_status;

typedef enum { HJCD_DH_MODIFIED = 0, HJCD_DH_STANDARD = 1 } hjcd_dh_convention;

typedef struct hjcd_ctx_s* hjcd_ctx;
typedef struct hjcd_robot_s* hjcd_robot;
typedef struct hjcd_scene_s* hjcd_scene;

/* Robot description (host memory, copied by hjcd_load_robot).
 * Kinematics (Sec. II, eq. fk): a serial chain of `dof` revolute joints.
 *   modified DH: {i-1}T_i = Rx(alpha_i) Tx(a_i) Rz(q_i + offset_i) Tz(d_i), joint i
 *                turns about z of frame i;
 *   standard DH: {i-1}T_i = Rz(q_i + offset_i) Tz(d_i) Tx(a_i) Rx(alpha_i), joint i
 *                turns about z of frame i-1;
 *   end effector = T_0n * tool (tool: row-major 4x4 rigid transform, NULL = I).
 * Joint limits q_min <= q <= q_max (eq. opt).
 * Collision geometry (Sec. IV-C): spheres (x, y, z, r) in the frame of link
 * sphere_link[i] (link 0 = base, link l moves with joint l).  Self pairs are
 * tested between spheres whose links differ by >= min_link_gap (0 = no
 * self test). */
typedef struct {
    int32_t dof;
    int32_t convention;           /* hjcd_dh_convention */
    const double* a;              /* [dof] m */
    const double* d;              /* [dof] m */
    const double* alpha;          /* [dof] rad */
    const double* offset;         /* [dof] rad */
    const double* q_min;          /* [dof] rad */
    const double* q_max;          /* [dof] rad */
    const double* tool;           /* [16] or NULL */
    int32_t n_spheres;            /* 0..HJCD_MAX_SPHERES */
    const int32_t* sphere_link;   /* [n_spheres] in 0..dof */
    const double* sphere_xyzr;    /* [n_spheres*4] */
    int32_t min_link_gap;
} hjcd_robot_desc;

/* Solver parameters.  The paper fixes none of these values (only lambda > 0);
 * hjcd_params_default() fills the defaults this library documents. */
typedef struct {
    int32_t cd_sweeps;       /* PO-CCD iterations (Alg. PO-CCD max_iters) */
    int32_t polish_iters;    /* PJ-IK iterations (Alg. PJ-IK max_iters) */
    float eps_cd, nu_cd;     /* PO-CCD exit: |r_p| < eps_cd (m) and phi < nu_cd (rad) */
    float gamma;             /* PO-CCD acceptance: improvement of |r_p|^2 or |omega|^2 > gamma */
    float delta0, delta_decay, delta_min;  /* delta(k) = max(delta_min, delta0 * decay^k) */
    float proj_eps;          /* position step is 0 when EE or target is closer than this (m) to the joint axis */
    float tie_eps;           /* greedy joint picks: candidates within tie_eps (m / rad) of the best tie; lowest joint wins */
    float lambda_;           /* LM damping lambda of eq. (normal-eqs) */
    float lambda_gn;         /* regulariser of the dogleg Gauss-Newton step */
    float trust_R;           /* trust radius R (rad) */
    float ls_beta;           /* line-search ratio beta */
    int32_t ls_A;            /* line search tries 1, 1/beta, ..., 1/beta^A */
    int32_t weight_mode;     /* 0: W normalises the rows of J; 1: W = I */
    float eps_pol, ups_pol;  /* PJ-IK exit: |r_p| < eps_pol (m) and phi < ups_pol (rad) */
    float sigma, mu;         /* perturbation N(mu, sigma^2 I) (rad) */
    int32_t resample_K;      /* > 0: keep the best K CD seeds per target ... */
    int32_t resample_B;      /* ... and polish floor(B/K)*K noisy copies (Alg. HJCD-IK); 0 = off */
    int32_t top_k;           /* solutions returned per target, 1..HJCD_MAX_TOPK */
    float succ_pos, succ_ori;/* success: collision free and |r_p| <= succ_pos, phi <= succ_ori */
    uint64_t rng_seed;       /* Philox key */
    int32_t collect_stats;   /* 0: none; 1: time each kernel and count executed work (the per-seed
                                kernels then run a build with counters); 2: time each kernel only
                                (the kernels of collect_stats = 0, counts read 0); hjcd_get_stats */
    int32_t polish_variant;  /* launch shape of the PJ-IK kernel: 0 default, 1 the other occupancy
                                (waves per SIMD 3 / 2 up to 8 joints, 2 / 1 up to 24, 1 / 2 above);
                                the arithmetic is the same, so results are bit-identical */
    int32_t cd_lanes_per_seed;  /* PO-CCD lanes per seed: 1 (or 0), or 2 for robots of 9 joints or
                                   more (a lane pair splits the per-joint candidates; smaller robots
                                   keep one lane); same steps and decisions either way */
} hjcd_params;

/* Per-call measurements of the last hjcd_solve / stage call made with
 * collect_stats = 1 or 2 on a context (work counts with 1 only).  Stage times
 * are HIP-event intervals on the call's stream: hjcd_solve reports its PO-CCD
 * kernels in ms_cd and its PJ-IK kernels in ms_polish (with resampling, the
 * replication in ms_resample). */
typedef struct {
    float ms_init, ms_cd, ms_resample, ms_polish, ms_collide, ms_select;
    float ms_total;          /* first to last event of the call */
    uint64_t seeds;          /* seeds processed */
    uint64_t cd_iters;       /* PO-CCD iterations executed (over all seeds) */
    uint64_t cd_perturb;
    uint64_t pol_iters;      /* PJ-IK iterations executed */
    uint64_t pol_trials;     /* trial cost evaluations */
    uint64_t pol_dogleg, pol_single, pol_perturb;
    uint64_t coll_coarse, coll_fine;  /* sphere-obstacle and sphere-sphere tests */
} hjcd_stats;

/* ---- context ------------------------------------------------------------- */

/* Bind to HIP device `device` (must be gfx950).  HJCD_E_DEVICE when no such
 * device exists (e.g. on a host without GPUs). */
hjcd_status hjcd_ctx_create(int device, hjcd_ctx* out);
/* Synchronises the device and frees the context's buffers.  Robots, scenes,
 * servers and plans created on it own their memory and may be destroyed
 * after it (but not used with it any more). */
void hjcd_ctx_destroy(hjcd_ctx ctx);
const char* hjcd_last_error(void);
void hjcd_params_default(hjcd_params* p);
const char* hjcd_version(void);

/* ---- models -------------------------------------------------------------- */

/* Validate and upload a robot (Sec. II kinematics, Sec. IV-C spheres).  Builds
 * the per-link coarse spheres and the self-collision link-pair list.  Host
 * only apart from one synchronous upload. */
hjcd_status hjcd_load_robot(hjcd_ctx ctx, const hjcd_robot_desc* desc, hjcd_robot* out);
void hjcd_robot_destroy(hjcd_robot robot);
int32_t hjcd_robot_dof(hjcd_robot robot);

/* Obstacles (eq. opt, g(q) >= 0): n_spheres x (x, y, z, r) and n_boxes x
 * (cx, cy, cz, hx, hy, hz) axis-aligned boxes, host float32, copied. */
hjcd_status hjcd_load_scene(hjcd_ctx ctx, int32_t n_spheres, const float* spheres, int32_t n_boxes,
                            const float* boxes, hjcd_scene* out);
void hjcd_scene_destroy(hjcd_scene scene);

/* ---- stages (one robot) ----------------------------------------------------
 * Each stage runs the same device code the whole solve runs. */

/* Forward kinematics (eq. fk) and geometric Jacobian (eq. jacobian) of S
 * configurations q [n][S]: pose [7][S] (px py pz qw qx qy qz, qw >= 0) and,
 * if jac != NULL, jac [6][n][S] (rows: linear xyz, angular xyz). */
hjcd_status hjcd_fk(hjcd_ctx ctx, hjcd_robot robot, int64_t S, const float* q, float* pose,
                    float* jac, void* stream);

/* Uniform seeds in the joint limits (Alg. PO-CCD, first lines): q [n][S]. */
hjcd_status hjcd_init_seeds(hjcd_ctx ctx, hjcd_robot robot, int32_t T,
                            const int64_t* seed_offsets /* host [T+1] */,
                            const uint32_t* target_keys, uint64_t rng_seed, float* q, void* stream);

/* PO-CCD (Alg. PO-CCD) on every seed, q [n][S] in/out.  Outputs (nullable):
 * err_p, err_o, cost [S] at the final configuration (|r_p|, phi, 0.5(|r_p|^2 +
 * phi^2)); traj [(cd_sweeps+1)][n+2][S]: configuration, |r_p|, phi before
 * each iteration and after the last. */
hjcd_status hjcd_cd(hjcd_ctx ctx, hjcd_robot robot, int32_t T, const float* targets,
                    const int64_t* seed_offsets /* host */, const uint32_t* target_keys,
                    const hjcd_params* params, float* q, float* err_p, float* err_o, float* cost,
                    float* traj, void* stream);

/* PJ-IK (Alg. PJ-IK) on every seed; same conventions with polish_iters. */
hjcd_status hjcd_polish(hjcd_ctx ctx, hjcd_robot robot, int32_t T, const float* targets,
                        const int64_t* seed_offsets /* host */, const uint32_t* target_keys,
                        const hjcd_params* params, float* q, float* err_p, float* err_o,
                        float* cost, float* traj, void* stream);

/* Collision filter (Sec. IV-C): flag [S] = 1 when any robot sphere overlaps
 * an obstacle or an allowed self pair overlaps, else 0.  scene may be NULL. */
hjcd_status hjcd_collide(hjcd_ctx ctx, hjcd_robot robot, hjcd_scene scene, int64_t S,
                         const float* q, uint8_t* flag, void* stream);

/* Top-K and noisy replication between the stages (Alg. HJCD-IK): per target,
 * the K seeds of smallest (cost, index) are copied floor(B/K) times with
 * N(mu, sigma^2 I) noise into q_out [n][T*B'], B' = floor(B/K)*K; copy i of
 * rank k lands at slot t*B' + i*K + k.  Targets with fewer than K seeds repeat
 * their seeds in rank order. */
hjcd_status hjcd_resample(hjcd_ctx ctx, hjcd_robot robot, int32_t T,
                          const int64_t* seed_offsets /* host */, const uint32_t* target_keys,
                          const hjcd_params* params, const float* q_in, const float* cost_in,
                          float* q_out, void* stream);

/* Final selection (Alg. HJCD-IK, last line, extended to top_k): per target,
 * order seeds by (flag != 0, cost, index) and return the first top_k:
 * q_out [T*k][n_stride] (row-major, unused joints 0), err_p/err_o [T*k],
 * flag_out [T*k] (255 = empty slot), n_free [T] (collision-free seeds),
 * solved [T] (a returned seed is collision free within succ_pos/succ_ori). */
hjcd_status hjcd_select(hjcd_ctx ctx, int32_t T, const int64_t* seed_offsets /* host */,
                        int32_t n, int32_t n_stride, const hjcd_params* params, const float* q,
                        const float* cost, const float* err_p, const float* err_o,
                        const uint8_t* flag, float* q_out, float* err_p_out, float* err_o_out,
                        uint8_t* flag_out, int32_t* n_free, uint8_t* solved, void* stream);

/* ---- tracking: targets along a path (Sec. V, hardware demonstration) -------
 * The paper's demonstration tracks a moving pose in real time, keeping the
 * returned solutions continuous.  Each pose of the path is solved from the
 * solution set of the previous pose, and the returned solution is the one
 * nearest the current configuration (readings: the paper gives no formula). */

/* Warm-start seeds: q_prev [T*k][n_stride] (row-major, e.g. the q_out of the
 * previous pose's hjcd_solve / hjcd_solve_near with top_k = k) -> q_out
 * [n][T*M] (SoA, usable as hjcd_solve's seeds with M seeds per target).
 * Seed m of target t starts at previous solution m mod k clipped to the
 * limits; for m >= k it is also moved to clip(. + mu + sigma z), z drawn for
 * seed index m at stage WARM (4) with the target's key. */
hjcd_status hjcd_warm_seeds(hjcd_ctx ctx, hjcd_robot robot, int32_t T, int32_t k, int32_t n_stride,
                            const float* q_prev, int32_t M, const uint32_t* target_keys,
                            const hjcd_params* params, float* q_out, void* stream);

/* hjcd_select with the nearest-solution order: per target, seeds that are
 * collision free with err_p <= succ_pos and err_o <= succ_ori come first,
 * ordered by squared joint distance to q_ref [T][n_stride] (device, row t =
 * target t's current configuration); then the other collision-free seeds and
 * then the colliding ones, each by cost; ties -> lower index.  n_free and
 * solved as hjcd_select. */
hjcd_status hjcd_select_near(hjcd_ctx ctx, int32_t T, const int64_t* seed_offsets /* host */, int32_t n,
                             int32_t n_stride, const hjcd_params* params, const float* q, const float* cost,
                             const float* err_p, const float* err_o, const uint8_t* flag, const float* q_ref,
                             float* q_out, float* err_p_out, float* err_o_out, uint8_t* flag_out,
                             int32_t* n_free, uint8_t* solved, void* stream);

/* ---- the whole batched solve (Alg. HJCD-IK) --------------------------------
 * T targets, each solved with the robot robots[robot_of_target[t]] (host,
 * NULL = robots[0]) from its seeds: seeds [n_max][S] (device, rows beyond a
 * robot's dof ignored, values clipped to the limits) or NULL for uniform
 * Philox seeds.  Outputs as hjcd_select with n_stride = n_max.  A target
 * whose seeds all collide or miss still returns its best top_k (solved = 0);
 * a target with no seeds returns empty slots. */
hjcd_status hjcd_solve(hjcd_ctx ctx, int32_t n_robots, const hjcd_robot* robots, hjcd_scene scene,
                       int32_t T, const int32_t* robot_of_target /* host */, const float* targets,
                       const int64_t* seed_offsets /* host [T+1] */, const uint32_t* target_keys,
                       const float* seeds, const hjcd_params* params, float* q_out, float* err_p,
                       float* err_o, uint8_t* flag, int32_t* n_free, uint8_t* solved, void* stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): hjcd_solve with the
 * same arguments, results and errors, whose work arrays (grouped seeds, CD and
 * PJ-IK state, costs, flags, the layout upload) live in a static device
 * workspace of HJCD_NOALLOC_SCRATCH_BYTES per device, held from library load
 * to process end, instead of context buffers grown on demand.  It calls no
 * allocating routine.  Limits: T <= HJCD_NOALLOC_MAX_TARGETS; the work must
 * fit the workspace: (n_max + 3) x 4 + 1 bytes per seed slot (also per
 * resampled slot, plus n_max x 4 per CD seed when resampling) and ~24 bytes
 * per target, else HJCD_E_INVALID (e.g. 1.6 M seeds of a 7-joint chain);
 * collect_stats must be 0 (HJCD_E_UNSUPPORTED).  Every call on one device
 * shares that device's workspace: calls that overlap on one device (other
 * streams, other contexts, other threads) race and must be serialised by the
 * caller.  Nothing in the workspace needs to start at zero. */
#define HJCD_NOALLOC_SCRATCH_BYTES (64u << 20)
#define HJCD_NOALLOC_MAX_TARGETS 65536
hjcd_status hjcd_solve_noalloc(hjcd_ctx ctx, int32_t n_robots, const hjcd_robot* robots, hjcd_scene scene,
                               int32_t T, const int32_t* robot_of_target /* host */, const float* targets,
                               const int64_t* seed_offsets /* host [T+1] */, const uint32_t* target_keys,
                               const float* seeds, const hjcd_params* params, float* q_out, float* err_p,
                               float* err_o, uint8_t* flag, int32_t* n_free, uint8_t* solved, void* stream);

/* hjcd_solve whose final selection is hjcd_select_near's order around
 * q_ref [T][n_max] (device): the tracking form of the whole solve. */
hjcd_status hjcd_solve_near(hjcd_ctx ctx, int32_t n_robots, const hjcd_robot* robots, hjcd_scene scene, int32_t T,
                            const int32_t* robot_of_target /* host */, const float* targets,
                            const int64_t* seed_offsets /* host [T+1] */, const uint32_t* target_keys,
                            const float* seeds, const hjcd_params* params, const float* q_ref, float* q_out,
                            float* err_p, float* err_o, uint8_t* flag, int32_t* n_free, uint8_t* solved,
                            void* stream);

/* Measurements of the last call made with collect_stats = 1 or 2
 * (synchronises the stream that call used). */
hjcd_status hjcd_get_stats(hjcd_ctx ctx, hjcd_stats* out);

/* ---- reusable plans (uneven batches) -----------------------------------------
 * A plan fixes one batch: robots, scene, targets grouped by robot, seed
 * offsets, params and the device buffers every execution reads and writes
 * (the arguments of hjcd_solve).  At creation it uploads the batch layout
 * once, optionally autotunes the per-seed kernels' launch shapes per robot
 * (PJ-IK occupancy variant x workgroup size, PO-CCD lanes per seed for
 * robots of 9 joints or more; timed on these buffers, fastest kept), and captures the whole solve into one hipGraph: the robots' solve
 * and collision kernels on concurrent branches, then the selection.
 * hjcd_plan_execute replays that graph on a stream: one launch for the whole
 * uneven batch.  The results equal hjcd_solve's on the same inputs, bit for
 * bit (the tuner chooses launch shapes only).  With resample_K > 0 each
 * robot's branch ranks its targets' CD seeds and polishes the replicated
 * ones (Alg. HJCD-IK) before its collision test.  Plans collect no
 * statistics.  The
 * caller keeps the buffers alive and unchanged in size until
 * hjcd_plan_destroy; their contents may change between executions. */
typedef struct hjcd_plan_s* hjcd_plan;

typedef struct {
    int32_t variant;        /* PJ-IK occupancy: 0 default, 1 the alternative (waves per SIMD
                               0 / 1: 3 / 2 up to 8 joints, 2 / 1 up to 24, 1 / 2 above) */
    int32_t block_threads;  /* workgroup size of the PJ-IK kernel (64 without tuning, as in
                               hjcd_solve; PO-CCD runs 256-thread workgroups) */
    float ms;               /* measured time of the chosen PJ-IK shape (0 when not tuned) */
    int64_t seeds;          /* seeds of this robot in the batch */
    int32_t cd_lanes;       /* PO-CCD lanes per seed chosen (1 or 2) */
    float cd_ms;            /* measured PO-CCD time with that choice (0 when not tuned) */
} hjcd_tune_choice;

hjcd_status hjcd_plan_create(hjcd_ctx ctx, int32_t n_robots, const hjcd_robot* robots, hjcd_scene scene,
                             int32_t T, const int32_t* robot_of_target /* host, or NULL */,
                             const float* targets, const int64_t* seed_offsets /* host [T+1] */,
                             const uint32_t* target_keys, const float* seeds, const hjcd_params* params,
                             float* q_out, float* err_p, float* err_o, uint8_t* flag, int32_t* n_free,
                             uint8_t* solved, int32_t tune, void* stream, hjcd_plan* out);
/* Replay the plan's graph on `stream` (asynchronous). */
hjcd_status hjcd_plan_execute(hjcd_plan plan, void* stream);
/* Launch shape used for robot index `robot` of the plan. */
hjcd_status hjcd_plan_choice(hjcd_plan plan, int32_t robot, hjcd_tune_choice* out);
void hjcd_plan_destroy(hjcd_plan plan);

/* ---- serving ----------------------------------------------------------------
 * A request loop over one robot and scene.  Requests (a few target poses with
 * a seed budget each) are submitted with a scheduled arrival time on the
 * server clock; a scheduler thread admits arrived requests as long as their
 * seeds fit in the resident slot pool (sized from a device-memory budget),
 * keeps every admitted seed's state resident in device memory, and advances
 * all of them together in chunks of `chunk_iters` iterations (continuous
 * batching: requests join and leave between chunks; a request whose PO-CCD
 * ends in a chunk also runs its first PJ-IK chunk in the same step).  A target retires at the
 * end of the first chunk in which one of its PJ-IK-converged seeds is
 * collision free within succ_pos / succ_ori (its best such seed by (cost,
 * index)); otherwise it returns its best seed by (collision, cost, index)
 * after the last PJ-IK iteration.  Every decision is taken at request-local
 * iteration counts and the random draws are keyed by the request tag, so a
 * request's result does not depend on what else is resident.
 * HJCD_SERVE_PLAIN runs the same stream one request at a time with
 * hjcd_solve (no cross-request batching, no early retirement), for
 * comparison; its scheduler thread calls hjcd_solve on the server's context,
 * which must not be used by other threads meanwhile.  Times are seconds since
 * hjcd_server_start.  Memory: the batched server allocates its slot pool
 * ((dof + 3) floats + 9 bytes per slot) and target table at create; nothing
 * is allocated per request on the device. */
typedef struct hjcd_server_s* hjcd_server;

typedef enum { HJCD_SERVE_BATCHED = 0, HJCD_SERVE_PLAIN = 1 } hjcd_serve_mode;

typedef struct {
    int32_t mode;          /* hjcd_serve_mode */
    int64_t max_slots;     /* resident seed slots (rounded up to 64); 0 = from hbm_budget */
    size_t hbm_budget;     /* bytes for resident state when max_slots = 0, rounded down to whole
                              64-slot blocks; HJCD_E_NOMEM below one block (0 = a quarter of
                              free memory, at most 8 GiB) */
    int32_t max_targets;   /* resident targets (0 = slots / 32, between 64 and 2^20) */
    int32_t chunk_iters;   /* iterations per chunk (>= 1); at least the stage lengths (one chunk per
                              stage, the first PJ-IK chunk in the step that ends PO-CCD) gives the
                              lowest latency, shorter chunks retire targets at more points */
    int32_t max_queue;     /* pending requests accepted before submit returns HJCD_E_BUSY */
    int32_t pipelines;     /* scheduler steps in flight at once, 1..HJCD_SERVE_MAX_PIPELINES (0 = 2):
                              each has its own stream and keeps the requests it admitted; a request
                              that arrives while steps run starts on a free one.  More pipelines
                              lower latency at high load and raise it at light load */
} hjcd_server_config;

#define HJCD_SERVE_MAX_PIPELINES 4

typedef struct {
    int64_t request_id;
    uint64_t tag;
    int32_t n_targets;
    int32_t n_solved;      /* targets solved (collision free within tolerance) */
    double arrival_s, admitted_s, done_s;
} hjcd_request_info;

typedef struct {
    int64_t submitted, admitted, completed, chunks;
    int64_t targets_solved, targets_done;
    int64_t max_slots, resident_slots_peak;
    double mean_resident_slots;  /* over chunks */
    double p50_latency_ms, p99_latency_ms;  /* done - arrival over completed requests */
    double first_arrival_s, last_done_s;
    double solves_per_s;   /* targets_solved / (last_done - first_arrival) */
    int64_t overlapped_steps;  /* steps launched while another pipeline's step was in flight */
} hjcd_server_stats;

hjcd_status hjcd_server_create(hjcd_ctx ctx, hjcd_robot robot, hjcd_scene scene /* nullable */,
                               const hjcd_params* params, const hjcd_server_config* config,
                               hjcd_server* out);
/* Set the server clock to 0 and start the scheduler thread. */
hjcd_status hjcd_server_start(hjcd_server srv);
/* Queue one request: targets host float [n_targets][7] (px py pz qw qx qy qz),
 * seeds_per_target >= 1, tag keys the random draws (target i of the request
 * uses Philox target key (uint32)(tag + i), the key hjcd_solve gives target
 * tag + i by default; seed m of it starts at the uniform draw of seed index
 * m), arrival_s on the server
 * clock (<= now: arrives immediately).  HJCD_E_NOMEM if it can never fit,
 * HJCD_E_BUSY if max_queue requests are pending.  Thread safe. */
hjcd_status hjcd_server_submit(hjcd_server srv, int32_t n_targets, const float* targets,
                               int32_t seeds_per_target, uint64_t tag, double arrival_s,
                               int64_t* request_id);
/* Completed requests not yet reported (up to max), oldest first. */
hjcd_status hjcd_server_poll(hjcd_server srv, int32_t max, hjcd_request_info* out, int32_t* n_out);
/* Per-target results of a completed request (host arrays, n_targets rows):
 * q [n_targets][dof], err_p, err_o, flag (0 free, 1 colliding, 255 none).
 * The request's record is released afterwards. */
hjcd_status hjcd_server_result(hjcd_server srv, int64_t request_id, float* q, float* err_p, float* err_o,
                               uint8_t* flag);
/* Block until every submitted request has completed or timeout_s elapsed
 * (HJCD_E_BUSY on timeout). */
hjcd_status hjcd_server_wait(hjcd_server srv, double timeout_s);
hjcd_status hjcd_server_get_stats(hjcd_server srv, hjcd_server_stats* out);
void hjcd_server_destroy(hjcd_server srv);

/* Diagnostics: raw Philox4x32-10 words, out[4*i .. 4*i+3] = Philox(ctr =
 * (ctr0 + i, ctr1, ctr2, ctr3), key = (key0, key1)) for i < count, device
 * uint32 [4*count]. */
hjcd_status hjcd_philox(hjcd_ctx ctx, const uint32_t ctr[4], const uint32_t key[2], int64_t count,
                        uint32_t* out, void* stream);

#ifdef __cplusplus
}
#endif
#endif
