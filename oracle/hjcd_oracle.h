/*
 * FP64 CPU oracle for the batched HJCD-IK solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or constant with the GPU library: it is a plain, slow,
 * step-by-step FP64 statement of what the method computes, written from the
 * paper (arXiv 2510.07514):
 *
 *   - forward kinematics and geometric Jacobian      Sec. II, eq. (fk), (jacobian)
 *   - task residual and quaternion error             Sec. II, eq. (task_residual), (quat_diff)
 *   - CCD position step                              Sec. II-A, eq. (vec_proj), (theta_proj)
 *   - orientation angle-axis step                    Sec. III, eq. (angle_axis), (ori_update)
 *   - PO-CCD greedy sweep, gamma test, perturbation  Sec. IV-A, Alg. PO-CCD
 *   - top-K + noisy replication                      Sec. IV, Alg. HJCD-IK
 *   - PJ-IK: weighted LM, trust region, line search,
 *     dogleg, single-coordinate step, perturbation   Sec. IV-B, eq. (normal-eqs),
 *                                                    (line-search), (dogleg), (single-coord),
 *                                                    Alg. PJ-IK
 *   - sphere collision filter and final argmin       Sec. IV-C, Alg. HJCD-IK
 *   - Philox4x32-10 (Salmon et al., SC'11) and Box-Muller normals for the
 *     random draws the paper leaves unspecified.
 *
 * Where the paper is silent or garbled the oracle follows the readings listed
 * in the design notes of the repository (sign conventions, annealing, line
 * search order, dogleg root, single-coordinate step length, constants).
 *
 * All arrays are host memory owned by the caller.  Angles in rad, lengths in m.
 * Functions return 0 on success and a negative value on invalid input.
 */
#ifndef HJCD_ORACLE_H
#define HJCD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAX_DOF 32

/* Categories of the operation counts (see or_ops_get).  A unit is one
 * execution of the step named. */
enum {
    OR_OPS_MISC = 0,       /* work outside any unit (inspection calls, target loading) */
    OR_OPS_EVAL = 1,       /* FK + residual of a configuration: the exit test at the start
                              of an iteration, the evaluation after a stage */
    OR_OPS_INIT = 2,       /* one uniform seed */
    OR_OPS_CD_ITER = 3,    /* one PO-CCD iteration past its exit test: candidates (a full FK
                              per candidate), greedy picks, combination, acceptance test */
    OR_OPS_CD_PERTURB = 4, /* one PO-CCD perturbation */
    OR_OPS_PJ_ITER = 5,    /* one PJ-IK iteration past its exit test: J, W, D, the n x n LM
                              system, its Cholesky solve, the trust-region clamp */
    OR_OPS_PJ_TRIAL = 6,   /* one trial configuration: clip + FK + residual + comparison */
    OR_OPS_PJ_DOGLEG = 7,  /* one dogleg step (its trial is a separate PJ_TRIAL unit) */
    OR_OPS_PJ_SINGLE = 8,  /* one single-coordinate step (trials separate) */
    OR_OPS_PJ_PERTURB = 9, /* one PJ-IK perturbation */
    OR_OPS_RESAMPLE = 10,  /* one replicated seed */
    OR_OPS_COLLIDE = 11,   /* one configuration's collision test (flat, every pair) */
    OR_OPS_SELECT = 12,    /* one target's final ordering */
    OR_OPS_INSTR = 13,     /* test instrumentation (margins, step sensitivity): no unit */
    OR_OPS_NCAT = 14
};

typedef struct {
    int32_t dof;                 /* 1..OR_MAX_DOF */
    int32_t convention;          /* 0 = modified DH (Craig), 1 = standard DH */
    const double* a;             /* [dof] */
    const double* d;             /* [dof] */
    const double* alpha;         /* [dof] */
    const double* offset;        /* [dof] */
    const double* q_min;         /* [dof] */
    const double* q_max;         /* [dof] */
    const double* tool;          /* [16] row-major 4x4 */
    int32_t n_spheres;
    const int32_t* sphere_link;  /* [n_spheres] link index 0..dof */
    const double* sphere_xyzr;   /* [n_spheres*4] centre in link frame, radius */
    int32_t min_link_gap;        /* self pairs need |la-lb| >= gap; 0 = no self test */
} or_robot;

typedef struct {
    int32_t n_spheres;
    const double* spheres;       /* [n*4] x y z r */
    int32_t n_boxes;
    const double* boxes;         /* [n*6] cx cy cz hx hy hz */
} or_scene;

typedef struct {
    int32_t cd_sweeps, polish_iters;
    double eps_cd, nu_cd, gamma, delta0, delta_decay, delta_min, proj_eps, tie_eps;
    double lam, lambda_gn, trust_R, ls_beta;
    int32_t ls_A, weight_mode;
    double eps_pol, ups_pol, sigma, mu;
    int32_t resample_K, resample_B, top_k;
    double succ_pos, succ_ori;
    uint64_t rng_seed;
    /* Test instrumentation, 0 = off: PJ-IK linearises with J and e carrying
     * single-precision-sized pseudo-random errors drawn from this key, and
     * PO-CCD projects its position candidates from joint-to-EE and
     * joint-to-target vectors carrying single-precision-sized absolute
     * errors (a "shadow" run that shows how far rounding alone can move a
     * trajectory). */
    uint64_t shadow;
} or_params;

/* Per-seed record of one stage run (PO-CCD or PJ-IK). */
typedef struct {
    int32_t iters_run;      /* iterations whose update step executed */
    int32_t frozen_at;      /* iteration index at which the exit test fired, -1 = never */
    int32_t n_perturb;      /* perturbations taken */
    int32_t n_trials;       /* PJ-IK: trial cost evaluations (line search + dogleg) */
    int32_t n_dogleg;       /* PJ-IK: dogleg steps computed */
    int32_t n_single;       /* PJ-IK: single-coordinate steps computed */
    int32_t n_tie_pick;     /* PO-CCD: iterations whose tie-tolerant greedy pick (position or
                               orientation joint) differs from the strict lowest-index argmin */
} or_stage_stats;

/* ---- kinematics ---------------------------------------------------------- */

/* FK at theta[dof].  Outputs (any may be NULL):
 *   p_ee[3], R_ee[9] (row-major), quat[4] (w x y z, w >= 0),
 *   joint_P[dof*3], joint_z[dof*3] (origin and unit axis of each joint),
 *   link_T[(dof+1)*12] (rows 0..2 of each link frame, row-major 3x4),
 *   J[6*dof] (row-major 6 x dof geometric Jacobian). */
int or_fk(const or_robot* rb, const double* theta, double* p_ee, double* R_ee, double* quat,
          double* joint_P, double* joint_z, double* link_T, double* J);

/* Rotation matrix -> unit quaternion (w x y z), Shepperd's method, w >= 0. */
void or_quat_from_R(const double* R, double* q);

/* Residual of a pose against a target (p_t[3], q_t[4] w x y z):
 * out[0..2] = r_p = p_t - p_ee, out[3..5] = omega, out[6] = phi,
 * out[7..9] = unit error axis a_hat (0 if phi = 0), out[10] = cost
 * 0.5 (|r_p|^2 + |omega|^2). */
void or_residual(const double* p_t, const double* q_t, const double* p_ee, const double* R_ee,
                 double* out);

/* ---- random numbers ------------------------------------------------------- */

void or_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out);

/* Standard normal draws for one seed: z[dof] keyed by (seed, target key, stage, iter). */
void or_normals(uint64_t rng_seed, uint32_t seed_idx, uint32_t target_key, uint32_t stage,
                uint32_t iter, int dof, double* z);

/* Uniform seed in the joint limits keyed the same way (stage 0). */
void or_uniform_seed(const or_robot* rb, uint64_t rng_seed, uint32_t seed_idx,
                     uint32_t target_key, double* theta);

/* ---- stages (one seed) ---------------------------------------------------- */

/* PO-CCD on one seed.  theta[dof] in/out.  target[7] = px py pz qw qx qy qz.
 * traj (nullable) receives (cd_sweeps+1) rows of (dof + 2) values:
 *   row 0 = start, row k+1 = after iteration k: theta, |r_p|, phi.
 * margin (nullable) receives cd_sweeps values: the smallest decision margin
 * (m or rad) met in each iteration, +inf when the iteration made no
 * consequential decision (see or_cd comments). */
int or_cd(const or_robot* rb, const double* target, const or_params* pr, uint32_t seed_idx,
          uint32_t target_key, double* theta, double* traj, double* margin, or_stage_stats* st);

/* PJ-IK on one seed; same conventions with polish_iters iterations.
 * sens (nullable) receives polish_iters values: how far the step taken in
 * that iteration moves (infinity norm, rad) when J and e carry
 * single-precision-sized errors (0 for perturbations and frozen iterations). */
int or_polish(const or_robot* rb, const double* target, const or_params* pr, uint32_t seed_idx,
              uint32_t target_key, double* theta, double* traj, double* margin, double* sens,
              or_stage_stats* st);

/* Inspection of one PO-CCD iteration k at theta: per-joint clipped position
 * steps dp[dof], orientation steps dor[dof] and their scores sp[dof]
 * (|r_p|^2 after moving that joint alone) and so[dof] (|omega|^2). */
int or_cd_candidates(const or_robot* rb, const double* target, const or_params* pr,
                     const double* theta, int32_t k, double* dp, double* dor, double* sp,
                     double* so);

/* Inspection of the PJ-IK steps at theta: lm[dof] (unclipped LM step),
 * gd[dof], gn[dof] (dogleg gradient and Gauss-Newton steps), dogleg[dof]
 * (blended step), single[dof] (single-coordinate step) and *single_idx. */
int or_pjik_steps(const or_robot* rb, const double* target, const or_params* pr,
                  const double* theta, double* lm, double* gd, double* gn, double* dogleg,
                  double* single, int32_t* single_idx);

/* Collision of one configuration: returns via flag (1 = collides) and
 * min_signed_dist (smallest distance - radii over every tested pair; +inf
 * when nothing was tested). */
int or_collide(const or_robot* rb, const or_scene* sc, const double* theta, int32_t* flag,
               double* min_signed_dist);

/* Final per-target selection over m seeds: stable order by (flag, cost,
 * index); order[k] receives the first k seed indices (-1 past m). */
int or_select(int32_t m, const int32_t* flag, const double* cost, int32_t k, int32_t* order);

/* Top-K ranking and noisy replication between the stages (Alg. HJCD-IK) for T
 * targets: q_in [S*dof] (AoS, CSR offsets[T+1], every target with >= 1 seed),
 * cost_in [S].  Per target t, its seeds are ranked by (cost, index); with
 * K = resample_K and B' = floor(resample_B / K) * K, copy i < floor(B/K) of
 * rank k < K lands at row t*B' + i*K + k of q_out [T*B'*dof] as
 * clip(q + mu + sigma z), z drawn for seed index i*K + k, stage RESAMPLE,
 * iteration 0.  A target with fewer than K seeds repeats its ranked seeds
 * cyclically (rank k takes the seed of rank k mod M).  -1 on invalid input. */
int or_resample(const or_robot* rb, int32_t T, const int64_t* offsets, const double* q_in,
                const double* cost_in, const uint32_t* target_keys, const or_params* pr,
                double* q_out);

/* Warm start for a target on a path (tracking, Sec. V demonstration): q_prev
 * [T*k*dof] holds each target's k previous solutions; seed m < M of target t
 * (row t*M + m of q_out [T*M*dof]) is previous solution m mod k clipped to the
 * limits, and for m >= k additionally moved by clip(. + mu + sigma z), z
 * drawn for seed index m, stage WARM (4), iteration 0.  -1 on invalid input. */
int or_warm_seeds(const or_robot* rb, int32_t T, int32_t k, const double* q_prev, int32_t M,
                  const uint32_t* target_keys, const or_params* pr, double* q_out);

/* Selection nearest to a reference configuration q_ref[dof] over m seeds
 * (q [m*dof]): seeds with flag 0, err_p <= succ_pos and err_o <= succ_ori
 * first, by squared joint distance to q_ref; then collision-free seeds, then
 * colliding ones, each by cost; ties -> lower index.  order[k] as or_select. */
int or_select_near(int32_t m, int32_t dof, const int32_t* flag, const double* cost, const double* err_p,
                   const double* err_o, const double* q, const double* q_ref, double succ_pos, double succ_ori,
                   int32_t k, int32_t* order);

/* ---- whole pipeline --------------------------------------------------------
 * T targets (targets[T*7]), CSR seed offsets[T+1], seeds (nullable, AoS
 * [S*dof] doubles; NULL = uniform Philox seeds), target_keys (nullable, [T];
 * NULL = target index).  Per-seed outputs (nullable, indexed by final seed
 * slot; with resampling the final slots are t*B' + j, B' = floor(B/K)*K):
 *   q_seed[S'*dof], errp_seed[S'], erro_seed[S'], cost_seed[S'], flag_seed[S']
 * Per-target outputs: q_out[T*k*dof], err_p[T*k], err_o[T*k], flag_out[T*k]
 * (255 for empty slots), n_free[T], solved[T] (1 if a returned seed is
 * collision free within succ_pos / succ_ori).  nthreads 0 = all cores. */
int or_solve(const or_robot* rb, const or_scene* sc, int32_t T, const double* targets,
             const int64_t* offsets, const double* seeds, const uint32_t* target_keys,
             const or_params* pr, double* q_seed, double* errp_seed, double* erro_seed,
             double* cost_seed, int32_t* flag_seed, double* q_out, double* err_p, double* err_o,
             int32_t* flag_out, int32_t* n_free, int32_t* solved, int32_t nthreads);

/* ---- operation counts (instrumentation) -------------------------------------
 * Every FP64 operation the oracle executes is counted in the category of the
 * unit it belongs to (add / subtract, multiply, divide, square root,
 * transcendental call; comparisons and sign changes are free).  Totals are
 * process wide and accumulate over calls until or_ops_reset.
 * or_ops_get: out[6] = add, mul, div, sqrt, trans, units of category cat. */
void or_ops_reset(void);
int or_ops_get(int32_t cat, uint64_t* out);

#ifdef __cplusplus
}
#endif
#endif
