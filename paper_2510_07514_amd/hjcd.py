"""Python binding of libhjcd (the C ABI in include/hjcd.h), same names.

Argument marshalling only: torch tensors supply device memory and streams,
every step of the solve runs in the library's HIP kernels.  Importing this
module fails loudly when libhjcd.so has not been built; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# HJCD_LIBRARY selects another build of the same ABI (e.g. a tuning variant).
LIB_PATH = os.environ.get("HJCD_LIBRARY", os.path.join(HERE, "libhjcd.so"))

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2510_07514_amd.build`")

_lib = C.CDLL(LIB_PATH)

HJCD_OK = 0
HJCD_E_INVALID = -1
HJCD_E_NOMEM = -2
HJCD_E_DEVICE = -3
HJCD_E_UNSUPPORTED = -4
HJCD_E_BUSY = -5
HJCD_E_INTERNAL = -6
HJCD_MAX_DOF = 32
HJCD_MAX_TOPK = 64

SYMBOLS = ("hjcd_ctx_create", "hjcd_ctx_destroy", "hjcd_last_error", "hjcd_params_default",
           "hjcd_version", "hjcd_load_robot", "hjcd_robot_destroy", "hjcd_robot_dof",
           "hjcd_load_scene", "hjcd_scene_destroy", "hjcd_fk", "hjcd_init_seeds", "hjcd_cd",
           "hjcd_polish", "hjcd_collide", "hjcd_resample", "hjcd_select", "hjcd_solve", "hjcd_solve_noalloc",
           "hjcd_warm_seeds", "hjcd_select_near", "hjcd_solve_near",
           "hjcd_get_stats", "hjcd_plan_create", "hjcd_plan_execute", "hjcd_plan_choice", "hjcd_plan_destroy",
           "hjcd_server_create", "hjcd_server_start", "hjcd_server_submit",
           "hjcd_server_poll", "hjcd_server_result", "hjcd_server_wait", "hjcd_server_get_stats",
           "hjcd_server_destroy", "hjcd_philox")


class HJCDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hjcd status {status}: {msg}")
        self.status = status


class hjcd_robot_desc(C.Structure):
    _fields_ = [("dof", C.c_int32), ("convention", C.c_int32),
                ("a", C.POINTER(C.c_double)), ("d", C.POINTER(C.c_double)),
                ("alpha", C.POINTER(C.c_double)), ("offset", C.POINTER(C.c_double)),
                ("q_min", C.POINTER(C.c_double)), ("q_max", C.POINTER(C.c_double)),
                ("tool", C.POINTER(C.c_double)), ("n_spheres", C.c_int32),
                ("sphere_link", C.POINTER(C.c_int32)), ("sphere_xyzr", C.POINTER(C.c_double)),
                ("min_link_gap", C.c_int32)]


class hjcd_params(C.Structure):
    _fields_ = [("cd_sweeps", C.c_int32), ("polish_iters", C.c_int32),
                ("eps_cd", C.c_float), ("nu_cd", C.c_float), ("gamma", C.c_float),
                ("delta0", C.c_float), ("delta_decay", C.c_float), ("delta_min", C.c_float),
                ("proj_eps", C.c_float), ("tie_eps", C.c_float), ("lambda_", C.c_float), ("lambda_gn", C.c_float),
                ("trust_R", C.c_float), ("ls_beta", C.c_float), ("ls_A", C.c_int32),
                ("weight_mode", C.c_int32), ("eps_pol", C.c_float), ("ups_pol", C.c_float),
                ("sigma", C.c_float), ("mu", C.c_float), ("resample_K", C.c_int32),
                ("resample_B", C.c_int32), ("top_k", C.c_int32), ("succ_pos", C.c_float),
                ("succ_ori", C.c_float), ("rng_seed", C.c_uint64), ("collect_stats", C.c_int32),
                ("polish_variant", C.c_int32), ("cd_lanes_per_seed", C.c_int32)]


class hjcd_stats(C.Structure):
    _fields_ = [("ms_init", C.c_float), ("ms_cd", C.c_float), ("ms_resample", C.c_float),
                ("ms_polish", C.c_float), ("ms_collide", C.c_float), ("ms_select", C.c_float),
                ("ms_total", C.c_float),
                ("seeds", C.c_uint64), ("cd_iters", C.c_uint64), ("cd_perturb", C.c_uint64),
                ("pol_iters", C.c_uint64), ("pol_trials", C.c_uint64), ("pol_dogleg", C.c_uint64),
                ("pol_single", C.c_uint64), ("pol_perturb", C.c_uint64),
                ("coll_coarse", C.c_uint64), ("coll_fine", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


HJCD_SERVE_BATCHED = 0
HJCD_SERVE_PLAIN = 1


class hjcd_tune_choice(C.Structure):
    _fields_ = [("variant", C.c_int32), ("block_threads", C.c_int32), ("ms", C.c_float), ("seeds", C.c_int64),
                ("cd_lanes", C.c_int32), ("cd_ms", C.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class hjcd_server_config(C.Structure):
    _fields_ = [("mode", C.c_int32), ("max_slots", C.c_int64), ("hbm_budget", C.c_size_t),
                ("max_targets", C.c_int32), ("chunk_iters", C.c_int32), ("max_queue", C.c_int32),
                ("pipelines", C.c_int32)]


class hjcd_request_info(C.Structure):
    _fields_ = [("request_id", C.c_int64), ("tag", C.c_uint64), ("n_targets", C.c_int32),
                ("n_solved", C.c_int32), ("arrival_s", C.c_double), ("admitted_s", C.c_double),
                ("done_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class hjcd_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("chunks", C.c_int64), ("targets_solved", C.c_int64), ("targets_done", C.c_int64),
                ("max_slots", C.c_int64), ("resident_slots_peak", C.c_int64),
                ("mean_resident_slots", C.c_double), ("p50_latency_ms", C.c_double),
                ("p99_latency_ms", C.c_double), ("first_arrival_s", C.c_double),
                ("last_done_s", C.c_double), ("solves_per_s", C.c_double), ("overlapped_steps", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = C.c_void_p
_i32, _i64, _u64 = C.c_int32, C.c_int64, C.c_uint64
_lib.hjcd_ctx_create.argtypes = [C.c_int, C.POINTER(_vp)]
_lib.hjcd_ctx_destroy.argtypes = [_vp]
_lib.hjcd_last_error.restype = C.c_char_p
_lib.hjcd_version.restype = C.c_char_p
_lib.hjcd_params_default.argtypes = [C.POINTER(hjcd_params)]
_lib.hjcd_load_robot.argtypes = [_vp, C.POINTER(hjcd_robot_desc), C.POINTER(_vp)]
_lib.hjcd_robot_destroy.argtypes = [_vp]
_lib.hjcd_robot_dof.argtypes = [_vp]
_lib.hjcd_load_scene.argtypes = [_vp, _i32, _vp, _i32, _vp, C.POINTER(_vp)]
_lib.hjcd_scene_destroy.argtypes = [_vp]
_lib.hjcd_fk.argtypes = [_vp, _vp, _i64, _vp, _vp, _vp, _vp]
_lib.hjcd_init_seeds.argtypes = [_vp, _vp, _i32, _vp, _vp, _u64, _vp, _vp]
_stage = [_vp, _vp, _i32, _vp, _vp, _vp, C.POINTER(hjcd_params), _vp, _vp, _vp, _vp, _vp, _vp]
_lib.hjcd_cd.argtypes = _stage
_lib.hjcd_polish.argtypes = _stage
_lib.hjcd_collide.argtypes = [_vp, _vp, _vp, _i64, _vp, _vp, _vp]
_lib.hjcd_resample.argtypes = [_vp, _vp, _i32, _vp, _vp, C.POINTER(hjcd_params), _vp, _vp, _vp, _vp]
_lib.hjcd_select.argtypes = [_vp, _i32, _vp, _i32, _i32, C.POINTER(hjcd_params), _vp, _vp, _vp, _vp,
                             _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.hjcd_select_near.argtypes = [_vp, _i32, _vp, _i32, _i32, C.POINTER(hjcd_params), _vp, _vp, _vp, _vp,
                                  _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.hjcd_solve.argtypes = [_vp, _i32, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp,
                            C.POINTER(hjcd_params), _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.hjcd_solve_noalloc.argtypes = _lib.hjcd_solve.argtypes
_lib.hjcd_solve_near.argtypes = [_vp, _i32, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp,
                                 C.POINTER(hjcd_params), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.hjcd_warm_seeds.argtypes = [_vp, _vp, _i32, _i32, _i32, _vp, _i32, _vp, C.POINTER(hjcd_params), _vp, _vp]
_lib.hjcd_get_stats.argtypes = [_vp, C.POINTER(hjcd_stats)]
_lib.hjcd_philox.argtypes = [_vp, _vp, _vp, _i64, _vp, _vp]
_lib.hjcd_plan_create.argtypes = [_vp, _i32, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp, C.POINTER(hjcd_params),
                                  _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, C.POINTER(_vp)]
_lib.hjcd_plan_execute.argtypes = [_vp, _vp]
_lib.hjcd_plan_choice.argtypes = [_vp, _i32, C.POINTER(hjcd_tune_choice)]
_lib.hjcd_plan_destroy.argtypes = [_vp]
_lib.hjcd_plan_destroy.restype = None
_lib.hjcd_server_create.argtypes = [_vp, _vp, _vp, C.POINTER(hjcd_params), C.POINTER(hjcd_server_config),
                                    C.POINTER(_vp)]
_lib.hjcd_server_start.argtypes = [_vp]
_lib.hjcd_server_submit.argtypes = [_vp, _i32, _vp, _i32, _u64, C.c_double, C.POINTER(_i64)]
_lib.hjcd_server_poll.argtypes = [_vp, _i32, C.POINTER(hjcd_request_info), C.POINTER(_i32)]
_lib.hjcd_server_result.argtypes = [_vp, _i64, _vp, _vp, _vp, _vp]
_lib.hjcd_server_wait.argtypes = [_vp, C.c_double]
_lib.hjcd_server_get_stats.argtypes = [_vp, C.POINTER(hjcd_server_stats)]
_lib.hjcd_server_destroy.argtypes = [_vp]
_lib.hjcd_server_destroy.restype = None
for _name in SYMBOLS:
    if _name not in ("hjcd_ctx_destroy", "hjcd_robot_destroy", "hjcd_scene_destroy", "hjcd_server_destroy",
                     "hjcd_plan_destroy",
                     "hjcd_last_error", "hjcd_version", "hjcd_params_default"):
        getattr(_lib, _name).restype = C.c_int32


def _check(status):
    if status != HJCD_OK:
        raise HJCDError(status, _lib.hjcd_last_error().decode())


def _ptr(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors passed to libhjcd must be contiguous")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


# ---------------------------------------------------------------------------
# handles
# ---------------------------------------------------------------------------

class Context:
    def __init__(self, handle):
        self.handle = handle

    def close(self):
        if self.handle:
            _lib.hjcd_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Robot:
    def __init__(self, ctx, handle, dof):
        self.ctx, self.handle, self.dof = ctx, handle, dof

    def close(self):
        if self.handle:
            _lib.hjcd_robot_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Scene:
    def __init__(self, ctx, handle):
        self.ctx, self.handle = ctx, handle

    def close(self):
        if self.handle:
            _lib.hjcd_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hjcd_version():
    return _lib.hjcd_version().decode()


def hjcd_last_error():
    return _lib.hjcd_last_error().decode()


def hjcd_params_default(**over) -> hjcd_params:
    p = hjcd_params()
    _lib.hjcd_params_default(C.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def params_from_dict(d: dict, collect_stats: int = 0) -> hjcd_params:
    """hjcd_params from the workload module's parameter dict (collect_stats:
    0 / False none, 1 / True stage times and work counts, 2 stage times)."""
    p = hjcd_params_default()
    for k, v in d.items():
        name = "lambda_" if k == "lam" else k
        if any(f == name for f, _ in hjcd_params._fields_):
            setattr(p, name, v)
    p.collect_stats = int(collect_stats)
    return p


def hjcd_ctx_create(device: int = 0) -> Context:
    h = _vp()
    _check(_lib.hjcd_ctx_create(device, C.byref(h)))
    return Context(h.value)


def hjcd_ctx_destroy(ctx: Context):
    ctx.close()


def hjcd_load_robot(ctx: Context, robot) -> Robot:
    """robot: any object with dof, convention, a, d, alpha, offset, q_min,
    q_max, tool (4x4), sphere_link, sphere_xyzr, min_link_gap."""
    bufs = [_host(getattr(robot, k), np.float64)[0] for k in ("a", "d", "alpha", "offset", "q_min", "q_max")]
    tool = _host(np.asarray(robot.tool).reshape(16), np.float64)[0]
    sl = _host(robot.sphere_link, np.int32)[0]
    sx = _host(np.asarray(robot.sphere_xyzr).reshape(-1), np.float64)[0]
    dp = C.POINTER(C.c_double)
    desc = hjcd_robot_desc(int(robot.dof), int(robot.convention),
                           *[b.ctypes.data_as(dp) for b in bufs], tool.ctypes.data_as(dp),
                           int(sl.shape[0]), sl.ctypes.data_as(C.POINTER(C.c_int32)),
                           sx.ctypes.data_as(dp), int(robot.min_link_gap))
    h = _vp()
    _check(_lib.hjcd_load_robot(ctx.handle, C.byref(desc), C.byref(h)))
    return Robot(ctx, h.value, int(robot.dof))


def hjcd_robot_destroy(robot: Robot):
    robot.close()


def hjcd_robot_dof(robot: Robot) -> int:
    return _lib.hjcd_robot_dof(robot.handle)


def hjcd_load_scene(ctx: Context, spheres, boxes) -> Scene:
    s, sp = _host(np.asarray(spheres).reshape(-1), np.float32)
    b, bp = _host(np.asarray(boxes).reshape(-1), np.float32)
    h = _vp()
    _check(_lib.hjcd_load_scene(ctx.handle, int(s.shape[0] // 4), sp if s.size else None,
                                int(b.shape[0] // 6), bp if b.size else None, C.byref(h)))
    return Scene(ctx, h.value)


def hjcd_scene_destroy(scene: Scene):
    scene.close()


# ---------------------------------------------------------------------------
# stages
# ---------------------------------------------------------------------------

def hjcd_fk(ctx, robot, q, pose, jac=None, stream=None):
    """q float32 [n][S] -> pose float32 [7][S], jac [6][n][S] (optional)."""
    S = q.shape[1] if q.dim() == 2 else 0
    _check(_lib.hjcd_fk(ctx.handle, robot.handle, S, _ptr(q), _ptr(pose), _ptr(jac), _stream(stream)))


def hjcd_init_seeds(ctx, robot, seed_offsets, q, rng_seed, target_keys=None, stream=None):
    offs, op = _host(seed_offsets, np.int64)
    _check(_lib.hjcd_init_seeds(ctx.handle, robot.handle, int(offs.shape[0] - 1), op, _ptr(target_keys),
                                int(rng_seed), _ptr(q), _stream(stream)))


def _stage(fn, ctx, robot, targets, seed_offsets, params, q, err_p, err_o, cost, traj, target_keys,
           stream):
    offs, op = _host(seed_offsets, np.int64)
    _check(fn(ctx.handle, robot.handle, int(offs.shape[0] - 1), _ptr(targets), op, _ptr(target_keys),
              C.byref(params), _ptr(q), _ptr(err_p), _ptr(err_o), _ptr(cost), _ptr(traj),
              _stream(stream)))


def hjcd_cd(ctx, robot, targets, seed_offsets, params, q, err_p=None, err_o=None, cost=None, traj=None,
            target_keys=None, stream=None):
    _stage(_lib.hjcd_cd, ctx, robot, targets, seed_offsets, params, q, err_p, err_o, cost, traj,
           target_keys, stream)


def hjcd_polish(ctx, robot, targets, seed_offsets, params, q, err_p=None, err_o=None, cost=None,
                traj=None, target_keys=None, stream=None):
    _stage(_lib.hjcd_polish, ctx, robot, targets, seed_offsets, params, q, err_p, err_o, cost, traj,
           target_keys, stream)


def hjcd_collide(ctx, robot, scene, q, flag, stream=None):
    S = q.shape[1] if q.dim() == 2 else 0
    _check(_lib.hjcd_collide(ctx.handle, robot.handle, scene.handle if scene else None, S, _ptr(q),
                             _ptr(flag), _stream(stream)))


def hjcd_resample(ctx, robot, seed_offsets, params, q_in, cost_in, q_out, target_keys=None,
                  stream=None):
    offs, op = _host(seed_offsets, np.int64)
    _check(_lib.hjcd_resample(ctx.handle, robot.handle, int(offs.shape[0] - 1), op, _ptr(target_keys),
                              C.byref(params), _ptr(q_in), _ptr(cost_in), _ptr(q_out), _stream(stream)))


def hjcd_select(ctx, seed_offsets, n, n_stride, params, q, cost, err_p, err_o, flag, q_out, err_p_out,
                err_o_out, flag_out, n_free, solved, stream=None):
    offs, op = _host(seed_offsets, np.int64)
    _check(_lib.hjcd_select(ctx.handle, int(offs.shape[0] - 1), op, int(n), int(n_stride),
                            C.byref(params), _ptr(q), _ptr(cost), _ptr(err_p), _ptr(err_o), _ptr(flag),
                            _ptr(q_out), _ptr(err_p_out), _ptr(err_o_out), _ptr(flag_out),
                            _ptr(n_free), _ptr(solved), _stream(stream)))


def hjcd_select_near(ctx, seed_offsets, n, n_stride, params, q, cost, err_p, err_o, flag, q_ref, q_out, err_p_out,
                     err_o_out, flag_out, n_free, solved, stream=None):
    offs, op = _host(seed_offsets, np.int64)
    _check(_lib.hjcd_select_near(ctx.handle, int(offs.shape[0] - 1), op, int(n), int(n_stride),
                                 C.byref(params), _ptr(q), _ptr(cost), _ptr(err_p), _ptr(err_o), _ptr(flag),
                                 _ptr(q_ref), _ptr(q_out), _ptr(err_p_out), _ptr(err_o_out), _ptr(flag_out),
                                 _ptr(n_free), _ptr(solved), _stream(stream)))


def hjcd_solve(ctx, robots, scene, targets, seed_offsets, params, q_out, err_p, err_o, flag, n_free,
               solved, robot_of_target=None, seeds=None, target_keys=None, stream=None, _fn=None):
    """The whole batched solve; see hjcd_solve in include/hjcd.h."""
    if isinstance(robots, Robot):
        robots = [robots]
    arr = (_vp * len(robots))(*[r.handle for r in robots])
    offs, op = _host(seed_offsets, np.int64)
    rot = None
    if robot_of_target is not None:
        rot, rotp = _host(robot_of_target, np.int32)
    _check((_fn or _lib.hjcd_solve)(ctx.handle, len(robots), C.cast(arr, _vp), scene.handle if scene else None,
                           int(offs.shape[0] - 1), rotp if rot is not None else None, _ptr(targets), op,
                           _ptr(target_keys), _ptr(seeds), C.byref(params), _ptr(q_out), _ptr(err_p),
                           _ptr(err_o), _ptr(flag), _ptr(n_free), _ptr(solved), _stream(stream)))


def hjcd_solve_near(ctx, robots, scene, targets, seed_offsets, params, q_ref, q_out, err_p, err_o, flag, n_free,
                    solved, robot_of_target=None, seeds=None, target_keys=None, stream=None):
    """The whole solve with the nearest-solution selection around q_ref
    [T][n_max]; see hjcd_solve_near in include/hjcd.h."""
    if isinstance(robots, Robot):
        robots = [robots]
    arr = (_vp * len(robots))(*[r.handle for r in robots])
    offs, op = _host(seed_offsets, np.int64)
    rot, rotp = None, None
    if robot_of_target is not None:
        rot, rotp = _host(robot_of_target, np.int32)
    _check(_lib.hjcd_solve_near(ctx.handle, len(robots), C.cast(arr, _vp), scene.handle if scene else None,
                                int(offs.shape[0] - 1), rotp, _ptr(targets), op, _ptr(target_keys), _ptr(seeds),
                                C.byref(params), _ptr(q_ref), _ptr(q_out), _ptr(err_p), _ptr(err_o), _ptr(flag),
                                _ptr(n_free), _ptr(solved), _stream(stream)))


def hjcd_warm_seeds(ctx, robot, q_prev, k, M, params, q_out, target_keys=None, stream=None):
    """q_prev [T*k][n_stride] -> q_out [n][T*M]; see hjcd_warm_seeds."""
    T = q_prev.shape[0] // k
    _check(_lib.hjcd_warm_seeds(ctx.handle, robot.handle, int(T), int(k), int(q_prev.shape[1]), _ptr(q_prev),
                                int(M), _ptr(target_keys), C.byref(params), _ptr(q_out), _stream(stream)))


def hjcd_solve_noalloc(ctx, robots, scene, targets, seed_offsets, params, q_out, err_p, err_o, flag, n_free,
                       solved, robot_of_target=None, seeds=None, target_keys=None, stream=None):
    """hjcd_solve over the library's static device workspace (allocates
    nothing); see hjcd_solve_noalloc in include/hjcd.h."""
    hjcd_solve(ctx, robots, scene, targets, seed_offsets, params, q_out, err_p, err_o, flag, n_free, solved,
               robot_of_target=robot_of_target, seeds=seeds, target_keys=target_keys, stream=stream,
               _fn=_lib.hjcd_solve_noalloc)


def hjcd_get_stats(ctx) -> dict:
    st = hjcd_stats()
    _check(_lib.hjcd_get_stats(ctx.handle, C.byref(st)))
    return st.as_dict()


def hjcd_philox(ctx, ctr, key, count, out, stream=None):
    c, cp = _host(ctr, np.uint32)
    k, kp = _host(key, np.uint32)
    _check(_lib.hjcd_philox(ctx.handle, cp, kp, int(count), _ptr(out), _stream(stream)))


# ---------------------------------------------------------------------------
# reusable plans
# ---------------------------------------------------------------------------

class Plan:
    def __init__(self, keep, handle, n_robots):
        # keep the context, robots, scene and buffers alive as long as the plan
        self.keep, self.handle, self.n_robots = keep, handle, n_robots

    def close(self):
        if self.handle:
            _lib.hjcd_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hjcd_plan_create(ctx, robots, scene, targets, seed_offsets, params, q_out, err_p, err_o, flag, n_free,
                     solved, robot_of_target=None, seeds=None, target_keys=None, tune=True, stream=None) -> Plan:
    """A reusable, graph-captured solve of one batch; see include/hjcd.h."""
    if isinstance(robots, Robot):
        robots = [robots]
    arr = (_vp * len(robots))(*[r.handle for r in robots])
    offs, op = _host(seed_offsets, np.int64)
    rot, rotp = None, None
    if robot_of_target is not None:
        rot, rotp = _host(robot_of_target, np.int32)
    h = _vp()
    _check(_lib.hjcd_plan_create(ctx.handle, len(robots), C.cast(arr, _vp), scene.handle if scene else None,
                                 int(offs.shape[0] - 1), rotp, _ptr(targets), op, _ptr(target_keys), _ptr(seeds),
                                 C.byref(params), _ptr(q_out), _ptr(err_p), _ptr(err_o), _ptr(flag), _ptr(n_free),
                                 _ptr(solved), 1 if tune else 0, _stream(stream), C.byref(h)))
    keep = (ctx, list(robots), scene, targets, q_out, err_p, err_o, flag, n_free, solved, seeds, target_keys)
    return Plan(keep, h.value, len(robots))


def hjcd_plan_execute(plan: Plan, stream=None):
    _check(_lib.hjcd_plan_execute(plan.handle, _stream(stream)))


def hjcd_plan_choice(plan: Plan, robot: int) -> dict:
    ch = hjcd_tune_choice()
    _check(_lib.hjcd_plan_choice(plan.handle, int(robot), C.byref(ch)))
    return ch.as_dict()


def hjcd_plan_destroy(plan: Plan):
    plan.close()


# ---------------------------------------------------------------------------
# serving loop
# ---------------------------------------------------------------------------

class Server:
    def __init__(self, ctx, robot, scene, handle, dof):
        # keep the context, robot and scene alive as long as the server
        self.ctx, self.robot, self.scene, self.handle, self.dof = ctx, robot, scene, handle, dof

    def close(self):
        if self.handle:
            _lib.hjcd_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hjcd_server_create(ctx, robot, scene, params, mode=HJCD_SERVE_BATCHED, max_slots=0, hbm_budget=0,
                       max_targets=0, chunk_iters=20, max_queue=0, pipelines=0) -> Server:
    cfg = hjcd_server_config(mode, max_slots, hbm_budget, max_targets, chunk_iters, max_queue, pipelines)
    h = _vp()
    _check(_lib.hjcd_server_create(ctx.handle, robot.handle, scene.handle if scene else None, C.byref(params),
                                   C.byref(cfg), C.byref(h)))
    return Server(ctx, robot, scene, h.value, robot.dof)


def hjcd_server_start(srv: Server):
    _check(_lib.hjcd_server_start(srv.handle))


def hjcd_server_submit(srv: Server, targets, seeds_per_target: int, tag: int, arrival_s: float) -> int:
    """targets: host array [n_targets][7] (px py pz qw qx qy qz)."""
    tg, p = _host(np.asarray(targets, np.float32).reshape(-1, 7), np.float32)
    rid = _i64()
    _check(_lib.hjcd_server_submit(srv.handle, tg.shape[0], p, int(seeds_per_target), int(tag) & (2**64 - 1),
                                   float(arrival_s), C.byref(rid)))
    return rid.value


def hjcd_server_poll(srv: Server, max_n: int = 1024) -> list:
    buf = (hjcd_request_info * max(1, max_n))()
    n = _i32()
    _check(_lib.hjcd_server_poll(srv.handle, max_n, buf, C.byref(n)))
    return [buf[i].as_dict() for i in range(n.value)]


REQUEST_INFO_DTYPE = np.dtype([("request_id", np.int64), ("tag", np.uint64), ("n_targets", np.int32),
                               ("n_solved", np.int32), ("arrival_s", np.float64), ("admitted_s", np.float64),
                               ("done_s", np.float64)])
assert REQUEST_INFO_DTYPE.itemsize == C.sizeof(hjcd_request_info)


def hjcd_server_poll_all(srv: Server, chunk: int = 65536) -> np.ndarray:
    """Every completed request not yet reported, as a numpy structured array
    (fields of hjcd_request_info), oldest first."""
    buf = (hjcd_request_info * chunk)()
    n = _i32()
    parts = []
    while True:
        _check(_lib.hjcd_server_poll(srv.handle, chunk, buf, C.byref(n)))
        if n.value == 0:
            break
        parts.append(np.frombuffer(buf, dtype=REQUEST_INFO_DTYPE, count=n.value).copy())
    return np.concatenate(parts) if parts else np.zeros(0, REQUEST_INFO_DTYPE)


def hjcd_server_result(srv: Server, request_id: int, n_targets: int) -> dict:
    q = np.zeros((n_targets, srv.dof), np.float32)
    ep = np.zeros(n_targets, np.float32)
    eo = np.zeros(n_targets, np.float32)
    fl = np.zeros(n_targets, np.uint8)
    _check(_lib.hjcd_server_result(srv.handle, int(request_id), q.ctypes.data, ep.ctypes.data, eo.ctypes.data,
                                   fl.ctypes.data))
    return {"q": q, "err_p": ep, "err_o": eo, "flag": fl}


def hjcd_server_wait(srv: Server, timeout_s: float):
    _check(_lib.hjcd_server_wait(srv.handle, float(timeout_s)))


def hjcd_server_get_stats(srv: Server) -> dict:
    st = hjcd_server_stats()
    _check(_lib.hjcd_server_get_stats(srv.handle, C.byref(st)))
    return st.as_dict()


def hjcd_server_destroy(srv: Server):
    srv.close()
