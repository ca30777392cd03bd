"""The C ABI library loads and exports what include/hjcd.h declares; argument
checks answer with the documented status before any device work (CPU only:
these calls never reach the GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hjcd.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hjcd_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def H():
    from paper_2510_07514_amd import hjcd
    return hjcd


def test_every_declared_symbol_is_exported(H):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(H._lib, n), n
    assert set(H.SYMBOLS) == set(names)


def test_defaults(H):
    p = H.hjcd_params_default()
    assert p.cd_sweeps == 20 and p.polish_iters == 20 and p.top_k == 1
    assert abs(p.lambda_ - 1e-3) < 1e-9 and abs(p.trust_R - 0.2) < 1e-7
    assert abs(p.succ_ori - np.pi / 180) < 1e-7
    assert "gfx950" in H.hjcd_version()


def test_no_device_reports_device_error(H):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    h = C.c_void_p()
    st = H._lib.hjcd_ctx_create(0, C.byref(h))
    assert st == H.HJCD_E_DEVICE
    assert h.value is None
    assert len(H.hjcd_last_error()) > 0


def _desc(H, rob, **over):
    from paper_2510_07514_amd import workload as W  # noqa: F401
    keep = []

    def arr(x, dt=np.float64):
        a = np.ascontiguousarray(x, dtype=dt)
        keep.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_double if dt == np.float64 else C.c_int32))
    d = H.hjcd_robot_desc(rob.dof, rob.convention, arr(rob.a), arr(rob.d), arr(rob.alpha),
                          arr(rob.offset), arr(rob.q_min), arr(rob.q_max),
                          arr(np.asarray(rob.tool).reshape(16)), len(rob.sphere_link),
                          arr(rob.sphere_link, np.int32), arr(np.asarray(rob.sphere_xyzr).reshape(-1)),
                          rob.min_link_gap)
    for k, v in over.items():
        setattr(d, k, v)
    return d, keep


def test_robot_validation_before_device(H):
    from paper_2510_07514_amd import workload as W
    rob = W.config_batched(T=1, M=1).robots[0]
    out = C.c_void_p()
    cases = [(dict(dof=0), H.HJCD_E_INVALID), (dict(dof=33), H.HJCD_E_UNSUPPORTED),
             (dict(convention=7), H.HJCD_E_INVALID), (dict(n_spheres=5000), H.HJCD_E_UNSUPPORTED),
             (dict(min_link_gap=-1), H.HJCD_E_INVALID)]
    for over, want in cases:
        d, keep = _desc(H, rob, **over)
        assert H._lib.hjcd_load_robot(None, C.byref(d), C.byref(out)) == want, over
    # limits reversed
    bad = W.panda_like()
    bad.q_min, bad.q_max = bad.q_max.copy(), bad.q_min.copy()
    d, keep = _desc(H, bad)
    assert H._lib.hjcd_load_robot(None, C.byref(d), C.byref(out)) == H.HJCD_E_INVALID
    assert "q_min" in H.hjcd_last_error()
    # non-rigid tool
    bad = W.panda_like()
    bad.tool = np.eye(4) * 2
    d, keep = _desc(H, bad)
    assert H._lib.hjcd_load_robot(None, C.byref(d), C.byref(out)) == H.HJCD_E_INVALID
    # a sphere on a link that does not exist
    bad = W.panda_like()
    bad.sphere_link = np.array([9], np.int32)
    bad.sphere_xyzr = np.array([[0, 0, 0, 0.1]])
    d, keep = _desc(H, bad)
    assert H._lib.hjcd_load_robot(None, C.byref(d), C.byref(out)) == H.HJCD_E_INVALID
    # a valid robot then fails only on the missing context
    d, keep = _desc(H, rob)
    assert H._lib.hjcd_load_robot(None, C.byref(d), C.byref(out)) == H.HJCD_E_INVALID
    assert "ctx" in H.hjcd_last_error()


def test_solve_validation_before_device(H):
    p = H.hjcd_params_default(top_k=8)
    offs = np.array([0, 4, 8], np.int64)
    bogus = C.c_void_p(0x1000)  # never dereferenced: checks fail first
    robots = (C.c_void_p * 1)(bogus)

    def solve(params, offsets, n_robots=1, rot=None):
        return H._lib.hjcd_solve(None, n_robots, C.cast(robots, C.c_void_p), None, len(offsets) - 1,
                                 rot, bogus, offsets.ctypes.data, None, None, C.byref(params),
                                 bogus, bogus, bogus, bogus, bogus, bogus, None)

    assert solve(H.hjcd_params_default(top_k=0), offs) == H.HJCD_E_INVALID
    assert solve(H.hjcd_params_default(top_k=65), offs) == H.HJCD_E_INVALID
    assert solve(H.hjcd_params_default(lambda_=0.0), offs) == H.HJCD_E_INVALID
    assert solve(H.hjcd_params_default(ls_beta=1.0), offs) == H.HJCD_E_INVALID
    assert solve(H.hjcd_params_default(gamma=float("nan")), offs) == H.HJCD_E_INVALID
    assert solve(H.hjcd_params_default(resample_K=4, resample_B=2), offs) == H.HJCD_E_INVALID
    assert solve(p, np.array([1, 4, 8], np.int64)) == H.HJCD_E_INVALID
    assert solve(p, np.array([0, 4, 3], np.int64)) == H.HJCD_E_INVALID
    assert "non-decreasing" in H.hjcd_last_error()
    assert solve(p, offs, n_robots=0) == H.HJCD_E_INVALID
    rot = np.array([0, 3], np.int32)
    assert solve(p, offs, rot=rot.ctypes.data) == H.HJCD_E_INVALID
    assert "robot_of_target" in H.hjcd_last_error()
    # resampling with an empty target
    assert solve(H.hjcd_params_default(resample_K=2, resample_B=4), np.array([0, 0, 8], np.int64)) \
        == H.HJCD_E_INVALID
    # all arguments fine: only the context is missing
    assert solve(p, offs) == H.HJCD_E_INVALID and "ctx" in H.hjcd_last_error()


def test_scene_and_stage_validation(H):
    out = C.c_void_p()
    sph = np.array([0, 0, 0, -0.1], np.float32)
    assert H._lib.hjcd_load_scene(None, 1, sph.ctypes.data, 0, None, C.byref(out)) == H.HJCD_E_INVALID
    box = np.array([0, 0, 0, 0.1, -0.1, 0.1], np.float32)
    assert H._lib.hjcd_load_scene(None, 0, None, 1, box.ctypes.data, C.byref(out)) == H.HJCD_E_INVALID
    nan = np.array([np.nan, 0, 0, 0.1], np.float32)
    assert H._lib.hjcd_load_scene(None, 1, nan.ctypes.data, 0, None, C.byref(out)) == H.HJCD_E_INVALID
    assert H._lib.hjcd_fk(None, None, -1, None, None, None, None) == H.HJCD_E_INVALID
    assert H._lib.hjcd_fk(None, None, 5, None, None, None, None) == H.HJCD_E_INVALID
    assert H._lib.hjcd_collide(None, None, None, 5, None, None, None) == H.HJCD_E_INVALID
    assert H._lib.hjcd_philox(None, None, None, 4, None, None) == H.HJCD_E_INVALID
    p = H.hjcd_params_default()
    offs = np.array([0, 4], np.int64)
    assert H._lib.hjcd_select(None, 1, offs.ctypes.data, 0, 7, C.byref(p), *([None] * 11), None) \
        == H.HJCD_E_INVALID
    assert H._lib.hjcd_resample(None, None, 1, offs.ctypes.data, None, C.byref(p), None, None, None,
                                None) == H.HJCD_E_INVALID
    assert "resample_K" in H.hjcd_last_error()


def test_struct_layouts_match_the_header(H, tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    the C compiler gives the header's struct of the same name."""
    structs = [H.hjcd_robot_desc, H.hjcd_params, H.hjcd_stats, H.hjcd_tune_choice, H.hjcd_server_config,
               H.hjcd_request_info, H.hjcd_server_stats]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "hjcd.h"', "int main(void) {"]
    for S in structs:
        lines.append(f'  printf("{S.__name__} %zu\\n", sizeof({S.__name__}));')
        for f in S._fields_:
            lines.append(f'  printf("{S.__name__}.{f[0]} %zu\\n", offsetof({S.__name__}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                 text=True).stdout.splitlines())
    for S in structs:
        assert int(got[S.__name__]) == C.sizeof(S), S.__name__
        for f in S._fields_:
            assert int(got[f"{S.__name__}.{f[0]}"]) == getattr(S, f[0]).offset, (S.__name__, f[0])


def test_server_config_validation_before_device(H):
    """Server configuration errors are reported before the context is used."""
    p = H.hjcd_params_default()
    h = C.c_void_p()
    for kw, status in [(dict(chunk_iters=0), H.HJCD_E_INVALID), (dict(mode=7), H.HJCD_E_INVALID),
                       (dict(pipelines=-1), H.HJCD_E_INVALID), (dict(pipelines=5), H.HJCD_E_INVALID),
                       (dict(max_queue=-1), H.HJCD_E_INVALID)]:
        cfg = H.hjcd_server_config(**dict(dict(chunk_iters=20), **kw))
        assert H._lib.hjcd_server_create(None, None, None, C.byref(p), C.byref(cfg), C.byref(h)) == status, kw
    cfg = H.hjcd_server_config(chunk_iters=20, pipelines=4)
    assert H._lib.hjcd_server_create(None, None, None, C.byref(p), C.byref(cfg), C.byref(h)) == H.HJCD_E_INVALID
    assert "ctx" in H.hjcd_last_error()
