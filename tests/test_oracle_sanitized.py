"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer runs
its whole pipeline (resampling with targets that have fewer seeds than K,
collision, both selections, tracking seeds, shadow runs) without a report
(CPU only)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
import numpy as np
import oracle as O
from paper_2510_07514_amd import workload as W
b = W.config_batched(T=3, M=40, host_seeds=True)
rob = b.robots[0]
tg = O.targets_from_qstar(rob, b.q_star).astype(np.float64)
offs = np.array([0, 3, 40, 120], np.int64)  # 3 < K = 8 seeds in the first target
seeds = W.uniform_configs(np.random.default_rng(1), rob, 120).astype(np.float64)
p = dict(b.params, cd_sweeps=4, polish_iters=4, resample_K=8, resample_B=20, top_k=5)
out = O.solve(rob, b.scene, tg, offs, p, seeds=seeds, nthreads=2)
assert out["q_seed"].shape[0] == 3 * 16
O.resample(rob, offs, seeds, np.arange(120.0), p)
for sh in (0, 1):
    O.cd(rob, tg[0], dict(p, shadow=sh), 0, 0, seeds[0])
    O.polish(rob, tg[0], dict(p, shadow=sh), 0, 0, seeds[1])
O.collide(rob, b.scene, seeds[2])
O.warm_seeds(rob, seeds[:6], 2, 7, p)
O.select_near(np.zeros(6, np.int32), np.arange(6.0), np.zeros(6), np.zeros(6), seeds[:6], seeds[0], 9, 1e-3, 0.02)
O.select(np.zeros(6, np.int32), np.arange(6.0), 9)
print("sanitized oracle ok")
"""


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    libasan = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    libubsan = subprocess.run(["g++", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    if not (os.path.isabs(libasan) and os.path.exists(libasan) and os.path.isabs(libubsan)):
        pytest.skip("no sanitizer runtime")
    lib = str(tmp_path / "liboracle_san.so")
    src = os.path.join(ROOT, "oracle", "hjcd_oracle.cpp")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                    "-o", lib, src, "-lpthread"], check=True)
    env = dict(os.environ, HJCD_ORACLE_LIBRARY=lib, LD_PRELOAD=f"{libasan}:{libubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", DRIVER], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitized oracle ok" in r.stdout
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
