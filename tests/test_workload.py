"""The seeded workload generator: determinism and the shape of its draws."""
import numpy as np

from paper_2510_07514_amd import workload as W


def test_batches_are_deterministic():
    for make in (W.config_tiny, lambda: W.config_batched(T=20, M=8, host_seeds=True),
                 lambda: W.config_uneven(T=30, host_seeds=True), lambda: W.config_large(T=5, M=4)):
        a, b = make(), make()
        for r1, r2 in zip(a.robots, b.robots):
            for k in ("a", "d", "alpha", "q_min", "q_max", "sphere_xyzr", "sphere_link"):
                assert np.array_equal(getattr(r1, k), getattr(r2, k))
        assert np.array_equal(a.seed_offsets, b.seed_offsets)
        assert np.array_equal(a.robot_of_target, b.robot_of_target)
        assert all(np.array_equal(x, y) for x, y in zip(a.q_star, b.q_star))
        assert np.array_equal(a.scene.spheres, b.scene.spheres)
        if a.seeds is not None:
            assert a.seeds.tobytes() == b.seeds.tobytes()


def test_draws_respect_their_ranges():
    b = W.config_batched(T=50, M=16, host_seeds=True)
    rob = b.robots[0]
    assert rob.sphere_xyzr.shape == (60, 4)
    assert np.all((rob.sphere_xyzr[:, 3] >= 0.03) & (rob.sphere_xyzr[:, 3] <= 0.08))
    assert np.bincount(rob.sphere_link).tolist() == [8, 8, 8, 8, 7, 7, 7, 7]
    sp = b.scene.spheres.astype(np.float64)
    assert sp.shape == (32, 4)
    assert np.all(np.linalg.norm(sp[:, :3], axis=1) >= 0.3)
    assert np.all((sp[:, 3] >= 0.02) & (sp[:, 3] <= 0.10))
    assert np.all(np.abs(sp[:, :2]) <= 0.6) and np.all((sp[:, 2] >= 0) & (sp[:, 2] <= 1.2))
    for q in b.q_star:
        assert np.all(q >= rob.q_min.astype(np.float32)) and np.all(q <= rob.q_max.astype(np.float32))
    s = b.seeds[:7]
    assert np.all(s >= rob.q_min[:, None].astype(np.float32))
    assert np.all(s <= rob.q_max[:, None].astype(np.float32))


def test_uneven_batch():
    b = W.config_uneven(T=4096)
    counts = np.diff(b.seed_offsets)
    assert counts.min() >= 16 and counts.max() < 2048
    assert 350 < counts.mean() < 480
    assert sorted(np.bincount(b.robot_of_target).tolist()) == [1365, 1365, 1366]
    assert [r.dof for r in b.robots] == [6, 7, 12]


def test_large_batch_shapes():
    b = W.config_large(T=10, M=256)
    rob = b.robots[0]
    assert rob.dof == 20 and rob.sphere_xyzr.shape == (120, 4)
    assert b.scene.spheres.shape == (128, 4) and b.scene.boxes.shape == (128, 6)
    assert b.params["cd_sweeps"] == 40 and b.params["top_k"] == 16


def test_serving_stream():
    s = W.serving_stream(2000.0, 1.0)
    n = s["arrival"].shape[0]
    assert 1800 < n < 2200
    assert np.all(np.diff(s["arrival"]) >= 0)
    assert s["n_targets"].min() >= 1 and s["n_targets"].max() <= 16
    assert s["seeds_per_target"].min() >= 32 and s["seeds_per_target"].max() < 1024
