"""Generator determinism and shape checks (inputs shared by oracle and GPU tests)."""
import numpy as np
import pytest

from paper_1801_09847_amd import synth


def test_heightfield_deterministic_and_shaped():
    a, b = synth.c1_heightfield(0), synth.c1_heightfield(0)
    for k in ("src", "tgt", "tgt_normals"):
        assert a[k].dtype == np.float32 and a[k].shape == (5000, 3) and a[k].flags.c_contiguous
        np.testing.assert_array_equal(a[k], b[k])
    assert np.abs(np.linalg.norm(a["tgt_normals"], axis=1) - 1).max() < 1e-6
    c = synth.c1_heightfield(1)
    assert not np.array_equal(a["src"], c["src"])
    # the applied motion is a rigid motion within the configured bounds
    R = a["G"][:3, :3]
    assert np.abs(R.T @ R - np.eye(3)).max() < 1e-12
    ang = np.degrees(np.arccos(np.clip((np.trace(R) - 1) / 2, -1, 1)))
    assert ang <= 5.0
    np.testing.assert_allclose(a["T_gt"] @ a["G"], np.eye(4), atol=1e-12)


def test_room_pair_small():
    d = synth.room_pair(3, 20000, 15000, 3.0, 2.0, 2.0, 4, 2, overlap=0.6)
    e = synth.room_pair(3, 20000, 15000, 3.0, 2.0, 2.0, 4, 2, overlap=0.6)
    np.testing.assert_array_equal(d["src"], e["src"])
    np.testing.assert_array_equal(d["tgt"], e["tgt"])
    assert d["tgt"].shape == (20000, 3) and d["src"].shape == (15000, 3)
    n = np.linalg.norm(d["tgt_normals"], axis=1)
    assert np.abs(n - 1).max() < 1e-6
    # target within the room (plus noise), source a slab of it before the motion
    assert d["tgt"].min() > -0.02 and d["tgt"][:, 0].max() < 3.02
    back = synth.apply(d["T_gt"], d["src"].astype(np.float64))
    if d["meta"]["from_low"]:
        assert back[:, 0].max() <= d["meta"]["cut"] + 1e-5
    else:
        assert back[:, 0].min() >= d["meta"]["cut"] - 1e-5
    assert d["area"] > 0


def test_c4_c5_sizes_in_range():
    rng_sizes = [synth.c5_request_size(q)[0] for q in range(200)]
    assert min(rng_sizes) >= 5000 and max(rng_sizes) <= 500000
    t = synth.poisson_arrivals(100, 10.0)
    assert np.all(np.diff(t) > 0)


def test_ransac_pair_structure():
    a = synth.ransac_pair(4, 3000, 2500)
    b = synth.ransac_pair(4, 3000, 2500)
    for k in ("src", "tgt", "src_feat", "tgt_feat", "true_match"):
        np.testing.assert_array_equal(a[k], b[k])
    assert a["src_feat"].shape == (2500, 33) and a["tgt_feat"].shape == (3000, 33)
    assert a["src_feat"].dtype == np.float32 and (a["src_feat"] >= 0).all()
    # three 11-bin sub-histograms summing to 100 for the targets
    s = a["tgt_feat"].reshape(-1, 3, 11).sum(axis=2)
    np.testing.assert_allclose(s, 100.0, rtol=1e-5)
    planted = a["true_match"] >= 0
    assert 0.0 < planted.mean() <= 0.3  # match_frac of the points whose counterpart is within 5 cm
    full = synth.ransac_pair(0)  # ~6 cm spacing: most points have a counterpart
    assert 0.2 < (full["true_match"] >= 0).mean() < 0.3
    # a planted feature is its counterpart's plus small noise
    diff = np.abs(a["src_feat"][planted] - a["tgt_feat"][a["true_match"][planted]])
    assert np.median(diff) < 2.0
    # the planted counterparts lie near the moved source points
    home = synth.apply(a["T_gt"], a["src"].astype(np.float64))
    dist = np.linalg.norm(home[planted] - a["tgt"][a["true_match"][planted]], axis=1)
    assert dist.max() < 0.05


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in (r.stdout + r.stderr)


def test_pooled_served_requests_numpy_equals_torch():
    """The served workload's requests are cut from a scene pool by a numpy
    definition and, in the benchmark, by the same steps in torch on the GPU;
    on the CPU the two give the same float32 clouds bit for bit."""
    torch = pytest.importorskip("torch")
    scenes = [synth.c5_scene(k, n_max=40_000) for k in range(2)]
    st = [{k: torch.from_numpy(np.ascontiguousarray(s[k])) for k in ("tgt", "tgt_normals", "src")}
          for s in scenes]
    for q in range(6):
        a = synth.c5_request_pooled(q, scenes)
        b = synth.c5_request_pooled_torch(q, scenes, st)
        for key in ("src", "tgt", "tgt_normals"):
            np.testing.assert_array_equal(a[key], b[key].numpy())
        assert a["spacing"] == b["spacing"] and np.array_equal(a["G"], b["G"])
        n = a["meta"]["n"]
        assert len(a["tgt"]) == n and 0 < len(a["src"]) <= n


def test_far_outliers_keep_the_target():
    d = synth.c1_heightfield(0)
    f = synth.with_far_outliers(d, seed=0, frac=0.01, dist=100.0)
    n = len(d["tgt"])
    assert len(f["tgt"]) == n + 50 and len(f["tgt_normals"]) == n + 50
    assert np.array_equal(f["tgt"][:n], d["tgt"]) and np.array_equal(f["src"], d["src"])
    centre = 0.5 * (d["tgt"].min(0) + d["tgt"].max(0))
    far = np.linalg.norm(f["tgt"][n:] - centre, axis=1)
    assert np.all(far > 95.0) and np.all(far < 105.0)
    # reproducible
    g = synth.with_far_outliers(d, seed=0, frac=0.01, dist=100.0)
    assert np.array_equal(f["tgt"], g["tgt"])
