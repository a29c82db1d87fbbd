"""RANSAC global registration on the GPU against the oracle, through the C ABI.

Bar: feature matches (indices and float32 distances) bit-exact; validation
scores (count, sumq) bit-exact for the same transforms; the validated
hypothesis sequence (indices h) identical, which requires that no distance
checker decision of the oracle lies within rounding of its threshold (the
two sides fit the transforms with different algorithms: SVD there, Horn's
quaternion here), checked through the oracle's smallest relative margin;
the fitted transforms within 1e-9 of the oracle's; the best hypothesis and
iteration count equal.
"""
import numpy as np
import pytest

from paper_1801_09847_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def icp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1801_09847_amd import icp as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def R():
    from oracle import ransac
    return ransac


def dev(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


@pytest.fixture(scope="module")
def small():
    return synth.ransac_pair(3, 4000, 3000)


@pytest.fixture(scope="module")
def full():
    return synth.ransac_pair(0)


@pytest.mark.parametrize("dim", [1, 5, 33, 64])
def test_feature_match_bit_exact(icp, R, dim):
    rng = np.random.default_rng(dim)
    fs = (rng.random((700, dim)) * 50).astype(np.float32)
    ft = (rng.random((1300, dim)) * 50).astype(np.float32)
    fs[::7] = ft[rng.integers(0, 1300, len(fs[::7]))]  # exact hits (distance 0)
    m, dist = icp.feature_match(dev(fs), dev(ft), with_dist=True)
    om, od = R.feature_match(fs, ft)
    np.testing.assert_array_equal(m.cpu().numpy(), om)
    np.testing.assert_array_equal(dist.cpu().numpy(), od)


def test_feature_match_ties_and_empty(icp, R):
    rng = np.random.default_rng(11)
    ft = rng.integers(0, 4, (900, 33)).astype(np.float32)
    ft[450:] = ft[:450]
    fs = rng.integers(0, 4, (513, 33)).astype(np.float32)
    m = icp.feature_match(dev(fs), dev(ft)).cpu().numpy()
    om, _ = R.feature_match(fs, ft)
    np.testing.assert_array_equal(m, om)
    assert m.max() < 450
    e = icp.feature_match(dev(fs), dev(ft[:0].reshape(0, 33))).cpu().numpy()
    assert (e == -1).all()
    assert icp.feature_match(dev(fs[:0].reshape(0, 33)), dev(ft)).numel() == 0


def test_feature_match_full_size_sampled(icp, R, full):
    m = icp.feature_match(dev(full["src_feat"]), dev(full["tgt_feat"])).cpu().numpy()
    rows = np.random.default_rng(0).choice(len(m), 400, replace=False)
    om, _ = R.feature_match(full["src_feat"][rows], full["tgt_feat"])
    np.testing.assert_array_equal(m[rows], om)
    planted = full["true_match"] >= 0
    assert (m[planted] == full["true_match"][planted]).mean() > 0.99


def test_validation_scores_bit_exact(icp, R, small):
    rng = np.random.default_rng(5)
    Ts = [np.eye(4), small["T_gt"]]
    for _ in range(30):
        from scipy.spatial.transform import Rotation
        T = np.eye(4)
        T[:3, :3] = Rotation.from_rotvec(rng.normal(size=3) * 0.05).as_matrix()
        T[:3, 3] = rng.normal(size=3) * 0.05
        Ts.append(T @ small["T_gt"])
    Ts = np.array(Ts)
    cnt, sq = icp.ransac_validate(dev(small["src"]), dev(small["tgt"]), 0.075, Ts)
    for k, T in enumerate(Ts):
        assert (cnt[k], int(sq[k])) == R.validate(small["src"], small["tgt"], T, 0.075), k


def _compare(icp, R, d, corr, **kw):
    prm = dict(max_corr_dist=0.075, ransac_n=4, edge_length=0.9, distance=0.075, max_iteration=200_000,
               max_validation=60, seed=7)
    prm.update(kw)
    g = icp.ransac_register(dev(d["src"]), dev(d["tgt"]), dev(corr, np.int32), trace=True, **prm)
    hs, Ts, n_iter, margin = R.hypotheses(d["src"], d["tgt"], corr, prm["ransac_n"], prm["edge_length"],
                                          prm["distance"], prm["max_iteration"], prm["max_validation"],
                                          prm["seed"], chunk=65536)
    print(f"validated {len(hs)} iterations {n_iter} margin {margin:.2e} best {g.best_hypothesis}")
    assert margin > 1e-9
    np.testing.assert_array_equal(g.trace["h"], hs)
    assert g.n_validated == len(hs) and g.n_iterations == n_iter
    np.testing.assert_allclose(g.trace["T"], Ts, rtol=0, atol=1e-9)
    return g, hs


def test_register_matches_oracle_small(icp, R, small):
    corr = icp.feature_match(dev(small["src_feat"]), dev(small["tgt_feat"])).cpu().numpy()
    g, hs = _compare(icp, R, small, corr)
    # every validated hypothesis's score, recomputed by the oracle at the
    # GPU's transform (bit-exact), and the selection among them
    keys = []
    for k in range(len(hs)):
        c, q = R.validate(small["src"], small["tgt"], g.trace["T"][k], 0.075)
        assert (g.trace["count"][k], int(g.trace["sumq"][k])) == (c, q)
        keys.append((-c, q, int(hs[k])))
    best = min(keys)
    assert g.best_hypothesis == best[2] and g.n_inliers == -best[0] and g.sumq == best[1]
    np.testing.assert_array_equal(g.T, g.trace["T"][keys.index(best)])
    o = R.ransac(small["src"], small["tgt"], corr, 0.075, 4, 0.9, 0.075, 200_000, 60, seed=7, chunk=65536)
    assert o["best_h"] == g.best_hypothesis and o["count"] == g.n_inliers and o["sumq"] == g.sumq
    np.testing.assert_allclose(g.T, o["T"], atol=1e-9)
    assert abs(g.fitness - o["fitness"]) == 0 and abs(g.inlier_rmse - o["rmse"]) <= 1e-15


def test_register_full_size(icp, R, full):
    """The paper's configuration (r = 0.075, ransac_n = 4, edge length 0.9,
    distance 0.075, 4e6 iterations, 500 validations) on the 20k/20k pair."""
    corr = icp.feature_match(dev(full["src_feat"]), dev(full["tgt_feat"])).cpu().numpy()
    g, hs = _compare(icp, R, full, corr, max_iteration=4_000_000, max_validation=500, seed=0)
    cnt = g.trace["count"]
    sq = g.trace["sumq"]
    for k in np.random.default_rng(1).choice(len(hs), 40, replace=False):
        assert (cnt[k], int(sq[k])) == R.validate(full["src"], full["tgt"], g.trace["T"][k], 0.075)
    k = np.lexsort((hs, sq, -cnt))[0]
    assert g.best_hypothesis == hs[k]
    assert (g.n_inliers, int(g.sumq)) == R.validate(full["src"], full["tgt"], g.T, 0.075)
    # the chosen pose is close to the truth (ICP refines from here)
    dR = g.T[:3, :3].T @ full["T_gt"][:3, :3]
    ang = np.degrees(np.arccos(np.clip((np.trace(dR) - 1) / 2, -1, 1)))
    assert ang < 3.0 and np.linalg.norm(g.T[:3, 3] - full["T_gt"][:3, 3]) < 0.1


@pytest.mark.parametrize("n", [3, 5, 8])
def test_register_other_sample_sizes(icp, R, small, n):
    corr = np.where(small["true_match"] >= 0, small["true_match"],
                    np.random.default_rng(n).integers(0, len(small["tgt"]), len(small["src"])))
    _compare(icp, R, small, corr, ransac_n=n, max_validation=20, max_iteration=400_000)


def test_register_checkers_off_and_limits(icp, R, small):
    rng = np.random.default_rng(2)
    corr = rng.integers(0, len(small["tgt"]), len(small["src"]))
    # no checker: every sample without a repeated index is validated
    g, hs = _compare(icp, R, small, corr, edge_length=0.0, distance=0.0, max_validation=30)
    assert g.n_iterations == hs[-1] + 1
    # the iteration cap ends the loop before max_validation
    g2, hs2 = _compare(icp, R, small, corr, edge_length=0.0, distance=0.0, max_validation=30,
                       max_iteration=int(hs[9]) + 1)
    assert g2.n_validated == 10 and g2.n_iterations == int(hs[9]) + 1
    # out-of-range matches count as no match: nothing passes
    bad = np.full(len(small["src"]), len(small["tgt"]), np.int32)
    bad[::2] = -1
    g3 = icp.ransac_register(dev(small["src"]), dev(small["tgt"]), dev(bad, np.int32), 0.075,
                             max_iteration=5000, max_validation=10)
    assert g3.status == icp.ICP_RANSAC_NO_HYPOTHESIS and g3.n_validated == 0 and g3.n_iterations == 5000
    np.testing.assert_array_equal(g3.T, np.eye(4))
    assert g3.best_hypothesis == -1 and g3.n_inliers == 0


def test_register_tiny_and_chunk_edges(icp, R, small):
    rng = np.random.default_rng(21)
    # one source point: every sample repeats it, nothing passes
    one = {"src": small["src"][:1], "tgt": small["tgt"]}
    g = icp.ransac_register(dev(one["src"]), dev(one["tgt"]), dev(np.zeros(1), np.int32), 0.075,
                            max_iteration=3000, max_validation=5)
    assert g.status == icp.ICP_RANSAC_NO_HYPOTHESIS and g.n_iterations == 3000
    # three points, ransac_n 3, exact matches: the permutations of {0, 1, 2} pass
    T = np.eye(4)
    T[:3, 3] = [0.1, -0.2, 0.05]
    src = rng.random((3, 3)).astype(np.float32)
    tgt = (src.astype(np.float64) + T[:3, 3]).astype(np.float32)
    three = {"src": src, "tgt": tgt}
    g, hs = _compare(icp, R, three, np.arange(3), ransac_n=3, max_validation=4, max_iteration=200)
    assert len(hs) == 4 and g.n_inliers == 3
    np.testing.assert_allclose(g.T, T, atol=1e-6)
    # one validation; iteration caps at and just past the first chunk
    corr = np.where(small["true_match"] >= 0, small["true_match"], 0)
    _compare(icp, R, small, corr, max_validation=1)
    for cap in (65536, 65537, 131072 + 65536 + 1):
        _compare(icp, R, small, corr, edge_length=0.99, max_validation=65535, max_iteration=cap)


def test_validation_in_several_launches(icp, R):
    """300k source points: 586 tiles, so 9543 hypotheses per launch; 10000
    hypotheses take two launches.  Scores at both ends of each launch and a
    few inside match the oracle bit for bit."""
    d = synth.room_pair_random(77, 300_000, 300_000, 6.0, 4.0, 3.0, 20, 10)
    rng = np.random.default_rng(77)
    from scipy.spatial.transform import Rotation
    Ts = np.empty((10_000, 4, 4))
    for k in range(len(Ts)):
        T = np.eye(4)
        T[:3, :3] = Rotation.from_rotvec(rng.normal(size=3) * 0.01).as_matrix()
        T[:3, 3] = rng.normal(size=3) * 0.01
        Ts[k] = T @ d["T_gt"]
    cnt, sq = icp.ransac_validate(dev(d["src"]), dev(d["tgt"]), 0.03, Ts)
    assert (cnt > 0).all()
    for k in (0, 9542, 9543, 9999, 4321):
        assert (cnt[k], int(sq[k])) == R.validate(d["src"], d["tgt"], Ts[k], 0.03), k


def test_nonfinite_inputs_are_rejected(icp, small):
    src = small["src"].copy()
    src[17, 1] = np.nan
    corr = dev(np.zeros(len(src)), np.int32)
    with pytest.raises(icp.IcpError) as e:
        icp.ransac_register(dev(src), dev(small["tgt"]), corr, 0.075, max_iteration=100, max_validation=5)
    assert e.value.code == icp.ICP_E_NONFINITE
    tgt = small["tgt"].copy()
    tgt[3, 0] = np.inf
    with pytest.raises(icp.IcpError) as e:
        icp.ransac_validate(dev(small["src"]), dev(tgt), 0.075, np.eye(4)[None])
    assert e.value.code == icp.ICP_E_NONFINITE
    with pytest.raises(icp.IcpError) as e:
        icp.compute_fpfh(dev(src), dev(np.tile([0.0, 0.0, 1.0], (len(src), 1))), 0.25, 30)
    assert e.value.code == icp.ICP_E_NONFINITE
