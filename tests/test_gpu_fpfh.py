"""FPFH descriptors on the GPU against the oracle, through the C ABI, and the
paper's pairwise workflow end to end (FPFH, feature matching, RANSAC, ICP).

Bar: neighbourhood sizes bit-exact; descriptors within one float32 ulp of
the oracle's.  The bins are decided by the same float64 operations on both
sides (atan2 may differ by an ulp, so each case first checks with the oracle
that no feature lies within 1e-9 of a bin edge); the weighted sum over the
neighbours runs in grid order here and in distance order in the oracle, a
float64 rounding difference below 1e-14 relative that can move the float32
result by at most one ulp.
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
def F():
    from oracle import fpfh
    return fpfh


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _compare(icp, F, pts, nrm, radius, max_nn):
    g, gnn = icp.compute_fpfh(dev(pts), dev(nrm), radius, max_nn, with_nn=True)
    o, counts, k, nn, margin = F.fpfh(pts, nrm, radius, max_nn)
    print(f"n {len(pts)} radius {radius} max_nn {max_nn}: margin {margin:.2e}, mean nn {nn.mean():.1f}")
    assert margin > 1e-9
    np.testing.assert_array_equal(gnn.cpu().numpy(), nn)
    g = g.cpu().numpy()
    ulp = np.spacing(np.abs(o))
    bad = np.abs(g - o) > ulp
    assert not bad.any(), (np.argwhere(bad)[:5], g[bad][:5], o[bad][:5])
    return g, o


def _sphere_plane(seed, n):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n // 2, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    sp, sn = 0.5 * v, v
    q = np.zeros((n - n // 2, 3))
    q[:, :2] = rng.random((len(q), 2)) * 2 - 1
    q[:, 2] = -0.7
    pts = np.concatenate([sp, q]) + rng.normal(scale=0.002, size=(n, 3))
    nrm = np.concatenate([sn, np.tile([0.0, 0.0, 1.0], (len(q), 1))])
    return pts.astype(np.float32), nrm.astype(np.float32)


@pytest.mark.parametrize("n,radius,max_nn", [(3001, 0.15, 30), (3001, 0.25, 100), (2000, 0.4, 128)])
def test_fpfh_matches_oracle(icp, F, n, radius, max_nn):
    pts, nrm = _sphere_plane(n, n)
    _compare(icp, F, pts, nrm, radius, max_nn)


def test_fpfh_full_size_room(icp, F):
    """The paper's setting (radius 0.25 m, max_nn 100) on the 20k-point
    downsampled room target with its normals."""
    d = synth.ransac_pair(0)
    g, o = _compare(icp, F, d["tgt"], d["tgt_normals"], 0.25, 100)
    assert np.abs(g).max() > 100


def test_fpfh_edge_cases(icp, F):
    pts, nrm = _sphere_plane(7, 65)
    _compare(icp, F, pts, nrm, 0.3, 1)     # only the point itself: all zero
    _compare(icp, F, pts, nrm, 1e-4, 10)   # isolated points
    _compare(icp, F, pts[:1], nrm[:1], 0.3, 10)
    dup = np.concatenate([pts, pts[:10]])  # duplicate points are skipped as pairs
    _compare(icp, F, dup, np.concatenate([nrm, nrm[:10]]), 0.3, 20)


def test_pairwise_workflow_end_to_end(icp):
    """FPFH of both clouds, nearest-feature matches, RANSAC with the paper's
    parameters, then point-to-plane ICP at 2 cm from the RANSAC pose."""
    d = synth.ransac_pair(1)
    s, t = dev(d["src"]), dev(d["tgt"])
    fs = icp.compute_fpfh(s, dev(d["src_normals"]), 0.25, 100)
    ft = icp.compute_fpfh(t, dev(d["tgt_normals"]), 0.25, 100)
    corr = icp.feature_match(fs, ft)
    g = icp.ransac_register(s, t, corr, 0.075, max_iteration=4_000_000, max_validation=500)
    res = icp.register(s, t, dev(d["tgt_normals"]), g.T, 0.02, 30)
    G = d["T_gt"]
    dR = res.T[:3, :3].T @ G[:3, :3]
    ang = np.degrees(np.arccos(np.clip((np.trace(dR) - 1) / 2, -1, 1)))
    print(f"RANSAC fitness {g.fitness:.3f} after {g.n_iterations} iterations; ICP fitness {res.fitness:.3f}, "
          f"rotation error {ang:.3f} deg, translation error {np.linalg.norm(res.T[:3, 3] - G[:3, 3]):.4f} m")
    assert g.status == icp.ICP_OK and ang < 0.5 and np.linalg.norm(res.T[:3, 3] - G[:3, 3]) < 0.02


def test_fpfh_from_estimated_normals(icp, F):
    """FPFH of the room target with normals estimated on the GPU (radius 0.1 m,
    max_nn 30, the paper's workflow; isolated points get zero normals, whose
    pairs are skipped on both sides)."""
    d = synth.ransac_pair(2, 12000, 100)
    t = dev(d["tgt"])
    nrm = icp.estimate_normals(t, 0.1, 30, (2.0, 1.5, 1.2)).cpu().numpy()
    _compare(icp, F, d["tgt"], nrm, 0.25, 100)
