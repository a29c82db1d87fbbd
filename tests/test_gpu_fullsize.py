"""Parity at the benchmark's full size: the 2M/2M room pair (12x8x3 m,
80 boxes, 40 spheres, r = 2 cm), single-pair path, the launch configuration
the benchmark times.

It checks
  * correspondences of a 20k-point random sample of the source, bit-exact
    (indices and pinned float32 distances), at the initial pose and at the
    pose the GPU reaches after 10 iterations;
  * the full normal equations at that pose, entry by entry within the
    float32-Kahan / float64 bounds of the sum of absolute terms;
  * the whole 50-iteration registration of the benchmark (51 passes, float32
    Kahan partials), both variants, against the oracle's (k-d tree, all host
    threads): equal inlier counts and iteration counts, pose within 1e-5 rad
    and 1e-6 m.
"""
import os
import sys

import numpy as np
import pytest

from paper_1801_09847_amd import synth

sys.path.insert(0, os.path.dirname(__file__))
from cases import pose_error  # noqa: E402

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

R = 0.02


@pytest.fixture(scope="module")
def icp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1801_09847_amd import icp as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def room():
    d = synth.c3_room(0)
    print(f"\nroom pair: {len(d['src'])} / {len(d['tgt'])} points", flush=True)
    return d


@pytest.fixture(scope="module")
def dev_room(room):
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    return f(room["src"]), f(room["tgt"]), f(room["tgt_normals"])


@pytest.fixture(scope="module")
def pose10(icp, dev_room):
    s, t, n = dev_room
    return icp.register(s, t, n, np.eye(4), R, 10, 0.0).T


@pytest.mark.parametrize("which", ["initial", "after_10"])
def test_sampled_correspondences_bit_exact(icp, oracle_lib, room, dev_room, pose10, which):
    T = np.eye(4) if which == "initial" else pose10
    s, t, _ = dev_room
    idx, d2 = icp.correspondences(s, T, t, R)
    idx, d2 = idx.cpu().numpy().astype(np.int64), d2.cpu().numpy()
    sel = np.random.default_rng(11).choice(len(room["src"]), 20000, replace=False)
    oi, of, _ = oracle_lib.correspondences(room["src"][sel], T, room["tgt"], R, search=2)
    np.testing.assert_array_equal(idx[sel], oi)
    m = oi >= 0
    np.testing.assert_array_equal(d2[sel][m], of[m])
    assert np.all(np.isinf(d2[sel][~m]))
    print(f"{which}: {m.sum()} of {len(sel)} sampled queries matched, all equal")


@pytest.mark.parametrize("precision,rel", [("kahan32", 1e-6), ("f64", 1e-12)])
def test_full_normal_equations(icp, oracle_lib, room, dev_room, pose10, precision, rel):
    import oracle.micro as micro
    s, t, n = dev_room
    A, b, sd2, nin = icp.normal_equations(s, pose10, t, n, R, "point_to_plane", precision)
    oA, ob, osd2, onin = oracle_lib.normal_equations(room["src"], pose10, room["tgt"],
                                                     room["tgt_normals"], R, search=2)
    assert nin == onin
    idx, _, _ = oracle_lib.correspondences(room["src"], pose10, room["tgt"], R, search=2)
    q = micro.transform64(pose10, room["src"])
    mk = idx >= 0
    p = room["tgt"][idx[mk]].astype(np.float64)
    nr = room["tgt_normals"][idx[mk]].astype(np.float64)
    r_, J = micro.jacobians("point_to_plane", q[mk], p, nr)
    SA = (np.abs(J).T @ np.abs(J))[np.triu_indices(6)]
    Sb = np.abs(J).T @ np.abs(r_)
    assert np.all(np.abs(np.asarray(A) - oA) <= rel * SA + 1e-300)
    assert np.all(np.abs(np.asarray(b) - ob) <= rel * Sb + 1e-300)
    assert abs(sd2 - osd2) <= rel * osd2 * 10


@pytest.mark.parametrize("variant", ["point_to_plane", "point_to_point"])
def test_full_registration_matches_oracle(icp, oracle_lib, room, dev_room, variant):
    s, t, n = dev_room
    K = room["max_iter"]
    g = icp.register(s, t, n, np.eye(4), R, K, 0.0, variant, "kahan32")
    o = oracle_lib.icp_register(room["src"], room["tgt"], room["tgt_normals"], np.eye(4), R, K,
                                variant=variant, search=2)
    ang, dt = pose_error(g.T, o.T)
    print(f"{variant}: rot {ang:.2e} rad, trans {dt:.2e} m, n_in {g.n_inliers}/{o.n_inliers}, "
          f"rmse diff {g.inlier_rmse - o.inlier_rmse:.2e}")
    assert g.n_inliers == o.n_inliers and g.n_iter == o.n_iter and g.status == o.status
    assert ang <= 1e-5 and dt <= 1e-6
