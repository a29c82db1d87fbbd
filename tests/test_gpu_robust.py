"""Robust (IRLS) variants on the GPU against the oracle, through the C ABI.

Bar: inlier counts equal; weighted normal equations within the plain hook's
bounds (1e-6 of sum |terms| with float32-Kahan partials, 1e-12 all-FP64; the
weight only scales a term by w in [0, 1], so the same bound holds, and the
float32 weight adds a relative error of a few ulp); final pose within 1e-5 rad
and 1e-6 m of the FP64 oracle; Huber above every residual equal to the plain
method bitwise.  With rel_tol = 0 the convergence test fires only at an
exact fixed point of the iteration, which one precision may reach and the
other not (float32-Kahan partials keep moving the last bits): iteration
counts must then agree unless one side stopped CONVERGED, in which case the
other may run on to max_iter, the poses still within the bound.
"""
import os
import sys

import numpy as np
import pytest
import scipy.linalg

from paper_1801_09847_amd import synth

sys.path.insert(0, os.path.dirname(__file__))
from cases import pose_error  # noqa: E402

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
def c1():
    return synth.c1_heightfield(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _twist(xi):
    w, v = xi[:3], xi[3:]
    X = np.zeros((4, 4))
    X[:3, :3] = [[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]
    X[:3, 3] = v
    return X


def _near(T, xi):
    return scipy.linalg.expm(_twist(np.asarray(xi, np.float64))) @ T


def _same_stop(g, o, icp):
    if icp.ICP_CONVERGED in (g.status, o.status):
        return {g.status, o.status} <= {icp.ICP_OK, icp.ICP_CONVERGED}
    return g.n_iter == o.n_iter and g.status == o.status


@pytest.mark.parametrize("precision,tol", [("kahan32", 1e-6), ("f64", 1e-12)])
@pytest.mark.parametrize("variant", ["point_to_plane", "point_to_point"])
@pytest.mark.parametrize("loss,k", [("huber", 0.002), ("tukey", 0.006), ("cauchy", 0.003)])
def test_weighted_normal_equations(icp, oracle_lib, c1, loss, k, variant, precision, tol):
    from oracle import micro
    T = _near(c1["T_gt"], [0.01, -0.008, 0.012, 0.004, -0.003, 0.005])
    s, t, n = dev(c1["src"]), dev(c1["tgt"]), dev(c1["tgt_normals"])
    A, b, sd2, nin = icp.normal_equations(s, T, t, n, 0.05, variant, precision, loss=loss, loss_k=k)
    oA, ob, osd2, onin = oracle_lib.normal_equations(c1["src"], T, c1["tgt"], c1["tgt_normals"], 0.05,
                                                     variant, loss=loss, loss_k=k)
    assert nin == onin
    idx, _, _ = oracle_lib.correspondences(c1["src"], T, c1["tgt"], 0.05)
    q = micro.transform64(T, c1["src"])
    m = idx >= 0
    p = c1["tgt"][idx[m]].astype(np.float64)
    nr = c1["tgt_normals"][idx[m]].astype(np.float64)
    r, J = micro.jacobians(variant, q[m], p, nr)
    SA = (np.abs(J).T @ np.abs(J))[np.triu_indices(6)]
    Sb = np.abs(J).T @ np.abs(r)
    assert np.all(np.abs(A - oA) <= tol * SA + 1e-300), np.max(np.abs(A - oA) / SA)
    assert np.all(np.abs(b - ob) <= tol * Sb + 1e-300), np.max(np.abs(b - ob) / Sb)
    assert abs(sd2 - osd2) <= tol * osd2 * 10


@pytest.mark.parametrize("variant", ["point_to_plane", "point_to_point"])
@pytest.mark.parametrize("loss,k", [("huber", 0.002), ("tukey", 0.01), ("cauchy", 0.003)])
def test_robust_registration_matches_oracle_c1(icp, oracle_lib, c1, loss, k, variant):
    T0 = _near(c1["T_gt"], [0.005, -0.004, 0.006, 0.002, -0.002, 0.001])
    s, t, n = dev(c1["src"]), dev(c1["tgt"]), dev(c1["tgt_normals"])
    for precision in ("kahan32", "f64"):
        g = icp.register(s, t, n, T0, 0.05, 30, 0.0, variant, precision, loss=loss, loss_k=k)
        o = oracle_lib.icp_register(c1["src"], c1["tgt"], c1["tgt_normals"], T0, 0.05, 30,
                                    variant=variant, loss=loss, loss_k=k)
        ang, dt = pose_error(g.T, o.T)
        print(f"{loss} {variant} {precision}: rot {ang:.2e} trans {dt:.2e} n_in {g.n_inliers}/{o.n_inliers}")
        assert g.n_inliers == o.n_inliers and _same_stop(g, o, icp), (g.n_iter, o.n_iter)
        assert ang <= 1e-5 and dt <= 1e-6


def test_robust_registration_matches_oracle_room(icp, oracle_lib):
    d = synth.c2_room(0)
    T0 = _near(d["T_gt"], [0.01, 0.01, -0.01, 0.01, -0.005, 0.005])
    s, t, n = dev(d["src"]), dev(d["tgt"]), dev(d["tgt_normals"])
    g = icp.register(s, t, n, T0, 0.03, 20, 0.0, "point_to_plane", "kahan32", loss="tukey", loss_k=0.01)
    o = oracle_lib.icp_register(d["src"], d["tgt"], d["tgt_normals"], T0, 0.03, 20, loss="tukey",
                                loss_k=0.01)
    ang, dt = pose_error(g.T, o.T)
    print(f"room 300k tukey: rot {ang:.2e} trans {dt:.2e} n_in {g.n_inliers}/{o.n_inliers}")
    assert g.n_inliers == o.n_inliers and _same_stop(g, o, icp), (g.n_iter, o.n_iter)
    assert ang <= 1e-5 and dt <= 1e-6


def test_huber_above_every_residual_is_plain(icp, c1):
    s, t, n = dev(c1["src"]), dev(c1["tgt"]), dev(c1["tgt_normals"])
    for precision in ("kahan32", "f64"):
        a = icp.register(s, t, n, np.eye(4), 0.05, 20, 0.0, "point_to_plane", precision)
        b = icp.register(s, t, n, np.eye(4), 0.05, 20, 0.0, "point_to_plane", precision,
                         loss="huber", loss_k=10.0)
        np.testing.assert_array_equal(a.T, b.T)
        assert (a.n_inliers, a.n_iter, a.inlier_rmse) == (b.n_inliers, b.n_iter, b.inlier_rmse)


def test_planted_outliers_on_gpu(icp, c1):
    rng = np.random.default_rng(9)
    src = c1["src"].copy()
    src[rng.random(len(src)) < 0.25, 2] += 0.025
    T0 = _near(c1["T_gt"], [0.005, -0.004, 0.006, 0.002, -0.002, 0.001])
    s, t, n = dev(src), dev(c1["tgt"]), dev(c1["tgt_normals"])
    plain = icp.register(s, t, n, T0, 0.05, 30)
    rob = icp.register(s, t, n, T0, 0.05, 30, loss="tukey", loss_k=0.01)
    ep = pose_error(plain.T, c1["T_gt"])[1]
    er = pose_error(rob.T, c1["T_gt"])[1]
    assert er < 0.5 * ep, (ep, er)
