"""Pose-graph optimisation (icp_pose_graph_optimize) against the oracle.

Bar: both sides are float64 throughout and differ only in summation order
and in the Cholesky implementation, so a consistent graph must be recovered
to 1e-10 and the optimised poses of a noisy graph must agree with the
oracle's within 1e-8 (rotation angle, rad / translation, m), F within 1e-9
relative.  Near convergence Levenberg-Marquardt's keep/refuse decisions
compare nearly equal F values, so the number of kept steps may differ; the
poses they reach may not.
"""
import os
import sys

import numpy as np
import pytest

from oracle import posegraph as opg
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


def _worst(Pa, Pb):
    errs = [pose_error(a, b) for a, b in zip(Pa, Pb)]
    return max(e[0] for e in errs), max(e[1] for e in errs)


def test_consistent_graph_recovered(icp):
    d = synth.pose_graph(1, 30, 20, noise_deg=0.0, noise_m=0.0)
    P, res = icp.pose_graph_optimize(d["init"], d["edges"], "gn", 30, 1e-14)
    assert res["F_initial"] > 1e-3 and res["F_final"] < 1e-18
    ang, dt = _worst(P, d["gt"])
    assert ang < 1e-10 and dt < 1e-10
    np.testing.assert_array_equal(P[0], d["init"][0])


@pytest.mark.parametrize("method", ["gn", "lm"])
@pytest.mark.parametrize("n,closures", [(12, 6), (64, 40), (200, 150), (256, 256)])
def test_noisy_graph_matches_oracle(icp, method, n, closures):
    d = synth.pose_graph(2 + n, n, closures)
    P, res = icp.pose_graph_optimize(d["init"], d["edges"], method, 100, 1e-13)
    O, F0, F, steps, status = opg.optimize(list(d["init"]), d["edges"], method, 100, 1e-13)
    ang, dt = _worst(P, O)
    print(f"\n[pose graph] n={n} {method}: F {res['F_initial']:.4g} -> {res['F_final']:.6g} "
          f"(oracle {F:.6g}), steps {res['steps']}/{steps}, status {res['status']}/{status}, "
          f"pose diff {ang:.2e} rad {dt:.2e} m", flush=True)
    assert abs(res["F_initial"] - F0) <= 1e-12 * F0
    assert abs(res["F_final"] - F) <= 1e-9 * F
    assert ang <= 1e-8 and dt <= 1e-8
    assert res["status"] != icp.ICP_DEGENERATE


def test_tree_graph_composes_measurements(icp):
    d = synth.pose_graph(5, 15, 0)
    edges = d["edges"][:-1]  # drop the loop-closing edge: a chain
    P, res = icp.pose_graph_optimize(d["init"], edges, "gn", 50, 1e-16)
    assert res["F_final"] < 1e-18
    T = np.eye(4)
    for k, (i, j, Z, L) in enumerate(edges):
        T = T @ Z
        ang, dt = pose_error(P[j], T)
        assert ang < 1e-9 and dt < 1e-9


def test_disconnected_node_is_degenerate(icp):
    d = synth.pose_graph(6, 10, 0)
    edges = [e for e in d["edges"] if 5 not in (e[0], e[1])]
    P, res = icp.pose_graph_optimize(d["init"], edges, "gn", 10, 0.0)
    assert res["status"] == icp.ICP_DEGENERATE and res["steps"] == 0
    np.testing.assert_array_equal(P, d["init"])
    O, F0, F, steps, status = opg.optimize(list(d["init"]), edges, "gn", 10, 0.0)
    assert status == opg.DEGENERATE and steps == 0


def test_disconnected_node_beyond_first_block_is_degenerate(icp):
    """A free node with no edge beyond the first 64 unknowns: its zero pivot
    is found by the diagonal factorisation fused into the trailing update
    (not by the first diagonal block), and the run stops degenerate."""
    d = synth.pose_graph(8, 30, 10)
    lost = 20  # unknowns 114..119, in the second 64-column block
    edges = [e for e in d["edges"] if lost not in (e[0], e[1])]
    P, res = icp.pose_graph_optimize(d["init"], edges, "lm", 10, 0.0)
    assert res["status"] == icp.ICP_DEGENERATE and res["steps"] == 0
    np.testing.assert_array_equal(P, d["init"])
    O, F0, F, steps, status = opg.optimize(list(d["init"]), edges, "lm", 10, 0.0)
    assert status == opg.DEGENERATE and steps == 0


@pytest.mark.parametrize("method", ["gn", "lm"])
def test_graph_with_whole_last_block(icp, method):
    """33 nodes: 32 free nodes, 192 unknowns, so the last 64-column block of
    the factorisation is full."""
    d = synth.pose_graph(9, 33, 20)
    P, res = icp.pose_graph_optimize(d["init"], d["edges"], method, 100, 1e-13)
    O, F0, F, steps, status = opg.optimize(list(d["init"]), d["edges"], method, 100, 1e-13)
    ang, dt = _worst(P, O)
    assert abs(res["F_final"] - F) <= 1e-9 * F
    assert ang <= 1e-8 and dt <= 1e-8
    assert res["status"] != icp.ICP_DEGENERATE
