"""GPU normal estimation (icp_estimate_normals) against the oracle.

Bar: neighbourhood sizes bit-exact (integer); normals within 1e-6 rad of the
oracle's wherever the least eigenvector is well defined (relative eigengap
(l1 - l0) / (l0 + l1 + l2) > 1e-6), same orientation wherever the point does
not lie within 1e-6 of the viewpoint's plane through it; zero exactly where
fewer than three neighbours exist; unit length elsewhere; where the least
eigenvector is not unique (duplicates, lattices, collinear or identical
points) the normal lies in the least eigenspace of the neighbourhood
covariance (n^T C n <= l0 + 1e-6 tr C).

Tolerance: both sides form the covariance in float64 from float32 points and
differ only in summation order and in the (shifted one-pass vs centred
two-pass) covariance formula, a relative difference of order 1e-15; divided by
a relative eigengap >= 1e-6 that moves the eigenvector by < 1e-9 rad, and the
float32 rounding of the output adds < 2e-7 rad.
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _angle(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    a = a / np.linalg.norm(a, axis=-1, keepdims=True)
    b = b / np.linalg.norm(b, axis=-1, keepdims=True)
    return np.arctan2(np.linalg.norm(np.cross(a, b), axis=-1), np.abs(np.sum(a * b, axis=-1)))


def _neighbourhood(P, i, radius, max_nn):
    """Hybrid neighbourhood of point i by brute force: the max_nn smallest
    (pinned float32 squared distance, index) within radius."""
    d = P - P[i]
    d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    r2 = np.float32(radius * radius)
    cand = np.nonzero(d2 <= r2)[0]
    order = np.lexsort((cand, d2[cand]))
    return cand[order[:max_nn]]


def _least_eigenspace_ok(P, sel, N, radius, max_nn, which):
    """For the points `which` (positions into sel) whose least eigenvector is
    not unique: the normal must lie in the least eigenspace of the
    neighbourhood covariance C, n^T C n <= l0 + 1e-6 tr C (a direction along
    a collinear neighbourhood, say, has n^T C n = l2 and fails)."""
    for k in which:
        nb = _neighbourhood(P, sel[k], radius, max_nn)
        X = P[nb].astype(np.float64)
        X = X - X.mean(0)
        C = X.T @ X / len(nb)
        l0 = np.linalg.eigvalsh(C)[0]
        n = N[k].astype(np.float64)
        assert n @ C @ n <= l0 + 1e-6 * np.trace(C) + 1e-300, (k, n @ C @ n, l0, np.trace(C))


def check(icp, oracle_lib, P, radius, max_nn, view, queries=None, label=""):
    P = np.ascontiguousarray(P, np.float32)
    print(f"\n[normals] {label} n={len(P)} radius={radius} max_nn={max_nn}", flush=True)
    N, cnt = icp.estimate_normals(_dev(P), radius, max_nn, view, with_counts=True)
    N, cnt = N.cpu().numpy(), cnt.cpu().numpy()
    sel = np.arange(len(P)) if queries is None else np.asarray(queries)
    oN, ocnt, oev = oracle_lib.estimate_normals(P, radius, max_nn, view, queries=queries, with_evals=True)
    N, cnt = N[sel], cnt[sel]
    np.testing.assert_array_equal(cnt, ocnt)
    few = ocnt < 3
    assert np.all(N[few] == 0)
    if (~few).any():
        assert np.abs(np.linalg.norm(N[~few].astype(np.float64), axis=1) - 1).max() < 1e-6
    gap = (oev[:, 1] - oev[:, 0]) / np.maximum(oev.sum(1), 1e-300)
    ok = ~few & (gap > 1e-6)
    if ok.any():
        ang = _angle(N[ok], oN[ok])
        assert ang.max() <= 1e-6, (ang.max(), np.argmax(ang))
        vp = np.asarray(view, np.float64) - P[sel].astype(np.float64)
        facing = np.abs(np.sum(oN.astype(np.float64) * vp, 1)) > 1e-6 * np.linalg.norm(vp, axis=1)
        both = ok & facing
        assert np.all(np.sum(N[both].astype(np.float64) * oN[both], 1) > 0)
    ill = np.nonzero(~few & ~ok)[0]
    _least_eigenspace_ok(P, sel, N, radius, max_nn, ill)
    print(f"[normals] {label}: {ok.sum()} compared, {few.sum()} with < 3 neighbours, "
          f"{(~few & ~ok).sum()} ill-conditioned, counts {cnt.min()}..{cnt.max()}", flush=True)
    return cnt


@pytest.mark.parametrize("radius,max_nn", [(0.05, 30), (0.03, 30), (0.05, 64), (0.05, 3), (0.02, 1)])
def test_heightfield(icp, oracle_lib, radius, max_nn):
    P, _ = synth.heightfield_surface(0, 5000)
    cnt = check(icp, oracle_lib, P, radius, max_nn, (0.5, 0.5, 2.0), label="heightfield")
    if max_nn == 30 and radius == 0.05:
        assert cnt.max() == 30  # the max_nn limit binds (heap path)


@pytest.mark.parametrize("sub", ["1", "2"])
def test_room_spanning_blocks_with_ragged_tail(icp, oracle_lib, sub, monkeypatch):
    monkeypatch.setenv("ICP_GRID_SUB", sub)
    d = synth.room_pair_random(3, 60000 + 37, 1000)
    check(icp, oracle_lib, d["tgt"], 0.06, 30, (3.0, 2.0, 1.5), label=f"room sub={sub}")


@pytest.mark.parametrize("scale", ["1.5", "3"])
def test_coarser_grids_give_the_same_neighbourhoods(icp, oracle_lib, scale, monkeypatch):
    # any cell edge above the radius bound is exact; only the scan order moves
    monkeypatch.setenv("ICP_GRID_SCALE", scale)
    d = synth.room_pair_random(4, 30000, 1000)
    check(icp, oracle_lib, d["tgt"], 0.06, 30, (3.0, 2.0, 1.5), label=f"room grid x{scale}")


def test_duplicates_ties_and_tiny_clouds(icp, oracle_lib):
    rng = np.random.default_rng(11)
    base = rng.uniform(0, 0.1, (10, 3))
    P = np.repeat(base, 50, axis=0)  # ties everywhere: selection by original index
    rng.shuffle(P)
    check(icp, oracle_lib, P, 0.05, 30, (1.0, 1.0, 1.0), label="duplicates")
    lat = np.stack(np.meshgrid(np.arange(6), np.arange(6), np.arange(2)), -1).reshape(-1, 3) * 0.5
    check(icp, oracle_lib, lat, 0.6, 4, (0.3, 0.2, 5.0), label="lattice ties")
    for n in (1, 2, 3, 4, 7):
        check(icp, oracle_lib, rng.uniform(0, 0.01, (n, 3)), 0.1, 30, (0.0, 0.0, 1.0), label=f"n={n}")
    # collinear neighbourhoods: the normal must be perpendicular to the line
    t = np.arange(40, dtype=np.float64)[:, None] * 0.01
    line = np.float32([0.1, 0.2, 0.3]) + t * np.float64([0.6, 0.0, 0.8])
    check(icp, oracle_lib, line, 0.05, 30, (1.0, 1.0, 1.0), label="collinear")
    N = icp.estimate_normals(_dev(line), 0.05, 30, (1.0, 1.0, 1.0)).cpu().numpy().astype(np.float64)
    assert np.abs(N @ np.float64([0.6, 0.0, 0.8])).max() < 1e-5


def test_identical_points(icp):
    P = np.tile(np.float32([[0.25, -0.5, 1.0]]), (100, 1))
    N, cnt = icp.estimate_normals(_dev(P), 0.1, 30, (0.0, 0.0, 0.0), with_counts=True)
    assert torch.all(cnt == 30)
    n = torch.linalg.norm(N.double(), dim=1)
    assert torch.allclose(n, torch.ones_like(n), atol=1e-6)  # any unit vector is valid


def test_full_size_room_sampled(icp, oracle_lib):
    d = synth.c3_room(0)
    P = d["tgt"]
    q = np.random.default_rng(12).choice(len(P), 20000, replace=False)
    check(icp, oracle_lib, P, 0.05, 30, (6.0, 4.0, 1.5), queries=q, label="room 2M, 20k sampled")


def test_argument_errors(icp):
    P = _dev(np.zeros((10, 3)))
    for kw in (dict(radius=0.0), dict(radius=float("nan")), dict(max_nn=0), dict(max_nn=65)):
        a = dict(radius=0.1, max_nn=30)
        a.update(kw)
        with pytest.raises(icp.IcpError):
            icp.estimate_normals(P, a["radius"], a["max_nn"])
    bad = P.clone()
    bad[3, 1] = float("inf")
    with pytest.raises(icp.IcpError) as e:
        icp.estimate_normals(bad, 0.1, 30)
    assert e.value.code == icp.ICP_E_NONFINITE
