"""Pins of the FPFH oracle, each against something outside it:

F1 a plane with a common normal: every pair feature is zero, so each SPFH
sub-histogram is 100 in its middle bin and FPFH adds (1/k') sum 100 / w_j
there (closed form from the neighbour distances);
F2 a sphere with outward normals: alpha = 0, phi = -d / 2 and
theta = atan2(-d sqrt(1 - d^2 / 4), 1 - d^2 / 2) for a chord of length d
(closed form of the Darboux frame on a sphere);
F3 an exact 90-degree rotation about z (coordinates and normals permuted and
negated without rounding) leaves every descriptor bit-identical, and a
general rigid motion leaves almost all of them equal;
F4 sub-histogram sums: SPFH blocks sum to 100, FPFH blocks to
100 [k_i > 0] + (1/k') sum 100 [k_j > 0] / w_j;
F5 the neighbour lists by brute force equal those of the k-d tree, sorted by
(distance, index) and capped at max_nn;
F6 degenerate inputs: an isolated point, a duplicate point and a normal
parallel to the line give no pair.
"""
import math

import numpy as np
from scipy.spatial.transform import Rotation

import oracle
from oracle import fpfh as F


def _plane(rng, n=400):
    p = np.zeros((n, 3), np.float32)
    p[:, :2] = rng.random((n, 2)).astype(np.float32)
    nrm = np.tile(np.array([0, 0, 1], np.float32), (n, 1))
    return p, nrm


def test_f1_plane_closed_form():
    rng = np.random.default_rng(1)
    p, nrm = _plane(rng)
    desc, counts, k, nn, _ = F.fpfh(p, nrm, 0.1, 30)
    nb, _ = oracle.hybrid_neighbors(p, 0.1, 30)
    P = p.astype(np.float64)
    for i in range(len(p)):
        js = [j for j in nb[i] if j >= 0 and j != i]
        assert k[i] == len(js)
        want = np.zeros(33)
        if js:
            w = np.linalg.norm(P[js] - P[i], axis=1)
            want[[5, 16, 27]] = 100.0 + 100.0 * np.sum(1.0 / w) / len(js)
            assert counts[i, 5] == counts[i, 16] == counts[i, 27] == len(js)
        np.testing.assert_allclose(desc[i], want.astype(np.float32), rtol=2e-7)


def _sphere(rng, n=2000):
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v.astype(np.float32), v.astype(np.float32)


def test_f2_sphere_closed_form():
    rng = np.random.default_rng(2)
    p, nrm = _sphere(rng)
    P, N = p.astype(np.float64), nrm.astype(np.float64)
    i = rng.integers(0, len(p), 500)
    j = rng.integers(0, len(p), 500)
    keep = i != j
    a, f, t, ok = F.pair_features(P[i[keep]], N[i[keep]], P[j[keep]], N[j[keep]])
    d = np.linalg.norm(P[j[keep]] - P[i[keep]], axis=1)
    assert ok.all()
    np.testing.assert_allclose(a, 0.0, atol=1e-6)
    np.testing.assert_allclose(f, -d / 2, atol=1e-6)
    np.testing.assert_allclose(t, np.arctan2(-d * np.sqrt(1 - d * d / 4), 1 - d * d / 2), atol=1e-6)


def test_f3_rotation_invariance():
    rng = np.random.default_rng(3)
    p, nrm = _sphere(rng, 1500)
    p = (p * np.float32(0.5) + rng.normal(scale=0.01, size=p.shape).astype(np.float32)).astype(np.float32)
    desc, *_ = F.fpfh(p, nrm, 0.15, 40)
    R90 = lambda a: np.stack([-a[:, 1], a[:, 0], a[:, 2]], axis=1).astype(np.float32)
    d90, *_ = F.fpfh(R90(p), R90(nrm), 0.15, 40)
    np.testing.assert_array_equal(d90, desc)
    R = Rotation.from_rotvec([0.3, -0.5, 0.7]).as_matrix()
    pr = (p.astype(np.float64) @ R.T + [1.0, -2.0, 0.5]).astype(np.float32)
    nr = (nrm.astype(np.float64) @ R.T).astype(np.float32)
    dr, *_ = F.fpfh(pr, nr, 0.15, 40)
    close = np.all(np.abs(dr - desc) <= 1e-3 * (1 + np.abs(desc)), axis=1)
    assert close.mean() > 0.9


def test_f4_histogram_sums():
    rng = np.random.default_rng(4)
    p, nrm = _sphere(rng, 1200)
    desc, counts, k, nn, _ = F.fpfh(p, nrm, 0.2, 25)
    nb, _ = oracle.hybrid_neighbors(p, 0.2, 25)
    P = p.astype(np.float64)
    for blk in range(3):
        s = counts[:, 11 * blk:11 * (blk + 1)].sum(axis=1)
        np.testing.assert_array_equal(s, k)
    for i in range(0, len(p), 7):
        js = [j for j in nb[i] if j >= 0 and j != i]
        w = np.linalg.norm(P[js] - P[i], axis=1)
        extra = np.sum(100.0 * (k[js] > 0) / w) / len(js) if js else 0.0
        for blk in range(3):
            want = 100.0 * (k[i] > 0) + extra
            assert abs(desc[i, 11 * blk:11 * (blk + 1)].astype(np.float64).sum() - want) <= 1e-5 * want


def test_f5_neighbour_lists():
    rng = np.random.default_rng(5)
    p = rng.random((800, 3)).astype(np.float32)
    a, ca = oracle.hybrid_neighbors(p, 0.15, 12, search=1)
    b, cb = oracle.hybrid_neighbors(p, 0.15, 12, search=2)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(ca, cb)
    r2f = np.float32(0.15 * 0.15)
    for i in range(0, 800, 37):
        dd = p - p[i]  # float32, as the selection's distance
        d2 = (dd[:, 0] * dd[:, 0] + dd[:, 1] * dd[:, 1]) + dd[:, 2] * dd[:, 2]
        inside = np.nonzero(d2 <= r2f)[0]
        order = inside[np.lexsort((inside, d2[inside]))][:12]
        assert ca[i] == len(order) and list(a[i, :len(order)]) == list(order)
        assert a[i, 0] == i


def test_f6_degenerate_pairs():
    p = np.array([[0, 0, 0], [0, 0, 0], [0.05, 0, 0], [5, 5, 5], [0, 0, 0.05]], np.float32)
    nrm = np.array([[0, 0, 1], [0, 0, 1], [1, 0, 0], [0, 0, 1], [0, 0, 1]], np.float32)
    desc, counts, k, nn, _ = F.fpfh(p, nrm, 0.1, 10)
    assert k[3] == 0 and not desc[3].any()  # isolated
    # point 0: point 1 is a duplicate (skipped); point 2 counts; point 4 lies
    # along both normals (frame undefined, skipped)
    assert k[0] == 1 and k[1] == 1
    a, f, t, ok = F.pair_features(p[[0]], nrm[[0]], p[[4]], nrm[[4]])
    assert not ok[0]
