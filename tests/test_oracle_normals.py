"""Pins of the normal-estimation oracle (hybrid radius / max_nn neighbourhood,
least-variance direction), each against something other than the oracle:
exact geometry (planes, a star of known covariance), numpy's symmetric
eigensolver, an independent numpy brute-force neighbourhood, and special
cases (ties, too few neighbours, orientation)."""
import numpy as np
import pytest

import oracle


def _angle(a, b):
    """Angle between the lines of a and b (atan2 form: accurate near 0)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    a = a / np.linalg.norm(a, axis=-1, keepdims=True)
    b = b / np.linalg.norm(b, axis=-1, keepdims=True)
    return np.arctan2(np.linalg.norm(np.cross(a, b), axis=-1), np.abs(np.sum(a * b, axis=-1)))


def test_axis_aligned_plane_is_exact():
    # all z equal: the covariance has an exactly zero z row, so the normal is e_z exactly
    rng = np.random.default_rng(1)
    P = np.column_stack([rng.uniform(-1, 1, 3000), rng.uniform(-1, 1, 3000), np.full(3000, 0.5)])
    P = P.astype(np.float32)
    N, cnt = oracle.estimate_normals(P, 0.1, 30, viewpoint=(0.0, 0.0, 10.0))
    assert cnt.min() >= 3
    np.testing.assert_array_equal(N, np.tile(np.float32([0, 0, 1]), (3000, 1)))
    N2, _ = oracle.estimate_normals(P, 0.1, 30, viewpoint=(0.0, 0.0, -10.0))
    np.testing.assert_array_equal(N2, np.tile(np.float32([0, 0, -1]), (3000, 1)))


def test_tilted_plane_within_input_rounding():
    rng = np.random.default_rng(2)
    n = np.array([0.3, -0.5, 0.8])
    n /= np.linalg.norm(n)
    u = np.cross(n, [1.0, 0.0, 0.0])
    u /= np.linalg.norm(u)
    v = np.cross(n, u)
    ab = rng.uniform(-1, 1, (4000, 2))
    P = (ab[:, :1] * u + ab[:, 1:] * v + np.array([0.1, 0.2, 0.3])).astype(np.float32)
    N, cnt = oracle.estimate_normals(P, 0.08, 30, viewpoint=10 * n)
    assert cnt.min() >= 3
    # float32 coordinates move points off the plane by ~1e-8 of the 0.08 m scale
    assert _angle(N, n).max() < 1e-5
    assert np.all(N.astype(np.float64) @ n > 0)


def test_star_of_known_covariance():
    # centre plus +-a R e1, +-b R e2, +-c R e3 (a > b > c): covariance R diag(2a^2, 2b^2, 2c^2)/7 R^T,
    # so the least-variance direction is R e3 (exact up to float32 rounding of the points)
    rng = np.random.default_rng(3)
    for trial in range(20):
        Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        a, b, c = 0.04, 0.025, 0.006
        ctr = rng.uniform(-1, 1, 3)
        pts = [ctr]
        for s, e in ((a, 0), (b, 1), (c, 2)):
            pts += [ctr + s * Q[:, e], ctr - s * Q[:, e]]
        P = np.array(pts, np.float32)
        N, cnt = oracle.estimate_normals(P, 0.2, 30, viewpoint=ctr + Q[:, 2])
        assert np.all(cnt == 7)
        assert _angle(N[0], Q[:, 2]) < 1e-5
        assert np.dot(N[0], Q[:, 2]) > 0


def test_eigensolver_matches_numpy():
    rng = np.random.default_rng(4)
    mats = []
    for _ in range(200):
        X = rng.normal(size=(3, 3))
        mats.append(X @ X.T)
    mats += [np.diag([3.0, 1.0, 2.0]), np.diag([1.0, 1.0, 1e-9]), np.zeros((3, 3)),
             np.array([[2.0, 1e-12, 0.0], [1e-12, 2.0, 0.0], [0.0, 0.0, 5.0]])]
    for A in mats:
        w, V = oracle.sym_eig3(A)
        w2, V2 = np.linalg.eigh(A)
        scale = max(np.abs(w2).max(), 1e-300)
        assert np.abs(w - w2).max() <= 1e-12 * scale
        np.testing.assert_allclose(V.T @ V, np.eye(3), atol=1e-12)
        np.testing.assert_allclose(A @ V, V * w, atol=1e-11 * scale)
        gaps = np.diff(w2)
        if gaps[0] > 1e-6 * scale:  # the least eigenvector is well defined
            assert _angle(V[:, 0], V2[:, 0]) < 1e-9


def _numpy_normals(P, radius, max_nn, view):
    """Independent brute-force definition in numpy: pinned float32 distances,
    lexicographic (d2, index) selection, float64 covariance, numpy eigh."""
    P = np.asarray(P, np.float32)
    r2f = np.float32(radius * radius)
    out = np.zeros((len(P), 3))
    cnt = np.zeros(len(P), np.int64)
    gap = np.zeros(len(P))
    for i in range(len(P)):
        d = P[i] - P
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        cand = np.nonzero(d2 <= r2f)[0]
        order = np.lexsort((cand, d2[cand]))
        nb = cand[order][:max_nn]
        cnt[i] = len(nb)
        if len(nb) < 3:
            continue
        X = P[nb].astype(np.float64)
        C = np.cov(X.T, bias=True)
        w, V = np.linalg.eigh(C)
        n = V[:, 0]
        if np.dot(n, np.asarray(view) - P[i].astype(np.float64)) < 0:
            n = -n
        out[i] = n
        gap[i] = (w[1] - w[0]) / max(w.sum(), 1e-300)
    return out, cnt, gap


@pytest.mark.parametrize("max_nn", [1, 3, 8, 30])
def test_selection_and_normals_match_numpy_brute_force(max_nn):
    rng = np.random.default_rng(5 + max_nn)
    # a noisy surface patch plus exact duplicates and lattice points (equal distances)
    xy = rng.uniform(0, 0.3, (250, 2))
    z = 0.05 * np.sin(10 * xy[:, 0]) + rng.normal(0, 0.002, 250)
    P = np.column_stack([xy, z])
    lat = np.stack(np.meshgrid(np.arange(4), np.arange(4), [0.0]), -1).reshape(-1, 3) * 0.0625
    P = np.concatenate([P, P[:10], lat + 0.5]).astype(np.float32)
    view = (0.1, 0.2, 1.0)
    N, cnt, ev = oracle.estimate_normals(P, 0.07, max_nn, viewpoint=view, with_evals=True)
    Nr, cntr, gap = _numpy_normals(P, 0.07, max_nn, view)
    np.testing.assert_array_equal(cnt, cntr)
    ok = (cnt >= 3) & (gap > 1e-6)
    assert ok.sum() > 100 or max_nn < 3
    if ok.any():
        assert _angle(N[ok], Nr[ok]).max() < 1e-6
    facing = np.abs(np.sum(Nr * (np.asarray(view) - P.astype(np.float64)), 1)) > 1e-6
    assert np.all(np.sign(np.sum(N[ok & facing] * Nr[ok & facing], 1)) > 0)
    assert np.all(N[cnt < 3] == 0)


def test_ties_go_to_smaller_index():
    # the query at the origin has six neighbours at exactly the same distance;
    # max_nn = 4 keeps itself and the three of smallest index: +x, -x, +y, whose
    # covariance lies in the xy-plane, so the normal is e_z (a wrong tie-break
    # that keeps +z gives a normal in the xy-plane)
    s = 0.5
    P = np.array([[0, 0, 0], [s, 0, 0], [-s, 0, 0], [0, s, 0], [0, 0, s], [0, -s, 0], [0, 0, -s]],
                 np.float32)
    N, cnt = oracle.estimate_normals(P, 0.6, 4, viewpoint=(0.0, 0.0, 5.0), queries=[0])
    assert cnt[0] == 4
    np.testing.assert_array_equal(N[0], np.float32([0, 0, 1]))


def test_too_few_neighbours_give_zero():
    P = np.array([[0, 0, 0], [0.01, 0, 0], [5, 5, 5], [9, 9, 9]], np.float32)
    N, cnt = oracle.estimate_normals(P, 0.1, 30)
    np.testing.assert_array_equal(cnt, [2, 2, 1, 1])
    assert np.all(N == 0)


def test_tree_and_brute_force_agree_bitwise():
    rng = np.random.default_rng(6)
    P = rng.uniform(0, 1, (4000, 3)).astype(np.float32)
    a = oracle.estimate_normals(P, 0.08, 16, search=1, with_evals=True)
    b = oracle.estimate_normals(P, 0.08, 16, search=2, with_evals=True)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_sphere_normals_are_radial_and_face_the_viewpoint():
    rng = np.random.default_rng(7)
    v = rng.normal(size=(20000, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    ctr = np.array([0.2, -0.1, 0.4])
    P = (ctr + 0.5 * v).astype(np.float32)
    N, cnt = oracle.estimate_normals(P, 0.03, 30, viewpoint=ctr)
    assert cnt.min() >= 3
    # a 3 cm cap of a 50 cm sphere tilts the fitted plane by at most ~0.03 rad
    assert np.percentile(_angle(N, v), 99) < 0.03
    assert np.all(np.sum(N * v, 1) < 0)  # facing the centre
