"""Pins of the pose-graph oracle, each against something outside it:
G1 Exp / Log against scipy's expm / logm and each other; G2 the adjoint
identity T Exp(xi) T^-1 = Exp(Ad_T xi); G3 the edge Jacobians by central
differences where the residual vanishes; G4 a consistent graph with loops is
recovered exactly from perturbed poses; G5 a tree graph reaches F = 0 with
T_j = T_i Z_ij (composition of the measurements); G7 LM decreases F and
ends at a stationary point (the Gauss-Newton one), node 0 untouched."""
import numpy as np
import scipy.linalg

from oracle import posegraph as pg


def _rand_T(rng, ang=1.0, trans=1.0):
    ax = rng.normal(size=3)
    ax /= np.linalg.norm(ax)
    return pg.exp_se3(np.concatenate([ax * rng.uniform(0, ang), rng.normal(size=3) * trans]))


def _twist(xi):
    X = np.zeros((4, 4))
    X[:3, :3] = pg.hat(xi[:3])
    X[:3, 3] = xi[3:]
    return X


def test_g1_exp_log_against_scipy():
    rng = np.random.default_rng(1)
    for k in range(200):
        xi = rng.normal(size=6) * (10.0 ** rng.uniform(-9, 0.3))
        if np.linalg.norm(xi[:3]) > 3.0:  # Log returns the angle in [0, pi)
            xi[:3] *= 3.0 / np.linalg.norm(xi[:3])
        T = pg.exp_se3(xi)
        np.testing.assert_allclose(T, scipy.linalg.expm(_twist(xi)), atol=1e-13)
        np.testing.assert_allclose(pg.log_se3(T), xi, atol=1e-12 * max(1, np.abs(xi).max()))
        L = np.real(scipy.linalg.logm(T))
        np.testing.assert_allclose(pg.log_se3(T)[3:], L[:3, 3], atol=1e-10)


def test_g2_adjoint_identity():
    rng = np.random.default_rng(2)
    for _ in range(50):
        T = _rand_T(rng)
        xi = rng.normal(size=6) * 0.3
        np.testing.assert_allclose(T @ pg.exp_se3(xi) @ pg.inv(T), pg.exp_se3(pg.adjoint(T) @ xi),
                                   atol=1e-12)


def test_g3_edge_jacobians_by_central_differences():
    rng = np.random.default_rng(3)
    for _ in range(20):
        Ti, Tj = _rand_T(rng), _rand_T(rng)
        Z = pg.inv(Ti) @ Tj  # consistent edge: e = 0
        poses = [Ti, Tj]
        edge = (0, 1, Z, np.eye(6))
        e0, J, _ = pg.edge_terms(poses, edge)
        assert np.abs(e0).max() < 1e-12
        h = 1e-6
        Jj = np.zeros((6, 6))
        Ji = np.zeros((6, 6))
        for m in range(6):
            d = np.zeros(6)
            d[m] = h
            ep = pg.edge_terms([Ti, pg.exp_se3(d) @ Tj], edge)[0]
            em = pg.edge_terms([Ti, pg.exp_se3(-d) @ Tj], edge)[0]
            Jj[:, m] = (ep - em) / (2 * h)
            ep = pg.edge_terms([pg.exp_se3(d) @ Ti, Tj], edge)[0]
            em = pg.edge_terms([pg.exp_se3(-d) @ Ti, Tj], edge)[0]
            Ji[:, m] = (ep - em) / (2 * h)
        np.testing.assert_allclose(Jj, J, atol=1e-7)
        np.testing.assert_allclose(Ji, -J, atol=1e-7)


def loop_graph(rng, n, closures, noise_rot=0.0, noise_t=0.0):
    """n poses on a closed trajectory, odometry edges plus random closures."""
    gt = [np.eye(4)]
    for k in range(1, n):
        step = pg.exp_se3(np.array([0, 0, 2 * np.pi / n, 0.5, 0, 0]) + rng.normal(size=6) * 0.02)
        gt.append(gt[-1] @ step)
    pairs = [(k, k + 1) for k in range(n - 1)] + [(n - 1, 0)]
    while len(pairs) < n + closures:
        i, j = sorted(rng.choice(n, 2, replace=False))
        if (i, j) not in pairs:
            pairs.append((int(i), int(j)))
    edges = []
    for i, j in pairs:
        Z = pg.inv(gt[i]) @ gt[j]
        if noise_rot or noise_t:
            Z = Z @ pg.exp_se3(np.concatenate([rng.normal(size=3) * noise_rot, rng.normal(size=3) * noise_t]))
        Q, _ = np.linalg.qr(rng.normal(size=(6, 6)))
        L = Q @ np.diag(rng.uniform(0.5, 5.0, 6)) @ Q.T
        edges.append((i, j, Z, L))
    return gt, edges


def test_g4_consistent_graph_recovered_exactly():
    rng = np.random.default_rng(4)
    gt, edges = loop_graph(rng, 20, 15)
    init = [gt[0]] + [pg.exp_se3(rng.normal(size=6) * 0.05) @ T for T in gt[1:]]
    P, F0, F, steps, status = pg.optimize(init, edges, "gn", 30, 1e-14)
    assert F0 > 1e-3 and F < 1e-20
    for a, b in zip(P, gt):
        np.testing.assert_allclose(a, b, atol=1e-10)


def test_g5_tree_graph_composes_measurements():
    rng = np.random.default_rng(5)
    n = 12
    edges = []
    parent = [None] + [int(rng.integers(0, k)) for k in range(1, n)]
    for k in range(1, n):
        Z = _rand_T(rng, 0.5, 0.5)
        edges.append((parent[k], k, Z, np.diag(rng.uniform(1, 3, 6))))
    init = [np.eye(4)] + [_rand_T(rng, 0.05, 0.05) for _ in range(1, n)]
    P, F0, F, steps, status = pg.optimize(init, edges, "gn", 50, 1e-16)
    assert F < 1e-18
    expect = [np.eye(4)] * n
    for k in range(1, n):  # parents precede children
        expect[k] = expect[parent[k]] @ edges[k - 1][2]
    for a, b in zip(P, expect):
        np.testing.assert_allclose(a, b, atol=1e-9)


def test_g7_lm_decreases_and_reaches_a_stationary_point():
    rng = np.random.default_rng(7)
    gt, edges = loop_graph(rng, 25, 20, noise_rot=0.01, noise_t=0.02)
    init = [gt[0]] + [pg.exp_se3(rng.normal(size=6) * 0.2) @ T for T in gt[1:]]
    P, F0, F, steps, status = pg.optimize(init, edges, "lm", 100, 1e-14)
    assert F < F0
    np.testing.assert_array_equal(P[0], gt[0])
    H, g, F2 = pg.normal_equations(P, edges)
    assert abs(F2 - F) <= 1e-12 * F
    assert np.linalg.norm(g) <= 1e-6 * np.linalg.norm(np.diag(H)) ** 0.5
    Pg, _, Fg, _, _ = pg.optimize(init, edges, "gn", 100, 1e-14)
    assert abs(Fg - F) <= 1e-6 * F
