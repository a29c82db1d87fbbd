"""Pose-graph optimisation oracle (multiway registration), plain numpy FP64.

TEST INFRASTRUCTURE ONLY: imported by the test-suite and the benchmark's
CPU-baseline leg, never by the GPU library or its binding; it shares no code
with the GPU path.

What it computes (paper: Sec. 3.3 "multiway registration using pose graph
optimization" and Sec. 2, the in-house Gauss-Newton and Levenberg-Marquardt
solvers).  The paper names the method only; the reading:

  * nodes carry poses T_i (node frame -> world); an edge (i, j, Z, L) carries a
    measured relative pose Z ~ T_i^-1 T_j and a 6x6 information matrix L;
  * residual e_ij = Log(Z^-1 T_i^-1 T_j) in R^6, rotation first (the same
    (omega, v) order and Exp as the ICP step); objective F = sum e^T L e;
  * node 0 is held fixed (gauge); the others move by left perturbations
    T_k <- Exp(d_k) T_k;
  * linearisation: de/dd_j = Ad(T_j^-1), de/dd_i = -Ad(T_j^-1), exact where
    e = 0 (the inverse right Jacobian of Log is taken as the identity), so a
    consistent graph is recovered exactly;
  * Gauss-Newton: H d = -g with H = sum J^T L J, g = sum J^T L e, solved by
    Cholesky; Levenberg-Marquardt: (H + lambda diag(H)) d = -g, lambda0 = 1e-4,
    a step is kept if F decreases (lambda / 10), else undone (lambda * 10);
  * stop after max_iter steps, or when a kept step changes F by at most
    rel_tol * F, or (LM) after 10 refusals in a row; a failed Cholesky pivot
    (<= 1e-12 max diag) ends the run as DEGENERATE.
"""
from __future__ import annotations

import numpy as np

OK, CONVERGED, DEGENERATE = 0, 1, 2


def hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def exp_se3(xi):
    """Exp of (omega, v): [[R, V v], [0, 1]] (Rodrigues, Taylor series near 0)."""
    w, v = np.asarray(xi[:3], np.float64), np.asarray(xi[3:], np.float64)
    th2 = float(w @ w)
    th = np.sqrt(th2)
    if th < 1e-4:
        A = 1 - th2 / 6 + th2 * th2 / 120
        B = 0.5 - th2 / 24 + th2 * th2 / 720
        C = 1 / 6 - th2 / 120 + th2 * th2 / 5040
    else:
        A, B, C = np.sin(th) / th, (1 - np.cos(th)) / th2, (th - np.sin(th)) / (th2 * th)
    W = hat(w)
    T = np.eye(4)
    T[:3, :3] = np.eye(3) + A * W + B * W @ W
    T[:3, 3] = (np.eye(3) + B * W + C * W @ W) @ v
    return T


def log_se3(T):
    """Log of a rigid transform with rotation angle below pi - 1e-6."""
    R, t = T[:3, :3], T[:3, 3]
    c = np.clip((np.trace(R) - 1) / 2, -1.0, 1.0)
    th = np.arccos(c)
    vee = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    if th < 1e-4:
        w = 0.5 * (1 + th * th / 6) * vee
        k = 1 / 12 + th * th / 720
    else:
        w = th / (2 * np.sin(th)) * vee
        k = (1 - th * np.sin(th) / (2 * (1 - np.cos(th)))) / (th * th)
    W = hat(w)
    Vinv = np.eye(3) - 0.5 * W + k * W @ W
    return np.concatenate([w, Vinv @ t])


def inv(T):
    Ti = np.eye(4)
    Ti[:3, :3] = T[:3, :3].T
    Ti[:3, 3] = -T[:3, :3].T @ T[:3, 3]
    return Ti


def adjoint(T):
    """Ad_T for (omega, v) twists: T Exp(xi) T^-1 = Exp(Ad_T xi)."""
    R, t = T[:3, :3], T[:3, 3]
    A = np.zeros((6, 6))
    A[:3, :3] = R
    A[3:, :3] = hat(t) @ R
    A[3:, 3:] = R
    return A


def edge_terms(poses, edge):
    i, j, Z, L = edge
    e = log_se3(inv(Z) @ inv(poses[i]) @ poses[j])
    J = adjoint(inv(poses[j]))
    return e, J, L


def objective(poses, edges):
    F = 0.0
    for ed in edges:
        e, _, L = edge_terms(poses, ed)
        F += float(e @ L @ e)
    return F


def normal_equations(poses, edges):
    """Dense H (6(N-1) square) and g over the free nodes 1..N-1, and F."""
    n = len(poses) - 1
    H = np.zeros((6 * n, 6 * n))
    g = np.zeros(6 * n)
    F = 0.0
    for ed in edges:
        i, j = ed[0], ed[1]
        e, J, L = edge_terms(poses, ed)
        K = J.T @ L @ J
        u = J.T @ L @ e
        F += float(e @ L @ e)
        for a, sa in ((i, -1.0), (j, 1.0)):
            if a == 0:
                continue
            g[6 * (a - 1):6 * a] += sa * u
            for b, sb in ((i, -1.0), (j, 1.0)):
                if b == 0:
                    continue
                H[6 * (a - 1):6 * a, 6 * (b - 1):6 * b] += sa * sb * K
    return H, g, F


def optimize(poses, edges, method="gn", max_iter=30, rel_tol=1e-10):
    """Returns (poses, F_initial, F_final, steps, status)."""
    P = [np.array(T, np.float64) for T in poses]
    H, g, F = normal_equations(P, edges)
    F0 = F
    lam = 1e-4
    steps, refusals = 0, 0
    status = OK
    while steps < max_iter:
        A = H.copy()
        if method == "lm":
            A[np.diag_indices_from(A)] *= 1.0 + lam
        d = np.diag(A)
        try:
            Lc = np.linalg.cholesky(A)
        except np.linalg.LinAlgError:
            status = DEGENERATE
            break
        if np.min(np.diag(Lc)) ** 2 <= 1e-12 * np.max(d):
            status = DEGENERATE
            break
        delta = -np.linalg.solve(Lc.T, np.linalg.solve(Lc, g))
        Pn = [P[0]] + [exp_se3(delta[6 * (k - 1):6 * k]) @ P[k] for k in range(1, len(P))]
        Hn, gn, Fn = normal_equations(Pn, edges)
        if method == "lm" and not Fn < F:
            lam *= 10.0
            refusals += 1
            if refusals >= 10:
                status = CONVERGED
                break
            continue
        refusals = 0
        if method == "lm":
            lam /= 10.0
        steps += 1
        done = abs(F - Fn) <= rel_tol * F
        P, H, g, F = Pn, Hn, gn, Fn
        if done:
            status = CONVERGED
            break
    return P, F0, F, steps, status
