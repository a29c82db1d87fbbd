"""Vectorised brute-force ICP in numpy, for tiny inputs (N_src * N_tgt <= ~4e6).

TEST INFRASTRUCTURE ONLY: a second, independently written oracle used to
cross-check the C++ oracle (``oracle.cpp``).  It follows the same readings of
the paper (Open3D, Sec. 3.3 ICP refinement with a maximum correspondence
distance; Sec. 4 eqs. (1)-(2), Gauss-Newton on the sum of squared residuals)
but written with array operations instead of loops: all pairwise distances,
then a lexicographic (distance, index) minimum per row.
"""
from __future__ import annotations

import numpy as np


def transform64(T, s):
    """FP64 transform in the pinned order ((R0 sx + R1 sy) + R2 sz) + t; numpy
    evaluates each elementwise op separately (no fused multiply-add)."""
    T = np.asarray(T, np.float64)
    s = np.asarray(s, np.float32).astype(np.float64)
    q = np.empty_like(s)
    for a in range(3):
        q[:, a] = ((T[a, 0] * s[:, 0] + T[a, 1] * s[:, 1]) + T[a, 2] * s[:, 2]) + T[a, 3]
    return q


def select(q64, tgt, r, pinned=True):
    """Brute-force nearest target per query.  Returns (idx, d2_f32, d2_f64);
    idx = -1 when nothing lies within r (inclusive)."""
    tgt = np.asarray(tgt, np.float32)
    if pinned:
        q32 = q64.astype(np.float32)
        d = q32[:, None, :] - tgt[None, :, :]                     # float32
        D = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
        thr = np.float32(r * r)
    else:
        d = q64[:, None, :] - tgt.astype(np.float64)[None, :, :]
        D = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
        thr = r * r
    ok = D <= thr
    Dm = np.where(ok, D, np.inf)
    # np.argmin returns the first (smallest index) minimum: the tie-break.
    j = np.argmin(Dm, axis=1)
    has = ok[np.arange(len(q64)), j]
    idx = np.where(has, j, -1)
    d2f = np.full(len(q64), np.inf, np.float32)
    if pinned:
        d2f[has] = D[np.arange(len(q64)), j][has]
    p = tgt.astype(np.float64)[np.maximum(idx, 0)]
    d2d = ((q64 - p) ** 2).sum(axis=1)
    d2d[~has] = np.inf
    return idx, d2f, d2d


def hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def se3_exp(xi):
    """Matrix exponential of the twist (omega, v), closed form (Rodrigues)."""
    w, v = np.asarray(xi[:3], float), np.asarray(xi[3:], float)
    th = np.linalg.norm(w)
    W = hat(w)
    if th < 1e-4:
        a = 1.0 - th ** 2 / 6.0 + th ** 4 / 120.0
        b = 0.5 - th ** 2 / 24.0 + th ** 4 / 720.0
        c = 1.0 / 6.0 - th ** 2 / 120.0 + th ** 4 / 5040.0
    else:
        a, b, c = np.sin(th) / th, 2.0 * np.sin(th / 2) ** 2 / th ** 2, (th - np.sin(th)) / th ** 3
    E = np.eye(4)
    E[:3, :3] = np.eye(3) + a * W + b * (W @ W)
    E[:3, 3] = (np.eye(3) + b * W + c * (W @ W)) @ v
    return E


def jacobians(variant, q, p, n):
    """Stacked residual vector and Jacobian (rows x 6) of all inliers."""
    if variant in ("point_to_plane", 1):
        r = ((q - p) * n).sum(axis=1)
        J = np.concatenate([np.cross(q, n), n], axis=1)
        return r, J
    m = len(q)
    r = (q - p).reshape(-1)
    J = np.zeros((m, 3, 6))
    # d(q)/d(omega) = -[q]_x
    J[:, :, :3] = -np.stack([hat(qi) for qi in q])
    J[:, :, 3:] = np.eye(3)[None]
    return r, J.reshape(3 * m, 6)


def icp_register(src, tgt, tgt_normals, T_init, r, max_iter, rel_tol=0.0,
                 variant="point_to_plane", pinned=True):
    """Same loop and termination rules as the C++ oracle."""
    T = np.array(T_init, dtype=np.float64).reshape(4, 4)
    tgt64 = np.asarray(tgt, np.float32).astype(np.float64)
    nrm64 = None if tgt_normals is None else np.asarray(tgt_normals, np.float32).astype(np.float64)
    n_prev, e_prev = 0, 0.0
    k = 0
    while True:
        q = transform64(T, src)
        idx, _, d2d = select(q, tgt, r, pinned)
        inl = idx >= 0
        nk = int(inl.sum())
        fk = nk / len(src)
        ek = float(np.sqrt(d2d[inl].sum() / nk)) if nk > 0 else 0.0
        if nk == 0:
            return T, fk, ek, nk, k, 2
        if k == max_iter:
            return T, fk, ek, nk, k, 0
        if k >= 1 and abs(nk - n_prev) <= rel_tol * n_prev and abs(ek - e_prev) <= rel_tol * e_prev:
            return T, fk, ek, nk, k, 1
        qi = q[inl]
        pi = tgt64[idx[inl]]
        ni = nrm64[idx[inl]] if nrm64 is not None else np.zeros_like(pi)
        res, J = jacobians(variant, qi, pi, ni)
        A = J.T @ J
        b = J.T @ res
        dmax = np.max(np.diag(A))
        try:
            L = np.linalg.cholesky(A)
        except np.linalg.LinAlgError:
            return T, fk, ek, nk, k, 2
        if np.min(np.diag(L) ** 2) <= 1e-12 * dmax:
            return T, fk, ek, nk, k, 2
        xi = -np.linalg.solve(A, b)
        T = se3_exp(xi) @ T
        n_prev, e_prev = nk, ek
        k += 1
