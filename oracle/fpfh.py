"""FPFH descriptor oracle, plain numpy FP64 plus the ICP oracle's hybrid
neighbourhood search.

TEST INFRASTRUCTURE ONLY: imported by the test-suite and the benchmark's
CPU-baseline leg, never by the GPU library or its binding; it shares no code
with the GPU path.

What it computes (paper: Sec. 3.3, `compute_fpfh_feature` with a hybrid
(radius, max_nn) neighbourhood ahead of RANSAC; the descriptor is the Fast
Point Feature Histogram of [17], Rusu, Blodow and Beetz, ICRA 2009).  The
reading:

  * the neighbourhood of point i is the hybrid selection of the normal
    estimation (the max_nn smallest (pinned float32 squared distance, index)
    within radius, i included); a neighbour j != i at zero distance is
    skipped;
  * pair (i, j), in FP64 from the float32 inputs: delta = p_j - p_i,
    d = |delta|; the source s is the end whose normal makes the smaller angle
    with the line to the other end: s = i iff n_i . delta >= -(n_j . delta),
    else s = j with the line reversed; e = line / d; Darboux frame u = n_s,
    v = (u x e) / |u x e| (pair skipped if |u x e| = 0), w = u x v;
    features alpha = v . n_t, phi = u . e, theta = atan2(w . n_t, u . n_t);
  * bins: floor((alpha + 1) 5.5), floor((phi + 1) 5.5),
    floor((theta + pi) (11 / (2 pi))), each clamped to [0, 10]; sub-histogram
    offsets 0, 11, 22 (33 bins);
  * SPFH(i) = counts c_i times q_i = 100 / k_i (k_i the pairs counted; 0 if
    none): each sub-histogram sums to 100;
  * FPFH(i) = SPFH(i) + (1 / k'_i) sum over neighbours j != i at non-zero
    distance w_ij of SPFH(j) / w_ij (neighbour order; k'_i their number;
    the sum term is 0 when k'_i = 0); rounded to float32 at the end.

Dot and cross products are evaluated left to right ((x + y) + z), without
FMA, so that another implementation doing the same operations reaches the
same bits; atan2 is the platform's, which may differ from another's by an
ulp, so `fpfh` also reports how close any feature came to a bin edge.
"""
from __future__ import annotations

import math

import numpy as np

import oracle

BINS = 11
THETA_SCALE = 11.0 / (2.0 * math.pi)


def _dot(a, b):
    return (a[..., 0] * b[..., 0] + a[..., 1] * b[..., 1]) + a[..., 2] * b[..., 2]


def _cross(a, b):
    return np.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                     a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                     a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], axis=-1)


def pair_features(pi, ni, pj, nj):
    """Features (alpha, phi, theta) of pairs (i, j) (arrays (m, 3), FP64) and
    a mask of the pairs that are defined (non-zero distance and frame)."""
    pi, ni, pj, nj = (np.asarray(a, np.float64) for a in (pi, ni, pj, nj))
    delta = pj - pi
    d = np.sqrt(_dot(delta, delta))
    fwd = _dot(ni, delta) >= -_dot(nj, delta)
    u = np.where(fwd[:, None], ni, nj)
    nt = np.where(fwd[:, None], nj, ni)
    line = np.where(fwd[:, None], delta, -delta)
    with np.errstate(invalid="ignore", divide="ignore"):
        e = line / d[:, None]
        c = _cross(u, e)
        cn = np.sqrt(_dot(c, c))
        v = c / cn[:, None]
        w = _cross(u, v)
        alpha = _dot(v, nt)
        phi = _dot(u, e)
        theta = np.arctan2(_dot(w, nt), _dot(u, nt))
    ok = (d > 0) & (cn > 0)
    return alpha, phi, theta, ok


def bin_positions(alpha, phi, theta):
    """Unclamped bin coordinates of the three features."""
    return (alpha + 1.0) * 5.5, (phi + 1.0) * 5.5, (theta + math.pi) * THETA_SCALE


def fpfh(pts, normals, radius, max_nn, search=0):
    """(n, 33) float32 descriptors, the SPFH counts (n, 33), pair counts k,
    neighbourhood sizes, and the smallest distance of any feature's bin
    coordinate to an interior bin edge."""
    pts = np.ascontiguousarray(pts, np.float32)
    P = pts.astype(np.float64)
    N = np.asarray(normals, np.float32).astype(np.float64)
    n = len(pts)
    nb, nn = oracle.hybrid_neighbors(pts, radius, max_nn, search)
    rows = np.arange(n)
    counts = np.zeros((n, 3 * BINS), np.int64)
    k = np.zeros(n, np.int64)
    margin = np.inf
    for slot in range(max_nn):
        j = nb[:, slot]
        sel = (j >= 0) & (j != rows)
        i, jj = rows[sel], j[sel]
        if len(i) == 0:
            continue
        a, f, t, ok = pair_features(P[i], N[i], P[jj], N[jj])
        i = i[ok]
        for off, x in zip((0, BINS, 2 * BINS), bin_positions(a[ok], f[ok], t[ok])):
            inner = (x > 0.5) & (x < BINS - 0.5)
            if inner.any():
                margin = min(margin, float(np.min(np.abs(x[inner] - np.round(x[inner])))))
            b = np.clip(np.floor(x), 0, BINS - 1).astype(np.int64)
            np.add.at(counts, (i, off + b), 1)
        np.add.at(k, i, 1)
    q = np.zeros(n)
    q[k > 0] = 100.0 / k[k > 0]
    S = counts * q[:, None]
    acc = np.zeros((n, 3 * BINS))
    kp = np.zeros(n, np.int64)
    for slot in range(max_nn):
        j = nb[:, slot]
        sel = (j >= 0) & (j != rows)
        delta = P[np.where(sel, j, 0)] - P
        w = np.sqrt(_dot(delta, delta))
        sel &= w > 0
        i = rows[sel]
        acc[i] = acc[i] + S[j[sel]] / w[sel][:, None]
        kp[i] += 1
    F = S.copy()
    m = kp > 0
    F[m] = S[m] + acc[m] / kp[m][:, None].astype(np.float64)
    return F.astype(np.float32), counts, k, nn, margin
