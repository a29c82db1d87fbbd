"""RANSAC global registration oracle (feature matching, hypothesis checks,
validation), plain numpy FP64 plus the k-d tree correspondence search of the
ICP oracle.

TEST INFRASTRUCTURE ONLY: imported by the test-suite and the benchmark's
CPU-baseline leg, never by the GPU library or its binding; it shares no code
with the GPU path.

What it computes (paper: Sec. 3.3, the global-registration step of the
pairwise workflow: FPFH features of both downsampled clouds, then RANSAC on
feature matches [17] with a point-to-point transformation estimate, the
edge-length and distance correspondence checkers, and a convergence criterion
of (max_iteration, max_validation); the paper notes that validating a
hypothesis dominates the cost).  The paper names the steps only; the reading:

  * feature match: c(i) = the target index j minimising (D_ij, j), with
    D_ij the float32 squared feature distance accumulated over the dimensions
    in index order, each term fl32(fl32(a_k - b_k)^2), no FMA;
  * hypothesis h draws ransac_n source indices with the Philox4x64-10
    counter-based generator (Salmon et al., SC'11): block b of hypothesis h is
    Philox(counter = (h, b, 0, 0), key = (seed, 0)); draw k is word k % 4 of
    block k // 4, mapped to [0, n_src) by ((z >> 32) * n_src) >> 32;
  * a sample with a repeated source index, or a source without a match
    (c(i) < 0), is rejected;
  * edge-length checker (sigma): for every pair (a, b) of the sample,
    ds2 = |s_a - s_b|^2 and dt2 = |t_a - t_b|^2 (FP64, ((dx^2 + dy^2) + dz^2),
    t = target point of the match) must satisfy ds2 >= sigma^2 dt2 and
    dt2 >= sigma^2 ds2; sigma <= 0 disables it;
  * the rigid transform (no scale) minimising sum |R s + t - p|^2 over the
    sample (Kabsch: SVD of the cross-covariance, reflection removed);
  * distance checker (d): every sampled pair has |T s - t|^2 <= d^2 (FP64,
    the pinned transform order ((R0 sx + R1 sy) + R2 sz) + t); d <= 0
    disables it;
  * a hypothesis that passes is validated: every source point is matched to
    its nearest target point under T with the ICP selection rule (pinned
    float32 squared distance, inlier iff <= fl32(r^2)); its score is (count,
    sumq) with sumq = sum over inliers of floor(d2 * 2^S), S = 40 - e where
    fl32(r^2) = m 2^e, m in [0.5, 1) (an exact integer sum, so the score
    does not depend on summation order);
  * the loop stops after max_iteration hypotheses or at the max_validation-th
    validated one; the best hypothesis is the lexicographic minimum of
    (-count, sumq, h); fitness = count / n_src, rmse = sqrt(sumq 2^-S /
    count).
"""
from __future__ import annotations

import math

import numpy as np

import oracle

OK, NO_HYPOTHESIS = 0, 1
M32 = np.uint64(0xFFFFFFFF)

# Philox4x64 round multipliers and key increments (Salmon et al., SC'11)
PHILOX_M0 = np.uint64(0xD2E7470EE14C6C93)
PHILOX_M1 = np.uint64(0xCA5A826395121157)
PHILOX_W0 = np.uint64(0x9E3779B97F4A7C15)
PHILOX_W1 = np.uint64(0xBB67AE8584CAA73B)


def mulhilo64(a, b):
    """(high, low) 64-bit halves of the 128-bit products a * b (uint64 arrays)."""
    a = np.asarray(a, np.uint64)
    b = np.asarray(b, np.uint64)
    a_lo, a_hi = a & M32, a >> np.uint64(32)
    b_lo, b_hi = b & M32, b >> np.uint64(32)
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> np.uint64(32)) + (lh & M32) + (hl & M32)
    hi = hh + (lh >> np.uint64(32)) + (hl >> np.uint64(32)) + (mid >> np.uint64(32))
    lo = a * b  # wraps modulo 2^64
    return hi, lo


def philox4x64(ctr, key, rounds=10):
    """Philox4x64-R of counters ctr (N, 4) under key (2,): (N, 4) uint64."""
    x = np.array(ctr, np.uint64).reshape(-1, 4).copy()
    k0 = np.uint64(key[0])
    k1 = np.uint64(key[1])
    with np.errstate(over="ignore"):
        for r in range(rounds):
            if r > 0:
                k0 = k0 + PHILOX_W0
                k1 = k1 + PHILOX_W1
            hi0, lo0 = mulhilo64(PHILOX_M0, x[:, 0])
            hi1, lo1 = mulhilo64(PHILOX_M1, x[:, 2])
            x = np.stack([hi1 ^ x[:, 1] ^ k0, lo1, hi0 ^ x[:, 3] ^ k1, lo0], axis=1)
    return x


def sample_indices(seed, h, ransac_n, n_src):
    """Source indices drawn by hypotheses h (array): (len(h), ransac_n) int64."""
    h = np.asarray(h, np.uint64).reshape(-1)
    nb = (ransac_n + 3) // 4
    out = np.empty((len(h), ransac_n), np.int64)
    for b in range(nb):
        ctr = np.zeros((len(h), 4), np.uint64)
        ctr[:, 0] = h
        ctr[:, 1] = b
        z = philox4x64(ctr, (np.uint64(seed), np.uint64(0)))
        for w in range(4):
            k = 4 * b + w
            if k < ransac_n:
                out[:, k] = ((z[:, w] >> np.uint64(32)) * np.uint64(n_src)) >> np.uint64(32)
    return out


def feature_match(fs, ft, chunk=512):
    """c(i) = argmin_j (D_ij, j) over target features ft (float32 sequential
    squared distance), and the minimum D_i."""
    fs = np.ascontiguousarray(fs, np.float32)
    ft = np.ascontiguousarray(ft, np.float32)
    assert fs.ndim == 2 and ft.ndim == 2 and fs.shape[1] == ft.shape[1]
    n, dim = fs.shape
    idx = np.full(n, -1, np.int64)
    dmin = np.full(n, np.inf, np.float32)
    if len(ft) == 0:
        return idx, dmin
    for a in range(0, n, chunk):
        q = fs[a:a + chunk]
        D = np.zeros((len(q), len(ft)), np.float32)
        for k in range(dim):
            t = q[:, k:k + 1] - ft[None, :, k]
            D = D + t * t
        j = np.argmin(D, axis=1)  # first minimum: smallest index among equals
        idx[a:a + chunk] = j
        dmin[a:a + chunk] = D[np.arange(len(q)), j]
    return idx, dmin


def rigid_fit(S, P):
    """(k, n, 3) source and target samples -> (k, 4, 4) transforms minimising
    sum |R s + t - p|^2 (Kabsch / Umeyama without scale)."""
    S = np.asarray(S, np.float64)
    P = np.asarray(P, np.float64)
    cs, cp = S.mean(axis=1), P.mean(axis=1)
    H = np.einsum("kni,knj->kij", S - cs[:, None], P - cp[:, None])
    U, _, Vt = np.linalg.svd(H)
    V = np.transpose(Vt, (0, 2, 1))
    d = np.sign(np.linalg.det(V @ np.transpose(U, (0, 2, 1))))
    d[d == 0] = 1.0
    D = np.zeros((len(S), 3, 3))
    D[:, 0, 0] = 1.0
    D[:, 1, 1] = 1.0
    D[:, 2, 2] = d
    R = V @ D @ np.transpose(U, (0, 2, 1))
    T = np.zeros((len(S), 4, 4))
    T[:, :3, :3] = R
    T[:, :3, 3] = cp - np.einsum("kij,kj->ki", R, cs)
    T[:, 3, 3] = 1.0
    return T


def _sq(d):
    return (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]


def edge_length_ok(S, P, sigma):
    """Edge-length checker on (k, n, 3) samples (FP64 squared lengths)."""
    S = np.asarray(S, np.float32).astype(np.float64)
    P = np.asarray(P, np.float32).astype(np.float64)
    k, n, _ = S.shape
    ok = np.ones(k, bool)
    if not sigma > 0:
        return ok
    s2 = float(sigma) * float(sigma)
    for a in range(n):
        for b in range(a + 1, n):
            ds2 = _sq(S[:, a] - S[:, b])
            dt2 = _sq(P[:, a] - P[:, b])
            ok &= (ds2 >= s2 * dt2) & (dt2 >= s2 * ds2)
    return ok


def transform_pinned(T, S):
    """q = R s + t per (k, n, 3) sample in the pinned order, FP64, no FMA."""
    S = np.asarray(S, np.float32).astype(np.float64)
    q = np.empty(S.shape)
    for r in range(3):
        q[..., r] = ((T[:, None, r, 0] * S[..., 0] + T[:, None, r, 1] * S[..., 1])
                     + T[:, None, r, 2] * S[..., 2]) + T[:, None, r, 3]
    return q


def distance_residuals(T, S, P):
    """|T s - t|^2 per sampled pair (k, n), FP64."""
    return _sq(transform_pinned(T, S) - np.asarray(P, np.float32).astype(np.float64))


def score_shift(max_corr_dist):
    """S = 40 - e with fl32(r^2) = m 2^e, m in [0.5, 1)."""
    r2f = float(np.float32(float(max_corr_dist) * float(max_corr_dist)))
    return 40 - math.frexp(r2f)[1]


def validate(src, tgt, T, max_corr_dist, search=0):
    """Score (count, sumq) of transform T over every source point (search as
    in the ICP oracle: 0 automatic, 1 brute force, 2 k-d tree)."""
    idx, d2f, _ = oracle.correspondences(src, T, tgt, max_corr_dist, search=search)
    m = idx >= 0
    S = score_shift(max_corr_dist)
    q = np.floor(d2f[m].astype(np.float64) * 2.0 ** S).astype(np.uint64)
    return int(m.sum()), int(q.sum(dtype=np.uint64))


def hypotheses(src, tgt, corr, ransac_n=4, edge_sim=0.9, dist=0.075, max_iteration=100_000,
               max_validation=500, seed=0, chunk=8192):
    """The first max_validation hypotheses (in h order) that pass both
    checkers: (h list, (k, 4, 4) transforms, n_iterations, smallest relative
    margin of the distance checker's decisions)."""
    src = np.ascontiguousarray(src, np.float32)
    tgt = np.ascontiguousarray(tgt, np.float32)
    corr = np.asarray(corr, np.int64)
    n_src = len(src)
    d2 = float(dist) * float(dist)
    hs_out, Ts_out = [], []
    margin = np.inf
    h0 = 0
    while h0 < max_iteration and len(hs_out) < max_validation and n_src > 0:
        hs = np.arange(h0, min(h0 + chunk, max_iteration), dtype=np.int64)
        I = sample_indices(seed, hs, ransac_n, n_src)
        ok = np.ones(len(hs), bool)
        srt = np.sort(I, axis=1)
        ok &= np.all(srt[:, 1:] != srt[:, :-1], axis=1)
        C = corr[I]
        ok &= np.all(C >= 0, axis=1)
        S, P = src[I], tgt[np.where(C >= 0, C, 0)]
        ok &= edge_length_ok(S, P, edge_sim)
        cand = np.nonzero(ok)[0]
        Ts = rigid_fit(S[cand], P[cand]) if len(cand) else np.zeros((0, 4, 4))
        if dist > 0 and len(cand):
            e2 = distance_residuals(Ts, S[cand], P[cand])
            margin = min(margin, float(np.min(np.abs(e2 - d2) / d2)))
            keep = np.all(e2 <= d2, axis=1)
        else:
            keep = np.ones(len(cand), bool)
        for c, T in zip(cand[keep], Ts[keep]):
            hs_out.append(int(hs[c]))
            Ts_out.append(T)
            if len(hs_out) == max_validation:
                break
        h0 += len(hs)
    n_iter = hs_out[-1] + 1 if len(hs_out) == max_validation else (max_iteration if n_src > 0 else 0)
    return np.array(hs_out, np.int64), np.array(Ts_out).reshape(-1, 4, 4), n_iter, margin


def ransac(src, tgt, corr, max_corr_dist, ransac_n=4, edge_sim=0.9, dist=None,
           max_iteration=100_000, max_validation=500, seed=0, chunk=8192):
    """RANSAC on putative correspondences corr (source i -> target corr[i]).

    dist defaults to max_corr_dist.  Returns a dict with T, fitness, rmse,
    count, sumq, best_h, n_iterations, n_validated, status and the trace of
    validated hypotheses (h, T, count, sumq) in order, plus the smallest
    relative margin of the distance checker's decisions (for judging how
    close a comparison with another implementation's fit may come)."""
    d = max_corr_dist if dist is None else dist
    hs, Ts, n_iter, margin = hypotheses(src, tgt, corr, ransac_n, edge_sim, d, max_iteration,
                                        max_validation, seed, chunk)
    counts, sums = [], []
    best = None
    for h, T in zip(hs, Ts):
        cnt, sq = validate(src, tgt, T, max_corr_dist)
        counts.append(cnt)
        sums.append(sq)
        key = (-cnt, sq, int(h))
        if best is None or key < best[0]:
            best = (key, T)
    S = score_shift(max_corr_dist)
    res = {"n_iterations": n_iter, "n_validated": len(hs), "trace_h": hs, "trace_T": Ts,
           "trace_count": np.array(counts, np.int64), "trace_sumq": np.array(sums, np.uint64),
           "min_distance_margin": margin, "shift": S}
    if best is None:
        res.update(T=np.eye(4), fitness=0.0, rmse=0.0, count=0, sumq=0, best_h=-1, status=NO_HYPOTHESIS)
    else:
        (negc, sq, h), T = best
        cnt = -negc
        res.update(T=T, fitness=cnt / len(src), rmse=math.sqrt(sq * 2.0 ** -S / cnt) if cnt else 0.0,
                   count=cnt, sumq=sq, best_h=h, status=OK)
    return res
