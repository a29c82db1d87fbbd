"""Pins of the RANSAC oracle, each against something outside it:

X1 its Philox4x64-10 equals numpy's Philox bit generator (an independent
implementation of the published generator) on random keys and counters;
X2 the sample indices equal the multiply-shift map of numpy's Philox stream;
X3 feature matching on small-integer features (float32 exact) equals the exact
integer argmin with ties to the smallest index, and on random features the
float64 argmin wherever the float64 gap is clear;
X4 the rigid fit recovers exact transforms, agrees with scipy's
Rotation.align_vectors on noisy data, and never returns a reflection;
X5 the edge-length checker's boundary (non-strict, squared lengths) on
power-of-two edges, congruent samples pass, scaled ones fail;
X6 the distance checker passes an exact sample and rejects one moved pair;
X7 validation: identical clouds score (n, 0); brute force and k-d tree agree;
the score is invariant under permutations of the source;
X8 exact correspondences give the true transform and full count; with 75%
wrong matches the transform is still recovered; X9 the stopping rules;
X10 the result does not depend on the chunking of the hypotheses.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import ransac as R


def test_x1_philox_matches_numpy():
    rng = np.random.default_rng(1)
    for _ in range(50):
        key = rng.integers(0, 2**63, 2, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, 2, dtype=np.uint64)
        ctr = rng.integers(0, 2**63, 4, dtype=np.uint64)
        ctr[0] = max(ctr[0], np.uint64(1))
        prev = ctr.copy()
        prev[0] -= np.uint64(1)  # numpy advances the counter before each block
        bg = np.random.Philox(key=key, counter=prev)
        np.testing.assert_array_equal(R.philox4x64(ctr[None], key)[0], bg.random_raw(4))


def test_x2_sample_indices_from_numpy_stream():
    seed, n = 12345, 7919
    hs = np.array([1, 2, 3, 1000, 2**40 + 7], np.int64)
    for ransac_n in (3, 4, 6):
        got = R.sample_indices(seed, hs, ransac_n, n)
        for row, h in zip(got, hs):
            want = []
            for b in range((ransac_n + 3) // 4):
                bg = np.random.Philox(key=np.array([seed, 0], np.uint64),
                                      counter=np.array([h - 1, b, 0, 0], np.uint64))
                want += [(int(z) >> 32) * n >> 32 for z in bg.random_raw(4)]
            assert list(row) == want[:ransac_n]
            assert all(0 <= x < n for x in row)
    # uniform over [0, n): chi-square over 10 bins of 40k draws
    d = R.sample_indices(7, np.arange(10_000), 4, 1000).ravel()
    c = np.bincount(d // 100, minlength=10)
    assert ((c - 4000) ** 2 / 4000).sum() < 30


def test_x3_feature_match_exact_and_float64():
    rng = np.random.default_rng(3)
    fs = rng.integers(0, 8, (300, 33)).astype(np.float32)
    ft = rng.integers(0, 8, (500, 33)).astype(np.float32)
    ft[250:] = ft[:250]  # duplicates: ties resolve to the smaller index
    idx, dmin = R.feature_match(fs, ft)
    D = ((fs[:, None, :].astype(np.int64) - ft[None].astype(np.int64)) ** 2).sum(axis=2)
    np.testing.assert_array_equal(idx, np.argmin(D, axis=1))
    np.testing.assert_array_equal(dmin, D.min(axis=1).astype(np.float32))
    assert np.all(idx < 250)
    fs = rng.random((200, 33)).astype(np.float32) * 100
    ft = rng.random((400, 33)).astype(np.float32) * 100
    idx, _ = R.feature_match(fs, ft)
    D = ((fs[:, None, :].astype(np.float64) - ft[None].astype(np.float64)) ** 2).sum(axis=2)
    Ds = np.sort(D, axis=1)
    clear = Ds[:, 1] - Ds[:, 0] > 1e-4 * Ds[:, 0]
    assert clear.mean() > 0.9
    np.testing.assert_array_equal(idx[clear], np.argmin(D, axis=1)[clear])
    e_idx, e_d = R.feature_match(fs[:0], ft)
    assert len(e_idx) == 0
    e_idx, _ = R.feature_match(fs[:3], ft[:0])
    assert list(e_idx) == [-1, -1, -1]


def _rand_T(rng, ang=math.pi, trans=2.0):
    T = np.eye(4)
    T[:3, :3] = Rotation.from_rotvec(rng.normal(size=3) / 2 * ang / 2).as_matrix()
    T[:3, 3] = rng.normal(size=3) * trans
    return T


def test_x4_rigid_fit():
    rng = np.random.default_rng(4)
    for n in (3, 4, 8):
        Ts = np.array([_rand_T(rng) for _ in range(30)])
        S = rng.normal(size=(30, n, 3))
        P = np.einsum("kij,knj->kni", Ts[:, :3, :3], S) + Ts[:, None, :3, 3]
        np.testing.assert_allclose(R.rigid_fit(S, P), Ts, atol=1e-11)
    S = rng.normal(size=(20, 6, 3))
    P = S @ Rotation.random(random_state=5).as_matrix().T + rng.normal(size=(20, 6, 3)) * 0.05
    Tf = R.rigid_fit(S, P)
    for k in range(20):
        a = P[k] - P[k].mean(axis=0)
        b = S[k] - S[k].mean(axis=0)
        rot, _ = Rotation.align_vectors(a, b)
        np.testing.assert_allclose(Tf[k, :3, :3], rot.as_matrix(), atol=1e-10)
    # mirrored planar-ish data: the best orthogonal map is a reflection
    S = rng.normal(size=(10, 5, 3))
    P = S * np.array([1.0, 1.0, -1.0]) + rng.normal(size=(10, 5, 3)) * 0.01
    dets = np.linalg.det(R.rigid_fit(S, P)[:, :3, :3])
    np.testing.assert_allclose(dets, 1.0, atol=1e-12)


def test_x5_edge_length_boundary():
    S = np.array([[[0, 0, 0], [1, 0, 0], [0, 2, 0]]], np.float32)
    P = S * np.float32(0.5)  # every edge ratio exactly 0.5
    assert R.edge_length_ok(S, P, 0.5)[0]
    assert not R.edge_length_ok(S, P, 0.5000001)[0]
    assert R.edge_length_ok(S, P, 0.0)[0]  # disabled
    rng = np.random.default_rng(5)
    S = rng.normal(size=(40, 4, 3)).astype(np.float32)
    Rm = Rotation.random(40, random_state=6).as_matrix()
    P = (np.einsum("kij,knj->kni", Rm, S) + 3.0).astype(np.float32)
    assert R.edge_length_ok(S, P, 0.9).all()
    assert not R.edge_length_ok(S, (P * 1.2).astype(np.float32), 0.9).any()
    assert R.edge_length_ok(S, (P * 1.2).astype(np.float32), 0.8).all()


def test_x6_distance_checker():
    rng = np.random.default_rng(6)
    T = _rand_T(rng)[None]
    S = rng.normal(size=(1, 4, 3)).astype(np.float32)
    P = np.einsum("ij,nj->ni", T[0, :3, :3], S[0]) + T[0, :3, 3]
    e2 = R.distance_residuals(T, S, P[None].astype(np.float32))
    assert e2.max() < 1e-12
    P2 = P.copy()
    P2[2, 0] += 0.1
    e2 = R.distance_residuals(T, S, P2[None].astype(np.float32))
    assert e2[0, 2] > 0.0099 and np.delete(e2[0], 2).max() < 1e-12


def test_x7_validation_score():
    rng = np.random.default_rng(7)
    pts = rng.random((800, 3)).astype(np.float32)
    cnt, sq = R.validate(pts, pts, np.eye(4), 0.05)
    assert (cnt, sq) == (800, 0)
    T = _rand_T(rng, 0.05, 0.01)
    src = rng.random((700, 3)).astype(np.float32)
    a = R.validate(src, pts, T, 0.06, search=1)
    b = R.validate(src, pts, T, 0.06, search=2)
    assert a == b and 0 < a[0] < 700
    perm = rng.permutation(700)
    assert R.validate(src[perm], pts, T, 0.06, search=1) == a
    # score quantum: sumq counts 2^-S units with fl32(r^2) < 2^(40 - S)
    S = R.score_shift(0.06)
    assert np.float32(0.06 * 0.06) < 2.0 ** (40 - S) <= 2 * np.float32(0.06 * 0.06)


def _matched_case(rng, n=600, wrong=0.0):
    src = rng.random((n, 3)).astype(np.float32) * 2
    T = _rand_T(rng)
    tgt = (src.astype(np.float64) @ T[:3, :3].T + T[:3, 3]).astype(np.float32)
    perm = rng.permutation(n)
    tgt = tgt[perm]
    corr = np.argsort(perm)  # tgt[corr[i]] is the image of src[i]
    bad = rng.random(n) < wrong
    corr = np.where(bad, rng.integers(0, n, n), corr)
    return src, tgt, corr, T


def test_x8_recovers_transform():
    rng = np.random.default_rng(8)
    src, tgt, corr, T = _matched_case(rng)
    res = R.ransac(src, tgt, corr, 0.05, 4, 0.9, None, 1000, 20, seed=3)
    assert res["status"] == R.OK and res["count"] == 600 and res["n_validated"] == 20
    np.testing.assert_allclose(res["T"], T, atol=1e-5)
    src, tgt, corr, T = _matched_case(rng, wrong=0.75)
    res = R.ransac(src, tgt, corr, 0.05, 4, 0.9, None, 200_000, 50, seed=4)
    assert res["count"] == 600 and res["n_validated"] == 50
    np.testing.assert_allclose(res["T"], T, atol=1e-5)
    # the best score is the lexicographic minimum of (-count, sumq, h)
    k = np.lexsort((res["trace_h"], res["trace_sumq"], -res["trace_count"]))[0]
    assert res["best_h"] == res["trace_h"][k]


def test_x9_stopping_rules():
    rng = np.random.default_rng(9)
    src, tgt, corr, T = _matched_case(rng, wrong=0.5)
    res = R.ransac(src, tgt, corr, 0.05, 4, 0.9, None, 100_000, 7, seed=1)
    assert res["n_validated"] == 7 and res["n_iterations"] == res["trace_h"][-1] + 1
    res2 = R.ransac(src, tgt, corr, 0.05, 4, 0.9, None, int(res["trace_h"][3]), 7, seed=1)
    assert res2["n_validated"] == 3 and res2["n_iterations"] == res["trace_h"][3]
    none = R.ransac(src, tgt, np.full(len(src), -1), 0.05, 4, 0.9, None, 500, 7, seed=1)
    assert none["status"] == R.NO_HYPOTHESIS and none["n_validated"] == 0 and none["n_iterations"] == 500
    np.testing.assert_array_equal(none["T"], np.eye(4))


def test_x10_chunking_invariance():
    rng = np.random.default_rng(10)
    src, tgt, corr, T = _matched_case(rng, wrong=0.6)
    a = R.ransac(src, tgt, corr, 0.05, 4, 0.9, 0.05, 50_000, 25, seed=9)
    b = R.ransac(src, tgt, corr, 0.05, 4, 0.9, 0.05, 50_000, 25, seed=9, chunk=37)
    for k in ("trace_h", "trace_count", "trace_sumq", "trace_T"):
        np.testing.assert_array_equal(a[k], b[k])
    assert a["best_h"] == b["best_h"] and a["n_iterations"] == b["n_iterations"]
