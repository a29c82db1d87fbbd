"""ctypes loader for the FP64 ICP oracle (``oracle.cpp``) and its build step.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library or its Python binding.
The oracle shares no code with the GPU path.  Functions mirror the GPU
library's entry points (same argument order) plus a ``selection`` mode and a
``search`` mode (0 automatic, 1 brute force, 2 k-d tree).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

SEL_PINNED_F32 = 0
SEL_F64 = 1
POINT_TO_POINT = 0
POINT_TO_PLANE = 1
STATUS_OK, STATUS_CONVERGED, STATUS_DEGENERATE = 0, 1, 2
_VARIANTS = {"point_to_point": 0, "point_to_plane": 1, 0: 0, 1: 1}


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile ``oracle.cpp`` into ``liboracle.so`` next to it (g++, FP64, no FMA
    contraction).  sanitize: clang++ with AddressSanitizer and
    UndefinedBehaviorSanitizer (the runtime must be preloaded; CPU test runs)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        if sanitize:
            cmd = ["/opt/rocm/llvm/bin/clang++", "-std=c++17", "-O1", "-g", "-ffp-contract=off", "-fopenmp",
                   "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                   "-shared-libsan", "-shared", "-fPIC", "-o", tmp, _SRC,
                   "-Wl,-rpath,/opt/rocm/llvm/lib"]
        else:
            cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math",
                   "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        L.oracle_num_threads.restype = C.c_int
        L.oracle_set_num_threads.argtypes = [C.c_int]
        L.oracle_pinned_d2.argtypes = [_f64p, _f32p, _f32p, C.c_int64, _f32p]
        L.oracle_transform64.argtypes = [_f64p, _f32p, C.c_int64, _f64p]
        L.oracle_se3_exp.argtypes = [_f64p, _f64p]
        L.oracle_residual_jacobian.argtypes = [C.c_int, _f64p, _f64p, _f64p, _f64p, _f64p]
        L.oracle_residual_jacobian.restype = C.c_int
        L.oracle_solve6.argtypes = [_f64p, _f64p, _f64p]
        L.oracle_estimate_normals.argtypes = [_f32p, C.c_int64, C.c_double, C.c_int, _f64p, C.c_int,
                                              C.c_void_p, C.c_int64, _f32p,
                                              np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS"),
                                              C.c_void_p]
        L.oracle_estimate_normals.restype = C.c_int
        L.oracle_sym_eig3.argtypes = [_f64p, _f64p, _f64p]
        L.oracle_sym_eig3.restype = None
        L.oracle_solve6.restype = C.c_int
        L.oracle_correspondences.argtypes = [_f32p, C.c_int64, _f64p, _f32p, C.c_int64, C.c_double,
                                             C.c_int, C.c_int, _i64p, _f32p, _f64p]
        L.oracle_correspondences.restype = C.c_int
        L.oracle_normal_equations.argtypes = [_f32p, C.c_int64, _f64p, _f32p, C.c_void_p, C.c_int64,
                                              C.c_double, C.c_int, C.c_int, C.c_int, _f64p, _f64p,
                                              C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.oracle_normal_equations.restype = C.c_int
        L.oracle_icp_register.argtypes = [
            _f32p, C.c_int64, _f32p, C.c_void_p, C.c_int64, _f64p, C.c_double, C.c_int32,
            C.c_double, C.c_int, C.c_int, C.c_int, _f64p, C.POINTER(C.c_double),
            C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int32),
            C.POINTER(C.c_int32), C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_icp_register.restype = C.c_int
        L.oracle_normal_equations_robust.argtypes = [
            _f32p, C.c_int64, _f64p, _f32p, C.c_void_p, C.c_int64, C.c_double, C.c_int, C.c_int,
            C.c_int, C.c_int, C.c_double, _f64p, _f64p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.oracle_normal_equations_robust.restype = C.c_int
        L.oracle_icp_register_robust.argtypes = [
            _f32p, C.c_int64, _f32p, C.c_void_p, C.c_int64, _f64p, C.c_double, C.c_int32,
            C.c_double, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, _f64p,
            C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int64),
            C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_icp_register_robust.restype = C.c_int
        L.oracle_loss_weight.argtypes = [C.c_int, C.c_double, C.c_double]
        L.oracle_loss_weight.restype = C.c_double
        L.oracle_voxel_downsample.argtypes = [_f32p, C.c_void_p, C.c_int64, C.c_double, _f32p,
                                              C.c_void_p]
        L.oracle_voxel_downsample.restype = C.c_int64
        L.oracle_hybrid_neighbors.argtypes = [_f32p, C.c_int64, C.c_double, C.c_int, C.c_int,
                                              C.c_void_p, C.c_void_p]
        L.oracle_hybrid_neighbors.restype = C.c_int
        _lib = L
    return _lib


def _pts(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float32)
    assert a.ndim == 2 and a.shape[1] == 3
    return a


def _T(T) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(T, dtype=np.float64).reshape(16))


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_num_threads(n: int) -> None:
    lib().oracle_set_num_threads(int(n))


def pinned_d2(T, s, p) -> np.ndarray:
    s, p = _pts(s), _pts(p)
    out = np.empty(len(s), np.float32)
    lib().oracle_pinned_d2(_T(T), s, p, len(s), out)
    return out


def transform64(T, s) -> np.ndarray:
    s = _pts(s)
    out = np.empty((len(s), 3), np.float64)
    lib().oracle_transform64(_T(T), s, len(s), out)
    return out


def se3_exp(xi) -> np.ndarray:
    E = np.empty(16, np.float64)
    lib().oracle_se3_exp(np.ascontiguousarray(xi, dtype=np.float64), E)
    return E.reshape(4, 4)


def residual_jacobian(variant, q, p, n):
    res = np.zeros(3, np.float64)
    J = np.zeros(18, np.float64)
    f = lambda v: np.ascontiguousarray(v, dtype=np.float64)
    rows = lib().oracle_residual_jacobian(_VARIANTS[variant], f(q), f(p), f(n), res, J)
    return res[:rows], J[:6 * rows].reshape(rows, 6)


def solve6(A21, b6):
    xi = np.zeros(6, np.float64)
    rc = lib().oracle_solve6(np.ascontiguousarray(A21, dtype=np.float64),
                             np.ascontiguousarray(b6, dtype=np.float64), xi)
    return (xi if rc == 0 else None)


def correspondences(src, T, tgt, max_corr_dist, selection=SEL_PINNED_F32, search=0):
    """Returns (idx int64, d2 pinned float32, d2 float64) per source point."""
    src, tgt = _pts(src), _pts(tgt)
    n = len(src)
    idx = np.empty(n, np.int64)
    d2f = np.empty(n, np.float32)
    d2d = np.empty(n, np.float64)
    rc = lib().oracle_correspondences(src, n, _T(T), tgt, len(tgt), float(max_corr_dist),
                                      selection, search, idx, d2f, d2d)
    if rc != 0:
        raise ValueError("oracle_correspondences: invalid arguments")
    return idx, d2f, d2d


LOSSES = {"none": 0, "huber": 1, "tukey": 2, "cauchy": 3}


def loss_weight(loss, k, s):
    """IRLS weight rho'(s) / s of a robust loss at residual magnitude s."""
    return lib().oracle_loss_weight(LOSSES[loss], float(k), float(s))


def normal_equations(src, T, tgt, tgt_normals, max_corr_dist, variant="point_to_plane",
                     selection=SEL_PINNED_F32, search=0, loss="none", loss_k=1.0):
    """Returns (A21, b6, sum_d2, n_in); with a robust loss the terms carry the
    IRLS weight of each correspondence."""
    src, tgt = _pts(src), _pts(tgt)
    nrm = _pts(tgt_normals) if tgt_normals is not None else None
    A21 = np.zeros(21, np.float64)
    b6 = np.zeros(6, np.float64)
    sd2 = C.c_double()
    nin = C.c_int64()
    rc = lib().oracle_normal_equations_robust(src, len(src), _T(T), tgt,
                                              nrm.ctypes.data if nrm is not None else None, len(tgt),
                                              float(max_corr_dist), _VARIANTS[variant], selection,
                                              search, LOSSES[loss], float(loss_k), A21, b6,
                                              C.byref(sd2), C.byref(nin))
    if rc != 0:
        raise ValueError("oracle_normal_equations: invalid arguments")
    return A21, b6, sd2.value, nin.value


def voxel_downsample(pts, voxel, normals=None):
    """(points, normals or None) of the voxel means, in voxel-key order."""
    pts = _pts(pts)
    nrm = _pts(normals) if normals is not None else None
    out = np.empty_like(pts)
    outn = np.empty_like(pts) if nrm is not None else None
    m = lib().oracle_voxel_downsample(pts, nrm.ctypes.data if nrm is not None else None, len(pts),
                                      float(voxel), out, outn.ctypes.data if outn is not None else None)
    if m < 0:
        raise ValueError("oracle_voxel_downsample: invalid arguments")
    return out[:m].copy(), (outn[:m].copy() if outn is not None else None)


def estimate_normals(pts, radius, max_nn, viewpoint=(0.0, 0.0, 0.0), search=0, queries=None,
                     with_evals=False):
    """(normals float32 (q, 3), neighbourhood sizes int32 (q,)[, eigenvalues
    float64 (q, 3) ascending]) with the hybrid neighbourhood: the max_nn
    nearest points within radius by (pinned FP32 squared distance, index);
    fewer than 3 neighbours give a zero normal; normals face the viewpoint.
    queries: original indices to evaluate (default: all points)."""
    pts = _pts(pts)
    q = None if queries is None else np.ascontiguousarray(queries, np.int64)
    nq = len(pts) if q is None else len(q)
    out = np.empty((nq, 3), np.float32)
    cnt = np.empty(nq, np.int32)
    ev = np.empty((nq, 3), np.float64) if with_evals else None
    rc = lib().oracle_estimate_normals(pts, len(pts), float(radius), int(max_nn),
                                       np.ascontiguousarray(viewpoint, np.float64), int(search),
                                       q.ctypes.data if q is not None else None, nq, out, cnt,
                                       ev.ctypes.data if ev is not None else None)
    if rc != 0:
        raise ValueError("oracle_estimate_normals: invalid arguments")
    return (out, cnt, ev) if with_evals else (out, cnt)


def hybrid_neighbors(pts, radius, max_nn, search=0):
    """(n, max_nn) int64 neighbour lists (sorted by (pinned distance, index),
    -1 padded, the point itself included) and their lengths."""
    pts = _pts(pts)
    n = len(pts)
    idx = np.empty((n, max_nn), np.int64)
    cnt = np.empty(n, np.int32)
    if lib().oracle_hybrid_neighbors(pts, n, float(radius), int(max_nn), int(search), idx.ctypes.data,
                                     cnt.ctypes.data) != 0:
        raise ValueError("oracle_hybrid_neighbors: invalid arguments")
    return idx, cnt


def sym_eig3(A):
    """Eigenvalues (ascending) and eigenvectors (columns) of a symmetric 3x3."""
    A = np.asarray(A, np.float64)
    a6 = np.array([A[0, 0], A[0, 1], A[0, 2], A[1, 1], A[1, 2], A[2, 2]], np.float64)
    w = np.zeros(3)
    V = np.zeros(9)
    lib().oracle_sym_eig3(a6, w, V)
    return w, V.reshape(3, 3)


def register_multiscale(src, tgt, tgt_normals, T_init, voxels, iters, dists, rel_tol=0.0,
                        variant="point_to_plane", selection=SEL_PINNED_F32):
    """Coarse-to-fine: per level, downsample both clouds (voxel 0: keep) and
    register from the previous level's pose; stops at a degenerate level."""
    T = np.asarray(T_init, np.float64).reshape(4, 4)
    total = 0
    res = None
    for v, k, r in zip(voxels, iters, dists):
        if v > 0:
            s, _ = voxel_downsample(src, v)
            t, tn = voxel_downsample(tgt, v, tgt_normals if variant in ("point_to_plane", 1) else None)
        else:
            s, t, tn = src, tgt, tgt_normals
        res = icp_register(s, t, tn, T, r, k, rel_tol, variant, selection)
        total += res.n_iter
        T = res.T
        if res.status == STATUS_DEGENERATE:
            break
    res.n_iter = total
    return res


@dataclass
class OracleResult:
    T: np.ndarray
    fitness: float
    inlier_rmse: float
    n_inliers: int
    n_iter: int
    status: int
    traj_T: np.ndarray | None = None
    traj_n: np.ndarray | None = None
    traj_rmse: np.ndarray | None = None


def icp_register(src, tgt, tgt_normals, T_init, max_corr_dist, max_iter, rel_tol=0.0,
                 variant="point_to_plane", selection=SEL_PINNED_F32, search=0,
                 trajectory=False, loss="none", loss_k=1.0) -> OracleResult:
    src, tgt = _pts(src), _pts(tgt)
    nrm = _pts(tgt_normals) if tgt_normals is not None else None
    T = np.zeros(16, np.float64)
    fit, rmse = C.c_double(), C.c_double()
    nin = C.c_int64()
    nit, st = C.c_int32(), C.c_int32()
    tT = tn = tr = None
    if trajectory:
        tT = np.zeros((max_iter + 1, 16), np.float64)
        tn = np.zeros(max_iter + 1, np.int64)
        tr = np.zeros(max_iter + 1, np.float64)
    rc = lib().oracle_icp_register_robust(
        src, len(src), tgt, nrm.ctypes.data if nrm is not None else None, len(tgt), _T(T_init),
        float(max_corr_dist), int(max_iter), float(rel_tol), _VARIANTS[variant], selection, search,
        LOSSES[loss], float(loss_k), T, C.byref(fit), C.byref(rmse), C.byref(nin), C.byref(nit), C.byref(st),
        tT.ctypes.data if trajectory else None, tn.ctypes.data if trajectory else None,
        tr.ctypes.data if trajectory else None)
    if rc != 0:
        raise ValueError("oracle_icp_register: invalid arguments")
    res = OracleResult(T.reshape(4, 4), fit.value, rmse.value, nin.value, nit.value, st.value)
    if trajectory:
        k = nit.value + 1
        res.traj_T, res.traj_n, res.traj_rmse = tT[:k].reshape(k, 4, 4), tn[:k], tr[:k]
    return res
