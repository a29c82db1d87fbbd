"""Python binding of libicp.so (argument marshalling only).

Every computation runs in the HIP library; this module converts torch tensors
and numpy arrays into the pointers and sizes of the C ABI (include/icp.h) and
raises ``IcpError`` on a negative return code.  Functions named ``icp_*`` take
raw integers (device pointers) exactly like the C entry points; the friendlier
``register`` / ``correspondences`` / ``normal_equations`` accept CUDA tensors.

The library is loaded from this package directory.  If it is missing, import
succeeds but every call raises: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libicp.so")

ICP_SUCCESS = 0
ICP_E_INVALID_ARG = -1
ICP_E_NONFINITE = -2
ICP_E_TOO_LARGE = -3
ICP_E_OOM = -4
ICP_E_DEVICE = -5
ICP_E_CANCELLED = -6
ICP_E_NOT_FOUND = -7
ICP_OK, ICP_CONVERGED, ICP_DEGENERATE, ICP_RANSAC_NO_HYPOTHESIS = 0, 1, 2, 3
ICP_POINT_TO_POINT, ICP_POINT_TO_PLANE = 0, 1
ICP_PREC_F32_KAHAN_F64, ICP_PREC_F64 = 0, 1

VARIANTS = {"point_to_point": ICP_POINT_TO_POINT, "point_to_plane": ICP_POINT_TO_PLANE,
            ICP_POINT_TO_POINT: ICP_POINT_TO_POINT, ICP_POINT_TO_PLANE: ICP_POINT_TO_PLANE}
PRECISIONS = {"kahan32": ICP_PREC_F32_KAHAN_F64, "f32_kahan_f64": ICP_PREC_F32_KAHAN_F64,
              "f64": ICP_PREC_F64, ICP_PREC_F32_KAHAN_F64: ICP_PREC_F32_KAHAN_F64,
              ICP_PREC_F64: ICP_PREC_F64}
ICP_LOSS_NONE, ICP_LOSS_HUBER, ICP_LOSS_TUKEY, ICP_LOSS_CAUCHY = 0, 1, 2, 3
LOSSES = {"none": ICP_LOSS_NONE, "huber": ICP_LOSS_HUBER, "tukey": ICP_LOSS_TUKEY,
          "cauchy": ICP_LOSS_CAUCHY, 0: 0, 1: 1, 2: 2, 3: 3}


class IcpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class icp_pose_edge_t(C.Structure):
    _fields_ = [("i", C.c_int32), ("j", C.c_int32), ("Z", C.c_double * 16),
                ("information", C.c_double * 36)]


class icp_pose_graph_result_t(C.Structure):
    _fields_ = [("F_initial", C.c_double), ("F_final", C.c_double), ("steps", C.c_int32),
                ("status", C.c_int32)]


class icp_result_t(C.Structure):
    _fields_ = [("T", C.c_double * 16), ("fitness", C.c_double), ("inlier_rmse", C.c_double),
                ("n_inliers", C.c_int64), ("n_iter", C.c_int32), ("status", C.c_int32)]


class icp_pair_t(C.Structure):
    _fields_ = [("src_xyz", C.c_void_p), ("tgt_xyz", C.c_void_p), ("tgt_normals", C.c_void_p),
                ("n_src", C.c_int64), ("n_tgt", C.c_int64), ("T_init", C.c_double * 16),
                ("max_corr_dist", C.c_double), ("rel_tol", C.c_double), ("max_iter", C.c_int32),
                ("reserved", C.c_int32)]


class icp_server_cfg_t(C.Structure):
    _fields_ = [("device", C.c_int32), ("max_slots", C.c_int32), ("hbm_budget_bytes", C.c_uint64),
                ("n_levels", C.c_int32), ("iters", C.c_int32 * 4), ("voxel", C.c_double * 4),
                ("corr_dist", C.c_double * 4), ("corr_factor", C.c_double), ("variant", C.c_int32),
                ("precision", C.c_int32), ("iters_per_step", C.c_int32),
                ("background_thread", C.c_int32), ("loss", C.c_int32), ("loss_k", C.c_double)]


class icp_request_t(C.Structure):
    _fields_ = [("src_xyz", C.c_void_p), ("tgt_xyz", C.c_void_p), ("tgt_normals", C.c_void_p),
                ("n_src", C.c_int64), ("n_tgt", C.c_int64), ("T_init", C.c_double * 16),
                ("rel_tol", C.c_double), ("spacing", C.c_double), ("host_memory", C.c_int32),
                ("reserved", C.c_int32), ("user_tag", C.c_uint64), ("stream", C.c_void_p)]


class icp_completion_t(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("user_tag", C.c_uint64), ("result", icp_result_t),
                ("error", C.c_int32), ("reserved", C.c_int32), ("t_submit_ns", C.c_int64),
                ("t_admit_ns", C.c_int64), ("t_done_ns", C.c_int64)]


class icp_profile_t(C.Structure):
    _fields_ = [("pass_ms", C.c_double), ("pass_launches", C.c_int64), ("pass_points", C.c_int64),
                ("call_ms", C.c_double), ("calls", C.c_int64), ("validate_ms", C.c_double),
                ("validate_launches", C.c_int64), ("validate_evals", C.c_int64), ("build_ms", C.c_double),
                ("builds", C.c_int64), ("build_points", C.c_int64), ("hashed_grids", C.c_int64), ("fine_grids", C.c_int64)]


class icp_ransac_params_t(C.Structure):
    _fields_ = [("max_corr_dist", C.c_double), ("edge_length", C.c_double), ("distance", C.c_double),
                ("max_iteration", C.c_int64), ("max_validation", C.c_int32), ("ransac_n", C.c_int32),
                ("seed", C.c_uint64)]


class icp_ransac_result_t(C.Structure):
    _fields_ = [("T", C.c_double * 16), ("fitness", C.c_double), ("inlier_rmse", C.c_double),
                ("n_inliers", C.c_int64), ("sumq", C.c_uint64), ("shift", C.c_int32), ("status", C.c_int32),
                ("n_iterations", C.c_int64), ("n_validated", C.c_int64), ("best_hypothesis", C.c_int64)]


class icp_ransac_trace_t(C.Structure):
    _fields_ = [("h", C.c_void_p), ("T", C.c_void_p), ("count", C.c_void_p), ("sumq", C.c_void_p)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise IcpError(ICP_E_DEVICE, f"HIP library not built: {LIB_PATH} is missing "
                                         "(run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        L.icp_version.restype = C.c_char_p
        L.icp_strerror.restype = C.c_char_p
        L.icp_strerror.argtypes = [C.c_int]
        L.icp_last_error.restype = C.c_char_p
        L.icp_ctx_create.argtypes = [C.c_int, vp, C.c_size_t, C.POINTER(vp)]
        L.icp_ctx_destroy.argtypes = [vp]
        L.icp_register.argtypes = [vp, vp, i64, vp, vp, i64, vp, dbl, i32, dbl, i32, i32,
                                   C.POINTER(icp_result_t)]
        L.icp_correspondences.argtypes = [vp, vp, i64, vp, vp, i64, dbl, vp, vp]
        L.icp_normal_equations.argtypes = [vp, vp, i64, vp, vp, vp, i64, dbl, i32, i32, vp, vp,
                                           C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.icp_register_robust.argtypes = [vp, vp, i64, vp, vp, i64, vp, dbl, i32, dbl, i32, i32, i32,
                                          dbl, C.POINTER(icp_result_t)]
        L.icp_normal_equations_robust.argtypes = [vp, vp, i64, vp, vp, vp, i64, dbl, i32, i32, i32,
                                                  dbl, vp, vp, C.POINTER(C.c_double),
                                                  C.POINTER(C.c_int64)]
        L.icp_register_batch.argtypes = [vp, C.POINTER(icp_pair_t), i32, i32, i32,
                                         C.POINTER(icp_result_t)]
        L.icp_register_batch_robust.argtypes = [vp, C.POINTER(icp_pair_t), i32, i32, i32, i32, dbl,
                                                C.POINTER(icp_result_t)]
        L.icp_voxel_downsample.argtypes = [vp, vp, vp, i64, dbl, vp, vp, i64, C.POINTER(C.c_int64)]
        L.icp_register_multiscale.argtypes = [vp, vp, i64, vp, vp, i64, vp, i32, vp, vp, vp, dbl, i32,
                                              i32, C.POINTER(icp_result_t)]
        L.icp_register_multiscale_robust.argtypes = [vp, vp, i64, vp, vp, i64, vp, i32, vp, vp, vp, dbl, i32,
                                                     i32, i32, dbl, C.POINTER(icp_result_t)]
        L.icp_estimate_normals.argtypes = [vp, vp, i64, dbl, i32, vp, vp, vp]
        L.icp_pose_graph_optimize.argtypes = [vp, i32, vp, i32, C.POINTER(icp_pose_edge_t), i32, i32,
                                              dbl, C.POINTER(icp_pose_graph_result_t)]
        L.icp_compute_fpfh.argtypes = [vp, vp, vp, i64, dbl, i32, vp, vp]
        L.icp_feature_match.argtypes = [vp, vp, i64, vp, i64, i32, vp, vp]
        L.icp_feature_match_noalloc.argtypes = [vp, i64, vp, i64, i32, vp, vp, vp]
        L.icp_ransac_validate.argtypes = [vp, vp, i64, vp, i64, dbl, i32, vp, vp, vp]
        L.icp_ransac_register.argtypes = [vp, vp, i64, vp, i64, vp, C.POINTER(icp_ransac_params_t),
                                          C.POINTER(icp_ransac_result_t), C.POINTER(icp_ransac_trace_t)]
        L.icp_server_create.argtypes = [C.POINTER(icp_server_cfg_t), C.POINTER(vp)]
        L.icp_server_submit.argtypes = [vp, C.POINTER(icp_request_t), C.POINTER(C.c_uint64)]
        L.icp_server_step.argtypes = [vp, C.POINTER(C.c_int32)]
        L.icp_server_poll.argtypes = [vp, C.POINTER(icp_completion_t), i32, C.POINTER(C.c_int32)]
        L.icp_server_wait.argtypes = [vp, C.c_uint64, C.POINTER(icp_completion_t)]
        L.icp_server_destroy.argtypes = [vp]
        L.icp_measure_valu.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.icp_measure_copy.argtypes = [C.c_int, i64, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.icp_ctx_set_profiling.argtypes = [vp, C.c_int]
        L.icp_ctx_get_profile.argtypes = [vp, C.POINTER(icp_profile_t)]
        for name in ("icp_ctx_create", "icp_ctx_destroy", "icp_register", "icp_correspondences",
                     "icp_normal_equations", "icp_ctx_set_profiling", "icp_ctx_get_profile",
                     "icp_register_batch", "icp_register_batch_robust", "icp_voxel_downsample", "icp_register_multiscale", "icp_register_multiscale_robust",
                     "icp_estimate_normals", "icp_register_robust", "icp_normal_equations_robust",
                     "icp_pose_graph_optimize", "icp_feature_match", "icp_feature_match_noalloc", "icp_ransac_validate", "icp_compute_fpfh",
                     "icp_ransac_register",
                     "icp_server_create", "icp_server_submit", "icp_server_step", "icp_server_poll",
                     "icp_server_wait", "icp_server_destroy", "icp_measure_valu", "icp_measure_copy"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != ICP_SUCCESS:
        L = lib()
        raise IcpError(rc, f"{L.icp_strerror(rc).decode()}: {L.icp_last_error().decode()}")


def measure_valu(kind: int, device: int = 0) -> tuple[float, float]:
    """(lane operations per second, best launch ms) of icp_measure_valu."""
    rate, ms = C.c_double(), C.c_double()
    _check(lib().icp_measure_valu(int(device), int(kind), C.byref(rate), C.byref(ms)))
    return rate.value, ms.value


def measure_copy(nbytes: int, kind: int = 0, device: int = 0) -> tuple[float, float]:
    """(GB/s, best launch ms) of icp_measure_copy."""
    rate, ms = C.c_double(), C.c_double()
    _check(lib().icp_measure_copy(int(device), int(nbytes), int(kind), C.byref(rate), C.byref(ms)))
    return rate.value, ms.value


def _pose(T) -> np.ndarray:
    T = np.ascontiguousarray(np.asarray(T, dtype=np.float64).reshape(16))
    return T


# ---------------------------------------------------------------- raw entry points
def icp_version() -> str:
    return lib().icp_version().decode()


def icp_ctx_create(device: int, hip_stream: int | None, arena_bytes: int = 0) -> int:
    h = C.c_void_p()
    _check(lib().icp_ctx_create(int(device), hip_stream or None, int(arena_bytes), C.byref(h)))
    return h.value


def icp_ctx_destroy(ctx: int | None) -> None:
    _check(lib().icp_ctx_destroy(ctx))


def icp_register(ctx, src_ptr, n_src, tgt_ptr, tgt_n_ptr, n_tgt, T_init, max_corr_dist, max_iter,
                 rel_tol, variant, precision, loss=0, loss_k=1.0) -> icp_result_t:
    """icp_register, or icp_register_robust when loss is not ICP_LOSS_NONE."""
    out = icp_result_t()
    T = _pose(T_init)
    if loss == ICP_LOSS_NONE:
        _check(lib().icp_register(ctx, src_ptr, int(n_src), tgt_ptr, tgt_n_ptr, int(n_tgt),
                                  T.ctypes.data, float(max_corr_dist), int(max_iter), float(rel_tol),
                                  int(variant), int(precision), C.byref(out)))
    else:
        _check(lib().icp_register_robust(ctx, src_ptr, int(n_src), tgt_ptr, tgt_n_ptr, int(n_tgt),
                                         T.ctypes.data, float(max_corr_dist), int(max_iter),
                                         float(rel_tol), int(variant), int(precision), int(loss),
                                         float(loss_k), C.byref(out)))
    return out


def icp_register_batch(ctx, pairs, variant, precision, loss=ICP_LOSS_NONE, loss_k=1.0):
    """pairs: sequence of icp_pair_t; returns a list of icp_result_t."""
    n = len(pairs)
    arr = (icp_pair_t * n)(*pairs)
    out = (icp_result_t * n)()
    if loss == ICP_LOSS_NONE:
        _check(lib().icp_register_batch(ctx, arr, n, int(variant), int(precision), out))
    else:
        _check(lib().icp_register_batch_robust(ctx, arr, n, int(variant), int(precision), int(loss),
                                               float(loss_k), out))
    return list(out)


def icp_correspondences(ctx, src_ptr, n_src, T, tgt_ptr, n_tgt, max_corr_dist, idx_ptr, d2_ptr):
    T = _pose(T)
    _check(lib().icp_correspondences(ctx, src_ptr, int(n_src), T.ctypes.data, tgt_ptr, int(n_tgt),
                                     float(max_corr_dist), idx_ptr, d2_ptr))


def icp_normal_equations(ctx, src_ptr, n_src, T, tgt_ptr, tgt_n_ptr, n_tgt, max_corr_dist, variant,
                         precision, loss=0, loss_k=1.0):
    T = _pose(T)
    A = np.zeros(21, np.float64)
    b = np.zeros(6, np.float64)
    sd2 = C.c_double()
    nin = C.c_int64()
    if loss == ICP_LOSS_NONE:
        _check(lib().icp_normal_equations(ctx, src_ptr, int(n_src), T.ctypes.data, tgt_ptr, tgt_n_ptr,
                                          int(n_tgt), float(max_corr_dist), int(variant),
                                          int(precision), A.ctypes.data, b.ctypes.data, C.byref(sd2),
                                          C.byref(nin)))
    else:
        _check(lib().icp_normal_equations_robust(ctx, src_ptr, int(n_src), T.ctypes.data, tgt_ptr,
                                                 tgt_n_ptr, int(n_tgt), float(max_corr_dist),
                                                 int(variant), int(precision), int(loss),
                                                 float(loss_k), A.ctypes.data, b.ctypes.data,
                                                 C.byref(sd2), C.byref(nin)))
    return A, b, sd2.value, nin.value


# ---------------------------------------------------------------- tensor-level helpers
def _dev_pts(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise IcpError(ICP_E_INVALID_ARG, f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32 or t.dim() != 2 or t.shape[1] != 3 or not t.is_contiguous():
        raise IcpError(ICP_E_INVALID_ARG, f"{name} must be a contiguous (N, 3) float32 tensor")
    return t.data_ptr(), t.shape[0]


class Context:
    """Owns an icp_ctx_t bound to a device and a HIP stream (default: torch's
    current stream of that device); arena_bytes > 0 gives it one fixed device
    arena, from which every call carves its buffers without allocating."""

    def __init__(self, device: int = 0, stream=None, arena_bytes: int = 0):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.device = device
        self.stream = stream
        self.handle = icp_ctx_create(device, stream.cuda_stream if stream is not None else None, arena_bytes)

    def set_profiling(self, enable: bool) -> None:
        _check(lib().icp_ctx_set_profiling(self.handle, 1 if enable else 0))

    def profile(self) -> dict:
        p = icp_profile_t()
        _check(lib().icp_ctx_get_profile(self.handle, C.byref(p)))
        return {k: getattr(p, k) for k, _ in icp_profile_t._fields_}

    def close(self):
        if self.handle:
            icp_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class IcpResult:
    T: np.ndarray
    fitness: float
    inlier_rmse: float
    n_inliers: int
    n_iter: int
    status: int


def register(src, tgt, tgt_normals, T_init, max_corr_dist, max_iter=30, rel_tol=0.0,
             variant="point_to_plane", precision="kahan32", ctx: Context | None = None,
             loss="none", loss_k=1.0) -> IcpResult:
    """ICP registration; loss "huber" / "tukey" / "cauchy" with scale loss_k
    gives the robust (IRLS) variant."""
    sp, ns = _dev_pts(src, "src")
    tp, nt = _dev_pts(tgt, "tgt")
    npn = None
    if tgt_normals is not None:
        npn, nn = _dev_pts(tgt_normals, "tgt_normals")
        if nn != nt:
            raise IcpError(ICP_E_INVALID_ARG, "tgt_normals must have as many rows as tgt")
    r = icp_register(ctx.handle if ctx else None, sp, ns, tp, npn, nt, T_init, max_corr_dist,
                     max_iter, rel_tol, VARIANTS[variant], PRECISIONS[precision], LOSSES[loss], loss_k)
    return IcpResult(np.array(r.T[:], dtype=np.float64).reshape(4, 4), r.fitness, r.inlier_rmse,
                     r.n_inliers, r.n_iter, r.status)


def make_pair(src, tgt, tgt_normals, T_init, max_corr_dist, max_iter=30, rel_tol=0.0) -> icp_pair_t:
    """Descriptor of one pair for register_batch (tensors must stay alive)."""
    sp, ns = _dev_pts(src, "src")
    tp, nt = _dev_pts(tgt, "tgt")
    npn = None
    if tgt_normals is not None:
        npn, nn = _dev_pts(tgt_normals, "tgt_normals")
        if nn != nt:
            raise IcpError(ICP_E_INVALID_ARG, "tgt_normals must have as many rows as tgt")
    p = icp_pair_t()
    p.src_xyz, p.tgt_xyz, p.tgt_normals = sp, tp, npn
    p.n_src, p.n_tgt = ns, nt
    p.T_init[:] = [float(x) for x in _pose(T_init)]
    p.max_corr_dist, p.rel_tol, p.max_iter, p.reserved = float(max_corr_dist), float(rel_tol), int(max_iter), 0
    return p


def register_batch(pairs, variant="point_to_plane", precision="kahan32",
                   ctx: Context | None = None, loss="none", loss_k=1.0) -> list[IcpResult]:
    """pairs: list of icp_pair_t (see make_pair); loss: a robust loss for every
    pair (as register)."""
    res = icp_register_batch(ctx.handle if ctx else None, pairs, VARIANTS[variant],
                             PRECISIONS[precision], LOSSES[loss], loss_k)
    return [IcpResult(np.array(r.T[:], dtype=np.float64).reshape(4, 4), r.fitness, r.inlier_rmse,
                      r.n_inliers, r.n_iter, r.status) for r in res]


def icp_voxel_downsample(ctx, pts_ptr, nrm_ptr, n, voxel, out_ptr, out_nrm_ptr, cap) -> int:
    n_out = C.c_int64()
    _check(lib().icp_voxel_downsample(ctx, pts_ptr, nrm_ptr, int(n), float(voxel), out_ptr,
                                      out_nrm_ptr, int(cap), C.byref(n_out)))
    return n_out.value


def voxel_downsample(pts, voxel, normals=None, ctx: Context | None = None):
    """(points, normals or None) as new device tensors."""
    import torch
    pp, n = _dev_pts(pts, "pts")
    npn = _dev_pts(normals, "normals")[0] if normals is not None else None
    out = torch.empty((n, 3), dtype=torch.float32, device=pts.device)
    outn = torch.empty((n, 3), dtype=torch.float32, device=pts.device) if normals is not None else None
    m = icp_voxel_downsample(ctx.handle if ctx else None, pp, npn, n, voxel, out.data_ptr(),
                             outn.data_ptr() if outn is not None else None, n)
    return out[:m], (outn[:m] if outn is not None else None)


def icp_estimate_normals(ctx, pts_ptr, n, radius, max_nn, viewpoint, normals_ptr, counts_ptr) -> None:
    v = np.ascontiguousarray(np.asarray(viewpoint, dtype=np.float64).reshape(3))
    _check(lib().icp_estimate_normals(ctx, pts_ptr, int(n), float(radius), int(max_nn),
                                      v.ctypes.data, normals_ptr, counts_ptr))


def estimate_normals(pts, radius, max_nn=30, viewpoint=(0.0, 0.0, 0.0), ctx: Context | None = None,
                     with_counts=False):
    """Normals (device (N, 3) float32) of a device cloud with the hybrid
    (radius, max_nn) neighbourhood, facing `viewpoint`; with_counts also
    returns the neighbourhood sizes (device int32)."""
    import torch
    pp, n = _dev_pts(pts, "pts")
    out = torch.empty((n, 3), dtype=torch.float32, device=pts.device)
    cnt = torch.empty((n,), dtype=torch.int32, device=pts.device) if with_counts else None
    icp_estimate_normals(ctx.handle if ctx else None, pp, n, radius, max_nn, viewpoint, out.data_ptr(),
                         cnt.data_ptr() if cnt is not None else None)
    return (out, cnt) if with_counts else out


PG_METHODS = {"gn": 0, "lm": 1, 0: 0, 1: 1}


def pose_graph_optimize(poses, edges, method="lm", max_iter=50, rel_tol=1e-10,
                        ctx: Context | None = None):
    """Multiway registration: optimise node poses (array (N, 4, 4), node 0
    fixed) over edges (i, j, Z ~ T_i^-1 T_j, 6x6 information).  Returns the
    new poses and a dict (F_initial, F_final, steps, status)."""
    P = np.ascontiguousarray(np.asarray(poses, np.float64).reshape(-1, 16)).copy()
    arr = (icp_pose_edge_t * len(edges))()
    for k, (i, j, Z, L) in enumerate(edges):
        arr[k].i, arr[k].j = int(i), int(j)
        arr[k].Z[:] = list(np.asarray(Z, np.float64).reshape(16))
        arr[k].information[:] = list(np.asarray(L, np.float64).reshape(36))
    out = icp_pose_graph_result_t()
    _check(lib().icp_pose_graph_optimize(ctx.handle if ctx else None, len(P), P.ctypes.data, len(edges),
                                         arr, int(PG_METHODS.get(method, method)), int(max_iter), float(rel_tol),
                                         C.byref(out)))
    return P.reshape(-1, 4, 4), {"F_initial": out.F_initial, "F_final": out.F_final,
                                 "steps": out.steps, "status": out.status}


def compute_fpfh(pts, normals, radius, max_nn=100, ctx: Context | None = None, with_nn=False):
    """FPFH descriptors (device (N, 33) float32) of a device cloud with unit
    normals, hybrid (radius, max_nn) neighbourhood; with_nn also returns the
    neighbourhood sizes (device int32)."""
    import torch
    pp, n = _dev_pts(pts, "pts")
    npn, nn_ = _dev_pts(normals, "normals")
    if nn_ != n:
        raise IcpError(ICP_E_INVALID_ARG, "normals must have one row per point")
    out = torch.empty((n, 33), dtype=torch.float32, device=pts.device)
    cnt = torch.empty((n,), dtype=torch.int32, device=pts.device) if with_nn else None
    _check(lib().icp_compute_fpfh(ctx.handle if ctx else None, pp, npn, n, float(radius), int(max_nn),
                                  out.data_ptr(), cnt.data_ptr() if cnt is not None else None))
    return (out, cnt) if with_nn else out


def feature_match(src_feat, tgt_feat, ctx: Context | None = None, with_dist=False):
    """Nearest target feature per source feature (device (N, dim) float32
    tensors): device int32 indices (-1 without targets), and with_dist the
    float32 squared feature distances."""
    import torch
    for name, t in (("src_feat", src_feat), ("tgt_feat", tgt_feat)):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or t.dim() != 2 \
                or not t.is_contiguous():
            raise IcpError(ICP_E_INVALID_ARG, f"{name} must be a contiguous 2-D float32 CUDA (HIP) tensor")
    if src_feat.shape[1] != tgt_feat.shape[1]:
        raise IcpError(ICP_E_INVALID_ARG, "feature dimensions differ")
    n = src_feat.shape[0]
    match = torch.empty((n,), dtype=torch.int32, device=src_feat.device)
    dist = torch.empty((n,), dtype=torch.float32, device=src_feat.device) if with_dist else None
    _check(lib().icp_feature_match(ctx.handle if ctx else None, src_feat.data_ptr(), n, tgt_feat.data_ptr(),
                                   tgt_feat.shape[0], int(src_feat.shape[1]), match.data_ptr(),
                                   dist.data_ptr() if dist is not None else None))
    return (match, dist) if with_dist else match


def icp_feature_match_noalloc(src_ptr, n_src, tgt_ptr, n_tgt, dim, match_ptr, dist_ptr, hip_stream) -> None:
    """Raw no-allocation feature match: enqueues on hip_stream (an int handle
    or None) into caller-provided outputs; complete when that stream is."""
    _check(lib().icp_feature_match_noalloc(src_ptr, int(n_src), tgt_ptr, int(n_tgt), int(dim), match_ptr,
                                           dist_ptr, hip_stream))


def ransac_validate(src, tgt, max_corr_dist, Ts, ctx: Context | None = None):
    """Scores (count int64, sumq uint64 arrays) of host transforms Ts (K, 4, 4)."""
    sp, ns = _dev_pts(src, "src")
    tp, nt = _dev_pts(tgt, "tgt")
    T = np.ascontiguousarray(np.asarray(Ts, np.float64).reshape(-1, 16))
    cnt = np.zeros(len(T), np.int64)
    sq = np.zeros(len(T), np.uint64)
    _check(lib().icp_ransac_validate(ctx.handle if ctx else None, sp, ns, tp, nt, float(max_corr_dist), len(T),
                                     T.ctypes.data, cnt.ctypes.data, sq.ctypes.data))
    return cnt, sq


class RansacResult:
    def __init__(self, r: icp_ransac_result_t, trace=None):
        self.T = np.array(r.T[:], np.float64).reshape(4, 4)
        self.fitness, self.inlier_rmse = r.fitness, r.inlier_rmse
        self.n_inliers, self.sumq, self.shift, self.status = r.n_inliers, r.sumq, r.shift, r.status
        self.n_iterations, self.n_validated, self.best_hypothesis = r.n_iterations, r.n_validated, r.best_hypothesis
        self.trace = trace

    def __repr__(self):
        return (f"RansacResult(fitness={self.fitness:.4f}, rmse={self.inlier_rmse:.3e}, inliers={self.n_inliers}, "
                f"iterations={self.n_iterations}, validated={self.n_validated}, best={self.best_hypothesis}, "
                f"status={self.status})")


def ransac_register(src, tgt, corr, max_corr_dist, ransac_n=4, edge_length=0.9, distance=None,
                    max_iteration=4_000_000, max_validation=500, seed=0, trace=False,
                    ctx: Context | None = None) -> RansacResult:
    """RANSAC registration from putative pairs (i, corr[i]) (device int32).
    distance defaults to max_corr_dist; trace=True also returns the validated
    hypotheses (h, T, count, sumq) as host arrays in result.trace."""
    import torch
    sp, ns = _dev_pts(src, "src")
    tp, nt = _dev_pts(tgt, "tgt")
    if not isinstance(corr, torch.Tensor) or not corr.is_cuda or corr.dtype != torch.int32 \
            or corr.shape != (ns,) or not corr.is_contiguous():
        raise IcpError(ICP_E_INVALID_ARG, "corr must be a contiguous (n_src,) int32 CUDA (HIP) tensor")
    prm = icp_ransac_params_t(float(max_corr_dist), float(edge_length),
                              float(max_corr_dist if distance is None else distance), int(max_iteration),
                              int(max_validation), int(ransac_n), int(seed))
    out = icp_ransac_result_t()
    tr = None
    bufs = None
    if trace:
        m = max(1, int(max_validation))
        dev = src.device
        bufs = {"h": torch.empty(m, dtype=torch.int64, device=dev),
                "T": torch.empty((m, 4, 4), dtype=torch.float64, device=dev),
                "count": torch.empty(m, dtype=torch.int64, device=dev),
                "sumq": torch.empty(m, dtype=torch.int64, device=dev)}
        tr = icp_ransac_trace_t(bufs["h"].data_ptr(), bufs["T"].data_ptr(), bufs["count"].data_ptr(),
                                bufs["sumq"].data_ptr())
    _check(lib().icp_ransac_register(ctx.handle if ctx else None, sp, ns, tp, nt, corr.data_ptr(), C.byref(prm),
                                     C.byref(out), C.byref(tr) if tr is not None else None))
    t = None
    if bufs is not None:
        k = out.n_validated
        t = {"h": bufs["h"][:k].cpu().numpy(), "T": bufs["T"][:k].cpu().numpy(),
             "count": bufs["count"][:k].cpu().numpy(), "sumq": bufs["sumq"][:k].cpu().numpy().view(np.uint64)}
    return RansacResult(out, t)


def register_multiscale(src, tgt, tgt_normals, T_init, voxels, iters, dists, rel_tol=0.0,
                        variant="point_to_plane", precision="kahan32",
                        ctx: Context | None = None, loss="none", loss_k=1.0) -> IcpResult:
    sp, ns = _dev_pts(src, "src")
    tp, nt = _dev_pts(tgt, "tgt")
    npn = _dev_pts(tgt_normals, "tgt_normals")[0] if tgt_normals is not None else None
    L = len(voxels)
    v = np.ascontiguousarray(voxels, dtype=np.float64)
    k = np.ascontiguousarray(iters, dtype=np.int32)
    r = np.ascontiguousarray(dists, dtype=np.float64)
    out = icp_result_t()
    T = _pose(T_init)
    _check(lib().icp_register_multiscale_robust(ctx.handle if ctx else None, sp, ns, tp, npn, nt, T.ctypes.data,
                                                L, v.ctypes.data, k.ctypes.data, r.ctypes.data,
                                                float(rel_tol), VARIANTS[variant], PRECISIONS[precision],
                                                LOSSES[loss], float(loss_k), C.byref(out)))
    return IcpResult(np.array(out.T[:], dtype=np.float64).reshape(4, 4), out.fitness, out.inlier_rmse,
                     out.n_inliers, out.n_iter, out.status)


def correspondences(src, T, tgt, max_corr_dist, ctx: Context | None = None):
    """(idx int32 tensor, d2 float32 tensor) per source point, on the device."""
    import torch
    sp, ns = _dev_pts(src, "src")
    tp, nt = _dev_pts(tgt, "tgt")
    idx = torch.empty(ns, dtype=torch.int32, device=src.device)
    d2 = torch.empty(ns, dtype=torch.float32, device=src.device)
    icp_correspondences(ctx.handle if ctx else None, sp, ns, T, tp, nt, max_corr_dist,
                        idx.data_ptr(), d2.data_ptr())
    return idx, d2


def normal_equations(src, T, tgt, tgt_normals, max_corr_dist, variant="point_to_plane",
                     precision="kahan32", ctx: Context | None = None, loss="none", loss_k=1.0):
    """(AtA21, Atb6, sum_d2, n_in) at pose T (IRLS-weighted with a robust loss)."""
    sp, ns = _dev_pts(src, "src")
    tp, nt = _dev_pts(tgt, "tgt")
    npn = _dev_pts(tgt_normals, "tgt_normals")[0] if tgt_normals is not None else None
    return icp_normal_equations(ctx.handle if ctx else None, sp, ns, T, tp, npn, nt, max_corr_dist,
                                VARIANTS[variant], PRECISIONS[precision], LOSSES[loss], loss_k)


def full_matrix(A21) -> np.ndarray:
    """Symmetric 6x6 matrix from its 21-entry upper triangle (row-major)."""
    A = np.zeros((6, 6))
    k = 0
    for u in range(6):
        for v in range(u, 6):
            A[u, v] = A[v, u] = A21[k]
            k += 1
    return A


# ---------------------------------------------------------------- served form
@dataclass
class Completion:
    ticket: int
    user_tag: int
    error: int
    result: IcpResult | None
    t_submit_ns: int
    t_admit_ns: int
    t_done_ns: int


def _completion(c: icp_completion_t) -> Completion:
    r = c.result
    res = IcpResult(np.array(r.T[:], dtype=np.float64).reshape(4, 4), r.fitness, r.inlier_rmse,
                    r.n_inliers, r.n_iter, r.status) if c.error == 0 else None
    return Completion(c.ticket, c.user_tag, c.error, res, c.t_submit_ns, c.t_admit_ns, c.t_done_ns)


class Server:
    """Continuous-batching registration server (icp_server_*)."""

    def __init__(self, voxels=(0.04, 0.02, 0.01), iters=(30, 20, 10), corr_dist=None,
                 corr_factor=2.0, max_slots=64, budget_bytes=8 << 30, variant="point_to_plane",
                 precision="kahan32", iters_per_step=5, background_thread=False, device=0, loss="none",
                 loss_k=1.0):
        cfg = icp_server_cfg_t()
        cfg.device, cfg.max_slots, cfg.hbm_budget_bytes = device, max_slots, int(budget_bytes)
        cfg.n_levels = len(voxels)
        for k, (v, it) in enumerate(zip(voxels, iters)):
            cfg.voxel[k], cfg.iters[k] = float(v), int(it)
            cfg.corr_dist[k] = float(corr_dist[k]) if corr_dist else 0.0
        cfg.corr_factor = float(corr_factor)
        cfg.variant, cfg.precision = VARIANTS[variant], PRECISIONS[precision]
        cfg.iters_per_step, cfg.background_thread = int(iters_per_step), int(background_thread)
        cfg.loss, cfg.loss_k = LOSSES[loss], float(loss_k)
        h = C.c_void_p()
        _check(lib().icp_server_create(C.byref(cfg), C.byref(h)))
        self.handle = h.value
        self.background = bool(background_thread)

    def submit(self, src, tgt, tgt_normals, T_init=None, rel_tol=0.0, spacing=0.0, tag=0) -> int:
        """src/tgt/tgt_normals: CUDA tensors or numpy arrays (host memory)."""
        q = icp_request_t()
        host = isinstance(src, np.ndarray)
        if host:
            arrs = [np.ascontiguousarray(a, dtype=np.float32) if a is not None else None
                    for a in (src, tgt, tgt_normals)]
            q.src_xyz, q.tgt_xyz = arrs[0].ctypes.data, arrs[1].ctypes.data
            q.tgt_normals = arrs[2].ctypes.data if arrs[2] is not None else None
            q.n_src, q.n_tgt = len(arrs[0]), len(arrs[1])
        else:
            q.src_xyz, q.n_src = _dev_pts(src, "src")
            q.tgt_xyz, q.n_tgt = _dev_pts(tgt, "tgt")
            q.tgt_normals = _dev_pts(tgt_normals, "tgt_normals")[0] if tgt_normals is not None else None
            # the server's copy is ordered after the work queued on the
            # producing (torch's current) stream
            import torch
            q.stream = torch.cuda.current_stream(src.device).cuda_stream
        q.T_init[:] = [float(x) for x in _pose(np.eye(4) if T_init is None else T_init)]
        q.rel_tol, q.spacing, q.host_memory, q.reserved, q.user_tag = float(rel_tol), float(spacing), int(host), 0, int(tag)
        t = C.c_uint64()
        _check(lib().icp_server_submit(self.handle, C.byref(q), C.byref(t)))
        return t.value

    def step(self) -> int:
        n = C.c_int32()
        _check(lib().icp_server_step(self.handle, C.byref(n)))
        return n.value

    def poll(self, cap=256) -> list[Completion]:
        buf = (icp_completion_t * cap)()
        n = C.c_int32()
        _check(lib().icp_server_poll(self.handle, buf, cap, C.byref(n)))
        return [_completion(buf[k]) for k in range(n.value)]

    def wait(self, ticket) -> Completion:
        c = icp_completion_t()
        _check(lib().icp_server_wait(self.handle, int(ticket), C.byref(c)))
        return _completion(c)

    def close(self):
        if self.handle:
            _check(lib().icp_server_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
