"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/icp.h, and rejects invalid arguments on the host before
any device work (so these calls are safe without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1801_09847_amd import icp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 1 << 20          # aligned, never dereferenced: validation fails first
MISALIGNED = FAKE + 2


def declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^[A-Za-z_][\w \*]*?\b(icp_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = icp.lib()
    names = declared_functions()
    assert "icp_register" in names and "icp_correspondences" in names
    for n in names:
        assert hasattr(L, n), n
    assert icp.icp_version().startswith("icp-mi355x")


def test_strerror_covers_codes():
    L = icp.lib()
    for code in range(0, -8, -1):
        assert L.icp_strerror(code).decode() not in ("", "unknown error code")
    assert L.icp_strerror(-99).decode() == "unknown error code"


def _reg(**kw):
    a = dict(ctx=None, src_ptr=FAKE, n_src=100, tgt_ptr=FAKE, tgt_n_ptr=FAKE, n_tgt=100,
             T_init=np.eye(4), max_corr_dist=0.05, max_iter=10, rel_tol=0.0,
             variant=icp.ICP_POINT_TO_PLANE, precision=icp.ICP_PREC_F32_KAHAN_F64)
    a.update(kw)
    with pytest.raises(icp.IcpError) as e:
        icp.icp_register(**a)
    return e.value.code


def test_register_validation_codes():
    bad_T = np.eye(4); bad_T[3, 0] = 1.0
    nan_T = np.eye(4); nan_T[0, 3] = np.nan
    skew_T = np.eye(4); skew_T[0, 1] = 0.01
    assert _reg(src_ptr=None) == icp.ICP_E_INVALID_ARG
    assert _reg(tgt_ptr=None) == icp.ICP_E_INVALID_ARG
    assert _reg(n_src=0) == icp.ICP_E_INVALID_ARG
    assert _reg(n_tgt=-5) == icp.ICP_E_INVALID_ARG
    assert _reg(n_src=2**31) == icp.ICP_E_TOO_LARGE
    assert _reg(max_corr_dist=0.0) == icp.ICP_E_INVALID_ARG
    assert _reg(max_corr_dist=float("nan")) == icp.ICP_E_INVALID_ARG
    assert _reg(max_corr_dist=float("inf")) == icp.ICP_E_INVALID_ARG
    assert _reg(max_iter=-1) == icp.ICP_E_INVALID_ARG
    assert _reg(rel_tol=-1e-3) == icp.ICP_E_INVALID_ARG
    assert _reg(rel_tol=float("nan")) == icp.ICP_E_INVALID_ARG
    assert _reg(T_init=bad_T) == icp.ICP_E_INVALID_ARG
    assert _reg(T_init=nan_T) == icp.ICP_E_INVALID_ARG
    assert _reg(T_init=skew_T) == icp.ICP_E_INVALID_ARG
    # point-to-plane needs normals with the target's record count (Sec. 3.1 field rule)
    assert _reg(tgt_n_ptr=None) == icp.ICP_E_INVALID_ARG
    assert _reg(variant=7) == icp.ICP_E_INVALID_ARG
    assert _reg(precision=3) == icp.ICP_E_INVALID_ARG
    assert _reg(src_ptr=MISALIGNED) == icp.ICP_E_INVALID_ARG
    assert "aligned" in icp.lib().icp_last_error().decode()
    # robust variant: loss kind and scale
    assert _reg(loss=9, loss_k=0.01) == icp.ICP_E_INVALID_ARG
    assert _reg(loss=icp.ICP_LOSS_TUKEY, loss_k=0.0) == icp.ICP_E_INVALID_ARG
    assert _reg(loss=icp.ICP_LOSS_HUBER, loss_k=float("inf")) == icp.ICP_E_INVALID_ARG
    assert _reg(loss=icp.ICP_LOSS_CAUCHY, loss_k=1e-300) == icp.ICP_E_INVALID_ARG  # 0 in float32


def test_null_out_and_hooks_validation():
    L = icp.lib()
    T = np.eye(4)
    rc = L.icp_register(None, FAKE, 10, FAKE, FAKE, 10, T.ctypes.data, 0.1, 3, 0.0, 1, 0, None)
    assert rc == icp.ICP_E_INVALID_ARG
    with pytest.raises(icp.IcpError) as e:
        icp.icp_correspondences(None, FAKE, 10, T, FAKE, 10, 0.1, None, FAKE)
    assert e.value.code == icp.ICP_E_INVALID_ARG
    with pytest.raises(icp.IcpError) as e:
        icp.icp_correspondences(None, FAKE, 10, T, FAKE, 10, -0.1, FAKE, FAKE)
    assert e.value.code == icp.ICP_E_INVALID_ARG
    with pytest.raises(icp.IcpError) as e:
        icp.icp_normal_equations(None, FAKE, 10, T, FAKE, None, 10, 0.1, 1, 0)
    assert e.value.code == icp.ICP_E_INVALID_ARG
    rc = L.icp_ctx_create(0, None, 0, None)
    assert rc == icp.ICP_E_INVALID_ARG
    assert L.icp_ctx_destroy(None) == 0


def test_product_path_has_no_oracle_or_cpu_fallback():
    """The package never imports the oracle, and the binding carries no
    computation of its own."""
    pkg = os.path.join(ROOT, "paper_1801_09847_amd")
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            src = open(os.path.join(pkg, f)).read()
            assert "import oracle" not in src and "from oracle" not in src, f
    for f in os.listdir(os.path.join(pkg, "csrc")):
        if not f.endswith((".hip", ".h", ".cpp")):
            continue
        src = open(os.path.join(pkg, "csrc", f)).read()
        assert "oracle" not in src.lower(), f


def _pair(**kw):
    p = icp.icp_pair_t()
    p.src_xyz, p.tgt_xyz, p.tgt_normals = FAKE, FAKE, FAKE
    p.n_src, p.n_tgt = 100, 100
    p.T_init[:] = list(np.eye(4).reshape(16))
    p.max_corr_dist, p.rel_tol, p.max_iter, p.reserved = 0.05, 0.0, 10, 0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_batch_validation():
    L = icp.lib()
    out = (icp.icp_result_t * 4)()
    arr = (icp.icp_pair_t * 4)(_pair(), _pair(), _pair(), _pair())
    assert L.icp_register_batch(None, arr, 0, 1, 0, out) == icp.ICP_E_INVALID_ARG
    assert L.icp_register_batch(None, None, 4, 1, 0, out) == icp.ICP_E_INVALID_ARG
    assert L.icp_register_batch(None, arr, 4, 1, 0, None) == icp.ICP_E_INVALID_ARG
    for bad in (dict(reserved=1), dict(max_corr_dist=-1.0), dict(max_iter=-2), dict(n_src=0),
                dict(tgt_normals=None), dict(rel_tol=float("nan"))):
        arr = (icp.icp_pair_t * 4)(_pair(), _pair(), _pair(**bad), _pair())
        assert L.icp_register_batch(None, arr, 4, 1, 0, out) == icp.ICP_E_INVALID_ARG, bad
        assert "pair 2" in L.icp_last_error().decode()
    big = (icp.icp_pair_t * 2)(_pair(n_src=2**30 + 10), _pair(n_src=2**30 + 10))
    assert L.icp_register_batch(None, big, 2, 1, 0, out) == icp.ICP_E_TOO_LARGE


def test_server_create_validation():
    L = icp.lib()
    h = C.c_void_p()
    good = icp.icp_server_cfg_t()
    good.max_slots, good.hbm_budget_bytes, good.n_levels = 4, 1 << 28, 1
    good.iters[0], good.voxel[0], good.corr_factor = 10, 0.02, 2.0
    good.variant, good.precision, good.iters_per_step = 1, 0, 4
    assert L.icp_server_create(None, C.byref(h)) == icp.ICP_E_INVALID_ARG
    for field, val in (("max_slots", 0), ("n_levels", 5), ("iters_per_step", 0),
                       ("hbm_budget_bytes", 1000), ("variant", 3), ("precision", 9),
                       ("corr_factor", 0.0)):
        cfg = icp.icp_server_cfg_t.from_buffer_copy(good)
        setattr(cfg, field, val)
        if field == "corr_factor":
            cfg.voxel[0] = 0.0
        assert L.icp_server_create(C.byref(cfg), C.byref(h)) == icp.ICP_E_INVALID_ARG, field
    assert L.icp_server_destroy(None) == 0


def test_pose_graph_validation():
    eye = np.eye(4)
    good = [(0, 1, eye, np.eye(6))]
    for poses, edges, kw in (
        (np.array([eye]), good, {}),                               # one node
        (np.array([eye] * 257), good, {}),                         # too many nodes
        (np.array([eye, eye]), [(0, 2, eye, np.eye(6))], {}),      # bad index
        (np.array([eye, eye]), [(1, 1, eye, np.eye(6))], {}),      # self edge
        (np.array([eye, eye]), [(0, 1, eye * 2, np.eye(6))], {}),  # not rigid
        (np.array([eye, eye]), [(0, 1, eye, np.full((6, 6), np.nan))], {}),
        (np.array([eye, eye]), [(0, 1, eye, np.eye(6) + np.triu(np.ones((6, 6)), 1) * 1e-3)], {}),  # asymmetric
        (np.array([eye, eye]), good, {"method": 7}),
        (np.array([eye, eye]), good, {"max_iter": -1}),
    ):
        with pytest.raises(icp.IcpError) as e:
            icp.pose_graph_optimize(poses, edges, **kw)
        assert e.value.code == icp.ICP_E_INVALID_ARG


def _ransac_rc(**kw):
    prm = dict(max_corr_dist=0.075, edge_length=0.9, distance=0.075, max_iteration=1000,
               max_validation=10, ransac_n=4, seed=0)
    args = dict(src=FAKE, n_src=100, tgt=FAKE, n_tgt=100, corr=FAKE)
    for k, v in kw.items():
        (prm if k in prm else args)[k] = v
    p = icp.icp_ransac_params_t(**prm)
    out = icp.icp_ransac_result_t()
    return icp.lib().icp_ransac_register(None, args["src"], args["n_src"], args["tgt"], args["n_tgt"],
                                         args["corr"], C.byref(p), C.byref(out), None)


def test_ransac_validation():
    E = icp.ICP_E_INVALID_ARG
    assert _ransac_rc(src=None) == E
    assert _ransac_rc(corr=None) == E
    assert _ransac_rc(corr=MISALIGNED) == E
    assert _ransac_rc(n_src=0) == E
    assert _ransac_rc(n_src=(1 << 23) + 1) == icp.ICP_E_TOO_LARGE
    assert _ransac_rc(max_corr_dist=0.0) == E
    assert _ransac_rc(max_corr_dist=float("nan")) == E
    assert _ransac_rc(ransac_n=2) == E
    assert _ransac_rc(ransac_n=9) == E
    assert _ransac_rc(edge_length=float("inf")) == E
    assert _ransac_rc(distance=float("nan")) == E
    assert _ransac_rc(max_iteration=0) == E
    assert _ransac_rc(max_validation=0) == E
    assert _ransac_rc(max_validation=65536) == E
    L = icp.lib()
    cnt = np.zeros(2, np.int64)
    sq = np.zeros(2, np.uint64)
    T = np.stack([np.eye(4)] * 2)
    bad = T.copy()
    bad[1, 0, 1] = 0.5
    for args in ((FAKE, 100, FAKE, 100, 0.05, 0, T), (FAKE, 100, FAKE, 100, 0.05, 65536, T),
                 (FAKE, 100, FAKE, 100, -1.0, 2, T), (FAKE, 100, FAKE, 100, 0.05, 2, bad),
                 (None, 100, FAKE, 100, 0.05, 2, T)):
        s, ns, t, nt, r, k, TT = args
        TT = np.ascontiguousarray(TT)
        assert L.icp_ransac_validate(None, s, ns, t, nt, r, k, TT.ctypes.data, cnt.ctypes.data,
                                     sq.ctypes.data) == E
    assert L.icp_ransac_validate(None, FAKE, 100, FAKE, 100, 0.05, 2, None, cnt.ctypes.data,
                                 sq.ctypes.data) == E
    m = np.zeros(4, np.int32)
    assert L.icp_feature_match(None, FAKE, 10, FAKE, 10, 0, m.ctypes.data, None) == E
    assert L.icp_feature_match(None, FAKE, 10, FAKE, 10, 65, m.ctypes.data, None) == E
    assert L.icp_feature_match(None, None, 10, FAKE, 10, 33, m.ctypes.data, None) == E
    assert L.icp_feature_match(None, FAKE, -1, FAKE, 10, 33, m.ctypes.data, None) == E
    assert L.icp_feature_match(None, FAKE, 10, FAKE, 10, 33, None, None) == E
    assert L.icp_feature_match(None, FAKE, 10, FAKE, 10, 33, MISALIGNED, None) == E


def test_fpfh_validation():
    L = icp.lib()
    E = icp.ICP_E_INVALID_ARG
    out = FAKE
    assert L.icp_compute_fpfh(None, None, FAKE, 10, 0.25, 100, out, None) == E
    assert L.icp_compute_fpfh(None, FAKE, None, 10, 0.25, 100, out, None) == E
    assert L.icp_compute_fpfh(None, FAKE, MISALIGNED, 10, 0.25, 100, out, None) == E
    assert L.icp_compute_fpfh(None, FAKE, FAKE, 0, 0.25, 100, out, None) == E
    assert L.icp_compute_fpfh(None, FAKE, FAKE, 10, 0.0, 100, out, None) == E
    assert L.icp_compute_fpfh(None, FAKE, FAKE, 10, float("inf"), 100, out, None) == E
    assert L.icp_compute_fpfh(None, FAKE, FAKE, 10, 0.25, 0, out, None) == E
    assert L.icp_compute_fpfh(None, FAKE, FAKE, 10, 0.25, 129, out, None) == E
    assert L.icp_compute_fpfh(None, FAKE, FAKE, 10, 0.25, 100, None, None) == E
    assert L.icp_compute_fpfh(None, FAKE, FAKE, 10, 0.25, 100, MISALIGNED, None) == E


def test_batch_robust_validation():
    p = _pair()
    out = (icp.icp_result_t * 1)()
    arr = (icp.icp_pair_t * 1)(p)
    L = icp.lib()
    assert L.icp_register_batch_robust(None, arr, 1, 1, 0, 7, 1.0, out) == icp.ICP_E_INVALID_ARG
    assert L.icp_register_batch_robust(None, arr, 1, 1, 0, icp.ICP_LOSS_TUKEY, 0.0, out) == icp.ICP_E_INVALID_ARG
    assert L.icp_register_batch_robust(None, arr, 1, 1, 0, icp.ICP_LOSS_TUKEY, float("nan"), out) == \
        icp.ICP_E_INVALID_ARG


def test_server_rejects_bad_loss():
    for loss, k in ((7, 1.0), (icp.ICP_LOSS_TUKEY, 0.0), (icp.ICP_LOSS_CAUCHY, float("nan"))):
        cfg = icp.icp_server_cfg_t()
        cfg.max_slots, cfg.hbm_budget_bytes, cfg.n_levels = 1, 1 << 30, 1
        cfg.iters[0], cfg.corr_factor, cfg.variant, cfg.iters_per_step = 5, 2.0, icp.ICP_POINT_TO_PLANE, 1
        cfg.loss, cfg.loss_k = loss, k
        h = C.c_void_p()
        assert icp.lib().icp_server_create(C.byref(cfg), C.byref(h)) == icp.ICP_E_INVALID_ARG
