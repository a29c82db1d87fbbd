"""Voxel downsampling and coarse-to-fine registration on the GPU against the
oracle.  Bars: downsampled positions bit-exact (same float64 sums in the same
order), normals within 2 ulp (float64 sqrt/division rounding), voxel counts
equal; multi-scale poses within 1e-5 rad / 1e-6 m with equal inlier counts."""
import os
import sys

import numpy as np
import pytest

from paper_1801_09847_amd import synth

sys.path.insert(0, os.path.dirname(__file__))
from cases import pose_error  # noqa: E402

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def icp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1801_09847_amd import icp as m
    m.lib()
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _ulp_diff(a, b):
    a = a.view(np.int32).astype(np.int64)
    b = b.view(np.int32).astype(np.int64)
    return np.abs(a - b)


@pytest.mark.parametrize("voxel", [0.04, 0.02, 0.01, 0.0137])
def test_voxel_downsample_matches_oracle(icp, oracle_lib, voxel):
    d = synth.room_pair_random(31, 60000, 1000, 4.0, 3.0, 2.5, 6, 3)
    pts, nrm = d["tgt"], d["tgt_normals"]
    g, gn = icp.voxel_downsample(dev(pts), voxel, dev(nrm))
    o, on = oracle_lib.voxel_downsample(pts, voxel, nrm)
    g, gn = g.cpu().numpy(), gn.cpu().numpy()
    assert g.shape == o.shape
    np.testing.assert_array_equal(g, o)
    assert _ulp_diff(gn, on).max() <= 2
    gp, _ = icp.voxel_downsample(dev(pts), voxel)
    np.testing.assert_array_equal(gp.cpu().numpy(), o)


def test_voxel_downsample_edges(icp, oracle_lib):
    rng = np.random.default_rng(3)
    one = np.array([[0.5, -0.25, 2.0]], np.float32)
    g, _ = icp.voxel_downsample(dev(one), 0.1)
    np.testing.assert_array_equal(g.cpu().numpy(), one)
    pts = rng.uniform(0, 1, (5000, 3)).astype(np.float32)
    for v in (5.0, 1e-4, 0.1):  # 1e-4: 1e12 voxels (keys wider than 32 bits)
        g, _ = icp.voxel_downsample(dev(pts), v)
        o, _ = oracle_lib.voxel_downsample(pts, v)
        np.testing.assert_array_equal(g.cpu().numpy(), o)
    with pytest.raises(icp.IcpError) as e:  # 1e15 voxels: beyond the 2^48 key range
        icp.voxel_downsample(dev(pts), 1e-5)
    assert e.value.code == icp.ICP_E_TOO_LARGE
    # capacity too small: error, count reported, nothing written past cap
    out = torch.full((10, 3), -7.0, device="cuda")
    with pytest.raises(icp.IcpError) as e:
        icp.icp_voxel_downsample(None, dev(pts).data_ptr(), None, 5000, 0.1, out.data_ptr(), None, 5)
    assert e.value.code == icp.ICP_E_TOO_LARGE
    assert (out[5:].cpu().numpy() == -7.0).all()
    bad = pts.copy()
    bad[10, 2] = np.nan
    with pytest.raises(icp.IcpError) as e:
        icp.voxel_downsample(dev(bad), 0.1)
    assert e.value.code == icp.ICP_E_NONFINITE


@pytest.mark.parametrize("seed,n_fixed", [(0, None), (1, None), (2, 450_000)])
def test_multiscale_matches_oracle(icp, oracle_lib, seed, n_fixed):
    """Requests of the served workload's recipe: two at their own size capped
    at 60k, one at 450k points (the upper end of the request sizes)."""
    n, o = synth.c5_request_size(seed)
    n = min(n, 60000) if n_fixed is None else n_fixed
    d = synth.room_pair_random(10_000 + seed, n, n, overlap=o)
    sp = np.sqrt(d["area"] / n)
    vox = [0.04, 0.02, 0.01]
    its = [30, 20, 10]
    dists = [2 * max(v, sp) for v in vox]
    g = icp.register_multiscale(dev(d["src"]), dev(d["tgt"]), dev(d["tgt_normals"]), np.eye(4), vox,
                                its, dists)
    r = oracle_lib.register_multiscale(d["src"], d["tgt"], d["tgt_normals"], np.eye(4), vox, its, dists)
    ang, dt = pose_error(g.T, r.T)
    print(f"multiscale seed {seed}: rot {ang:.2e} trans {dt:.2e} n_in {g.n_inliers}/{r.n_inliers}")
    assert g.n_inliers == r.n_inliers
    assert ang <= 1e-5 and dt <= 1e-6
