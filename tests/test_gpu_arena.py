"""Contexts with a fixed device arena (icp_ctx_create with arena_bytes > 0).

Bars:
  * results bit-identical to those of a context whose buffers grow on demand,
    for a sequence of calls of different kinds and sizes on one context
    (plain registrations of C1 and the 300k room, a batch, a multi-scale
    registration, normal estimation);
  * no device memory allocated by the calls: the device's free memory is the
    same before and after the sequence (a growing context's first run of the
    same sequence takes more than 32 MB);
  * a call that does not fit fails with ICP_E_OOM and leaves the context
    usable for calls that fit.
"""
import numpy as np
import pytest

from paper_1801_09847_amd import synth

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


@pytest.fixture(scope="module")
def clouds():
    c1, c2 = synth.c1_heightfield(0), synth.c2_room(0)
    return [(d, dev(d["src"]), dev(d["tgt"]), dev(d["tgt_normals"])) for d in (c1, c2)]


def _sequence(icp, ctx, clouds):
    out = []
    for d, s, t, n in clouds:
        r = icp.register(s, t, n, np.eye(4), d["max_corr_dist"], 20, 0.0, ctx=ctx)
        out.append(("register", r.T.copy(), r.n_iter, r.n_inliers))
    d, s, t, n = clouds[0]
    descs = [icp.make_pair(s, t, n, np.eye(4), 0.05, 15, 0.0), icp.make_pair(s, t, n, d["T_gt"], 0.05, 15, 0.0)]
    for r in icp.register_batch(descs, ctx=ctx):
        out.append(("batch", r.T.copy(), r.n_iter, r.n_inliers))
    d, s, t, n = clouds[1]
    r = icp.register_multiscale(s, t, n, np.eye(4), [0.04, 0.02], [10, 10], [0.08, 0.04], ctx=ctx)
    out.append(("multiscale", r.T.copy(), r.n_iter, r.n_inliers))
    nr = icp.estimate_normals(t, 0.05, 30, ctx=ctx)
    out.append(("normals", nr.cpu().numpy().copy(), 0, 0))
    torch.cuda.synchronize()
    return out


def test_arena_results_equal_growing_and_allocate_nothing(icp, clouds):
    grow = icp.Context(0)
    torch.cuda.synchronize()
    g0, _ = torch.cuda.mem_get_info()
    ref = _sequence(icp, grow, clouds)
    g1, _ = torch.cuda.mem_get_info()
    grow.close()
    assert g0 - g1 > 32 << 20, (g0, g1)  # the growing context allocated its buffers
    arena = icp.Context(0, arena_bytes=1 << 30)
    _sequence(icp, arena, clouds)  # first use (code objects, events)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    got = _sequence(icp, arena, clouds)
    free1, _ = torch.cuda.mem_get_info()
    arena.close()
    assert free1 == free0, (free0, free1)
    for (k0, a0, i0, n0), (k1, a1, i1, n1) in zip(ref, got):
        assert k0 == k1
        assert np.array_equal(a0, a1), k0
        assert (i0, n0) == (i1, n1), k0


def test_arena_too_small_fails_and_recovers(icp, clouds):
    ctx = icp.Context(0, arena_bytes=8 << 20)
    d1, s1, t1, n1 = clouds[0]
    d2, s2, t2, n2 = clouds[1]
    small = icp.register(s1, t1, n1, np.eye(4), d1["max_corr_dist"], 20, 0.0, ctx=ctx)
    with pytest.raises(icp.IcpError) as e:
        icp.register(s2, t2, n2, np.eye(4), d2["max_corr_dist"], 20, 0.0, ctx=ctx)
    assert e.value.code == icp.ICP_E_OOM
    again = icp.register(s1, t1, n1, np.eye(4), d1["max_corr_dist"], 20, 0.0, ctx=ctx)
    ctx.close()
    assert np.array_equal(small.T, again.T) and small.n_iter == again.n_iter
