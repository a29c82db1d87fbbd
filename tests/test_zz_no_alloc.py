"""The no-allocation entry point icp_feature_match_noalloc (static device
scratch) against icp_feature_match on the same inputs: indices bit-exact and
distances equal (the same kernels on the same data), on two calls in a row,
the second with fewer source features, called through the C ABI on torch's
current stream; sizes beyond the scratch are rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def icp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1801_09847_amd import icp as m
    m.lib()
    return m


def _noalloc(icp, s, t):
    n = s.shape[0]
    match = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    dist = torch.full((n,), -7.0, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    icp.icp_feature_match_noalloc(s.data_ptr(), n, t.data_ptr(), t.shape[0], s.shape[1], match.data_ptr(),
                                  dist.data_ptr(), stream)
    torch.cuda.current_stream().synchronize()
    return match, dist


def test_noalloc_matches_feature_match_twice(icp):
    rng = np.random.default_rng(5)
    for n_src, n_tgt, dim in ((30000, 20000, 33), (7001, 20000, 33)):
        s = torch.from_numpy(rng.random((n_src, dim), dtype=np.float32)).cuda()
        t = torch.from_numpy(rng.random((n_tgt, dim), dtype=np.float32)).cuda()
        ref_m, ref_d = icp.feature_match(s, t, with_dist=True)
        m, d = _noalloc(icp, s, t)
        assert torch.equal(m, ref_m)
        assert torch.equal(d, ref_d)
        assert int(m.min()) >= 0


def test_noalloc_rejects_oversize(icp):
    s = torch.zeros((1 << 20) + 1, 4, dtype=torch.float32, device="cuda")
    t = torch.zeros(10, 4, dtype=torch.float32, device="cuda")
    out = torch.empty((1 << 20) + 1, dtype=torch.int32, device="cuda")
    with pytest.raises(icp.IcpError) as e:
        icp.icp_feature_match_noalloc(s.data_ptr(), s.shape[0], t.data_ptr(), 10, 4, out.data_ptr(), None,
                                      None)
    assert e.value.code == icp.ICP_E_TOO_LARGE
