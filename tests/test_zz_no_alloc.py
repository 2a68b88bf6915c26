"""The no-allocation vMF fit (lbessel_vmf_fit_f32_noalloc, static device
workspace) against the workspace entry point lbessel_vmf_fit_f32: the same
kernels in the same order, so the four result words must agree bit for bit,
on consecutive calls that reuse the one static buffer, the later ones with
smaller inputs (stale contents of a larger call must not leak into them)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the -m gpu tests need an MI355X")
    import paper_2409_08729_amd as m
    m.lib()
    return m


def _low_concentration(n, p, a, seed):
    g = np.random.default_rng(seed)
    X = g.normal(size=(n, p))
    X[:, 0] += a
    return torch.from_numpy(X.astype(np.float32)).to("cuda:0")


def _same(lb, X, res):
    out = lb.vmf_fit_noalloc(X, res)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = np.array(lb.vmf_fit(X), dtype=np.float64)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), (tuple(X.shape), got, ref)
    assert np.isfinite(got).all() and got[3] >= 1
    return got


def test_noalloc_fit_matches_workspace_fit_on_shrinking_calls(lb):
    from paper_2409_08729_amd import workloads as wl
    res = torch.empty(4, dtype=torch.float64, device="cuda:0")
    # the 4-column pass with the most slices, then smaller inputs of both passes
    cases = [wl.vmf_features(50_000, 32768, seed=11, device="cuda:0"),
             wl.vmf_features(5_000, 8192, seed=12, device="cuda:0"),
             wl.vmf_features(700, 2048, seed=13, device="cuda:0"),
             _low_concentration(4000, 3, 1.0, seed=14),      # I series region of the solve
             _low_concentration(300, 2, 3.0, seed=15)]
    for X in cases:
        print(f"noalloc fit n={X.shape[0]} p={X.shape[1]}", flush=True)
        _same(lb, X, res)
    # and a large call again after the small ones
    _same(lb, cases[1], res)


def test_noalloc_fit_rejects_oversized_requests(lb):
    """Shapes whose workspace exceeds the static buffer come back as
    LBESSEL_ENOSPACE before anything is launched (X is a small real tensor:
    the call never reads it)."""
    res = torch.full((4,), -1.0, dtype=torch.float64, device="cuda:0")
    X = torch.zeros((4, 4), dtype=torch.float32, device="cuda:0")
    fn = lb.lib().lbessel_vmf_fit_f32_noalloc
    assert fn(X.data_ptr(), 1_015_808, 32768, res.data_ptr(), None) == -7
    assert fn(X.data_ptr(), 2_619_392, 2048, res.data_ptr(), None) == -7
    torch.cuda.synchronize()
    assert (res.cpu() == -1.0).all()
