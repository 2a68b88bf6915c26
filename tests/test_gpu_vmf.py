"""vMF fit on the GPU (paper, Sec. "Metric learning"): mean resultant, kappa
estimates, likelihood fit with the analytic gradient, checked against numpy
(float64) and the binary128 oracle."""
import math

import numpy as np
import pytest
import torch

from parity import TOL64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the -m gpu tests need an MI355X")
    import paper_2409_08729_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("n,p", [(3001, 257), (700, 2048), (1, 5), (129, 1), (64, 8192)])
def test_colsum_matches_numpy(lb, n, p):
    g = np.random.default_rng(n * 7 + p)
    X = np.abs(g.normal(size=(n, p))).astype(np.float32)
    X[0, :] = 0.0                                    # a zero row contributes nothing
    cs, ss = lb.vmf_colsum(torch.from_numpy(X).to("cuda:0"))
    cs = cs.cpu().numpy()
    X64 = X.astype(np.float64)
    nrm = np.sqrt((X64 * X64).sum(1))
    ref = (X64[nrm > 0] / nrm[nrm > 0, None]).sum(0)
    np.testing.assert_allclose(cs, ref, rtol=1e-13, atol=1e-13)
    assert abs(ss.item() - float((cs * cs).sum())) <= 1e-13 * max(1.0, float((cs * cs).sum()))
    # same bits on a second call (fixed reduction order)
    cs2, _ = lb.vmf_colsum(torch.from_numpy(X).to("cuda:0"))
    assert np.array_equal(cs, cs2.cpu().numpy())


@pytest.mark.parametrize("p", [2048, 8192])
def test_kappa_fit_solves_likelihood_equation(lb, oracle, p):
    from paper_2409_08729_amd import vmf, workloads as wl
    X = wl.vmf_features(4000, p, seed=p, device="cuda:0")
    _, R = vmf.mean_resultant(X)
    assert 0.8 < R < 0.99
    ks = vmf.kappa_estimates(R, p)
    k = ks[-1]
    # A_p(k) from the oracle: exp(log I_{p/2}(k) - log I_{p/2-1}(k))
    v = np.array([p / 2 - 1, p / 2])
    hi, lo = oracle.log_iv(v, np.array([k, k]))
    a_ref = math.exp((hi[1] - hi[0]) + (lo[1] - lo[0]))
    s = sum(max(abs(h), 1 + math.hypot(vv, k)) for h, vv in zip(hi, v))
    assert abs(a_ref - R) <= TOL64 * s * a_ref + 1e-15, (p, k, a_ref, R)
    # kappa_0 within a few percent, kappa_2 already converged to ~1e-10
    assert abs(ks[0] - k) / k < 0.05
    assert abs(ks[2] - k) / k < 1e-9
    # likelihood maximisation with the analytic gradient reaches the same kappa
    # (to the ~sqrt(eps) resolution of a minimum located from function values)
    k_lbfgs = vmf.fit_kappa_lbfgs(R, p)
    assert abs(k_lbfgs - k) / k < 1e-7, (k_lbfgs, k)


def test_vmf_log_norm_gradient_vs_finite_difference(lb):
    for p in (3.0, 2048.0, 32768.0):
        k = torch.tensor([0.5 * p, 3.0 * p, 6.2 * p], dtype=torch.float64, device="cuda:0")
        g = lb.vmf_log_norm_grad(k, p).cpu().numpy()
        for i in range(3):
            kk = float(k[i])
            h = 1e-4 * kk
            pts = torch.tensor([kk - 2 * h, kk - h, kk + h, kk + 2 * h], dtype=torch.float64,
                               device="cuda:0")
            f = lb.vmf_log_norm(pts, p).cpu().numpy()
            fd = (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * h)
            assert abs(fd - g[i]) <= 1e-7 * abs(g[i]) + 1e-9, (p, kk, fd, g[i])
        # autograd path gives the same numbers
        kr = k.clone().requires_grad_(True)
        (gk,) = torch.autograd.grad(lb.VmfLogNorm.apply(kr, p).sum(), kr)
        assert torch.equal(gk, lb.vmf_log_norm_grad(k, p))


@pytest.mark.parametrize("p", [2, 3, 10, 30])
@pytest.mark.parametrize("a", [1.0, 3.0])
def test_device_kappa_solve_low_concentration(lb, oracle, p, a):
    """The device kappa solve where log I_{p/2-1}(kappa) takes the power series
    (order p/2 - 1 <= 14 and kappa in ~1..20): rows a e_1 + N(0, I) give
    mean resultant lengths from ~0.06 to ~0.94.  The solve must satisfy
    A_p(kappa) = R (paper, eq. kappa estimates) with A_p from the oracle, and
    kappa_0 must be R (p - R^2) / (1 - R^2)."""
    import math
    g = np.random.default_rng(1000 + p)
    X = g.normal(size=(4000, p))
    X[:, 0] += a
    Xd = torch.from_numpy(X.astype(np.float32)).to("cuda:0")
    k, R, k0, steps = lb.vmf_fit(Xd)
    X64 = X.astype(np.float32).astype(np.float64)
    U = X64 / np.linalg.norm(X64, axis=1, keepdims=True)
    R_ref = float(np.linalg.norm(U.sum(0))) / X.shape[0]
    assert abs(R - R_ref) <= 1e-12 * R_ref, (R, R_ref)
    assert abs(k0 - R * (p - R * R) / (1 - R * R)) <= 1e-13 * k0
    assert 0.5 < k < 25.0, k                    # inside the series region of the order
    assert 1 <= steps <= 12, steps
    v = np.array([p / 2 - 1, p / 2])
    hi, lo = oracle.log_iv(v, np.array([k, k]))
    a_ref = math.exp((hi[1] - hi[0]) + (lo[1] - lo[0]))
    s = sum(max(abs(h), 1 + math.hypot(vv, k)) for h, vv in zip(hi, v))
    assert abs(a_ref - R) <= TOL64 * s * a_ref + 1e-15, (p, k, a_ref, R)
