"""Fitting a von Mises-Fisher distribution (paper, Sec. "Metric learning").

mean_resultant(X)      xbar = (1/N) sum_i x_i/||x_i|| and R = ||xbar|| (eq. mean
                       direction estimate), from lbessel_vmf_colsum_f32
kappa_estimates(R, p)  kappa_0 = R (p - R^2) / (1 - R^2) and the Newton steps
                       kappa_{t+1} = F(kappa_t),
                       F(k) = k - (A_p(k) - R) / (1 - A_p(k)^2 - (p-1) A_p(k)/k),
                       A_p = I_{p/2} / I_{p/2-1} (eq. kappa estimates), iterated
                       to convergence
fit_kappa_lbfgs(R, p)  maximum likelihood: minimise
                       NLL(k) = -(log C_p(k) + k R) with L-BFGS and the analytic
                       gradient -A_p(k) + ... (the paper's gradient-based fit)

A_p and log C_p come from the GPU library; only O(1) scalar bookkeeping runs
on the host.
"""
from __future__ import annotations

import math

import torch

import paper_2409_08729_amd as lb


def mean_resultant(X: torch.Tensor):
    """(xbar float64 (p,), R float) of the L2-normalised rows of X (N, p) float32."""
    colsum, sumsq = lb.vmf_colsum(X)
    n = X.shape[0]
    return colsum / n, math.sqrt(float(sumsq.item())) / n


def a_p(kappa: float, p: float, device="cuda:0") -> float:
    """A_p(kappa) = I_{p/2}(kappa) / I_{p/2-1}(kappa) on the GPU."""
    k = torch.tensor([kappa], dtype=torch.float64, device=device)
    return -float(lb.vmf_log_norm_grad(k, p).item())


def kappa_estimates(R: float, p: float, steps: int = 8, device="cuda:0") -> list[float]:
    """[kappa_0, kappa_1, ...]: kappa_0 then Newton steps F until the update is
    below 1e-15 relative or stops shrinking (at most `steps`).

    The second test ends the iteration at its noise floor: A_p comes from two
    log-values of size ~kappa, so it carries a relative error of ~kappa * 1e-16,
    and with A_p'(kappa) ~ 1e-2 / p the root is only defined to ~1e-11 relative
    for the vMF fits here; past that point Newton updates no longer contract."""
    if not (0.0 < R < 1.0):
        raise ValueError("mean resultant length must be in (0, 1)")
    k = R * (p - R * R) / (1.0 - R * R)
    out = [k]
    prev = math.inf
    for _ in range(steps):
        A = a_p(k, p, device)
        k_new = k - (A - R) / (1.0 - A * A - (p - 1.0) * A / k)
        out.append(k_new)
        d = abs(k_new - k)
        if d <= 1e-15 * abs(k_new) or d >= prev:
            break
        prev = d
        k = k_new
    return out


def neg_log_likelihood(kappa: torch.Tensor, R: float, p: float) -> torch.Tensor:
    """Per-sample NLL of the vMF model at concentration kappa, given R = mu^T xbar."""
    return -(lb.VmfLogNorm.apply(kappa, p) + kappa * R)


def fit_kappa_lbfgs(R: float, p: float, kappa0: float | None = None, device="cuda:0",
                    max_iter: int = 100) -> float:
    """Maximum-likelihood kappa by L-BFGS on log kappa with the analytic gradient."""
    k0 = kappa0 if kappa0 is not None else R * (p - R * R) / (1.0 - R * R)
    t = torch.tensor([math.log(k0)], dtype=torch.float64, device=device, requires_grad=True)
    opt = torch.optim.LBFGS([t], lr=1.0, max_iter=max_iter, tolerance_grad=1e-15,
                            tolerance_change=1e-18, history_size=20,
                            line_search_fn="strong_wolfe")

    def closure():
        opt.zero_grad()
        loss = neg_log_likelihood(torch.exp(t), R, p).sum() / p
        loss.backward()
        return loss

    opt.step(closure)
    return float(torch.exp(t).item())
