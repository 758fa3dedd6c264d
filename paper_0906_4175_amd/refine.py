"""Gradient refinement of triggers off the template grid.

A trigger is a bank template (M_c, eta) and a peak time j* dt.  Its statistic
rho^2 is a smooth function F(M_c, eta, t_c) once the frequency band is frozen
at the starting template (F is z(t) of Eq. (1) at continuous t = t_c, squared
and normalised by Eq. (4)).  `refine` climbs F with Newton steps in the
template-space metric g (mf_template_metric: near a maximum
F(theta* + d) ~ F* (1 - d^T g d)), damped Levenberg-Marquardt style when a
step fails.  Chirp mass and eta are
strongly correlated (the metric is nearly singular in their difference), which
plain preconditioned gradient ascent handles poorly.  F and its
gradient come from the hand-written forward and adjoint kernels (mf_snr_grad)
through `SnrSq`, so `torch.autograd.grad` drives the kernels.
"""
from __future__ import annotations

import torch

from . import Grid, SnrSq, filter as mf_filter


def triggers_from_peaks(grid: Grid, bank, stilde: torch.Tensor, Sn: torch.Tensor, mc, eta, n_windows: int = 4,
                        precision: str = "fp32_ph64"):
    """One trigger per template and time window: the window's rho peak.

    The segment is split into n_windows equal windows; windows are at least
    N / n_windows samples apart, so triggers of one template are >= 1 s apart
    for 256 s segments.  Returns theta [n, 3] (M_c, eta, t), k_hi [n], seg [n],
    rho [n] on the stilde device.
    """
    dev = stilde.device
    n = grid.n
    edges = [round(i * n / n_windows) for i in range(n_windows + 1)]
    n_seg = stilde.shape[0] if stilde.dim() == 2 else 1
    thetas, khis, segs, rhos = [], [], [], []
    mc_t = torch.as_tensor(mc, dtype=torch.float64, device=dev)
    eta_t = torch.as_tensor(eta, dtype=torch.float64, device=dev)
    khi_t = torch.as_tensor(bank.k_hi, dtype=torch.int32, device=dev)
    for w in range(n_windows):
        res = mf_filter(grid, bank, stilde, Sn, precision, window=(edges[w], edges[w + 1]))
        for s in range(n_seg):
            t = res["j"][:, s].to(torch.float64) / grid.fs
            thetas.append(torch.stack([mc_t, eta_t, t], dim=1))
            khis.append(khi_t)
            segs.append(torch.full_like(khi_t, s))
            rhos.append(res["rho"][:, s].clone())
    return torch.cat(thetas), torch.cat(khis), torch.cat(segs), torch.cat(rhos)


def rho2_and_grad(grid: Grid, theta: torch.Tensor, seg, stilde, Sn, khi, precision: str = "fp32_ph64"):
    th = theta.detach().clone().requires_grad_(True)
    F = SnrSq.apply(th, grid, seg, stilde, Sn, khi, precision)
    (g,) = torch.autograd.grad(F.sum(), th)
    return F.detach(), g


def _solve3(A: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """Batched 3x3 solve A x = b by cofactors (no library call)."""
    a00, a01, a02 = A[:, 0, 0], A[:, 0, 1], A[:, 0, 2]
    a10, a11, a12 = A[:, 1, 0], A[:, 1, 1], A[:, 1, 2]
    a20, a21, a22 = A[:, 2, 0], A[:, 2, 1], A[:, 2, 2]
    c00 = a11 * a22 - a12 * a21
    c01 = a12 * a20 - a10 * a22
    c02 = a10 * a21 - a11 * a20
    det = a00 * c00 + a01 * c01 + a02 * c02
    inv = torch.stack([
        torch.stack([c00, a02 * a21 - a01 * a22, a01 * a12 - a02 * a11], -1),
        torch.stack([c01, a00 * a22 - a02 * a20, a02 * a10 - a00 * a12], -1),
        torch.stack([c02, a01 * a20 - a00 * a21, a00 * a11 - a01 * a10], -1),
    ], -2) / det[:, None, None]
    return (inv * b[:, None, :]).sum(-1)


def refine(grid: Grid, theta0: torch.Tensor, seg, stilde, Sn, khi, steps: int = 20,
           precision: str = "fp32_ph64"):
    """Newton ascent on F with the template metric; returns (theta, F, evaluations).

    Near a maximum F(theta* + d) ~ F* (1 - d^T g d), so grad F ~ -2 F* g d and
    the step is d = (2 F g)^-1 grad F, shortened so that eta stays in (0, 1/4].
    A step that lowers F is retried with Levenberg-Marquardt damping,
    (2 F (g + lambda diag g))^-1 grad F for lambda = 1e-2 ... 1e3 (each larger
    lambda shortens the step towards a metric-scaled gradient step); the
    trigger keeps its point if all fail.  One evaluation is one forward,
    adjoint or metric pass over every trigger.
    """
    theta = theta0.detach().clone()
    n = theta.shape[0]
    dev = theta.device
    F, g = _eval_grad(grid, theta, seg, stilde, Sn, khi, precision)
    evals = 2
    lambdas = (0.0, 1e-2, 1e-1, 1.0, 10.0, 1e2, 1e3)
    for _ in range(steps):
        G = _metric(grid, theta, Sn, khi)
        evals += 1
        diag = torch.diag_embed(torch.diagonal(G, dim1=1, dim2=2))
        accepted = torch.zeros(n, dtype=torch.bool, device=dev)
        new_theta = theta.clone()
        for lam in lambdas:
            p = _solve3(2.0 * F.clamp_min(1e-30)[:, None, None] * (G + lam * diag), g)
            # keep eta inside (0, 1/4]: cap the step length along p
            pe = p[:, 1]
            cap = torch.where(pe > 0, 0.999 * (0.25 - theta[:, 1]) / pe.clamp_min(1e-300),
                              torch.where(pe < 0, 0.999 * theta[:, 1] / (-pe).clamp_min(1e-300),
                                          torch.ones_like(pe)))
            trial = theta + cap.clamp(max=1.0)[:, None] * p
            Ft = _eval(grid, trial, seg, stilde, Sn, khi, precision)
            evals += 1
            ok = (Ft >= F) & ~accepted & torch.isfinite(Ft)
            new_theta[ok] = trial[ok]
            accepted |= ok
            if bool(accepted.all()):
                break
        if not bool(accepted.any()):
            break
        theta = torch.where(accepted[:, None], new_theta, theta)
        F_new, g_new = _eval_grad(grid, theta, seg, stilde, Sn, khi, precision)
        evals += 2
        F = torch.where(accepted, F_new, F)
        g = torch.where(accepted[:, None], g_new, g)
    return theta, F, evals


def _forward_only(grid, theta, seg, stilde, Sn, khi, precision):
    from . import snr_sq
    return snr_sq(grid, theta, seg, stilde, Sn, khi, precision)


# Objective hooks used by `refine` (module attributes so that the optimiser can
# be exercised on the CPU with an analytic surface).
def _eval(grid, theta, seg, stilde, Sn, khi, precision):
    return _forward_only(grid, theta, seg, stilde, Sn, khi, precision)[0]


def _eval_grad(grid, theta, seg, stilde, Sn, khi, precision):
    return rho2_and_grad(grid, theta, seg, stilde, Sn, khi, precision)


def _metric(grid, theta, Sn, khi):
    from . import template_metric
    return template_metric(grid, theta, Sn, khi)


def finite_difference_grad(grid: Grid, theta: torch.Tensor, seg, stilde, Sn, khi, rel: float = 1e-6,
                           precision: str = "fp32_ph64"):
    """Central differences of F on the GPU: relative steps for M_c, eta; 1e-6 dt for t_c."""
    from . import snr_sq
    h = torch.stack([rel * theta[:, 0], rel * theta[:, 1], torch.full_like(theta[:, 0], rel / grid.fs)], dim=1)
    out = torch.empty_like(theta)
    for q in range(3):
        tp = theta.clone()
        tm = theta.clone()
        tp[:, q] += h[:, q]
        tm[:, q] -= h[:, q]
        Fp = snr_sq(grid, tp, seg, stilde, Sn, khi, precision)[0]
        Fm = snr_sq(grid, tm, seg, stilde, Sn, khi, precision)[0]
        out[:, q] = (Fp - Fm) / (2.0 * h[:, q])
    return out

