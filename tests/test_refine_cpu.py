"""The refinement optimiser on an analytic, strongly correlated surface (CPU)."""
import torch

from paper_0906_4175_amd import refine as R


def test_metric_newton_ascent_converges_on_correlated_peak(monkeypatch):
    # F = 200 exp(-1/2 (x - x*)^T A (x - x*)), A in the preconditioned units of
    # (M_c, eta, t_c) with a 0.999 correlation between the first two.
    xs = torch.tensor([[1.2, 0.24, 10.0], [2.0, 0.2, 3.0]], dtype=torch.float64)
    d = torch.tensor([1e-3, 1e-3, 1e-4], dtype=torch.float64)
    C = torch.tensor([[1.0, 0.999, 0.3], [0.999, 1.0, 0.3], [0.3, 0.3, 1.0]], dtype=torch.float64)
    A = torch.linalg.inv(C)

    def F_of(theta):
        z = (theta - xs) / (d * torch.stack([xs[:, 0], torch.ones(2, dtype=torch.float64),
                                            torch.ones(2, dtype=torch.float64)], 1))
        return 200.0 * torch.exp(-0.5 * ((z @ A) * z).sum(1)), z

    def ev(grid, theta, *a):
        return F_of(theta)[0]

    def evg(grid, theta, *a):
        th = theta.detach().clone().requires_grad_(True)
        F, _ = F_of(th)
        (g,) = torch.autograd.grad(F.sum(), th)
        return F.detach(), g

    def met(grid, theta, *a):
        # exact metric of the surface: F ~ F*(1 - 1/2 z^T A z), z = (theta - x*)/scale
        sc = d * torch.stack([xs[:, 0], torch.ones(2, dtype=torch.float64), torch.ones(2, dtype=torch.float64)], 1)
        return 0.5 * A[None] / (sc[:, :, None] * sc[:, None, :])

    monkeypatch.setattr(R, "_eval", ev)
    monkeypatch.setattr(R, "_eval_grad", evg)
    monkeypatch.setattr(R, "_metric", met)
    theta0 = xs + torch.tensor([[1.5e-3 * 1.2, 1.2e-3, -1.2e-4], [-1e-3 * 2.0, -0.8e-3, 0.9e-4]],
                               dtype=torch.float64)
    F0 = F_of(theta0)[0]
    theta, F, evals = R.refine(None, theta0, None, None, None, None, steps=20)
    assert bool((F > F0).all())
    assert bool((F > 0.999 * 200.0).all()), F
    assert evals >= 2
