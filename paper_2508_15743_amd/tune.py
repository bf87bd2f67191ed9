"""Fitting decoder parameters with the differentiable decoder.

The soft-syndrome loss of K unrolled min-sum iterations (Graph.bp_grad,
computed by the gradient kernel) is minimised over the channel LLRs lambda
and one min-sum scaling factor shared by every iteration, with Adam on the
device.  The result can be turned into a decoder graph: priors
p_v = 1 / (1 + exp(lambda_v)) and the fitted scaling factor.  The paper
trains nothing; whether the fitted decoder is better is for the caller to
measure against the untuned one.

The loss is continuous and piecewise smooth (min, sign and clamp), and its
pieces shrink quickly with the number of unrolled iterations: on the d = 5
circuit graph Adam lowers the loss of 8 iterations steadily, while at 20
iterations no step size tried made it descend.  The fit therefore returns
the parameters of the lowest loss it evaluated.
"""
from __future__ import annotations

import numpy as np


def fit(graph, syndromes, K, steps=30, lr_lam=0.01, lr_alpha=0.003, lam0=None, alpha0=0.625,
        alpha_range=(0.05, 1.0), eps=1e-7):
    """Minimise the loss of `graph` (its members and schedule) on device
    syndromes uint8 [B, m].  Returns (lam float64 [n], alpha float, losses):
    the parameters of the lowest loss seen, and the per-shot loss before
    each step and after the last."""
    import torch

    from . import bp_loss

    dev = syndromes.device
    B = syndromes.shape[0]
    if lam0 is None:
        raise ValueError("lam0 (the starting channel LLRs) is required")
    lam = torch.tensor(np.asarray(lam0, np.float64), dtype=torch.float32, device=dev, requires_grad=True)
    a = torch.tensor([float(alpha0)], dtype=torch.float32, device=dev, requires_grad=True)
    opt = torch.optim.Adam([{"params": [lam], "lr": lr_lam}, {"params": [a], "lr": lr_alpha}])
    losses = []
    best = (float("inf"), None, None)

    def keep(value):
        nonlocal best
        losses.append(value)
        if value < best[0]:
            best = (value, lam.detach().double().cpu().numpy(), float(a.item()))

    for _ in range(steps):
        opt.zero_grad()
        loss = bp_loss(graph, syndromes, lam, a.expand(K), eps)
        keep(float(loss.item()) / B)
        loss.backward()
        opt.step()
        with torch.no_grad():
            a.clamp_(*alpha_range)
            lam.clamp_(min=1e-3)
    with torch.no_grad():
        keep(float(bp_loss(graph, syndromes, lam, a.expand(K), eps).item()) / B)
    return best[1], best[2], losses


def priors_from_llr(lam):
    """p_v = 1 / (1 + exp(lambda_v)), the priors whose channel LLRs are lam."""
    lam = np.asarray(lam, np.float64)
    return 1.0 / (1.0 + np.exp(lam))
