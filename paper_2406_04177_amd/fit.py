"""Fitting the parameters of the explicit loop to target curves.

The gradient of the loss comes from the library's discrete adjoint
(``autograd.simulate_totals``, checkpointed); the update is the paper's
stochastic gradient descent with a normalised gradient (Sec. V.A): each
fitted parameter moves by the learning rate against the sign of its own
derivative, the learning rate starting at 0.1 and halved every 10 epochs
(Sec. V.B), applied on the device by ``vg_sign_update``.  The step is taken
in units of the parameter's starting value,
so factors that start at 1 (the region conductances) move exactly as in the
paper, while diffusion coefficients and rates move by the same fraction of
themselves; a derivative of exactly zero gives no move.  After each update a
fitted parameter is held inside ``box`` times its starting value (default
[0.5, 1.5]), so that a fixed time step chosen for the box stays below the
explicit stability bound.  ``method="adam"`` runs Adam on the same scaled
coordinates instead (torch's optimiser: an option outside the paper).

The loss is the mean over (step, volume) of the squared difference between
the per-volume CO2 total and the target curve; an epoch uses every volume, or
the subset of volumes given for it (``inputs.epoch_subsets``).
"""
from __future__ import annotations

import numpy as np
import torch

from .autograd import simulate_totals
from .pngm import sign_update


def epoch_loss(sim, theta, x0, target, nsteps, dt, checkpoint_every, vols=None):
    """Differentiable loss of one epoch ([nsteps+1, nvol] target, CUDA)."""
    tot = simulate_totals(sim, theta, x0, nsteps, dt, checkpoint_every)
    if vols is None:
        return ((tot[:, :, 4] - target) ** 2).mean()
    idx = torch.as_tensor(np.asarray(vols), device=tot.device)
    return ((tot[:, idx, 4] - target[:, idx]) ** 2).mean()


def fit(sim, x0, target, theta0, nsteps, dt, which, epochs=30, checkpoint_every=100, lr=0.1,
        halve_every=10, subsets=None, method="sign", box=(0.5, 1.5)):
    """Returns (theta history [epochs+1, 20] FP64, loss history [epochs])."""
    theta = theta0.detach().to(torch.float64).cpu().clone()
    scale = theta.clone()
    lo = scale * box[0]
    hi = scale * box[1]
    which = list(which)
    dev = x0.device
    scale_d, lo_d, hi_d = scale.to(dev), lo.to(dev), hi.to(dev)
    hist, losses = [theta.clone()], []
    u = torch.ones(len(which), dtype=torch.float64, requires_grad=True)   # Adam's coordinates
    opt = torch.optim.Adam([u], lr=lr) if method == "adam" else None
    for e in range(epochs):
        rate = lr * 0.5 ** (e // halve_every)
        th = theta.clone().requires_grad_(True)
        vols = None if subsets is None else subsets[e]
        loss = epoch_loss(sim, th, x0, target, nsteps, dt, checkpoint_every, vols)
        loss.backward()
        g = th.grad.detach()
        losses.append(float(loss.detach()))
        if method == "sign":
            # the parameters not fitted get a zero derivative: no move
            g_fit = torch.zeros_like(g)
            g_fit[which] = g[which]
            theta_d = theta.to(dev)
            sign_update(theta_d, g_fit.to(dev).contiguous(), rate, scale_d, lo_d, hi_d)
            theta = theta_d.cpu()
        elif method == "adam":
            for group in opt.param_groups:
                group["lr"] = rate
            opt.zero_grad()
            u.grad = torch.stack([g[q] * scale[q] for q in which])
            opt.step()
            with torch.no_grad():
                for k, q in enumerate(which):
                    theta[q] = scale[q] * u[k].detach()
        else:
            raise ValueError("method must be 'sign' or 'adam'")
        if method == "adam":
            for q in which:
                theta[q] = min(max(float(theta[q]), float(lo[q])), float(hi[q]))
            with torch.no_grad():
                for k, q in enumerate(which):
                    u[k] = theta[q] / scale[q]
        hist.append(theta.clone())
    return torch.stack(hist).numpy(), np.array(losses)
