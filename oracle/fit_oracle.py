"""Oracle of the parameter fitting driven by the discrete adjoint.

TEST INFRASTRUCTURE ONLY (callers: the test suite).  Plain FP64 CPU code on
top of ``oracle.py``; shares nothing with the HIP path.

What is fitted: the parameters of the explicit loop (region conductance
factors, diffusion coefficients, rates) so that the per-volume CO2 total
curves match target curves, loss = mean over (step, volume) of the squared
difference.  The update is the paper's stochastic gradient descent with a
normalised gradient (Sec. V.A): every fitted parameter moves by the learning
rate against the sign of its own derivative; the learning rate starts at 0.1
and is halved every 10 epochs (Sec. V.B).  Readings (the paper fits O(1)
conductances): the step is taken in units of each parameter's starting value
(theta_q <- theta_q - lr * theta0_q * sign(dL/dtheta_q)), which leaves
factors that start at 1 exactly as in the paper; a derivative of exactly
zero gives no move; after each update a fitted parameter is held inside a
box of its starting value (default [0.5, 1.5] times it: a fixed time step
chosen for the box stays stable); each epoch uses the whole batch of volumes, or the
subset of volumes given for that epoch (drawn by the caller, e.g.
``inputs.epoch_subsets``), and only their curves enter the loss.  Options:
other pools' curves (each divided by a scale) and one segment per octant of
every volume (``octant_graph``).
"""
from __future__ import annotations

import numpy as np

from . import oracle as orc

NTHETA = 20


def theta_to_params(theta, base):
    """[D0..D4, v_dom, k_dom, rho, mu, beta, v_som, v_p4, c0..c7] -> (params, c)."""
    t = [float(v) for v in theta]
    p = base.replace(D=tuple(t[0:5]), v_dom=t[5], k_dom=t[6], rho=t[7], mu=t[8], beta=t[9],
                     v_som=t[10], v_p4=t[11])
    return p, t[12:20]


def octant_graph(og):
    """The same graph with one segment per (volume, octant), for compacted
    lists that are octant-major inside each volume (bricks of half the side
    of a cubic volume); checks that order."""
    nz, ny, nx = og.shape
    v = og.vox.astype(np.int64)
    oct_ = 4 * (v // (nx * ny) >= nz // 2) + 2 * ((v // nx) % ny >= ny // 2) + (v % nx >= nx // 2)
    vol = np.repeat(np.arange(og.nseg), np.diff(og.seg_off))
    key = vol * 8 + oct_
    if np.any(np.diff(key) < 0):
        raise ValueError("the compacted list is not octant-major inside each volume")
    counts = np.bincount(key, minlength=og.nseg * 8)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return orc.OracleGraph(og.shape, og.vox, og.nbr, off)


def loss_and_gradient(theta, base, dt, og, x0, target, vols=None, curves=(4,), scale=None, segs_per_vol=1):
    """Loss and its gradient with respect to the 20 parameters, by the
    oracle's discrete adjoint over the whole run (all states kept).  The loss
    is the mean over (step, segment, curve) of ((T - target) / scale)^2 for
    the pools in `curves` (default: the CO2 total alone, target
    [nsteps+1][nseg]; else target [nsteps+1][nseg][len(curves)]); `vols`
    selects whole volumes of `segs_per_vol` segments each."""
    p, c = theta_to_params(theta, base)
    reg = orc.octant_regions(og)
    w = orc.edge_weights(og, reg, c)
    nsteps = target.shape[0] - 1
    states = orc.run_states(p, dt, og, x0, nsteps, w=w)
    tot = np.stack([orc.totals(og, states[t]) for t in range(nsteps + 1)])
    curves = list(curves)
    tgt = target if target.ndim == 3 else target[:, :, None]
    sc = np.ones(len(curves)) if scale is None else np.asarray(scale, np.float64)
    if vols is None:
        segs = np.arange(og.nseg)
    else:
        segs = np.concatenate([np.arange(v * segs_per_vol, (v + 1) * segs_per_vol) for v in np.asarray(vols)])
    diff = (tot[:, segs][:, :, curves] - tgt[:, segs]) / sc
    loss = float(np.mean(diff ** 2))
    seeds = np.zeros((nsteps + 1, og.nseg, 5))
    for k, s in enumerate(curves):
        seeds[:, segs, s] = 2.0 * diff[:, :, k] / sc[k] / diff.size
    _, grad = orc.adjoint(p, dt, og, states, seeds, w=w, region=reg, nreg=8)
    return loss, grad


def sign_sgd(theta0, grad_fn, epochs, which, lr=0.1, halve_every=10, box=(0.5, 1.5)):
    """Normalised-gradient descent: returns (theta history [epochs+1][20],
    loss history [epochs]); grad_fn(theta, epoch) -> (loss, gradient)."""
    theta = np.array(theta0, np.float64)
    scale = np.array(theta0, np.float64)
    lo, hi = scale * box[0], scale * box[1]
    hist, losses = [theta.copy()], []
    for e in range(epochs):
        rate = lr * 0.5 ** (e // halve_every)
        loss, g = grad_fn(theta, e)
        losses.append(loss)
        for q in which:
            if g[q] > 0:
                theta[q] -= rate * scale[q]
            elif g[q] < 0:
                theta[q] += rate * scale[q]
            theta[q] = min(max(theta[q], lo[q]), hi[q])
        hist.append(theta.copy())
    return np.array(hist), np.array(losses)


def fit(theta0, base, dt, og, x0, target, epochs, which, lr=0.1, halve_every=10, subsets=None, box=(0.5, 1.5),
        curves=(4,), scale=None, segs_per_vol=1):
    """The fitting loop on the oracle; see the module docstring."""

    def grad_fn(theta, epoch):
        vols = None if subsets is None else subsets[epoch]
        return loss_and_gradient(theta, base, dt, og, x0, target, vols, curves, scale, segs_per_vol)

    return sign_sgd(theta0, grad_fn, epochs, which, lr, halve_every, box)
