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
the subset of volumes given for it (``inputs.epoch_subsets``).  Options: other
curves (e.g. DOM and CO2, each divided by a scale) and finer segments (the
eight octants of every volume, ``octant_segments``), on which the region
factors act separately.  D_DOM and the region factors enter the model only as
the products D_DOM c_r (the edge weights scale D), so no loss on the totals
separates them: ``sensitivity`` / ``identifiability`` show which parameter
combinations a loss sees.

``gauss_newton`` is a refinement outside the paper: Gauss-Newton on the
logarithms of the fitted parameters for the same least-squares misfit, with
the Jacobian from central differences of the forward run and a truncated
SVD solve, so that directions the curves cannot see (such as the common scale
of D_DOM and the region factors) are left where they are.  With the FP64
forward it recovers combinations that the sign-normalised SGD leaves
barely moved because the loss is nearly flat along them.
"""
from __future__ import annotations

import numpy as np
import torch

from .autograd import simulate_totals
from .pngm import sign_update


def octant_segments(graph) -> np.ndarray:
    """Segment offsets [nvol * 8 + 1] that split every volume of a graph into
    its eight octants, for graphs whose compacted lists are octant-major:
    cubic volumes of even side N enumerated in bricks of side N / 2 (brick
    k of a volume is then octant k, 4 [z >= N/2] + 2 [y >= N/2] + [x >= N/2]).
    The per-segment totals of a simulation given these segments are the
    octant totals (the counts come from the library's region codes)."""
    nz, ny, nx = graph.shape
    if not (nx == ny == nz and nx % 2 == 0 and graph.brick == nx // 2):
        raise ValueError("octant segments need cubic volumes of even side N in bricks of side N / 2")
    codes = graph.rcode if graph.rcode is not None else graph.make_region_codes()
    octant = (codes.to(torch.int64) & 7)
    vol = torch.repeat_interleave(torch.arange(graph.nseg, device=octant.device),
                                  torch.as_tensor(np.diff(graph.seg_off), device=octant.device))
    counts = torch.bincount(vol * 8 + octant, minlength=graph.nseg * 8).cpu().numpy()
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    # octant-major inside each volume: the boundaries of the volumes are kept
    assert np.array_equal(off[::8], graph.seg_off)
    return off


def segments_of(vols, per_vol: int):
    """Segments of the given volumes when each volume has `per_vol` segments."""
    return np.concatenate([np.arange(v * per_vol, (v + 1) * per_vol) for v in np.asarray(vols)])


def curves_loss(tot, target, curves=(4,), scale=None, segs=None):
    """Mean over (step, segment, curve) of ((total - target) / scale)^2:
    tot [nsteps+1, nseg, 5] totals, target [nsteps+1, nseg] (one curve) or
    [nsteps+1, nseg, len(curves)], scale one factor per curve (or None)."""
    sel = tot[:, :, list(curves)]
    if target.dim() == 2:
        target = target[:, :, None]
    d = sel - target
    if scale is not None:
        d = d / torch.as_tensor(scale, dtype=d.dtype, device=d.device)
    if segs is not None:
        d = d[:, torch.as_tensor(np.asarray(segs), device=d.device)]
    return (d ** 2).mean()


def epoch_loss(sim, theta, x0, target, nsteps, dt, checkpoint_every, vols=None, curves=(4,), scale=None,
               segs_per_vol=1):
    """Differentiable loss of one epoch (target on the device: [nsteps+1,
    nseg] for the CO2 curve alone, else [nsteps+1, nseg, len(curves)]);
    with `segs_per_vol` segments per volume (8: octants), `vols` selects
    whole volumes."""
    tot = simulate_totals(sim, theta, x0, nsteps, dt, checkpoint_every)
    segs = None if vols is None else segments_of(vols, segs_per_vol)
    return curves_loss(tot, target, curves, scale, segs)


def sensitivity(sim, theta, x0, nsteps, dt, which, curves=(4,), scale=None, rel_eps=1e-4, checkpoint_every=100):
    """Sensitivity of the totals curves (every step and segment, divided by
    `scale` per curve) to the logarithm of each parameter in `which`, by
    central differences of the forward run: J [n_outputs, len(which)].  Its
    singular values tell which parameter combinations a loss on these curves
    identifies (a zero singular value: a direction the curves cannot see)."""
    cols = []
    with torch.no_grad():
        for q in which:
            tp, tm = theta.clone(), theta.clone()
            h = rel_eps * float(theta[q])
            tp[q] += h
            tm[q] -= h
            up = simulate_totals(sim, tp, x0, nsteps, dt, checkpoint_every)[:, :, list(curves)]
            dn = simulate_totals(sim, tm, x0, nsteps, dt, checkpoint_every)[:, :, list(curves)]
            d = (up - dn) / (2 * rel_eps)
            if scale is not None:
                d = d / torch.as_tensor(scale, dtype=d.dtype, device=d.device)
            cols.append(d.reshape(-1))
    return torch.stack(cols, 1)


def identifiability(J, names):
    """Singular values of J (descending, relative to the largest) and, for
    the smallest, the parameter direction (unit vector over `names`)."""
    U, S, Vh = torch.linalg.svd(J.to(torch.float64), full_matrices=False)
    s = (S / S[0]).cpu().numpy()
    weakest = Vh[-1].cpu().numpy()
    return s, dict(zip(names, map(float, weakest)))


def fit(sim, x0, target, theta0, nsteps, dt, which, epochs=30, checkpoint_every=100, lr=0.1,
        halve_every=10, subsets=None, method="sign", box=(0.5, 1.5), curves=(4,), curve_scale=None, segs_per_vol=1):
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
        loss = epoch_loss(sim, th, x0, target, nsteps, dt, checkpoint_every, vols, curves, curve_scale, segs_per_vol)
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


def lstsq_step(J: torch.Tensor, r: torch.Tensor, rcond: float = 1e-9):
    """The least-squares step d minimising |J d + r| over the span of the
    right singular vectors of J whose singular value is at least rcond times
    the largest (zero along the others).  Returns (d, relative singular
    values)."""
    U, S, Vh = torch.linalg.svd(J.to(torch.float64), full_matrices=False)
    keep = S >= S[0] * rcond
    d = -(Vh[keep].T @ ((U[:, keep].T @ r.to(torch.float64)) / S[keep]))
    return d, (S / S[0])


def gauss_newton(sim, theta0, x0, target, nsteps, dt, which, curves=(4,), scale=None, iters=3, rel_eps=1e-4,
                 rcond=1e-9, checkpoint_every=100, box=(0.5, 1.5)):
    """Gauss-Newton on log(theta[q]) for q in `which`, for the residual
    (totals[:, :, curves] - target) / scale over every step and segment:
    the Jacobian by central differences of the forward run (step rel_eps in
    each log-parameter, two runs per parameter), the step by ``lstsq_step``,
    each parameter then held inside box times its start.  Returns (theta
    history [iters + 1, 20] FP64, squared residual norm per iterate)."""
    theta = theta0.detach().to(torch.float64).cpu().clone()
    lo, hi = theta * box[0], theta * box[1]
    which = list(which)
    if target.dim() == 2:
        target = target[:, :, None]
    sc = None if scale is None else torch.as_tensor(scale, dtype=torch.float64, device=target.device)

    def resid(th):
        with torch.no_grad():
            d = simulate_totals(sim, th, x0, nsteps, dt, checkpoint_every)[:, :, list(curves)].to(torch.float64)
            d = d - target.to(torch.float64)
            if sc is not None:
                d = d / sc
            return d.reshape(-1)

    hist, norms = [theta.clone()], []
    for it in range(iters + 1):
        r = resid(theta)
        norms.append(float(r @ r))
        if it == iters:
            break
        cols = []
        for q in which:
            tp, tm = theta.clone(), theta.clone()
            tp[q] *= float(np.exp(rel_eps))
            tm[q] *= float(np.exp(-rel_eps))
            cols.append((resid(tp) - resid(tm)) / (2 * rel_eps))
        d, _ = lstsq_step(torch.stack(cols, 1), r, rcond)
        d = d.cpu()
        for k, q in enumerate(which):
            theta[q] = min(max(float(theta[q]) * float(np.exp(float(d[k]))), float(lo[q])), float(hi[q]))
        hist.append(theta.clone())
    return torch.stack(hist).numpy(), np.array(norms)
