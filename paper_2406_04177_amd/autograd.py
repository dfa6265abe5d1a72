"""Gradients of losses on mass-total curves through the explicit time loop.

``simulate_totals(sim, theta, x0, nsteps, dt, checkpoint_every)`` returns the
per-volume pool totals after every step ([nsteps+1, nseg, 5], FP64) as a
differentiable function of

    theta = [D_0..D_4, v_DOM, K_DOM, rho, mu, beta, v_SOM, v_P4, c_0..c_7]

(diffusion coefficients, kinetic rates, region conductance factors; 20
values) and of the initial fields ``x0``.  The backward pass is the library's
hand-written discrete adjoint (``vg_adjoint``) with checkpointed recomputation:
the forward keeps the state at the start of every ``checkpoint_every`` steps;
the backward re-records each segment (``vg_record``) and sweeps it in reverse.
Segments whose recorded states fit ``tape_bytes`` (default:
``default_tape_bytes`` of the free device memory at the forward; 0 turns it
off) are recorded by the forward
itself (``vg_step_record``: the same kernels, bit-identical states and
totals), so the backward sweeps them without running them again; the last
segments are the ones kept, and each is freed once swept.  When only DOM
diffuses, the recordings keep each step's diffused DOM (the adjoint option
``tape_dom``: the totals' CO2 adjoint is uniform over each volume, which it
needs), so the reverse steps need not diffuse again; the gradient is
bit-identical either way.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from .inputs import ModelParams

NTHETA = 20
VG_POOLS = 5
THETA_NAMES = ("D_MB", "D_DOM", "D_SOM", "D_P4", "D_CO2", "v_dom", "k_dom", "rho", "mu", "beta",
               "v_som", "v_p4") + tuple("c%d" % r for r in range(8))


def theta_of(params: ModelParams, c=None) -> torch.Tensor:
    c = [1.0] * 8 if c is None else list(c)
    return torch.tensor(list(params.D) + [params.v_dom, params.k_dom, params.rho, params.mu, params.beta,
                                          params.v_som, params.v_p4] + c, dtype=torch.float64)


def params_of(theta, base: ModelParams) -> tuple:
    t = [float(v) for v in theta.detach().cpu().tolist()]
    p = dataclasses.replace(base, D=tuple(t[0:5]), v_dom=t[5], k_dom=t[6], rho=t[7], mu=t[8], beta=t[9],
                            v_som=t[10], v_p4=t[11])
    return p, t[12:20]


def default_tape_bytes(free: int, seg_bytes: int, total_bytes: int, field_bytes: int, nseg: int) -> int:
    """The forward's recording budget: every segment when all of them fit
    with a tenth of the free memory and the backward's two adjoint field sets
    to spare; else what fits beside those, the checkpoints of the segments
    not recorded (at most nseg field sets) and the one segment's states that
    the backward records again."""
    spare = free // 10 + 2 * field_bytes
    if total_bytes + spare <= free:
        return total_bytes
    return max(0, free - spare - seg_bytes - nseg * field_bytes)


class _TotalsFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, x0, sim, nsteps, dt, K, tape_bytes):
        # recordings and their sweeps take the same option; the caller's is
        # restored afterwards
        ctx.tape_dom = not sim.mobile_all
        prev_tape_dom = sim.adjoint_options["tape_dom"]
        sim.set_adjoint_options(tape_dom=ctx.tape_dom)
        try:
            return _TotalsFn._forward(ctx, theta, x0, sim, nsteps, dt, K, tape_bytes)
        finally:
            sim.set_adjoint_options(tape_dom=prev_tape_dom)

    @staticmethod
    def _forward(ctx, theta, x0, sim, nsteps, dt, K, tape_bytes):
        p, c = params_of(theta, sim.params)
        sim.set_params(p)
        sim.set_regions(c)
        sim.set_fields(x0)
        nseg = sim.nseg
        dev = sim.fields.device
        tot = torch.empty((nsteps + 1, nseg, 6), dtype=torch.float64, device=dev)
        tot[0] = torch.from_numpy(sim.totals()).to(dev)
        ckpts = []
        keep = any(ctx.needs_input_grad[:2])      # no checkpoints when no gradient is wanted
        segs = [(k0, min(K, nsteps - k0)) for k0 in range(0, nsteps, K)]
        # the last segments whose states fit the budget are recorded on the way
        rows = sim.tape_rows
        per_step = rows * sim.graph.n * torch.empty((), dtype=sim.dtype).element_size()
        if tape_bytes is None:
            # free device memory, and what torch's allocator holds unused
            # (e.g. the states buffer of an earlier backward)
            free = 0 if dev.type != "cuda" else (torch.cuda.mem_get_info(dev)[0] + torch.cuda.memory_reserved(dev)
                                                 - torch.cuda.memory_allocated(dev))
            field = VG_POOLS * sim.graph.n * torch.empty((), dtype=sim.dtype).element_size()
            tape_bytes = default_tape_bytes(free, min(K, nsteps) * per_step, nsteps * per_step, field, len(segs))
        taped, budget = set(), int(tape_bytes) if keep else 0
        for k0, k in reversed(segs):
            if k * per_step > budget:
                break
            budget -= k * per_step
            taped.add(k0)
        for k0, k in segs:
            if k0 in taped:
                tape = torch.empty((k, rows, sim.graph.n), dtype=sim.dtype, device=dev)
                sim.step_record(k, dt, tape, tot[k0 + 1:k0 + 1 + k])
                ckpts.append((k0, k, tape))
            else:
                ckpts.append((k0, k, sim.fields.clone() if keep else None))
                sim.step(k, dt, log_every=1, totals_out=tot[k0 + 1:k0 + 1 + k])
        ctx.taped = taped
        sim.last_taped_segments = len(taped)   # for reporting
        ctx.sim, ctx.dt, ctx.ckpts, ctx.nsteps = sim, dt, ckpts, nsteps
        ctx.params, ctx.regions = p, c       # the backward differentiates at this forward's theta
        ctx.theta_device = theta.device
        ctx.x0_dtype = x0.dtype
        return tot[:, :, :5].clone()

    @staticmethod
    def backward(ctx, gout):
        sim = ctx.sim
        prev_tape_dom = sim.adjoint_options["tape_dom"]
        sim.set_adjoint_options(tape_dom=ctx.tape_dom)
        try:
            return _TotalsFn._backward(ctx, gout)
        finally:
            sim.set_adjoint_options(tape_dom=prev_tape_dom)

    @staticmethod
    def _backward(ctx, gout):
        sim, dt = ctx.sim, ctx.dt
        # another forward on the same simulation may have changed its
        # parameters since: re-record at this forward's, restore afterwards
        prev_p, prev_c = sim.params, getattr(sim, "regions", None)
        sim.set_params(ctx.params)
        sim.set_regions(ctx.regions)
        dev = sim.fields.device
        n = sim.graph.n
        seeds = gout.detach().to(device=dev, dtype=torch.float64).contiguous()
        lam = torch.zeros((5, n), dtype=sim.dtype, device=dev)
        sim.seed_lambda(seeds[ctx.nsteps], lam, zero=True)
        grad = torch.zeros(NTHETA, dtype=torch.float64, device=dev)
        kmax = max((k for k0, k, _ in ctx.ckpts if k0 not in ctx.taped), default=0)
        states = torch.empty((kmax, sim.tape_rows, n), dtype=sim.dtype, device=dev) if kmax else None
        for idx in range(len(ctx.ckpts) - 1, -1, -1):
            k0, k, ck = ctx.ckpts[idx]
            if k0 in ctx.taped:
                sim.adjoint(k, dt, ck, seeds[k0:k0 + k], lam, grad)
                ctx.ckpts[idx] = (k0, k, None)   # free the tape once swept
                continue
            sim.set_fields(ck)
            sim.record(k, dt, states)
            sim.adjoint(k, dt, states, seeds[k0:k0 + k], lam, grad)
        sim.set_params(prev_p)
        if prev_c is not None:
            sim.set_regions(prev_c)
        return (grad.to(ctx.theta_device), lam.to(ctx.x0_dtype), None, None, None, None, None)


def simulate_totals(sim, theta: torch.Tensor, x0: torch.Tensor, nsteps: int, dt: float,
                    checkpoint_every: int = 100, tape_bytes=None) -> torch.Tensor:
    """Differentiable [nsteps+1, nseg, 5] totals; see the module docstring."""
    if nsteps < 1 or checkpoint_every < 1:
        raise ValueError("need nsteps >= 1 and checkpoint_every >= 1")
    return _TotalsFn.apply(theta, x0, sim, int(nsteps), float(dt), int(checkpoint_every), tape_bytes)


def co2_mse(totals: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """Mean over (step, volume) of (CO2 total - target)^2."""
    return ((totals[:, :, 4] - target) ** 2).mean()
