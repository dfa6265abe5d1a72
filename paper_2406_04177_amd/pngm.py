"""Pore-network (PNGM) conductances from voxel-method data (Sec. V).

Primitives are the bricks of side b of the image (pore voxels of one brick);
their graph, volumes, contact surfaces and centre distances are assembled on
the device by ``vg_pngm_partition`` from the voxel graph; the data pairs (X^p, Y^p) are
primitive masses of voxel-method diffusion runs taken dt apart (range sums
over a brick-ordered compacted list, where each brick is one contiguous
range); the objective (L1 or L2) and its gradient come from
``vg_pngm_loss_grad``; the parameters are fitted with the normalised-gradient
SGD of Sec. V (``vg_sign_update``) starting from theta = S / d; the fitted
network is run with the explicit PNGM scheme (``vg_pngm_step``).
Readings are those of the library header (inner term x_j / v_j, one theta per
ordered pair, the minus sign of dL2/dtheta)."""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import _lib, inputs
from .graph import Graph, range_sums
from .sim import Simulation


@dataclasses.dataclass
class Partition:
    b: int
    q: int
    v: torch.Tensor          # [q] FP64 pore voxels per primitive
    row: torch.Tensor        # [q+1] int64
    col: torch.Tensor        # [E] int32
    S: np.ndarray            # [E] contact faces
    d: np.ndarray            # [E] centre distance (voxels)
    offsets: torch.Tensor    # [q+1] int64: primitive ranges of the brick-ordered list
    bricks: np.ndarray       # [q] brick index of each primitive


def partition(g: Graph, b: int) -> Partition:
    """The brick partition of a single, non-periodic volume whose compacted
    list is brick-ordered with bricks of side b (assembled by
    ``vg_pngm_partition``; the outputs are allocated at their capacities
    and cut to q primitives and E edges)."""
    if g.nseg != 1 or g.periodic or g.brick != b:
        raise ValueError("need one volume, no periodic axis, brick order with bricks of side b")
    L = _lib.load()
    nz, ny, nx = g.shape
    wb, mp, me = ctypes.c_size_t(0), ctypes.c_int64(0), ctypes.c_int64(0)
    _lib.check(L.vg_pngm_partition_bytes(nx, ny, nz, b, ctypes.byref(wb), ctypes.byref(mp), ctypes.byref(me)),
               "vg_pngm_partition_bytes")
    dev = g.vox.device
    f64, i64, i32 = torch.float64, torch.int64, torch.int32
    work = torch.empty(wb.value, dtype=torch.uint8, device=dev)
    v = torch.empty(mp.value, dtype=f64, device=dev)
    offsets = torch.empty(mp.value + 1, dtype=i64, device=dev)
    bricks = torch.empty(mp.value, dtype=i32, device=dev)
    row = torch.empty(mp.value + 1, dtype=i64, device=dev)
    col = torch.empty(max(me.value, 1), dtype=i32, device=dev)
    S = torch.empty(max(me.value, 1), dtype=f64, device=dev)
    d = torch.empty(max(me.value, 1), dtype=f64, device=dev)
    q, e = ctypes.c_int64(0), ctypes.c_int64(0)
    _lib.check(L.vg_pngm_partition(g.vox.data_ptr(), g.nbr.data_ptr(), g.n, nx, ny, nz, b, work.data_ptr(), wb.value,
                                   v.data_ptr(), offsets.data_ptr(), bricks.data_ptr(), row.data_ptr(), col.data_ptr(),
                                   S.data_ptr(), d.data_ptr(), ctypes.byref(q), ctypes.byref(e),
                                   _lib.stream_ptr(None)), "vg_pngm_partition")
    q, e = q.value, e.value
    return Partition(b, q, v[:q].clone(), row[:q + 1].clone(), col[:e].clone(), S[:e].cpu().numpy(),
                     d[:e].cpu().numpy(), offsets[:q + 1].clone(), bricks[:q].cpu().numpy().astype(np.int64))


def primitive_masses(part: Partition, m: torch.Tensor) -> torch.Tensor:
    """[q] FP64 masses per primitive of a voxel field (brick-ordered list)."""
    return range_sums(m, part.offsets)


def loss_grad(part: Partition, X: torch.Tensor, Y: torch.Tensor, theta: torch.Tensor, c: float, objective: int):
    L = _lib.load()
    X = X.contiguous()
    Y = Y.contiguous()
    lq = X.shape[0]
    rowloss = torch.empty(part.q, dtype=torch.float64, device=X.device)
    loss = torch.empty(1, dtype=torch.float64, device=X.device)
    grad = torch.empty_like(theta)
    _lib.check(L.vg_pngm_loss_grad(X.data_ptr(), Y.data_ptr(), lq, part.q, part.v.data_ptr(), part.row.data_ptr(),
                                   part.col.data_ptr(), theta.data_ptr(), float(c), int(objective),
                                   rowloss.data_ptr(), loss.data_ptr(), grad.data_ptr(), _lib.stream_ptr(None)),
               "vg_pngm_loss_grad")
    return loss, grad


def step(part: Partition, m: torch.Tensor, theta: torch.Tensor, c: float) -> torch.Tensor:
    L = _lib.load()
    out = torch.empty_like(m)
    _lib.check(L.vg_pngm_step(m.data_ptr(), out.data_ptr(), part.q, part.v.data_ptr(), part.row.data_ptr(),
                              part.col.data_ptr(), theta.data_ptr(), float(c), _lib.stream_ptr(None)), "vg_pngm_step")
    return out


def implicit_step(part: Partition, m: torch.Tensor, theta: torch.Tensor, c: float, rtol: float = 1e-12,
                  max_iter: int = 20000, work: torch.Tensor = None):
    """One implicit PNGM step (scheme 4); returns (masses, sweeps, relative residual)."""
    L = _lib.load()
    out = torch.empty_like(m)
    if work is None:
        work = torch.empty(3 * part.q + 2, dtype=torch.float64, device=m.device)
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    _lib.check(L.vg_pngm_implicit_step(m.data_ptr(), out.data_ptr(), part.q, part.v.data_ptr(), part.row.data_ptr(),
                                       part.col.data_ptr(), theta.data_ptr(), float(c), float(rtol), int(max_iter),
                                       work.data_ptr(), ctypes.byref(it), ctypes.byref(rel), _lib.stream_ptr(None)),
               "vg_pngm_implicit_step")
    return out, it.value, rel.value


def sign_update(theta, grad, lr, scale, lo, hi):
    L = _lib.load()
    _lib.check(L.vg_sign_update(theta.data_ptr(), grad.data_ptr(), theta.numel(), float(lr), scale.data_ptr(),
                                lo.data_ptr(), hi.data_ptr(), _lib.stream_ptr(None)), "vg_sign_update")


def pngm_params(dt_vga: float = 0.1) -> inputs.ModelParams:
    """DOM-only diffusion with the paper's D = 100950 voxel^2/day (voxel units)."""
    d = 100950.0 / 86400.0
    return inputs.ModelParams(D=(0.0, d, 0.0, 0.0, 0.0), h=1.0, v_dom=0.0, k_dom=1.0, rho=0.0, mu=0.0, beta=0.0,
                              v_som=0.0, v_p4=0.0)


def generate(g: Graph, part: Partition, mask: np.ndarray, scenarios, records: int, every_s: float,
             dt_vga: float = 0.1, precision: str = "f64"):
    """Voxel-method runs from each scenario's initial DOM: primitive masses at
    t = 0, every_s, ..., records * every_s.  Returns [scenarios, records+1, q]."""
    p = pngm_params()
    sim = Simulation(g, p, precision=precision, implicit=False)
    nper = int(round(every_s / dt_vga))
    out = torch.empty((len(scenarios), records + 1, part.q), dtype=torch.float64, device=g.vox.device)
    for k, seed in enumerate(scenarios):
        sim.set_fields(g.fields_from_specs(inputs.init_scenario(mask, seed), torch.float64))
        out[k, 0] = primitive_masses(part, sim.fields[1])
        for r in range(records):
            sim.step(nper, dt_vga)
            out[k, r + 1] = primitive_masses(part, sim.fields[1])
    return out


def fit(part: Partition, X: torch.Tensor, Y: torch.Tensor, c: float, epochs: int, batch: int = 4, lr: float = 0.1,
        halve_every: int = 10, objective: int = 2, seed: int = 0, box=(0.05, 20.0), theta0=None, record=False):
    """Normalised-gradient SGD on theta from theta0 = S / d: each epoch draws
    `batch` data pairs (default_rng(seed)), steps by lr (halved every
    `halve_every` epochs) in units of theta0, held within box * theta0.
    Returns (theta, loss per epoch on its batch[, theta per epoch, batches])."""
    dev = X.device
    t0 = torch.as_tensor(part.S / part.d, dtype=torch.float64, device=dev) if theta0 is None else theta0.clone()
    theta = t0.clone()
    lo, hi = t0 * box[0], t0 * box[1]
    rng = np.random.default_rng(seed)
    losses, hist, batches = [], [theta.cpu().numpy()] if record else [], []
    for e in range(epochs):
        sel = np.sort(rng.choice(X.shape[0], size=min(batch, X.shape[0]), replace=False))
        idx = torch.as_tensor(sel, device=dev)
        loss, g = loss_grad(part, X[idx], Y[idx], theta, c, objective)
        losses.append(loss)
        sign_update(theta, g, lr * 0.5 ** (e // halve_every), t0, lo, hi)
        if record:
            hist.append(theta.cpu().numpy())
            batches.append(sel)
    if record:
        return theta, torch.cat(losses).cpu().numpy(), np.array(hist), batches
    return theta, torch.cat(losses).cpu().numpy()
