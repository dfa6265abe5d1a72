"""The paper's diffusion comparison (Sec. IV.B) on a synthetic volume.

A mass M0 = 592.7593 (mg) of DOM is spread uniformly over the pore voxels of
the first two z-layers; DOM diffuses alone (no transformation) with the
paper's D = 100950 voxel^2/day for 1.76 h; the result is the DOM mass per
z-layer.  Explicit (Scheme 1, 0.1 s steps, Fig. 8) and implicit (Scheme 2,
30 s steps, Figs. 7-8) runs go through the library; the layer profile is a
range sum over the raster-ordered compacted list (every layer is one
contiguous range).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .graph import Graph, layer_offsets, range_sums
from .inputs import ModelParams
from .sim import Simulation

M0 = 592.7593                      # mg on the first two layers
D_VOXEL2_PER_DAY = 100950.0        # the paper's DOM diffusion coefficient
T_END = 1.76 * 3600.0              # s
H = 24e-6                          # m (voxel size; only D / h^2 matters)


def params() -> ModelParams:
    """DOM-only diffusion in SI units: D = (100950 / 86400) voxel^2/s * h^2."""
    d = D_VOXEL2_PER_DAY / 86400.0 * H * H
    return ModelParams(D=(0.0, d, 0.0, 0.0, 0.0), h=H, v_dom=0.0, k_dom=1.0, rho=0.0, mu=0.0, beta=0.0,
                       v_som=0.0, v_p4=0.0)


def initial_fields(mask: np.ndarray, g: Graph, dtype=torch.float64) -> torch.Tensor:
    """[5, n]: DOM = M0 / (pore voxels in layers 0-1) on those voxels."""
    off = layer_offsets(mask)
    k = int(off[2])
    x = torch.zeros((5, g.n), dtype=torch.float64)
    x[1, :k] = M0 / k
    return x.to(device=g.vox.device, dtype=dtype)


def layer_profile(sim: Simulation, mask: np.ndarray) -> np.ndarray:
    """DOM mass per z-layer of the simulation's current state."""
    off = torch.as_tensor(layer_offsets(mask), device=sim.fields.device)
    return range_sums(sim.fields[1], off).cpu().numpy()


def run_explicit(mask, g, dt=0.1, t_end=T_END, precision="f32", kernel=0):
    p = params()
    sim = Simulation(g, p, precision=precision, implicit=False)
    sim.set_kernel(kernel)
    sim.set_fields(initial_fields(mask, g))
    nsteps = int(round(t_end / dt))
    sim.step(nsteps, dt)
    return sim, nsteps


def run_implicit(mask, g, dt=30.0, t_end=T_END, precision="f32", rtol=1e-10, kernel=0, multigrid=False):
    """Whole steps of dt, then one step of the remainder so the run ends at
    t_end; CG preconditioned by the diagonal (the paper's) or, with
    multigrid=True, by the library's multigrid V-cycle."""
    p = params()
    sim = Simulation(g, p, precision=precision, implicit=True, multigrid=multigrid)
    if multigrid:
        sim.set_preconditioner("mg")
    sim.set_kernel(kernel)
    sim.set_fields(initial_fields(mask, g))
    nfull = int(math.floor(t_end / dt + 1e-9))
    its = []
    for _ in range(nfull):
        its.append(sim.implicit_step(dt, rtol=rtol)[0][1])
    rest = t_end - nfull * dt
    if rest > 1e-9 * dt:
        its.append(sim.implicit_step(rest, rtol=rtol)[0][1])
    return sim, its
