"""Degenerate volumes (single voxels, single rows, planes or columns, raw
random masks down to one pore voxel): every neighbour source, the band
kernel where it can be chosen, and the implicit step, against the oracle."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2406_04177_amd import inputs

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1), (1, 5, 7), (3, 1, 9), (2, 2, 2), (5, 9, 1), (40, 3, 2), (7, 17, 3), (4, 8, 64), (9, 9, 9),
          (1, 40, 40), (33, 1, 1), (6, 65, 5)]
RELATIVE, BAND = 4, 5


def masks():
    rng = np.random.default_rng(5)
    for shape in SHAPES:
        for por in (0.3, 0.7, 1.0):
            mask = (rng.random(shape) < por).astype(np.uint8)
            if mask.sum():
                yield shape, por, mask


def params():
    return inputs.ModelParams(v_dom=0.05, k_dom=0.5, rho=0.01, mu=0.02, v_som=0.01, v_p4=0.02)


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_explicit_every_source(precision):
    from paper_2406_04177_amd import _lib
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    p = params()
    dt = inputs.explicit_dt(p, 0.9)
    for shape, por, mask in masks():
        print("explicit", precision, shape, por, flush=True)
        g = Graph.from_masks(mask)
        spec = inputs.init_random_all(mask, 2)
        og = orc.build_graph(mask)
        ref, _ = orc.run(p, dt, og, orc.fields_from_spec(og, spec), 9, with_totals=False)
        outs = {}
        for kernel in (1, 2, 3, RELATIVE, BAND):
            sim = Simulation(g, p, precision=precision, implicit=False)
            try:
                sim.set_kernel(kernel)
            except _lib.VgError:
                assert kernel == BAND, (shape, kernel)   # the band kernel may decline a volume
                continue
            sim.set_fields(g.fields_from_specs(spec, torch.float64))
            sim.step(9, dt)
            outs[kernel] = sim.fields.cpu().numpy().astype(np.float64)
        for kernel, got in outs.items():
            if precision == "f64":
                assert np.array_equal(got, ref), (shape, por, kernel)
            else:
                np.testing.assert_array_equal(got, outs[1], err_msg=str((shape, por, kernel)))
                np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-6 * np.abs(ref).max())


def test_implicit_step():
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    p = inputs.ModelParams(mu=1e-4, rho=5e-5)
    dt = 20 * inputs.explicit_dt(p, 1.0)
    a = p.D[1] * dt / p.h ** 2
    for shape, por, mask in masks():
        print("implicit", shape, por, flush=True)
        g = Graph.from_masks(mask)
        spec = inputs.init_random_all(mask, 4)
        og = orc.build_graph(mask)
        sim = Simulation(g, p, precision="f64", implicit=True)
        sim.set_fields(g.fields_from_specs(spec, torch.float64))
        its, rel, rc = sim.implicit_step(dt, rtol=1e-12)
        assert rc == 0, (shape, por)
        got = sim.fields.cpu().numpy()
        b = orc.transform(p, dt, orc.fields_from_spec(og, spec))[1]
        res = np.linalg.norm(b - orc.apply_B(a, og, got[1]))
        assert res <= 2e-12 * np.linalg.norm(b) + 1e-300, (shape, por, res)


def test_adjoint_fp64_batch_of_degenerate_volumes():
    """A batch of degenerate volumes of one shape (a single pore voxel, a
    column, a row, a plane, a 2^3 cube, isolated voxels, an empty volume)
    through the checkpointed FP64 adjoint with region factors: totals,
    dL/dx0 and the parameter gradient against the oracle's discrete adjoint."""
    from paper_2406_04177_amd.autograd import simulate_totals, theta_of
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    rng = np.random.default_rng(9)
    shape = (5, 6, 7)
    masks = [np.zeros(shape, np.uint8) for _ in range(7)]
    masks[0][2, 3, 4] = 1
    masks[1][:, 2, 3] = 1
    masks[2][1, 4, :] = 1
    masks[3][3] = 1
    masks[4][3:5, 4:6, 5:7] = 1
    masks[5] = (rng.random(shape) < 0.15).astype(np.uint8)
    specs = [inputs.init_random_all(m, b) for b, m in enumerate(masks)]
    p = inputs.ModelParams(v_dom=2e-3, k_dom=0.5, rho=3e-4, mu=2e-4, beta=0.55, v_som=1e-4, v_p4=2e-4)
    c = [0.8, 0.9, 1.0, 0.85, 0.95, 0.75, 0.9, 1.0]
    dt = inputs.explicit_dt(p, 0.8)
    nsteps = 12
    seeds = rng.standard_normal((nsteps + 1, len(masks), 5))
    g = Graph.from_masks(masks, regions=True)
    sim = Simulation(g, p, precision="f64", implicit=False, adjoint=True, regions=c)
    x0 = g.fields_from_specs(specs, torch.float64).requires_grad_(True)
    theta = theta_of(p, c).requires_grad_(True)
    tot = simulate_totals(sim, theta, x0, nsteps, dt, checkpoint_every=5)
    (tot * torch.as_tensor(seeds, device=tot.device)).sum().backward()
    og = orc.build_batch(masks)
    reg = orc.octant_regions(og)
    w = orc.edge_weights(og, reg, c)
    ox0 = orc.fields_from_spec(og, specs)
    states = orc.run_states(p, dt, og, ox0, nsteps, w=w)
    lam0, grad = orc.adjoint(p, dt, og, states, seeds, w=w, region=reg, nreg=8)
    _, otot = orc.run(p, dt, og, ox0, nsteps, w=w)
    np.testing.assert_allclose(tot.detach().cpu().numpy(), otot[:, :, :5], rtol=1e-13, atol=1e-300)
    lam = x0.grad.detach().cpu().numpy()
    np.testing.assert_allclose(lam, lam0, rtol=1e-11, atol=1e-12 * np.abs(lam0).max())
    gg = theta.grad.numpy()
    scale = np.abs(grad).max()
    np.testing.assert_allclose(gg, grad, rtol=1e-9, atol=1e-9 * scale)
