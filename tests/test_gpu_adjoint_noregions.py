"""The reverse sweep without region weights (unit edge weights, the
configuration of the 512^3 benchmark row) against the oracle's discrete
adjoint: small volumes in FP64 for every neighbour source, both dL/dD
options and a uniform or varying CO2 adjoint; FP32 against the FP64 oracle;
the checkpointed autograd gradient; and three reverse steps of the 512^3
volume itself in FP32 and FP64."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2406_04177_amd import _lib, inputs

pytestmark = pytest.mark.gpu


def rates():
    return inputs.ModelParams(v_dom=2e-3, k_dom=0.5, rho=3e-4, mu=2e-4, beta=0.55, v_som=1e-4, v_p4=2e-4)


def batch(seed=0):
    masks = [inputs.synthetic_volume((14, 16, 12), porosity=por, seed=seed + b) for b, por in enumerate((0.2, 0.25))]
    return masks, [inputs.init_random_all(m, seed + b) for b, m in enumerate(masks)]


def final_adjoint(og, seed, uniform_co2):
    lam = np.random.default_rng(seed).standard_normal((5, og.n))
    if uniform_co2:
        for k in range(og.nseg):
            lam[4, og.seg_off[k]:og.seg_off[k + 1]] = 0.3 + k
    return lam


def gpu_sweep(g, spec_fields, p, dt, precision, nsteps, lam_end, seeds, skip=False, kernel=0):
    from paper_2406_04177_amd.sim import Simulation
    sim = Simulation(g, p, precision=precision, implicit=False, adjoint=True)
    sim.set_kernel(kernel)
    sim.set_adjoint_options(skip_static_d=skip)
    dtype = torch.float64 if precision == "f64" else torch.float32
    sim.set_fields(spec_fields(dtype))
    states = torch.empty((nsteps, 5, g.n), dtype=dtype, device="cuda")
    sim.record(nsteps, dt, states)
    lam = torch.as_tensor(lam_end, device="cuda").to(dtype).contiguous()
    grad = torch.zeros(20, dtype=torch.float64, device="cuda")
    sim.adjoint(nsteps, dt, states, torch.as_tensor(seeds, device="cuda").contiguous(), lam, grad)
    torch.cuda.synchronize()
    out = lam.cpu().numpy().astype(np.float64), grad.cpu().numpy()
    del sim, states, lam
    return out


def oracle_sweep(og, x0, p, dt, nsteps, lam_end, seeds):
    states = orc.run_states(p, dt, og, x0, nsteps)
    oseeds = np.concatenate([seeds, np.zeros((1, og.nseg, 5))])
    return orc.adjoint(p, dt, og, states, oseeds, lam_final=lam_end)


@pytest.mark.parametrize("uniform_co2", [True, False], ids=["co2_uniform", "co2_varying"])
@pytest.mark.parametrize("skip", [False, True], ids=["all_d", "skip_static_d"])
@pytest.mark.parametrize("kernel", [_lib.VG_KERNEL_TABLE, _lib.VG_KERNEL_OFFSET, _lib.VG_KERNEL_RELATIVE],
                         ids=["table", "offset", "relative"])
def test_fp64_reverse_sweep_equals_oracle(kernel, skip, uniform_co2):
    from paper_2406_04177_amd.graph import Graph
    masks, specs = batch(seed=2)
    p = rates()
    dt = inputs.explicit_dt(p, 0.8)
    og = orc.build_batch(masks)
    g = Graph.from_masks(masks)
    nsteps = 11
    lam_end = final_adjoint(og, 3, uniform_co2)
    seeds = np.random.default_rng(4).standard_normal((nsteps, og.nseg, 5))
    lam, grad = gpu_sweep(g, lambda dt_: g.fields_from_specs(specs, dt_), p, dt, "f64", nsteps, lam_end, seeds,
                          skip, kernel)
    lam_or, g_or = oracle_sweep(og, orc.fields_from_spec(og, specs), p, dt, nsteps, lam_end, seeds)
    np.testing.assert_allclose(lam, lam_or, rtol=1e-11, atol=1e-12 * np.abs(lam_or).max())
    scale = np.abs(g_or).max()
    for q in range(5, 12):   # the kinetic rates
        assert abs(grad[q] - g_or[q]) <= 1e-9 * abs(g_or[q]) + 1e-12 * scale, (q, grad[q], g_or[q])
    # dL/dD_s: sums of differences of adjoints that largely cancel
    for q in range(5):
        if skip and q != 1:
            assert np.isnan(grad[q])
        else:
            assert abs(grad[q] - g_or[q]) <= 1e-7 * abs(g_or[q]) + 1e-9 * scale, (q, grad[q], g_or[q])
    np.testing.assert_array_equal(grad[12:], 0.0)   # no regions: no dL/dc_r


def test_fp32_reverse_sweep_close_to_oracle():
    """FP32 fields and adjoint (FP64 accumulators) against the FP64 oracle:
    lambda within FP32 rounding over the sweep, the diffusing pool's D and the
    kinetic rates within 1e-3."""
    from paper_2406_04177_amd.graph import Graph
    masks, specs = batch(seed=6)
    p = rates()
    dt = inputs.explicit_dt(p, 0.8)
    og = orc.build_batch(masks)
    g = Graph.from_masks(masks)
    nsteps = 16
    lam_end = final_adjoint(og, 7, True)
    seeds = np.random.default_rng(8).standard_normal((nsteps, og.nseg, 5))
    lam, grad = gpu_sweep(g, lambda dt_: g.fields_from_specs(specs, dt_), p, dt, "f32", nsteps, lam_end, seeds)
    lam_or, g_or = oracle_sweep(og, orc.fields_from_spec(og, specs), p, dt, nsteps, lam_end, seeds)
    np.testing.assert_allclose(lam, lam_or, rtol=2e-5, atol=2e-6 * np.abs(lam_or).max())
    for q in [1] + list(range(5, 12)):
        assert abs(grad[q] - g_or[q]) <= 1e-3 * abs(g_or[q]) + 1e-9 * np.abs(g_or).max(), (q, grad[q], g_or[q])


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_checkpointed_gradient_without_regions(precision):
    """simulate_totals over 25 steps with checkpoints every 7 (each segment's
    first reverse step reads the stored state itself) against the oracle's
    adjoint of the same totals loss: dL/dx0 and the parameter gradient."""
    from paper_2406_04177_amd.autograd import simulate_totals, theta_of
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    masks, specs = batch(seed=10)
    p = rates()
    dt = inputs.explicit_dt(p, 0.8)
    nsteps = 25
    og = orc.build_batch(masks)
    g = Graph.from_masks(masks)
    w = np.random.default_rng(11).standard_normal((nsteps + 1, og.nseg, 5))
    sim = Simulation(g, p, precision=precision, implicit=False, adjoint=True)
    dtype = torch.float64 if precision == "f64" else torch.float32
    x0 = g.fields_from_specs(specs, dtype).requires_grad_(True)
    theta = theta_of(p).requires_grad_(True)
    (simulate_totals(sim, theta, x0, nsteps, dt, checkpoint_every=7) * torch.as_tensor(w, device="cuda")).sum().backward()
    gx = x0.grad.cpu().numpy().astype(np.float64)
    gt = theta.grad.numpy()
    states = orc.run_states(p, dt, og, orc.fields_from_spec(og, specs), nsteps)
    lam_or, g_or = orc.adjoint(p, dt, og, states, w)
    rt = 1e-10 if precision == "f64" else 1e-4
    np.testing.assert_allclose(gx, lam_or, rtol=rt, atol=rt * np.abs(lam_or).max())
    for q in [1] + list(range(5, 12)):
        tol = (1e-9 if precision == "f64" else 1e-3) * abs(g_or[q]) + 1e-9 * np.abs(g_or).max()
        assert abs(gt[q] - g_or[q]) <= tol, (q, gt[q], g_or[q])


def test_512_reverse_steps_against_oracle():
    """Three reverse steps of the 512^3 benchmark volume (the relative-code
    kernel AUTO takes; static pools' dL/dD skipped, as in the benchmark's
    second timing) against the oracle: FP64 lambda to 1e-11 and the kinetic
    rates to 1e-9, FP32 lambda within FP32 rounding."""
    from paper_2406_04177_amd.graph import Graph
    mask = inputs.synthetic_volume((512,) * 3, porosity=0.17, seed=0)
    spec = inputs.init_uniform(mask, seed=0)
    p = inputs.ModelParams()
    dt = inputs.explicit_dt(p, 0.9)
    og = orc.build_graph(mask)
    g = Graph.from_masks(mask)
    assert g.n == og.n
    nsteps = 3
    lam_end = final_adjoint(og, 12, True)
    seeds = np.zeros((nsteps, 1, 5))
    seeds[:, :, 4] = 1.0
    seeds[:, :, 1] = 0.25
    lam_or, g_or = oracle_sweep(og, orc.fields_from_spec(og, spec), p, dt, nsteps, lam_end, seeds)
    scale = np.abs(g_or).max()
    lam64, g64 = gpu_sweep(g, lambda dt_: g.fields_from_specs(spec, dt_), p, dt, "f64", nsteps, lam_end, seeds,
                           skip=True)
    np.testing.assert_allclose(lam64, lam_or, rtol=1e-11, atol=1e-12 * np.abs(lam_or).max())
    for q in range(5, 12):
        assert abs(g64[q] - g_or[q]) <= 1e-9 * abs(g_or[q]) + 1e-12 * scale, (q, g64[q], g_or[q])
    del lam64
    lam32, g32 = gpu_sweep(g, lambda dt_: g.fields_from_specs(spec, dt_), p, dt, "f32", nsteps, lam_end, seeds,
                           skip=True)
    np.testing.assert_allclose(lam32, lam_or, rtol=1e-5, atol=1e-6 * np.abs(lam_or).max())
    for q in range(5, 12):
        assert abs(g32[q] - g_or[q]) <= 1e-3 * abs(g_or[q]) + 1e-9 * scale, (q, g32[q], g_or[q])
