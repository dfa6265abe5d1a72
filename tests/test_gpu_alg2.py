"""Algorithm 2 (sequential transformation) and unequal transformation /
diffusion steps on the GPU against the oracle: FP64 bit for bit, FP32 within
1e-5."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2406_04177_amd import inputs

pytestmark = pytest.mark.gpu

TABLE, RANK, OFFSET, RELATIVE = 1, 2, 3, 4


def setup(shape=(30, 28, 26), seed=2, dense=True, regions=None):
    from paper_2406_04177_amd.graph import Graph
    mask = inputs.synthetic_volume(shape, seed=seed)
    spec = inputs.init_random_all(mask, seed) if dense else inputs.init_uniform(mask, seed, frac_dom=0.05)
    g = Graph.from_masks(mask, regions=regions is not None)
    og = orc.build_graph(mask)
    return g, og, spec


def sim_of(g, p, precision, kernel=0, regions=None, implicit=False):
    from paper_2406_04177_amd.sim import Simulation
    sim = Simulation(g, p, precision=precision, implicit=implicit, regions=regions)
    sim.set_kernel(kernel)
    return sim


def fast_rates(**kw):
    # rates high enough for every branch of Algorithm 2 to fire somewhere
    base = dict(v_dom=0.8, k_dom=0.5, rho=0.3, mu=0.4, beta=0.55, v_som=0.2, v_p4=0.5, sequential=True)
    base.update(kw)
    return inputs.ModelParams(**base)


@pytest.mark.parametrize("kernel", [TABLE, RANK, RELATIVE], ids=["table", "rank", "relative"])
@pytest.mark.parametrize("route", [False, True], ids=["paper", "to_p4"])
def test_algorithm2_fp64_bitwise(kernel, route):
    g, og, spec = setup()
    p = fast_rates(mort_to_p4=route)
    dt = inputs.explicit_dt(p, 0.9)
    sim = sim_of(g, p, "f64", kernel)
    sim.set_fields(g.fields_from_specs(spec, torch.float64))
    log = sim.step(60, dt, log_every=20)
    ref, tot = orc.run(p, dt, og, orc.fields_from_spec(og, spec), 60)
    np.testing.assert_array_equal(sim.fields.cpu().numpy(), ref)
    np.testing.assert_allclose(log.cpu().numpy(), tot[20::20], rtol=1e-13, atol=1e-300)


def test_algorithm2_clamps_fire():
    """Large steps for the rates (dt = 4 s): uptake, mortality, respiration
    and both turnovers take whole pools in some voxels."""
    g, og, spec = setup()
    p = fast_rates(v_dom=1.5, mu=0.2, rho=0.3, v_som=0.3, v_p4=0.4)
    x0 = orc.fields_from_spec(og, spec)
    dt_t = 4.0
    y = orc.transform(p, dt_t, x0)
    assert np.count_nonzero(y[0] == 0) > 0 and np.count_nonzero(y[3] == 0) > np.count_nonzero(x0[3] == 0)
    sim = sim_of(g, p, "f64")
    sim.set_fields(g.fields_from_specs(spec, torch.float64))
    dt_d = inputs.explicit_dt(p, 0.9)
    sim.step_subcycled(3, dt_t, dt_d)
    ref = orc.run_subcycled(p, dt_t, dt_d, og, x0, 3)
    np.testing.assert_array_equal(sim.fields.cpu().numpy(), ref)


@pytest.mark.parametrize("steps,bound", [(40, 1e-5), (100, 4 * 100 * 2.0 ** -24)])
def test_algorithm2_fp32(steps, bound):
    """Within 1e-5 for short runs; longer runs within the FP32 rounding bound
    c k 2^-24 (c = 4): Algorithm 2 rounds MB up to three times per step."""
    g, og, spec = setup(dense=False)
    p = inputs.ModelParams(sequential=True)
    dt = inputs.explicit_dt(p, 0.9)
    sim = sim_of(g, p, "f32")
    sim.set_fields(g.fields_from_specs(spec, torch.float64))
    sim.step(steps, dt)
    ref, _ = orc.run(p, dt, og, orc.fields_from_spec(og, spec), steps, with_totals=False)
    got = sim.fields.cpu().numpy().astype(np.float64)
    for s in range(5):
        scale = np.abs(ref[s]).max()
        if scale > 0:
            err = np.abs(got[s] - ref[s]).max() / scale
            assert err <= bound, (s, err)


@pytest.mark.parametrize("ratio,nt", [(1.0, 20), (4.3, 9), (0.5, 30), (3.0, 8)])
@pytest.mark.parametrize("sequential", [False, True], ids=["alg1", "alg2"])
@pytest.mark.parametrize("kernel", [TABLE, RELATIVE], ids=["table", "relative"])
def test_subcycled_fp64_bitwise(ratio, nt, sequential, kernel):
    c = [0.8, 1.0, 0.9, 1.1, 0.95, 1.05, 0.85, 1.0]
    g, og, spec = setup(regions=c)
    p = fast_rates(sequential=sequential, v_dom=0.05, rho=0.01, mu=0.02, v_som=0.01, v_p4=0.02)
    dt_d = inputs.explicit_dt(p, 0.8)
    dt_t = ratio * dt_d
    sim = sim_of(g, p, "f64", kernel, regions=c)
    sim.set_fields(g.fields_from_specs(spec, torch.float64))
    sim.step_subcycled(nt, dt_t, dt_d)
    w = orc.edge_weights(og, orc.octant_regions(og), c)
    ref = orc.run_subcycled(p, dt_t, dt_d, og, orc.fields_from_spec(og, spec), nt, w=w)
    np.testing.assert_array_equal(sim.fields.cpu().numpy(), ref)


def test_subcycled_equal_steps_match_the_plain_loop_fp32():
    g, og, spec = setup(dense=False)
    p = inputs.ModelParams()
    dt = inputs.explicit_dt(p, 0.9)
    a = sim_of(g, p, "f32")
    a.set_fields(g.fields_from_specs(spec, torch.float64))
    a.step(40, dt)
    b = sim_of(g, p, "f32")
    b.set_fields(g.fields_from_specs(spec, torch.float64))
    b.step_subcycled(40, dt, dt)
    np.testing.assert_array_equal(a.fields.cpu().numpy(), b.fields.cpu().numpy())


def test_subcycled_fp32_within_1e5():
    g, og, spec = setup(dense=False)
    p = inputs.ModelParams(sequential=True)
    dt_d = inputs.explicit_dt(p, 0.9)
    dt_t = 4.3 * dt_d
    sim = sim_of(g, p, "f32")
    sim.set_fields(g.fields_from_specs(spec, torch.float64))
    sim.step_subcycled(25, dt_t, dt_d)
    ref = orc.run_subcycled(p, dt_t, dt_d, og, orc.fields_from_spec(og, spec), 25)
    got = sim.fields.cpu().numpy().astype(np.float64)
    for s in range(5):
        scale = np.abs(ref[s]).max()
        if scale > 0:
            assert np.abs(got[s] - ref[s]).max() / scale <= 1e-5, s


def test_implicit_step_with_algorithm2():
    g, og, spec = setup()
    p = fast_rates(v_dom=0.05, rho=0.01, mu=0.02, v_som=0.01, v_p4=0.02)
    dt = 20 * inputs.explicit_dt(p, 1.0)
    sim = sim_of(g, p, "f64", implicit=True)
    sim.set_fields(g.fields_from_specs(spec, torch.float64))
    its, rel, rc = sim.implicit_step(dt, rtol=1e-12)
    assert rc == 0
    ref, _, _ = orc.implicit_step(p, dt, og, orc.fields_from_spec(og, spec), rtol=1e-14)
    got = sim.fields.cpu().numpy()
    for s in (0, 2, 3, 4):
        np.testing.assert_array_equal(got[s], ref[s])      # transformation half, bit for bit
    a = p.D[1] * dt / p.h ** 2
    assert np.abs(got[1] - ref[1]).max() / np.abs(ref[1]).max() <= (1 + 12 * a) * 1e-12


def test_adjoint_refuses_algorithm2():
    from paper_2406_04177_amd import _lib
    from paper_2406_04177_amd.sim import Simulation
    g, og, spec = setup(shape=(12, 12, 12))
    p = inputs.ModelParams(sequential=True)
    sim = Simulation(g, p, precision="f32", implicit=False, adjoint=True)
    states = torch.empty((2, 5, g.n), dtype=torch.float32, device="cuda")
    with pytest.raises(_lib.VgError):
        sim.record(2, inputs.explicit_dt(p), states)
