"""Runs of fused passes replayed from captured HIP graphs (vg_set_launch_options)
give the same state, bit for bit, as plain launches: the same kernels with
the same arguments in the same order.  Each graph is replayed many times,
with the program's own eager work (totals, other steps, state loads,
synchronisations) between replays, and every replay's result is checked;
changes of dt, parameters, regions and kernel force a new capture."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2406_04177_amd import inputs

pytestmark = pytest.mark.gpu


def _pair(mask_or_masks, precision, params, regions=None, kernel=0, band=True):
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    g = Graph.from_masks(mask_or_masks, regions=regions is not None)
    sims = []
    for mode in ("off", "on"):
        sim = Simulation(g, params, precision=precision, implicit=False, regions=regions, band=band)
        sim.set_kernel(kernel)
        sim.set_launch_options(mode)
        sims.append(sim)
    return g, sims


def _same(a, b):
    torch.cuda.synchronize()
    assert torch.equal(a.state(), b.state())


@pytest.mark.parametrize("precision", ["f64", "f32", "f32c"])
@pytest.mark.parametrize("order", [0, 1])
def test_replays_equal_plain_launches(precision, order):
    mask = inputs.synthetic_volume((40, 36, 44), seed=3)
    spec = [inputs.init_random_all(mask, 3)]
    p = inputs.ModelParams(mu=1e-4, rho=1e-4)
    dt = inputs.explicit_dt(p)
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    g, (plain, graph) = _pair(mask, precision, p)
    for s in (plain, graph):
        s.step_order = order
        s.set_params(p)
        s.set_fields(g.fields_from_specs(spec, torch.float64))
    # runs of various lengths (several captured runs, remainders, logged steps
    # breaking runs), with eager work between the calls
    for steps, every in ((70, 0), (33, 0), (100, 25), (17, 0), (64, 16), (200, 7)):
        la = plain.step(steps, dt, log_every=every)
        lb = graph.step(steps, dt, log_every=every)
        _same(plain, graph)
        if every:
            assert torch.equal(la, lb)
        np.testing.assert_array_equal(plain.totals(), graph.totals())
    # the result is also the oracle's (FP64)
    if precision == "f64":
        og = orc.build_graph(mask)
        ref, _ = orc.run(p, dt, og, orc.fields_from_spec(og, spec), 70 + 33 + 100 + 17 + 64 + 200, order=order,
                         with_totals=False)
        np.testing.assert_array_equal(graph.state().cpu().numpy(), ref)


def test_recapture_after_changes():
    """dt, parameters, regions, kernel choice and a state reload between calls:
    each call's result equals plain launches."""
    mask = inputs.synthetic_volume((30, 32, 34), seed=5)
    spec = [inputs.init_random_all(mask, 5)]
    p = inputs.ModelParams(mu=1e-4, rho=1e-4)
    c = [0.7, 1.0, 0.8, 0.9, 1.1, 0.75, 0.95, 0.85]
    g, (plain, graph) = _pair(mask, "f64", p, regions=c)
    x0 = g.fields_from_specs(spec, torch.float64)
    for s in (plain, graph):
        s.set_fields(x0)
    dt1, dt2 = inputs.explicit_dt(p, 0.5), inputs.explicit_dt(p, 0.6)
    for k in range(3):                       # replays of one captured run
        for s in (plain, graph):
            s.step(40, dt1)
        _same(plain, graph)
    for s in (plain, graph):
        s.step(40, dt2)                      # new dt
    _same(plain, graph)
    p2 = p.replace(rho=3e-4, v_dom=2e-4)
    for s in (plain, graph):
        s.set_params(p2)
        s.step(40, dt2)
    _same(plain, graph)
    for s in (plain, graph):
        s.set_regions([1.1, 0.9, 1.0, 1.2, 0.8, 1.0, 0.95, 1.05])
        s.step(40, dt2)
    _same(plain, graph)
    for s in (plain, graph):
        s.set_kernel(1)                      # the table kernel
        s.step(40, dt2)
    _same(plain, graph)
    for s in (plain, graph):
        s.set_fields(x0)                     # same pointers, new contents
        s.step(40, dt2)
    _same(plain, graph)


def test_band_runs_and_batches():
    """The band kernel's runs (forced on a small volume) and a batch of
    volumes with an empty one."""
    p = inputs.ModelParams(mu=1e-4, rho=1e-4)
    dt = inputs.explicit_dt(p)
    mask = inputs.synthetic_volume((48, 40, 36), seed=2)
    spec = [inputs.init_random_all(mask, 2)]
    g, (plain, graph) = _pair(mask, "f32", p, kernel=5)
    assert graph.kernel_in_use() == 5
    for s in (plain, graph):
        s.set_fields(g.fields_from_specs(spec, torch.float64))
        s.step(123, dt, log_every=50)
    _same(plain, graph)
    masks = [inputs.synthetic_volume((24, 20, 16), porosity=por, seed=b) for b, por in enumerate((0.12, 0.25))]
    masks.insert(1, np.zeros((24, 20, 16), np.uint8))
    specs = [inputs.init_random_all(m, 1) for m in masks]
    g, (plain, graph) = _pair(masks, "f32", p)
    for s in (plain, graph):
        s.set_fields(g.fields_from_specs(specs, torch.float64))
        s.step(77, dt)
    _same(plain, graph)
