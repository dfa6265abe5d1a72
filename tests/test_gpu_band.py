"""The two-pass band kernel (pairs of fused passes in one launch, rows of a
band marching along z with the intermediate DOM in LDS) against the
single-pass relative-code kernel (bit-identical fields and totals, FP32 and
FP64, both step orders, runs whose logged steps split the band runs at every
offset) and against the FP64 oracle; when it is used and when not."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2406_04177_amd import inputs

pytestmark = pytest.mark.gpu

RELATIVE, BAND = 4, 5

SHAPES = [((30, 36, 40), 0.35, 0), ((23, 17, 130), 0.30, 1), ((64, 64, 64), 0.17, 2), ((9, 70, 33), 0.5, 3),
          ((40, 30, 20), 0.6, 4)]


def sim_of(g, params, precision, kernel, order=0, band=True, regions=None):
    from paper_2406_04177_amd.sim import Simulation
    sim = Simulation(g, params, precision=precision, implicit=False, step_order=order, band=band, regions=regions)
    sim.set_kernel(kernel)
    return sim


def fast_params(**kw):
    # rates large enough that the transformation moves every pool within a few steps
    base = dict(v_dom=0.05, k_dom=0.5, rho=0.01, mu=0.02, v_som=0.01, v_p4=0.02)
    base.update(kw)
    return inputs.ModelParams(**base)


@pytest.mark.parametrize("shape,por,seed", SHAPES)
@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("order", [0, 1], ids=["TD", "DT"])
def test_band_bitwise_equals_single_passes(shape, por, seed, precision, order):
    from paper_2406_04177_amd.graph import Graph
    mask = inputs.synthetic_volume(shape, porosity=por, seed=seed)
    g = Graph.from_masks(mask)
    p = fast_params()
    dt = inputs.explicit_dt(p, 0.9)
    spec = inputs.init_random_all(mask, seed)
    dtype = torch.float32 if precision == "f32" else torch.float64
    a = sim_of(g, p, precision, BAND, order)
    b = sim_of(g, p, precision, RELATIVE, order)
    assert a.kernel_in_use() == BAND and b.kernel_in_use() == RELATIVE
    for steps, log_every in ((1, 0), (4, 0), (5, 0), (9, 0), (13, 0), (50, 0), (21, 3), (29, 7), (40, 5)):
        x0 = g.fields_from_specs(spec, torch.float64)
        a.set_fields(x0)
        b.set_fields(x0)
        la = a.step(steps, dt, log_every=log_every)
        lb = b.step(steps, dt, log_every=log_every)
        assert torch.equal(a.fields, b.fields), (steps, log_every)
        assert a.fields.dtype == dtype
        if log_every:
            assert torch.equal(la, lb), (steps, log_every)


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_band_raw_mask_with_empty_rows_and_planes(precision):
    """Unfiltered random mask with empty planes, an empty row in every plane
    and an empty x range (isolated voxels, bands and planes with no voxel):
    band kernel = single passes bit for bit; FP64 = the oracle."""
    from paper_2406_04177_amd.graph import Graph
    shape = (40, 33, 29)
    mask = (np.random.default_rng(17).random(shape) < 0.35).astype(np.uint8)
    mask[5:7] = 0
    mask[30] = 0
    mask[:, 3] = 0
    mask[:, 16:24] = 0
    mask[:, :, :4] = 0
    g = Graph.from_masks(mask)
    p = fast_params()
    dt = inputs.explicit_dt(p, 0.9)
    spec = inputs.init_random_all(mask, 8)
    a = sim_of(g, p, precision, BAND)
    b = sim_of(g, p, precision, RELATIVE)
    assert a.kernel_in_use() == BAND
    for steps, log_every in ((1, 0), (2, 0), (7, 0), (30, 0), (17, 4)):
        x0 = g.fields_from_specs(spec, torch.float64)
        a.set_fields(x0)
        b.set_fields(x0)
        la = a.step(steps, dt, log_every=log_every)
        lb = b.step(steps, dt, log_every=log_every)
        assert torch.equal(a.fields, b.fields), (steps, log_every)
        if log_every:
            assert torch.equal(la, lb)
    if precision == "f64":
        og = orc.build_graph(mask)
        ref, _ = orc.run(p, dt, og, orc.fields_from_spec(og, spec), 30, with_totals=False)
        a.set_fields(g.fields_from_specs(spec, torch.float64))
        a.step(30, dt)
        assert np.array_equal(a.fields.cpu().numpy(), ref)


def test_band_fp64_equals_oracle():
    """FP64 through the band kernel is the oracle bit for bit (200 steps, the
    48^3 workload's generator at 35 % porosity)."""
    from paper_2406_04177_amd.graph import Graph
    mask = inputs.synthetic_volume((48, 48, 48), porosity=0.35, seed=5)
    g = Graph.from_masks(mask)
    p = fast_params()
    dt = inputs.explicit_dt(p, 0.9)
    spec = inputs.init_random_all(mask, 5)
    sim = sim_of(g, p, "f64", BAND)
    sim.set_fields(g.fields_from_specs(spec, torch.float64))
    sim.step(200, dt)
    og = orc.build_graph(mask)
    ref, _ = orc.run(p, dt, og, orc.fields_from_spec(og, spec), 200, with_totals=False)
    assert np.array_equal(sim.fields.cpu().numpy(), ref)


def test_band_use_and_fallbacks():
    """AUTO leaves a volume this short in z to single passes; chosen
    explicitly, the band kernel is used unless regions, other diffusing
    pools or Algorithm 2 send the passes to the single-pass kernel (with the
    same results); brick order, batches or a handle without the feature
    cannot choose it."""
    from paper_2406_04177_amd import _lib
    from paper_2406_04177_amd.graph import Graph
    mask = inputs.synthetic_volume((32, 30, 28), porosity=0.3, seed=6)
    g = Graph.from_masks(mask)
    p = fast_params()
    assert sim_of(g, p, "f32", 0).kernel_in_use() == RELATIVE
    assert sim_of(g, p, "f32", BAND).kernel_in_use() == BAND
    # (region factors attach region codes to the graph: a graph of its own)
    assert sim_of(Graph.from_masks(mask), p, "f32", BAND, regions=[1.0] * 8).kernel_in_use() == RELATIVE
    assert sim_of(g, fast_params(sequential=True), "f32", BAND).kernel_in_use() == RELATIVE
    assert sim_of(g, fast_params(D=(1e-9, 1e-9, 0, 0, 0)), "f32", BAND).kernel_in_use() == RELATIVE
    with pytest.raises(_lib.VgError):
        sim_of(g, p, "f32", BAND, band=False)
    gb = Graph.from_masks(mask, brick=4)
    with pytest.raises(_lib.VgError):
        sim_of(gb, p, "f32", BAND)
    g2 = Graph.from_masks([mask, mask])
    with pytest.raises(_lib.VgError):
        sim_of(g2, p, "f32", BAND)
    # a band-capable handle whose parameters turn to Algorithm 2 steps on the single-pass kernel
    dt = inputs.explicit_dt(p, 0.9)
    spec = inputs.init_random_all(mask, 6)
    a = sim_of(g, p, "f64", BAND)
    assert a.kernel_in_use() == BAND
    a.set_params(fast_params(sequential=True))
    assert a.kernel_in_use() == RELATIVE
    b = sim_of(g, fast_params(sequential=True), "f64", RELATIVE)
    for s in (a, b):
        s.set_fields(g.fields_from_specs(spec, torch.float64))
        s.step(12, dt)
    assert torch.equal(a.fields, b.fields)


def test_band_512_auto_and_bitwise():
    """The 512^3 workload (20.8 M pore voxels): AUTO takes the band kernel,
    and 9 FP32 steps through it equal 9 single passes bit for bit."""
    from paper_2406_04177_amd.graph import Graph
    mask = inputs.synthetic_volume((512, 512, 512), porosity=0.17, seed=0)
    g = Graph.from_masks(mask)
    p = inputs.ModelParams()
    dt = inputs.explicit_dt(p)
    spec = inputs.init_uniform(mask, 0)
    x0 = g.fields_from_specs(spec, torch.float64)
    a = sim_of(g, p, "f32", 0)
    assert a.kernel_in_use() == BAND
    a.set_fields(x0)
    a.step(9, dt)
    fa = a.fields.clone()
    del a
    torch.cuda.empty_cache()
    b = sim_of(g, p, "f32", RELATIVE, band=False)
    b.set_fields(x0)
    b.step(9, dt)
    assert torch.equal(fa, b.fields)
