"""Recordings that keep each step's diffused DOM (adjoint option tape_dom:
four rows per state, MB, DOM, SOM, P4, with the DOM of x^k after the first
state): the reverse sweep reads x^k directly instead of diffusing the stored
state again.  Lambda, the gradient, the totals and the stepped fields must be
bit-identical to the five-row recording, for every neighbour source, both
field types, with and without region weights, both dL/dD options, one to
several steps, vg_record and vg_step_record; the kept rows themselves are
checked against the oracle's states."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2406_04177_amd import _lib, inputs

pytestmark = pytest.mark.gpu

KERNELS = [_lib.VG_KERNEL_TABLE, _lib.VG_KERNEL_OFFSET, _lib.VG_KERNEL_RELATIVE]
STATIC = [0, 2, 3]   # MB, SOM, P4: the rows both recordings hold alike
KERNEL_IDS = ["table", "offset", "relative"]


def rates():
    return inputs.ModelParams(v_dom=2e-3, k_dom=0.5, rho=3e-4, mu=2e-4, beta=0.55, v_som=1e-4, v_p4=2e-4)


def batch(seed):
    masks = [inputs.synthetic_volume((14, 16, 12), porosity=por, seed=seed + b) for b, por in enumerate((0.2, 0.25))]
    return masks, [inputs.init_random_all(m, seed + b) for b, m in enumerate(masks)]


def final_adjoint(seg_off, n, seed, uniform_co2):
    lam = np.random.default_rng(seed).standard_normal((5, n))
    if uniform_co2:
        for k in range(len(seg_off) - 1):
            lam[4, seg_off[k]:seg_off[k + 1]] = 0.3 + k
    return lam


def make_sim(g, precision, kernel, regions, skip, tape_dom, mobile_all=None):
    from paper_2406_04177_amd.sim import Simulation
    p = rates()
    c = [1.0, 0.9, 0.8, 1.05, 0.95, 0.85, 1.0, 0.9] if regions else None
    sim = Simulation(g, p, precision=precision, implicit=False, adjoint=True, regions=c, mobile_all=mobile_all)
    sim.set_kernel(kernel)
    sim.set_adjoint_options(skip_static_d=skip, tape_dom=tape_dom)
    return sim


def sweep(sim, g, x0, dt, nsteps, lam_end, seeds):
    """vg_record then vg_adjoint from x0; returns (states, lambda^0, grad)."""
    sim.set_fields(x0)
    states = torch.empty((nsteps, sim.tape_rows, g.n), dtype=x0.dtype, device="cuda")
    sim.record(nsteps, dt, states)
    lam = torch.as_tensor(lam_end, device="cuda").to(x0.dtype).contiguous()
    grad = torch.zeros(20, dtype=torch.float64, device="cuda")
    sim.adjoint(nsteps, dt, states, torch.as_tensor(seeds, device="cuda").contiguous(), lam, grad)
    torch.cuda.synchronize()
    return states, lam, grad


@pytest.mark.parametrize("nsteps", [1, 2, 11])
@pytest.mark.parametrize("skip", [False, True], ids=["all_d", "skip_static_d"])
@pytest.mark.parametrize("regions", [False, True], ids=["unit_w", "regions"])
@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("kernel", KERNELS, ids=KERNEL_IDS)
def test_sweep_bit_identical(kernel, precision, regions, skip, nsteps):
    from paper_2406_04177_amd.graph import Graph
    masks, specs = batch(seed=21)
    g = Graph.from_masks(masks, regions=regions)
    dtype = torch.float64 if precision == "f64" else torch.float32
    x0 = g.fields_from_specs(specs, dtype)
    dt = inputs.explicit_dt(rates(), 0.8)
    lam_end = final_adjoint(g.seg_off, g.n, 5, True)
    seeds = np.random.default_rng(6).standard_normal((nsteps, len(masks), 5))
    out = []
    for tape_dom in (False, True):
        sim = make_sim(g, precision, kernel, regions, skip, tape_dom)
        out.append(sweep(sim, g, x0, dt, nsteps, lam_end, seeds))
        del sim
    (s0, l0, g0), (s1, l1, g1) = out
    assert s0.shape[1] == 5 and s1.shape[1] == 4
    assert torch.equal(l1, l0)
    assert torch.equal(torch.nan_to_num(g1, nan=7.0), torch.nan_to_num(g0, nan=7.0))
    # MB, SOM and P4 of every state and the first state's DOM as recorded
    # without the kept DOM
    assert torch.equal(s1[:, STATIC], s0[:, STATIC])
    assert torch.equal(s1[0, 1], s0[0, 1])


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_varying_co2_adjoint(precision):
    """A CO2 adjoint that varies within a volume: with the static pools' dL/dD
    skipped the sweep is bit-identical; dL/dD_CO2 would need the CO2 state
    the recording no longer holds, so asking for it is an error."""
    from paper_2406_04177_amd.graph import Graph
    masks, specs = batch(seed=31)
    g = Graph.from_masks(masks)
    dtype = torch.float64 if precision == "f64" else torch.float32
    x0 = g.fields_from_specs(specs, dtype)
    dt = inputs.explicit_dt(rates(), 0.8)
    nsteps = 6
    lam_end = final_adjoint(g.seg_off, g.n, 7, False)
    seeds = np.random.default_rng(8).standard_normal((nsteps, len(masks), 5))
    ref = sweep(make_sim(g, precision, _lib.VG_KERNEL_AUTO, False, True, False), g, x0, dt, nsteps, lam_end, seeds)
    sim = make_sim(g, precision, _lib.VG_KERNEL_AUTO, False, True, True)
    got = sweep(sim, g, x0, dt, nsteps, lam_end, seeds)
    assert torch.equal(got[1], ref[1])
    assert torch.equal(torch.nan_to_num(got[2], nan=7.0), torch.nan_to_num(ref[2], nan=7.0))
    sim.set_adjoint_options(skip_static_d=False)
    with pytest.raises(_lib.VgError, match="CO2"):
        sweep(sim, g, x0, dt, nsteps, lam_end, seeds)


def test_kept_dom_equals_oracle_states():
    """FP64: the DOM row of recorded state j >= 1 holds x^j's DOM (the
    oracle's state after j steps), the MB, SOM and P4 rows T(x^(j-1))'s;
    state 0 is x^0 without CO2."""
    from paper_2406_04177_amd.graph import Graph
    masks, specs = batch(seed=41)
    p = rates()
    dt = inputs.explicit_dt(p, 0.8)
    nsteps = 9
    g = Graph.from_masks(masks)
    og = orc.build_batch(masks)
    sim = make_sim(g, "f64", _lib.VG_KERNEL_AUTO, False, False, True)
    sim.set_fields(g.fields_from_specs(specs, torch.float64))
    assert sim.tape_rows == 4
    states = torch.empty((nsteps, 4, g.n), dtype=torch.float64, device="cuda")
    sim.record(nsteps, dt, states)
    st = states.cpu().numpy()
    ref = orc.run_states(p, dt, og, orc.fields_from_spec(og, specs), nsteps)
    np.testing.assert_array_equal(st[0], ref[0][:4])
    for j in range(1, nsteps):
        dom = ref[j][1]
        np.testing.assert_allclose(st[j][1], dom, rtol=1e-12, atol=1e-14 * np.abs(dom).max())
        tj = orc.transform(p, dt, ref[j - 1])
        np.testing.assert_allclose(st[j][STATIC], tj[STATIC], rtol=1e-12, atol=1e-14 * np.abs(tj).max())


@pytest.mark.parametrize("k", [1, 2, 7])
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_step_record_bit_identical(precision, k):
    """vg_step_record with the diffused DOM kept: the stepped fields and
    totals bit-identical to the recording without it, the states to
    vg_record's with it, and the sweep over them to the sweep without it."""
    from paper_2406_04177_amd.graph import Graph
    masks, specs = batch(seed=51)
    g = Graph.from_masks(masks, regions=True)
    dtype = torch.float64 if precision == "f64" else torch.float32
    x0 = g.fields_from_specs(specs, dtype)
    dt = inputs.explicit_dt(rates(), 0.8)
    lam_end = final_adjoint(g.seg_off, g.n, 9, True)
    seeds = np.random.default_rng(10).standard_normal((k, len(masks), 5))
    res = {}
    for tape_dom in (False, True):
        sim = make_sim(g, precision, _lib.VG_KERNEL_AUTO, True, False, tape_dom)
        sim.set_fields(x0)
        sim.step(3, dt)
        start = sim.fields.clone()
        rec = torch.empty((k, sim.tape_rows, g.n), dtype=dtype, device="cuda")
        sim.record(k, dt, rec)
        states = torch.empty_like(rec)
        tot = torch.empty((k, g.nseg, 6), dtype=torch.float64, device="cuda")
        sim.set_fields(start)
        sim.step_record(k, dt, states, tot)
        fields = sim.fields.clone()
        lam = torch.as_tensor(lam_end, device="cuda").to(dtype).contiguous()
        grad = torch.zeros(20, dtype=torch.float64, device="cuda")
        sim.adjoint(k, dt, states, torch.as_tensor(seeds, device="cuda").contiguous(), lam, grad)
        torch.cuda.synchronize()
        assert torch.equal(states, rec)
        res[tape_dom] = (fields, tot, lam, grad)
        del sim
    for a, b in zip(res[False], res[True]):
        assert torch.equal(a, b)


def test_ignored_when_every_pool_diffuses():
    """With every pool diffusing the option changes nothing: the recorded
    states keep CO2."""
    from paper_2406_04177_amd.graph import Graph
    masks, specs = batch(seed=61)
    g = Graph.from_masks(masks)
    x0 = g.fields_from_specs(specs, torch.float64)
    dt = inputs.explicit_dt(rates(), 0.8)
    lam_end = final_adjoint(g.seg_off, g.n, 11, False)
    seeds = np.random.default_rng(12).standard_normal((5, len(masks), 5))
    out = [sweep(make_sim(g, "f64", _lib.VG_KERNEL_AUTO, False, False, td, mobile_all=True), g, x0, dt, 5, lam_end,
                 seeds) for td in (False, True)]
    for a, b in zip(out[0], out[1]):
        assert torch.equal(a, b)


def test_unknown_option_rejected():
    from paper_2406_04177_amd.graph import Graph
    masks, _ = batch(seed=71)
    sim = make_sim(Graph.from_masks(masks), "f32", _lib.VG_KERNEL_AUTO, False, False, False)
    for flags in range(4):
        assert sim.L.vg_set_adjoint_options(sim.h, flags) == _lib.VG_OK
    assert sim.L.vg_set_adjoint_options(sim.h, 4) == _lib.VG_EINVAL


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("brick", [0, 4], ids=["raster", "brick4"])
def test_rank_index_recording_bit_identical(brick, precision):
    """A single volume recorded through the rank-index pass (raster and brick
    order, region weights): the same bit-identity with and without the kept
    DOM, for vg_record and vg_step_record."""
    from paper_2406_04177_amd.graph import Graph
    mask = inputs.synthetic_volume((16, 16, 16), porosity=0.22, seed=81)
    spec = inputs.init_random_all(mask, 81)
    g = Graph.from_masks(mask, brick=brick, regions=True)
    dtype = torch.float64 if precision == "f64" else torch.float32
    x0 = g.fields_from_specs(spec, dtype)
    dt = inputs.explicit_dt(rates(), 0.8)
    nsteps = 7
    lam_end = final_adjoint(g.seg_off, g.n, 13, True)
    seeds = np.random.default_rng(14).standard_normal((nsteps, 1, 5))
    out = []
    for tape_dom in (False, True):
        sim = make_sim(g, precision, _lib.VG_KERNEL_RANK, True, False, tape_dom)
        states, lam, grad = sweep(sim, g, x0, dt, nsteps, lam_end, seeds)
        sim.set_fields(x0)
        taped = torch.empty_like(states)
        tot = torch.empty((nsteps, 1, 6), dtype=torch.float64, device="cuda")
        sim.step_record(nsteps, dt, taped, tot)
        torch.cuda.synchronize()
        assert torch.equal(taped, states)
        out.append((lam, grad, states[:, STATIC].clone(), tot, sim.fields.clone()))
        del sim
    for a, b in zip(out[0], out[1]):
        assert torch.equal(a, b)


def test_states_shape_checked():
    """A states tensor with fewer rows per step than the recording writes is
    refused before any launch; the kept-DOM recording takes four."""
    from paper_2406_04177_amd.graph import Graph
    masks, specs = batch(seed=91)
    g = Graph.from_masks(masks)
    sim = make_sim(g, "f32", _lib.VG_KERNEL_AUTO, False, False, False)
    sim.set_fields(g.fields_from_specs(specs, torch.float32))
    small = torch.empty((3, 4, g.n), dtype=torch.float32, device="cuda")
    assert sim.tape_rows == 5
    with pytest.raises(ValueError):
        sim.record(3, inputs.explicit_dt(rates(), 0.8), small)
    sim.set_adjoint_options(tape_dom=True)
    assert sim.tape_rows == 4
    sim.record(3, inputs.explicit_dt(rates(), 0.8), small)
    torch.cuda.synchronize()
    # a five-row recording swept under the four-row option (or the reverse)
    five = torch.empty((3, 5, g.n), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        sim.record(3, inputs.explicit_dt(rates(), 0.8), five)
