"""Pins of the oracle's transformation (Sec. II.C eq. (3); Appendix A,
Algorithm 1) and of the whole time step (Sec. II.A, Sec. III).

Expected values: closed forms of explicit Euler on the linear sub-models,
hand-computed clamp cases with binary-exact numbers, eq. (3) written out,
carbon conservation, uniform-state and mirror invariance, the splitting
identity, and printed numbers of the paper.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2406_04177_amd.inputs import ModelParams

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")


def one_voxel():
    return orc.build_graph(np.ones((1, 1, 1), np.uint8))


def T1(params, dt, x5):
    x = np.array(x5, np.float64).reshape(5, 1)
    return orc.transform(params, dt, x)[:, 0]


NOFLOW = dict(D=(0.0,) * 5)


def test_p4_and_som_decay_closed_forms():
    """FOM only decays: x4 (1 - v_FOM dt)^n.  Without mortality SOM decays as
    x3 (1 - v_SOM dt)^n and all of it ends in DOM."""
    p = ModelParams(**NOFLOW, v_dom=0.0, rho=0.0, mu=0.0, v_som=2e-3, v_p4=5e-3)
    dt, n = 1.5, 300
    g = one_voxel()
    x0 = np.array([[0.0], [0.0], [0.7], [0.9], [0.0]])
    x, _ = orc.run(p, dt, g, x0, n, with_totals=False)
    assert math.isclose(x[3, 0], 0.9 * (1 - 5e-3 * dt) ** n, rel_tol=1e-13)
    assert math.isclose(x[2, 0], 0.7 * (1 - 2e-3 * dt) ** n, rel_tol=1e-13)
    gained = 0.9 * (1 - (1 - 5e-3 * dt) ** n) + 0.7 * (1 - (1 - 2e-3 * dt) ** n)
    assert math.isclose(x[1, 0], gained, rel_tol=1e-12)


def test_biomass_and_co2_closed_forms():
    """No uptake (v_DOM = 0): MB = x1 q^n with q = 1 - (rho + mu) dt; CO2 =
    rho dt x1 (1 - q^n) / (1 - q); DOM and SOM split the dead mass beta : 1-beta."""
    rho, mu, beta, dt, n = 3e-3, 2e-3, 0.55, 2.0, 400
    p = ModelParams(**NOFLOW, v_dom=0.0, rho=rho, mu=mu, beta=beta, v_som=0.0, v_p4=0.0)
    x0 = np.array([[0.8], [0.0], [0.0], [0.0], [0.1]])
    x, _ = orc.run(p, dt, one_voxel(), x0, n, with_totals=False)
    q = 1 - (rho + mu) * dt
    geo = (1 - q ** n) / (1 - q)
    assert math.isclose(x[0, 0], 0.8 * q ** n, rel_tol=1e-12)
    assert math.isclose(x[4, 0], 0.1 + rho * dt * 0.8 * geo, rel_tol=1e-12)
    assert math.isclose(x[1, 0], beta * mu * dt * 0.8 * geo, rel_tol=1e-12)
    assert math.isclose(x[2, 0], (1 - beta) * mu * dt * 0.8 * geo, rel_tol=1e-12)


def test_monod_uptake_without_losses():
    """Only uptake: MB + DOM is constant and MB grows by v x2/(K + x2) x1 dt."""
    p = ModelParams(**NOFLOW, v_dom=0.5, k_dom=0.25, rho=0.0, mu=0.0, v_som=0.0, v_p4=0.0)
    y = T1(p, 0.5, [0.5, 0.25, 0, 0, 0])
    # uptake = 0.5 * 0.25 / 0.5 * 0.5 * 0.5 = 0.0625 (binary exact)
    np.testing.assert_array_equal(y, [0.5625, 0.1875, 0, 0, 0])


def test_clamp_uptake_exceeds_dom():
    p = ModelParams(**NOFLOW, v_dom=10.0, k_dom=0.125, rho=0.0, mu=0.0, v_som=0.0, v_p4=0.0)
    y = T1(p, 1.0, [1.0, 0.125, 0, 0, 0])  # raw uptake 5 > 0.125
    np.testing.assert_array_equal(y, [1.125, 0.0, 0, 0, 0])


def test_clamp_respiration_takes_the_rest():
    """resp + mort > x1 with mort <= x1: resp = x1 - mort."""
    p = ModelParams(**NOFLOW, v_dom=0.0, rho=0.75, mu=0.5, beta=0.5, v_som=0.0, v_p4=0.0)
    y = T1(p, 1.0, [1.0, 0, 0, 0, 0])
    np.testing.assert_array_equal(y, [0.0, 0.25, 0.25, 0.0, 0.5])


def test_clamp_mortality_exceeds_biomass():
    """mort > x1: all biomass dies, no respiration."""
    p = ModelParams(**NOFLOW, v_dom=0.0, rho=0.25, mu=2.0, beta=0.75, v_som=0.0, v_p4=0.0)
    y = T1(p, 1.0, [0.5, 0, 0, 0, 0])
    np.testing.assert_array_equal(y, [0.0, 0.375, 0.125, 0.0, 0.0])


def test_clamp_turnovers():
    p = ModelParams(**NOFLOW, v_dom=0.0, rho=0.0, mu=0.0, v_som=3.0, v_p4=4.0)
    y = T1(p, 1.0, [0, 0, 0.25, 0.5, 0])
    np.testing.assert_array_equal(y, [0, 0.75, 0.0, 0.0, 0])


def test_mortality_to_p4_routing():
    p = ModelParams(**NOFLOW, v_dom=0.0, rho=0.0, mu=0.5, v_som=0.0, v_p4=0.0, mort_to_p4=True)
    y = T1(p, 1.0, [0.5, 0, 0, 0, 0])
    np.testing.assert_array_equal(y, [0.25, 0.0, 0.0, 0.25, 0.0])


def test_no_clamp_equals_equation_3():
    """Without an active clamp Algorithm 1 is the forward-Euler step eq. (3)."""
    rng = np.random.default_rng(0)
    v, K, rho, mu, beta, vS, vF, dt = 1e-4, 0.5, 2e-6, 5e-7, 0.55, 1e-7, 3e-7, 0.0864
    p = ModelParams(**NOFLOW, v_dom=v, k_dom=K, rho=rho, mu=mu, beta=beta, v_som=vS, v_p4=vF)
    for _ in range(20):
        x1, x2, x3, x4, x5 = rng.random(5)
        monod = v * x2 / (K + x2) * x1
        eq3 = [x1 + monod * dt - (rho * x1 + mu * x1) * dt,
               x2 - monod * dt + (vS * x3 + vF * x4 + beta * mu * x1) * dt,
               x3 + ((1 - beta) * mu * x1 - vS * x3) * dt,
               x4 - vF * x4 * dt,
               x5 + rho * x1 * dt]
        np.testing.assert_allclose(T1(p, dt, [x1, x2, x3, x4, x5]), eq3, rtol=1e-14, atol=1e-16)


def random_state(g, seed):
    rng = np.random.default_rng(seed)
    return rng.random((5, g.n)) * np.array([[0.5], [1.0], [0.3], [0.2], [0.1]])


def test_total_carbon_conserved_2000_steps():
    rng = np.random.default_rng(3)
    mask = (rng.random((16, 16, 16)) < 0.5).astype(np.uint8)
    g = orc.build_graph(mask)
    x = random_state(g, 1)
    p = ModelParams(D=(2e-10, 1e-9, 3e-10, 1e-10, 5e-10), mu=5e-5, rho=2e-5, v_som=1e-5, v_p4=2e-5)
    dt = 0.9 * p.h ** 2 / (6 * 1e-9)
    reg = orc.octant_regions(g)
    for w in (None, orc.edge_weights(g, reg, rng.uniform(0.6, 1.0, 8))):
        out, tot = orc.run(p, dt, g, x, 2000, w=w)
        c = tot[:, 0, 5]
        assert np.abs(c - c[0]).max() / c[0] <= 1e-12
        # per-pool totals change only through the transformation
        assert abs(tot[-1, 0, 4] - tot[0, 0, 4]) > 0


def test_uniform_state_stays_uniform_and_equals_scalar_recurrence():
    g = orc.build_graph(np.ones((6, 5, 4), np.uint8))
    p = ModelParams(D=(1e-9,) * 5)
    dt = 0.08
    x0 = np.array([0.4, 0.9, 0.2, 0.1, 0.05])
    x = np.repeat(x0[:, None], g.n, axis=1)
    out, _ = orc.run(p, dt, g, x, 300, with_totals=False)
    single, _ = orc.run(p, dt, one_voxel(), x0[:, None], 300, with_totals=False)
    np.testing.assert_array_equal(out, np.repeat(single, g.n, axis=1))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_mirror_symmetry_bitwise(axis):
    rng = np.random.default_rng(10 + axis)
    mask = (rng.random((9, 10, 11)) < 0.55).astype(np.uint8)
    dense = rng.random((5,) + mask.shape)
    p = ModelParams(D=(0.0, 1e-9, 0.0, 2e-10, 0.0), mu=1e-4, rho=3e-5, v_som=2e-5, v_p4=1e-5)
    dt = 0.08

    def simulate(m, d):
        g = orc.build_graph(m)
        x = d.reshape(5, -1)[:, g.vox]
        out, _ = orc.run(p, dt, g, x, 50, with_totals=False)
        full = np.zeros((5, m.size))
        full[:, g.vox] = out
        return full.reshape((5,) + m.shape)

    a = simulate(mask, dense)
    flip = lambda arr, ax: np.ascontiguousarray(np.flip(arr, ax))
    b = simulate(flip(mask, axis), flip(dense, axis + 1))
    np.testing.assert_array_equal(flip(b, axis + 1), a)


def test_splitting_identity_bitwise():
    """(D o T)^n = D o (T o D)^(n-1) o T, exactly."""
    rng = np.random.default_rng(8)
    mask = (rng.random((10, 10, 10)) < 0.55).astype(np.uint8)
    g = orc.build_graph(mask)
    x = random_state(g, 2)
    p = ModelParams(mu=1e-4, rho=3e-5)
    dt, n = 0.08, 40
    ref, _ = orc.run(p, dt, g, x, n, order=0, with_totals=False)
    y = orc.transform(p, dt, x)
    y, _ = orc.run(p, dt, g, y, n - 1, order=1, with_totals=False)
    y = orc.diffuse(p, dt, g, y)
    np.testing.assert_array_equal(y, ref)


def test_totals_match_fsum():
    rng = np.random.default_rng(12)
    x = (rng.random((5, 10000)) - 0.3) * 10.0 ** rng.integers(-8, 8, size=(5, 10000))
    g = orc.OracleGraph((1, 1, 10000), np.arange(10000, dtype=np.int32),
                        np.full((6, 10000), -1, np.int32), np.array([0, 4000, 10000]))
    tot = orc.totals(g, x)
    for seg, (lo, hi) in enumerate([(0, 4000), (4000, 10000)]):
        for s in range(5):
            exact = math.fsum(x[s, lo:hi])
            assert abs(tot[seg, s] - exact) <= 2 * np.spacing(abs(exact))


def test_paper_printed_numbers():
    gold = json.load(open(GOLDEN))
    b = gold["bacterial_carbon"]
    assert math.isclose(b["cells"] * b["carbon_per_cell_ug"], b["total_ug"], rel_tol=1e-12)
    sh = gold["initial_shares"]
    tot = sh["dom_ug"] + b["total_ug"]
    assert round(100 * sh["dom_ug"] / tot, 4) == sh["dom_percent"]
    assert round(100 * b["total_ug"] / tot, 3) == sh["mb_percent"]
    v = gold["sample_volume"]
    assert round((v["voxels_per_side"] * v["voxel_um"] * 1e-4) ** 3, 3) == v["volume_cm3"]
    e = gold["explicit_limit"]
    D_vox_per_s = e["D_voxel2_per_day"] / 86400.0
    assert e["largest_dt_s"] <= 1.0 / (6.0 * D_vox_per_s)
    # the workloads' rates are the paper's Arthrobacter rates to within a factor
    # of 1.2 (mortality is 10x lower in the workloads, as given)
    r = gold["arthrobacter_rates_per_day"]
    w = ModelParams()
    for name, ours in (("rho", w.rho), ("v_dom", w.v_dom), ("v_som", w.v_som)):
        ratio = ours / (r[name] / 86400.0)
        assert 0.8 < ratio < 1.2, (name, ratio)
