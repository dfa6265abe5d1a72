"""Pins of the oracle's Algorithm 2 (Appendix A, sequential transformation,
read with its three corrections) and of the sub-cycled time loop for unequal
transformation and diffusion steps (Sec. III)."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2406_04177_amd import inputs


def seq_params(**kw):
    base = dict(D=(0.0, 0.0, 0.0, 0.0, 0.0), h=1.0, v_dom=0.5, k_dom=1.0, rho=0.125, mu=0.25, beta=0.5,
                v_som=0.25, v_p4=0.5, sequential=True)
    base.update(kw)
    return inputs.ModelParams(**base)


def one(p, m, dt=1.0):
    x = np.array(m, np.float64).reshape(5, 1)
    return orc.transform(p, dt, x)[:, 0]


# Hand-derived results (binary-exact numbers): the processes act one after the
# other, each on what the previous left.
@pytest.mark.parametrize("kw,m,expected", [
    # no clamp: uptake 0.25; mortality 0.3125 (half to DOM, half to SOM);
    # respiration 0.1171875; SOM turnover 0.2890625; FOM turnover 0.5
    ({}, [1, 1, 1, 1, 0], [0.8203125, 1.6953125, 0.8671875, 0.5, 0.1171875]),
    # uptake would take 2 > DOM 1: MB takes all DOM; then all MB (2) dies;
    # SOM (1.5) and FOM (0.25) turn over completely
    (dict(v_dom=4.0, mu=1.0, v_som=2.0, v_p4=1.0), [1, 1, 0.5, 0.25, 0], [0, 2.75, 0, 0, 0]),
    # no DOM: no uptake; mortality 0.25; respiration 1.5 > MB 0.75: all
    # respires; then SOM turnover 0.03125 of the 0.125 it received
    (dict(rho=2.0), [1, 0, 0, 0, 0], [0, 0.15625, 0.09375, 0, 0.75]),
    # no MB: only the turnovers
    ({}, [0, 0, 1, 1, 0], [0, 0.75, 0.75, 0.5, 0]),
    # dead biomass routed to pool 4 instead of DOM / SOM
    (dict(mort_to_p4=True), [1, 1, 1, 1, 0], [0.8203125, 1.65625, 0.75, 0.65625, 0.1171875]),
])
def test_hand_cases(kw, m, expected):
    got = one(seq_params(**kw), m)
    np.testing.assert_array_equal(got, np.array(expected, np.float64))
    assert got.sum() == float(np.sum(m))         # binary-exact: carbon conserved exactly


def test_conservation_on_random_voxels():
    rng = np.random.default_rng(0)
    x = rng.random((5, 4000)) * np.array([[2.0], [1.0], [3.0], [0.5], [0.0]])
    x[:, :200] = 0.0
    p = seq_params(v_dom=3.0, rho=0.9, mu=0.7, v_som=1.3, v_p4=2.2)
    for dt in (0.01, 0.3, 1.0, 3.0):
        y = orc.transform(p, dt, x)
        np.testing.assert_allclose(y.sum(axis=0), x.sum(axis=0), rtol=1e-15, atol=0)   # a few roundings
        assert np.all(y >= 0)


def test_first_order_agreement_with_algorithm_1():
    """Both algorithms are first-order consistent with eq. (3): one step
    differs by O(dt^2), so halving dt divides the difference by ~4."""
    rng = np.random.default_rng(1)
    x = 0.2 + rng.random((5, 500))
    p2 = seq_params(v_dom=2.0, rho=0.5, mu=0.4, v_som=0.3, v_p4=0.6)
    p1 = p2.replace(sequential=False)
    diffs = []
    for dt in (0.02, 0.01, 0.005):
        diffs.append(np.abs(orc.transform(p2, dt, x) - orc.transform(p1, dt, x)).max())
    r1, r2 = diffs[0] / diffs[1], diffs[1] / diffs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, (diffs, r1, r2)


def test_closed_form_biomass_decay_without_dom():
    """No uptake (v_DOM = 0): each step MB loses mu dt of itself, then rho dt
    of the rest, so MB_n = MB_0 ((1 - mu dt)(1 - rho dt))^n and CO2 collects
    the respired parts."""
    p = seq_params(mu=0.3, rho=0.2, v_dom=0.0, v_som=0.0, v_p4=0.0)
    dt, n = 0.1, 40
    x = np.zeros((5, 1))
    x[0] = 1.7
    q = (1 - 0.3 * dt) * (1 - 0.2 * dt)
    co2 = 0.0
    y = x.copy()
    for k in range(n):
        y = orc.transform(p, dt, y)
        co2 += 0.2 * dt * 1.7 * q ** k * (1 - 0.3 * dt)
    np.testing.assert_allclose(y[0, 0], 1.7 * q ** n, rtol=1e-13)
    np.testing.assert_allclose(y[4, 0], co2, rtol=1e-12)


# ---------------------------------------------------------------------------
# unequal time steps
# ---------------------------------------------------------------------------
def small():
    mask = inputs.synthetic_volume((12, 14, 10), seed=3)
    g = orc.build_graph(mask)
    x = orc.fields_from_spec(g, inputs.init_random_all(mask, 3))
    p = inputs.ModelParams(mu=1e-3, rho=2e-3, v_dom=5e-3)
    return g, x, p


@pytest.mark.parametrize("sequential", [False, True])
def test_equal_steps_are_the_plain_loop(sequential):
    g, x, p = small()
    p = p.replace(sequential=sequential)
    dt = inputs.explicit_dt(p, 0.9)
    ref, _ = orc.run(p, dt, g, x, 13, with_totals=False)
    np.testing.assert_array_equal(orc.run_subcycled(p, dt, dt, g, x, 13), ref)


def test_integer_ratio_is_t_then_m_diffusions():
    g, x, p = small()
    dd = 0.0625
    dtt = 4 * dd
    y = x.copy()
    for _ in range(5):
        y = orc.transform(p, dtt, y)
        for _ in range(4):
            y = orc.diffuse(p, dd, g, y)
    np.testing.assert_array_equal(orc.run_subcycled(p, dtt, dd, g, x, 5), y)


@pytest.mark.parametrize("dtt,dd,nt", [(0.043, 0.01, 7), (0.01, 0.043, 31), (0.05, 0.03, 6)])
def test_event_order_by_start_time(dtt, dd, nt):
    """The steps of an independent event list: (start, kind) sorted by start,
    transformation first on ties; the last diffusion step ends at nt*dtt."""
    g, x, p = small()
    t_end = nt * dtt
    ev = [(k * dtt, 0, dtt) for k in range(nt)]
    k = 0
    while k * dd < t_end:
        ev.append((k * dd, 1, min(dd, t_end - k * dd) if (k + 1) * dd > t_end else dd))
        k += 1
    ev.sort(key=lambda e: (e[0], e[1]))
    y = x.copy()
    for _, kind, length in ev:
        y = orc.transform(p, length, y) if kind == 0 else orc.diffuse(p, length, g, y)
    np.testing.assert_array_equal(orc.run_subcycled(p, dtt, dd, g, x, nt), y)


def test_partial_last_step_fourier_mode():
    """Pure diffusion in a periodic channel: full steps of dt_d, then one of the
    remainder; the mode decays by the product of (1 - a_k lambda)."""
    W, H, Lz, k = 3, 4, 32, 3
    mask = np.ones((Lz, H, W), np.uint8)
    g = orc.build_graph(mask, periodic=7)
    p = inputs.ModelParams(D=(0, 0.2, 0, 0, 0), h=1.0, v_dom=0.0, rho=0.0, mu=0.0, v_som=0.0, v_p4=0.0)
    z = g.vox // (W * H)
    mode = np.cos(2 * np.pi * k * z / Lz)
    x = np.zeros((5, g.n))
    x[1] = 1.0 + 0.5 * mode
    lam = 4 * np.sin(np.pi * k / Lz) ** 2
    dtt, dd, nt = 2.6, 0.7, 3          # t_end 7.8 = 11 steps of 0.7 + 0.1
    out = orc.run_subcycled(p, dtt, dd, g, x, nt)
    amp = (1 - 0.2 * 0.7 * lam) ** 11 * (1 - 0.2 * (7.8 - 11 * 0.7) * lam)
    np.testing.assert_allclose(out[1], 1.0 + 0.5 * amp * mode, rtol=0, atol=1e-13)
