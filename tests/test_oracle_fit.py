"""Pins of the fitting oracle (oracle/fit_oracle.py): the normalised-gradient
descent of Sec. V on a function with a known minimum, the loss gradient
against central differences of the oracle's own loss, and recovery of a
respiration rate from CO2 curves."""
import numpy as np
import pytest

from oracle import fit_oracle as fo
from oracle import oracle as orc
from paper_2406_04177_amd import inputs


def test_sign_descent_on_a_quadratic_reaches_the_minimum_within_one_step():
    """L = sum (theta_q - a_q)^2: each coordinate walks toward a_q by
    lr * 0.5^(e // 10) * theta0_q per epoch, then oscillates around it with an
    amplitude of at most the current step; a coordinate whose derivative is
    exactly zero stays; one whose minimum lies outside the box [0.5, 1.5]
    stops at the box's edge."""
    a = np.array([1.3731, 0.6452, 1.9, 1.0])
    theta0 = np.array([1.0, 1.0, 1.0, 1.0])

    def grad(theta, e):
        return float(np.sum((theta - a) ** 2)), 2 * (theta - a)

    epochs = 40
    hist, losses = fo.sign_sgd(theta0, grad, epochs, which=[0, 1, 2, 3])
    # first epochs: straight toward the minimum by 0.1 per epoch
    np.testing.assert_allclose(hist[1], [1.1, 0.9, 1.1, 1.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(hist[3], [1.3, 0.7, 1.3, 1.0], rtol=0, atol=1e-15)
    assert hist[-1][3] == 1.0                     # zero derivative: no move
    assert hist[-1][2] == 1.5                     # held at the box's edge
    last_step = 0.1 * 0.5 ** ((epochs - 1) // 10)
    assert np.all(np.abs(hist[-1][:2] - a[:2]) <= last_step + 1e-12)
    # the loss never ends above where the walk started
    assert losses[-1] < losses[0]


def tiny():
    masks = [inputs.synthetic_volume((14, 16, 12), porosity=por, seed=b) for b, por in enumerate((0.2, 0.25, 0.15))]
    specs = [inputs.init_random_all(m, b) for b, m in enumerate(masks)]
    og = orc.build_batch(masks)
    p = inputs.ModelParams(D=(0, 1e-9, 0, 0, 0), v_dom=2e-3, k_dom=0.5, rho=3e-4, mu=2e-4, beta=0.55,
                           v_som=1e-4, v_p4=2e-4)
    dt = inputs.explicit_dt(p, 0.8)
    return og, p, dt, orc.fields_from_spec(og, specs)


def theta_of(p, c=None):
    return np.array(list(p.D) + [p.v_dom, p.k_dom, p.rho, p.mu, p.beta, p.v_som, p.v_p4] + list(c or [1.0] * 8))


def curves(og, p, dt, x0, theta, nsteps):
    tp, tc = fo.theta_to_params(theta, p)
    _, tot = orc.run(tp, dt, og, x0, nsteps, w=orc.edge_weights(og, orc.octant_regions(og), tc))
    return tot[:, :, 4]


@pytest.mark.parametrize("vols", [None, [0, 2]])
def test_loss_gradient_matches_central_differences(vols):
    og, p, dt, x0 = tiny()
    nsteps = 20
    truth = theta_of(p, [1.1, 0.9, 1.0, 1.05, 0.95, 1.0, 0.92, 1.08])
    target = curves(og, p, dt, x0, truth, nsteps)
    theta = theta_of(p)
    loss, g = fo.loss_and_gradient(theta, p, dt, og, x0, target, vols)
    def central(q, h):
        tp, tm = theta.copy(), theta.copy()
        tp[q] += h
        tm[q] -= h
        lp, _ = fo.loss_and_gradient(tp, p, dt, og, x0, target, vols)
        lm, _ = fo.loss_and_gradient(tm, p, dt, og, x0, target, vols)
        return (lp - lm) / (2 * h)

    for q in (1, 5, 7, 8, 12, 15, 19):
        # Richardson-extrapolated central differences (error O(h^4)); the
        # region factors change the loss (~1e-17) so little that much smaller
        # steps drown in rounding
        h = 1e-3 * theta[q]
        fd = (4 * central(q, h / 2) - central(q, h)) / 3
        assert abs(g[q] - fd) <= 1e-4 * abs(fd), (q, g[q], fd)


def test_fit_recovers_the_respiration_rate():
    """Only rho moves: it starts 19 % low and ends within the last step
    (0.0125 of its start) of the rate that made the target, so the loss (about
    quadratic in the error) ends below (0.0125 / 0.19)^2 < 1e-2 of its start."""
    og, p, dt, x0 = tiny()
    nsteps = 30
    truth = theta_of(p)
    target = curves(og, p, dt, x0, truth, nsteps)
    theta0 = truth.copy()
    theta0[7] *= 0.8137
    hist, losses = fo.fit(theta0, p, dt, og, x0, target, 40, which=[7])
    assert abs(hist[-1][7] - truth[7]) <= 0.0125 * theta0[7]
    assert losses[-1] < 1e-2 * losses[0]
    np.testing.assert_array_equal(np.delete(hist[-1], 7), np.delete(theta0, 7))


def octant_case():
    """Three 16^3 volumes enumerated in bricks of 8 (octant-major inside each)."""
    masks = [inputs.synthetic_volume((16, 16, 16), porosity=por, seed=b) for b, por in enumerate((0.3, 0.35, 0.25))]
    specs = [inputs.init_random_all(m, b) for b, m in enumerate(masks)]
    og = fo.octant_graph(orc.build_batch(masks, brick=8))
    p = inputs.ModelParams(D=(0, 1e-9, 0, 0, 0), v_dom=2e-3, k_dom=0.5, rho=3e-4, mu=2e-4, beta=0.55,
                           v_som=1e-4, v_p4=2e-4)
    dt = inputs.explicit_dt(p, 0.8)
    return og, p, dt, orc.fields_from_spec(orc.build_batch(masks, brick=8), specs)


def test_octant_graph_by_hand():
    """Two all-pore 4^3 volumes in bricks of 2: every octant holds 2^3 voxels,
    segment k of volume v holds exactly octant k of v (named voxels), and the
    octant totals add up to the volume totals."""
    masks = [np.ones((4, 4, 4), np.uint8)] * 2
    og = fo.octant_graph(orc.build_batch(masks, brick=2))
    assert og.seg_off.tolist() == list(range(0, 129, 8))
    lin = lambda x, y, z: x + 4 * (y + 4 * z)
    seg = np.repeat(np.arange(16), 8)
    where = {int(v): s for v, s in zip(og.vox[:64], seg[:64])}
    assert where[lin(0, 0, 0)] == 0 and where[lin(1, 1, 1)] == 0
    assert where[lin(2, 0, 0)] == 1 and where[lin(3, 1, 1)] == 1
    assert where[lin(0, 2, 0)] == 2 and where[lin(0, 0, 2)] == 4
    assert where[lin(3, 3, 3)] == 7 and where[lin(2, 2, 2)] == 7
    assert int(seg[64 + 8 * 3]) == 11                    # volume 1, octant 3
    x = np.random.default_rng(0).random((5, og.n))
    t8 = orc.totals(og, x)
    gvol = orc.OracleGraph(og.shape, og.vox, og.nbr, og.seg_off[::8])
    np.testing.assert_allclose(t8.reshape(2, 8, 6).sum(axis=1), orc.totals(gvol, x), rtol=1e-14)
    # raster order is not octant-major: refused
    with pytest.raises(ValueError):
        fo.octant_graph(orc.build_batch(masks))


@pytest.mark.parametrize("vols", [None, [0, 2]])
def test_octant_dom_co2_loss_gradient_matches_central_differences(vols):
    """The loss on the per-octant DOM and CO2 curves (each divided by a scale),
    on whole volumes or a subset."""
    og, p, dt, x0 = octant_case()
    nsteps = 16
    truth = theta_of(p, [1.1, 0.9, 1.0, 1.05, 0.95, 1.0, 0.92, 1.08])
    tp, tc = fo.theta_to_params(truth, p)
    _, tot = orc.run(tp, dt, og, x0, nsteps, w=orc.edge_weights(og, orc.octant_regions(og), tc))
    target = tot[:, :, [1, 4]]
    scale = np.abs(target).max(axis=(0, 1))
    theta = theta_of(p)
    kw = dict(vols=vols, curves=(1, 4), scale=scale, segs_per_vol=8)
    loss, g = fo.loss_and_gradient(theta, p, dt, og, x0, target, **kw)

    def central(q, h):
        tp_, tm_ = theta.copy(), theta.copy()
        tp_[q] += h
        tm_[q] -= h
        return (fo.loss_and_gradient(tp_, p, dt, og, x0, target, **kw)[0]
                - fo.loss_and_gradient(tm_, p, dt, og, x0, target, **kw)[0]) / (2 * h)

    for q in (1, 5, 7, 12, 15, 19):
        h = 1e-3 * theta[q]
        fd = (4 * central(q, h / 2) - central(q, h)) / 3
        assert abs(g[q] - fd) <= 1e-4 * abs(fd), (q, g[q], fd)
