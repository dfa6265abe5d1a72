"""The fitting loop on the GPU (library adjoint + normalised-gradient SGD of
Sec. V) against the fitting oracle: at every epoch of the GPU's trajectory
the loss equals the oracle's loss at the same parameters, and every move is
the one the oracle's gradient prescribes (several moves are correct only
where a derivative is within rounding of zero: there any of -step, 0, +step
is accepted)."""
import numpy as np
import pytest
import torch

from oracle import fit_oracle as fo
from oracle import oracle as orc
from paper_2406_04177_amd import inputs

pytestmark = pytest.mark.gpu


def case():
    masks = [inputs.synthetic_volume((18, 16, 14), porosity=por, seed=b) for b, por in enumerate((0.25, 0.3, 0.2))]
    specs = [inputs.init_random_all(m, b) for b, m in enumerate(masks)]
    p = inputs.ModelParams(D=(0, 1e-9, 0, 0, 0), v_dom=2e-3, k_dom=0.5, rho=3e-4, mu=2e-4, beta=0.55,
                           v_som=1e-4, v_p4=2e-4)
    dt = inputs.explicit_dt(p, 0.8)
    return masks, specs, p, dt


def theta_np(p, c=None):
    return np.array(list(p.D) + [p.v_dom, p.k_dom, p.rho, p.mu, p.beta, p.v_som, p.v_p4] + list(c or [1.0] * 8))


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_fit_follows_the_oracle(precision):
    from paper_2406_04177_amd.fit import fit
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    masks, specs, p, dt = case()
    og = orc.build_batch(masks)
    x0o = orc.fields_from_spec(og, specs)
    nsteps, epochs = 30, 14
    truth = theta_np(p, [1.08, 0.93, 1.05, 0.9, 1.1, 0.95, 1.02, 0.97])
    truth[1] *= 1.07
    truth[7] *= 0.9137
    tp, tc = fo.theta_to_params(truth, p)
    _, tot = orc.run(tp, dt, og, x0o, nsteps, w=orc.edge_weights(og, orc.octant_regions(og), tc))
    target = tot[:, :, 4]
    theta0 = theta_np(p)
    which = [1, 5, 7] + list(range(12, 20))
    subsets = inputs.epoch_subsets(len(masks), 2, epochs, seed=0)
    g = Graph.from_masks(masks, regions=True)
    sim = Simulation(g, p, precision=precision, implicit=False, adjoint=True, regions=[1.0] * 8)
    x0 = g.fields_from_specs(specs, torch.float64 if precision == "f64" else torch.float32)
    hist, losses = fit(sim, x0, torch.as_tensor(target, device="cuda"), torch.as_tensor(theta0), nsteps, dt, which,
                       epochs=epochs, checkpoint_every=7, subsets=subsets)
    # FP64: loss to rounding and every robust move.  FP32: the CO2 totals
    # carry up to 4 k 2^-24 relative error after k steps, which moves the
    # loss (a mean of squared differences d) by up to 2 eps max|T| sqrt(L);
    # moves are checked where the derivative is well above the FP32 gradient
    # error
    robust = 1e-6 if precision == "f64" else 1e-2
    eps = 4 * nsteps * 2.0 ** -24
    tmax = np.abs(tot[:, :, 4]).max()
    others = [q for q in range(20) if q not in which]
    for e in range(epochs):
        lo, go = fo.loss_and_gradient(hist[e], p, dt, og, x0o, target, subsets[e])
        tol = 1e-10 * lo if precision == "f64" else 2 * eps * tmax * np.sqrt(lo) + 1e-6 * lo
        assert abs(losses[e] - lo) <= tol, (e, losses[e], lo)
        rate = 0.1 * 0.5 ** (e // 10)
        gmax = np.abs(go[which]).max()
        for q in which:
            lo_q, hi_q = 0.5 * theta0[q], 1.5 * theta0[q]       # the fit's box
            moves = [-np.sign(go[q])] if abs(go[q]) > robust * gmax else [-1.0, 0.0, 1.0]
            allowed = [min(max(hist[e][q] + m * rate * theta0[q], lo_q), hi_q) for m in moves]
            assert min(abs(hist[e + 1][q] - a) for a in allowed) <= 1e-12 * theta0[q], (e, q, hist[e + 1][q], allowed)
        np.testing.assert_array_equal(hist[e + 1][others], theta0[others])
    assert losses[-1] < losses[0]


def test_adam_variant_reduces_the_loss():
    from paper_2406_04177_amd.fit import fit
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    masks, specs, p, dt = case()
    og = orc.build_batch(masks)
    x0o = orc.fields_from_spec(og, specs)
    truth = theta_np(p)
    truth[7] *= 0.9137
    tp, tc = fo.theta_to_params(truth, p)
    _, tot = orc.run(tp, dt, og, x0o, 30, w=orc.edge_weights(og, orc.octant_regions(og), tc))
    g = Graph.from_masks(masks, regions=True)
    sim = Simulation(g, p, precision="f64", implicit=False, adjoint=True, regions=[1.0] * 8)
    hist, losses = fit(sim, g.fields_from_specs(specs, torch.float64), torch.as_tensor(tot[:, :, 4], device="cuda"),
                       torch.as_tensor(theta_np(p)), 30, dt, [7], epochs=30, checkpoint_every=10, lr=0.05,
                       method="adam")
    assert losses[-1] < 0.1 * losses[0]
    assert abs(hist[-1][7] / truth[7] - 1) < 0.03


def test_octant_dom_co2_fit_follows_the_oracle():
    """The loss on per-octant DOM and CO2 curves (three 16^3 volumes in
    bricks of 8, one segment per octant; D_DOM held as the gauge of the
    D c_r products): segment offsets, every epoch's loss and every move
    against the oracle (FP64)."""
    from paper_2406_04177_amd.fit import fit, octant_segments
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    masks = [inputs.synthetic_volume((16, 16, 16), porosity=por, seed=b) for b, por in enumerate((0.3, 0.35, 0.25))]
    specs = [inputs.init_random_all(m, b) for b, m in enumerate(masks)]
    p = inputs.ModelParams(D=(0, 1e-9, 0, 0, 0), v_dom=2e-3, k_dom=0.5, rho=3e-4, mu=2e-4, beta=0.55,
                           v_som=1e-4, v_p4=2e-4)
    dt = inputs.explicit_dt(p, 0.8 / 1.5 ** 2)
    ogb = orc.build_batch(masks, brick=8)
    og = fo.octant_graph(ogb)
    x0o = orc.fields_from_spec(ogb, specs)
    nsteps, epochs = 24, 12
    truth = theta_np(p, [1.08, 0.93, 1.05, 0.9, 1.1, 0.95, 1.02, 0.97])
    truth[5] *= 1.06
    truth[7] *= 0.93
    tp, tc = fo.theta_to_params(truth, p)
    _, tot = orc.run(tp, dt, og, x0o, nsteps, w=orc.edge_weights(og, orc.octant_regions(og), tc))
    target = tot[:, :, [1, 4]]
    scale = np.abs(target).max(axis=(0, 1))
    theta0 = theta_np(p)
    which = [5, 7] + list(range(12, 20))
    subsets = inputs.epoch_subsets(len(masks), 2, epochs, seed=1)
    g = Graph.from_masks(masks, brick=8, regions=True)
    seg = octant_segments(g)
    np.testing.assert_array_equal(seg, og.seg_off)
    sim = Simulation(g, p, precision="f64", implicit=False, adjoint=True, regions=[1.0] * 8, segments=seg)
    x0 = g.fields_from_specs(specs, torch.float64)
    hist, losses = fit(sim, x0, torch.as_tensor(target, device="cuda"), torch.as_tensor(theta0), nsteps, dt, which,
                       epochs=epochs, checkpoint_every=5, subsets=subsets, curves=(1, 4), curve_scale=scale, segs_per_vol=8)
    others = [q for q in range(20) if q not in which]
    for e in range(epochs):
        lo, go = fo.loss_and_gradient(hist[e], p, dt, og, x0o, target, subsets[e], curves=(1, 4), scale=scale,
                                      segs_per_vol=8)
        assert abs(losses[e] - lo) <= 1e-10 * lo, (e, losses[e], lo)
        rate = 0.1 * 0.5 ** (e // 10)
        gmax = np.abs(go[which]).max()
        for q in which:
            lo_q, hi_q = 0.5 * theta0[q], 1.5 * theta0[q]
            moves = [-np.sign(go[q])] if abs(go[q]) > 1e-6 * gmax else [-1.0, 0.0, 1.0]
            allowed = [min(max(hist[e][q] + m * rate * theta0[q], lo_q), hi_q) for m in moves]
            assert min(abs(hist[e + 1][q] - a) for a in allowed) <= 1e-12 * theta0[q], (e, q, hist[e + 1][q], allowed)
        np.testing.assert_array_equal(hist[e + 1][others], theta0[others])
    assert losses[-1] < losses[0]


def test_gauss_newton_recovers_the_identifiable_parameters():
    """The Gauss-Newton refinement (FP64 forward, central-difference
    Jacobian, truncated SVD) on the per-octant DOM and CO2 curves of three
    16^3 volumes, against a target the oracle computes at perturbed
    parameters: v_DOM, rho and the products D_DOM c_r return to the
    generating values, D_DOM (the gauge) and the parameters not fitted stay,
    and the misfit falls to rounding."""
    from paper_2406_04177_amd.fit import gauss_newton, octant_segments
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    masks = [inputs.synthetic_volume((16, 16, 16), porosity=por, seed=b) for b, por in enumerate((0.3, 0.35, 0.25))]
    specs = [inputs.init_random_all(m, b) for b, m in enumerate(masks)]
    p = inputs.ModelParams(D=(0, 1e-9, 0, 0, 0), v_dom=2e-3, k_dom=0.5, rho=3e-4, mu=2e-4, beta=0.55,
                           v_som=1e-4, v_p4=2e-4)
    dt = inputs.explicit_dt(p, 0.8 / 1.5 ** 2)
    ogb = orc.build_batch(masks, brick=8)
    og = fo.octant_graph(ogb)
    x0o = orc.fields_from_spec(ogb, specs)
    nsteps = 24
    truth = theta_np(p, [1.08, 0.93, 1.05, 0.9, 1.1, 0.95, 1.02, 0.97])
    truth[1] *= 1.04
    truth[5] *= 1.06
    truth[7] *= 0.93
    tp, tc = fo.theta_to_params(truth, p)
    _, tot = orc.run(tp, dt, og, x0o, nsteps, w=orc.edge_weights(og, orc.octant_regions(og), tc))
    target = tot[:, :, [1, 4]]
    scale = np.abs(target).max(axis=(0, 1))
    theta0 = theta_np(p)
    which = [5, 7] + list(range(12, 20))
    g = Graph.from_masks(masks, brick=8, regions=True)
    seg = octant_segments(g)
    sim = Simulation(g, p, precision="f64", implicit=False, adjoint=False, regions=[1.0] * 8, segments=seg)
    x0 = g.fields_from_specs(specs, torch.float64)
    hist, norms = gauss_newton(sim, torch.as_tensor(theta0), x0, torch.as_tensor(target, device="cuda"), nsteps, dt,
                               which, curves=(1, 4), scale=scale, iters=4, checkpoint_every=5)

    def combos(t):
        return np.array([t[1] * t[12 + r] for r in range(8)] + [t[5], t[7]])

    err = np.abs(combos(hist[-1]) / combos(truth) - 1)
    print("Gauss-Newton: squared misfit", norms, "combination errors", err)
    assert err.max() < 1e-8, err
    others = [q for q in range(20) if q not in which]
    np.testing.assert_array_equal(hist[-1][others], theta0[others])
    assert norms[-1] < 1e-18 * norms[0]
