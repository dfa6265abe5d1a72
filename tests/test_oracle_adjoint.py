"""Pins of the oracle's discrete adjoint (gradients of a loss on the mass-total
curves with respect to the initial state, the diffusion coefficients, the
kinetic rates and the region conductance factors).

Independent references: torch autograd through the vectorised FP64 restatement
in ``oracle/torch_ref.py`` (exact to rounding), central finite differences of
the C oracle's forward, the transposition identity <J v, w> = <v, J^T w>, and
the invariant that a CO2-only loss leaves dL/dD_CO2 = 0.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from oracle import torch_ref
from paper_2406_04177_amd.inputs import ModelParams

torch.set_default_dtype(torch.float64)


def setup(seed=0, nvol=2, shape=(6, 7, 6), clamps=False):
    rng = np.random.default_rng(seed)
    masks = [(rng.random(shape) < 0.6).astype(np.uint8) for _ in range(nvol)]
    g = orc.build_batch(masks)
    x = rng.random((5, g.n)) * np.array([[0.5], [1.0], [0.3], [0.2], [0.1]])
    if clamps:
        p = ModelParams(D=(2e-10, 1e-9, 0.0, 4e-10, 0.0), v_dom=0.9, k_dom=0.05, rho=0.4, mu=0.3,
                        beta=0.55, v_som=0.9, v_p4=1.5)
        dt = 0.8
    else:
        p = ModelParams(D=(2e-10, 1e-9, 0.0, 4e-10, 0.0), v_dom=2e-2, k_dom=0.5, rho=3e-3, mu=2e-3,
                        beta=0.55, v_som=1e-3, v_p4=2e-3)
        dt = 0.08
    region = orc.octant_regions(g)
    c = rng.uniform(0.6, 1.0, 8)
    w = orc.edge_weights(g, region, c)
    return rng, g, x, p, dt, region, c, w


def torch_grads(g, x, p, dt, region, c, seeds, nsteps, order, mort_to_p4=False):
    D = torch.tensor(p.D, requires_grad=True)
    names = torch_ref.RATE_NAMES
    vals = dict(v_dom=p.v_dom, k_dom=p.k_dom, rho=p.rho, mu=p.mu, beta=p.beta, v_som=p.v_som,
                v_p4=p.v_p4)
    r = {k: torch.tensor(vals[k], requires_grad=True) for k in names}
    ct = torch.tensor(c, requires_grad=True)
    x0 = torch.tensor(x, requires_grad=True)
    tot = torch_ref.run_totals(x0, torch.tensor(g.nbr), torch.tensor(region), ct, D, r, dt, p.h,
                               nsteps, g.seg_off, order=order, mort_to_p4=mort_to_p4)
    loss = (tot * torch.tensor(seeds)).sum()
    loss.backward()
    grad = np.concatenate([D.grad.numpy(), [r[k].grad.item() if r[k].grad is not None else 0.0 for k in names], ct.grad.numpy()])
    return x0.grad.numpy(), grad, tot.detach().numpy()


@pytest.mark.parametrize("order,clamps,route", [(0, False, False), (1, False, False),
                                                (0, True, False), (0, False, True),
                                                (1, True, True)])
def test_adjoint_equals_torch_autograd(order, clamps, route):
    rng, g, x, p, dt, region, c, w = setup(seed=order + 2 * clamps, clamps=clamps)
    p = p.replace(mort_to_p4=route)
    nsteps = 6
    seeds = rng.standard_normal((nsteps + 1, g.nseg, 5))
    states = orc.run_states(p, dt, g, x, nsteps, order=order, w=w)
    lam0, grad = orc.adjoint(p, dt, g, states, seeds, order=order, w=w, region=region, nreg=8)
    lam_t, grad_t, tot_t = torch_grads(g, x, p, dt, region, c, seeds, nsteps, order, route)
    # same forward
    _, tot = orc.run(p, dt, g, x, nsteps, order=order, w=w)
    np.testing.assert_allclose(tot[:, :, :5], tot_t, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(lam0, lam_t, rtol=1e-11, atol=1e-13)
    scale = np.abs(grad_t).max()
    np.testing.assert_allclose(grad, grad_t, rtol=1e-9, atol=1e-12 * scale)


def test_transposition_identity():
    """<J v, u> = <v, J^T u> for the Jacobian of x^S with respect to x^0."""
    rng, g, x, p, dt, region, c, w = setup(seed=5)
    nsteps = 4
    v = rng.standard_normal(x.shape)
    u = rng.standard_normal(x.shape)
    states = orc.run_states(p, dt, g, x, nsteps, w=w)
    seeds = np.zeros((nsteps + 1, g.nseg, 5))
    JTu, _ = orc.adjoint(p, dt, g, states, seeds, w=w, region=region, nreg=8, lam_final=u)

    D = torch.tensor(p.D)
    r = {k: torch.tensor(getattr(p, k)) for k in torch_ref.RATE_NAMES}

    def f(x0):
        return torch_ref.run_state(x0, torch.tensor(g.nbr), torch.tensor(region), torch.tensor(c),
                                   D, r, dt, p.h, nsteps)

    _, Jv = torch.func.jvp(f, (torch.tensor(x),), (torch.tensor(v),))
    lhs = float((Jv.numpy() * u).sum())
    rhs = float((v * JTu).sum())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # and central differences of the C forward
    eps = 1e-6
    fp, _ = orc.run(p, dt, g, x + eps * v, nsteps, w=w, with_totals=False)
    fm, _ = orc.run(p, dt, g, x - eps * v, nsteps, w=w, with_totals=False)
    fd = float((((fp - fm) / (2 * eps)) * u).sum())
    assert abs(fd - rhs) <= 1e-7 * abs(rhs)


def co2_mse_loss_and_seeds(tot, target):
    """L = mean over (step, volume) of (CO2 total - target)^2 and dL/dTotals."""
    S1, B = tot.shape[0], tot.shape[1]
    diff = tot[:, :, 4] - target
    L = (diff ** 2).sum() / (S1 * B)
    seeds = np.zeros((S1, B, 5))
    seeds[:, :, 4] = 2 * diff / (S1 * B)
    return L, seeds


def test_parameter_gradient_matches_central_differences():
    rng, g, x, p, dt, region, c, w = setup(seed=7)
    # every pool that a step of -eps could push below zero gets D > 0, so both
    # sides of the difference take the same clamp branches
    p = p.replace(D=(2e-10, 1e-9, 1e-10, 4e-10, 0.0))
    nsteps = 20
    target = orc.run(p.replace(rho=p.rho * 1.05, v_dom=p.v_dom * 0.95), dt, g, x, nsteps, w=w)[1][:, :, 4]
    states = orc.run_states(p, dt, g, x, nsteps, w=w)
    _, tot = orc.run(p, dt, g, x, nsteps, w=w)
    L0, seeds = co2_mse_loss_and_seeds(tot, target)
    _, grad = orc.adjoint(p, dt, g, states, seeds, w=w, region=region, nreg=8)

    def loss_at(pp, cc):
        ww = orc.edge_weights(g, region, cc)
        _, t = orc.run(pp, dt, g, x, nsteps, w=ww)
        return co2_mse_loss_and_seeds(t, target)[0]

    names = ["D%d" % s for s in range(5)] + list(torch_ref.RATE_NAMES)
    for q, name in enumerate(names):
        if q < 5:
            # pools with D = 0 have tiny gradients: a wider step keeps the
            # difference above the rounding of L (the loss is nearly linear in D)
            eps = max(1e-4 * p.D[q], 1e-11)
            Dp, Dm = list(p.D), list(p.D)
            Dp[q] += eps
            Dm[q] -= eps
            fd = (loss_at(p.replace(D=tuple(Dp)), c) - loss_at(p.replace(D=tuple(Dm)), c)) / (2 * eps)
        else:
            attr = torch_ref.RATE_NAMES[q - 5]
            val = getattr(p, attr)
            eps = 1e-4 * val
            fd = (loss_at(p.replace(**{attr: val + eps}), c) - loss_at(p.replace(**{attr: val - eps}), c)) / (2 * eps)
        assert abs(grad[q] - fd) <= 1e-4 * abs(fd) + 1e-9 * np.abs(grad).max(), (name, grad[q], fd)
    for r in range(8):
        eps = 1e-4 * c[r]
        cp, cm = c.copy(), c.copy()
        cp[r] += eps
        cm[r] -= eps
        fd = (loss_at(p, cp) - loss_at(p, cm)) / (2 * eps)
        assert abs(grad[12 + r] - fd) <= 1e-4 * abs(fd) + 1e-9 * np.abs(grad).max(), (r, grad[12 + r], fd)


def test_co2_only_loss_gives_zero_dD_co2():
    """A loss on CO2 totals only seeds a spatially uniform adjoint on CO2 in each
    volume; since every row of the Laplacian sums to zero, dL/dD_CO2 = 0."""
    rng, g, x, p, dt, region, c, w = setup(seed=9, nvol=3)
    nsteps = 10
    states = orc.run_states(p, dt, g, x, nsteps, w=w)
    seeds = np.zeros((nsteps + 1, g.nseg, 5))
    seeds[:, :, 4] = rng.standard_normal((nsteps + 1, g.nseg))
    lam0, grad = orc.adjoint(p, dt, g, states, seeds, w=w, region=region, nreg=8)
    # bound on what rounding can leave of sum_i lambda_i sum_j w_ij (u_j - u_i)
    lam_max = np.abs(np.cumsum(seeds[::-1, :, 4], axis=0)).max()
    gross = 0.0
    for t in range(nsteps):
        u = states[t, 4]
        for k in range(6):
            j = g.nbr[k]
            ok = j >= 0
            gross += np.abs(w[k, ok] * (u[j[ok]] - u[ok])).sum()
    gross *= lam_max * dt / p.h ** 2
    assert gross > 0
    assert abs(grad[4]) <= 1e-12 * gross
    for b in range(g.nseg):
        seg = lam0[4, g.seg_off[b]:g.seg_off[b + 1]]
        assert np.all(seg == seg[0])
