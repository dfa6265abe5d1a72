"""Pins of the PNGM oracle (oracle/pngm_oracle.py): the partition against a
voxel-by-voxel construction, scheme 3's and scheme 4's conservation and
fixed points, the two-primitive closed forms of both schemes, the objectives'
gradients against central differences and autograd, and zero loss on data
the network itself generated."""
import numpy as np
import pytest
import torch

from oracle import pngm_oracle as po
from paper_2406_04177_amd import inputs


def tiny_mask(seed=0, shape=(9, 11, 10)):
    return (np.random.default_rng(seed).random(shape) < 0.55).astype(np.uint8)


@pytest.mark.parametrize("seed,b", [(0, 3), (1, 4), (2, 5)])
def test_partition_brute_force(seed, b):
    mask = tiny_mask(seed)
    part = po.partition(mask, b)
    nz, ny, nx = mask.shape
    vox = [(z, y, x) for z in range(nz) for y in range(ny) for x in range(nx) if mask[z, y, x]]
    bricks = sorted({(z // b, y // b, x // b) for z, y, x in vox})
    bid = {br: k for k, br in enumerate(bricks)}
    prim = [bid[(z // b, y // b, x // b)] for z, y, x in vox]
    np.testing.assert_array_equal(part["prim"], prim)
    v = np.zeros(len(bricks))
    cen = np.zeros((len(bricks), 3))
    for (z, y, x), k in zip(vox, prim):
        v[k] += 1
        cen[k] += (x, y, z)
    cen /= v[:, None]
    np.testing.assert_array_equal(part["v"], v)
    S = {}
    pore = set(vox)
    for z, y, x in vox:
        for dz, dy, dx in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            o = (z + dz, y + dy, x + dx)
            if o in pore:
                i, j = bid[(z // b, y // b, x // b)], bid[(o[0] // b, o[1] // b, o[2] // b)]
                if i != j:
                    S[(i, j)] = S.get((i, j), 0) + 1
    keys = sorted(S)
    got = [(i, part["col"][e]) for i in range(part["q"]) for e in range(part["row"][i], part["row"][i + 1])]
    assert got == keys
    np.testing.assert_array_equal(part["S"], [S[k] for k in keys])
    np.testing.assert_allclose(part["d"], [np.linalg.norm(cen[i] - cen[j]) for i, j in keys], rtol=1e-14)


def setup(seed=3, b=4):
    mask = tiny_mask(seed, (12, 13, 14))
    part = po.partition(mask, b)
    theta = part["S"] / part["d"]
    rng = np.random.default_rng(seed)
    X = rng.random((3, part["q"])) * part["v"]
    return part, theta, X


def test_scheme3_conserves_mass_and_keeps_uniform_concentration():
    part, theta, X = setup()
    c = 0.3
    y = po.scheme3_step(part, X[0], theta, c)
    np.testing.assert_allclose(y.sum(), X[0].sum(), rtol=1e-14)      # theta symmetric
    uni = 2.5 * part["v"]
    np.testing.assert_allclose(po.scheme3_step(part, uni, theta, c), uni, rtol=1e-15)


@pytest.mark.parametrize("objective", [1, 2])
def test_gradient_matches_central_differences_and_autograd(objective):
    part, theta, X = setup()
    c = 0.3
    rng = np.random.default_rng(9)
    Y = X * (1 + 0.1 * rng.standard_normal(X.shape))
    th = theta * (1 + 0.2 * rng.standard_normal(theta.shape))
    loss, g = po.loss_grad(part, X, Y, th, c, objective)
    for e in rng.choice(th.size, 8, replace=False):
        h = 1e-6 * th[e]
        tp, tm = th.copy(), th.copy()
        tp[e] += h
        tm[e] -= h
        fd = (po.loss_grad(part, X, Y, tp, c, objective)[0] - po.loss_grad(part, X, Y, tm, c, objective)[0]) / (2 * h)
        assert abs(g[e] - fd) <= 1e-6 * abs(fd) + 1e-12 * loss, (e, g[e], fd)
    # an independent vectorised restatement, differentiated by torch
    v = torch.tensor(part["v"])
    src = torch.tensor(np.repeat(np.arange(part["q"]), np.diff(part["row"])))
    col = torch.tensor(part["col"])
    t = torch.tensor(th, requires_grad=True)
    Xt, Yt = torch.tensor(X), torch.tensor(Y)
    z = Xt if objective == 1 else Yt
    flux = torch.zeros_like(Xt).index_add_(1, src, t * (z[:, src] / v[src] - z[:, col] / v[col]))
    r = (Yt - Xt + c * flux) if objective == 1 else (Xt - Yt - c * flux)
    L = (r ** 2).mean()
    L.backward()
    np.testing.assert_allclose(float(L), loss, rtol=1e-13)
    np.testing.assert_allclose(t.grad.numpy(), g, rtol=1e-10, atol=1e-14 * np.abs(g).max())


def test_zero_loss_on_data_of_the_network_itself():
    part, theta, X = setup()
    c = 0.3
    Y1 = np.stack([po.scheme3_step(part, x, theta, c) for x in X])
    l1, g1 = po.loss_grad(part, X, Y1, theta, c, 1)
    assert l1 <= 1e-28 * np.mean(X ** 2)
    # scheme 4 data: x = y + c sum theta (y_i/v_i - y_j/v_j)
    Y2 = X
    X2 = np.stack([2 * y - po.scheme3_step(part, y, theta, c) for y in Y2])
    l2, _ = po.loss_grad(part, X2, Y2, theta, c, 2)
    assert l2 <= 1e-28 * np.mean(X ** 2)


def test_scheme4_two_primitives_closed_form():
    """Two primitives joined by theta both ways: the concentration difference
    is divided by 1 + c theta (1/v1 + 1/v2) per implicit step (the explicit
    step multiplies it by 1 - c theta (1/v1 + 1/v2)); total mass is kept."""
    mask = np.zeros((1, 1, 6), np.uint8)
    mask[0, 0, 1:5] = 1                       # bricks of 3: voxels {1,2} and {3,4}
    part = po.partition(mask, 3)
    assert part["q"] == 2 and list(part["v"]) == [2.0, 2.0] and list(part["S"]) == [1.0, 1.0]
    theta = np.array([0.7, 0.7])
    c = 1.3
    m = np.array([3.0, 1.0])
    ds = m[0] / 2 - m[1] / 2
    k = c * 0.7 * (1 / 2 + 1 / 2)
    y = po.scheme4_step(part, m, theta, c)
    np.testing.assert_allclose(y[0] / 2 - y[1] / 2, ds / (1 + k), rtol=1e-14)
    np.testing.assert_allclose(y.sum(), m.sum(), rtol=1e-15)
    y3 = po.scheme3_step(part, m, theta, c)
    np.testing.assert_allclose(y3[0] / 2 - y3[1] / 2, ds * (1 - k), rtol=1e-14)


def test_scheme4_conserves_keeps_uniform_and_zeroes_L2():
    part, theta, X = setup()
    c = 0.8
    y = po.scheme4_step(part, X[0], theta, c)
    np.testing.assert_allclose(y.sum(), X[0].sum(), rtol=1e-13)        # theta symmetric
    uni = 1.5 * part["v"]
    np.testing.assert_allclose(po.scheme4_step(part, uni, theta, c), uni, rtol=1e-13)
    # data the implicit network generated leaves objective 2 at zero (up to the solve's rounding)
    Y = np.stack([po.scheme4_step(part, x, theta, c) for x in X])
    l2, _ = po.loss_grad(part, X, Y, theta, c, 2)
    assert l2 <= 1e-26 * np.mean(X ** 2)
    # for small c the implicit and explicit steps agree to O(c^2)
    e1 = np.abs(po.scheme4_step(part, X[0], theta, 1e-3) - po.scheme3_step(part, X[0], theta, 1e-3)).max()
    e2 = np.abs(po.scheme4_step(part, X[0], theta, 5e-4) - po.scheme3_step(part, X[0], theta, 5e-4)).max()
    assert 3.5 < e1 / e2 < 4.5


def test_normalised_gradient_descent_recovers_known_conductances():
    """Data made by scheme 4 with known conductances theta* (0.5-2x the
    starting S/d, symmetric): the normalised-gradient descent of Sec. V.A on
    objective 2, started from S/d, lowers the loss by more than 100x and
    moves theta towards theta*."""
    from oracle import fit_oracle as fo
    part, theta0, X = setup(seed=5)
    rng = np.random.default_rng(11)
    # one factor per unordered pair: theta* symmetric like the truth it stands for
    fac = {}
    theta_true = theta0.copy()
    for i in range(part["q"]):
        for e in range(part["row"][i], part["row"][i + 1]):
            key = (min(i, part["col"][e]), max(i, part["col"][e]))
            fac.setdefault(key, rng.uniform(0.5, 2.0))
            theta_true[e] *= fac[key]
    c = 0.8
    Xs = rng.random((6, part["q"])) * part["v"]
    Ys = np.stack([po.scheme4_step(part, x, theta_true, c) for x in Xs])

    def grad_fn(theta, epoch):
        return po.loss_grad(part, Xs, Ys, theta, c, 2)
    which = range(theta0.size)
    hist, losses = fo.sign_sgd(theta0, grad_fn, 60, which, lr=0.1, halve_every=10, box=(0.05, 20.0))
    final_loss = grad_fn(hist[-1], 0)[0]
    assert final_loss < 1e-2 * losses[0]
    err0 = np.mean(np.abs(theta0 - theta_true) / theta_true)
    err1 = np.mean(np.abs(hist[-1] - theta_true) / theta_true)
    assert err1 < 0.5 * err0, (err0, err1)
