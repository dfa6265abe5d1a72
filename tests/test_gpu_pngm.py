"""Pore-network objectives on the GPU (brick partition, primitive masses,
L1/L2 and gradients, scheme 3, the normalised-gradient update, data from the
voxel method, fitting) against the PNGM oracle."""
import numpy as np
import pytest
import torch

from oracle import fit_oracle as fo
from oracle import oracle as orc
from oracle import pngm_oracle as po
from paper_2406_04177_amd import inputs

pytestmark = pytest.mark.gpu

B = 8


@pytest.fixture(scope="module")
def vol():
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd import pngm
    mask = inputs.synthetic_volume((44, 40, 36), porosity=0.3, seed=4)
    g = Graph.from_masks(mask, brick=B)
    return mask, g, pngm.partition(g, B), po.partition(mask, B)


def test_partition_equals_oracle(vol):
    mask, g, part, ref = vol
    assert part.q == ref["q"]
    np.testing.assert_array_equal(part.v.cpu().numpy(), ref["v"])
    np.testing.assert_array_equal(part.row.cpu().numpy(), ref["row"])
    np.testing.assert_array_equal(part.col.cpu().numpy(), ref["col"])
    np.testing.assert_array_equal(part.S, ref["S"])
    np.testing.assert_array_equal(part.d, ref["d"])     # same operations in the same order
    np.testing.assert_array_equal(part.offsets.cpu().numpy(), np.concatenate([[0], np.cumsum(ref["v"])]))


@pytest.mark.parametrize("shape,por,b,seed", [((13, 11, 17), 0.5, 3, 1), ((20, 9, 14), 0.2, 5, 2),
                                              ((8, 8, 8), 0.9, 16, 3), ((6, 7, 5), 0.6, 1, 4),
                                              ((33, 18, 25), 0.35, 8, 5), ((10, 10, 10), 0.0, 4, 6)])
def test_partition_raw_masks(shape, por, b, seed):
    """Unfiltered random masks (isolated voxels, empty bricks, ragged bricks
    at the far faces, one brick bigger than the box, one voxel per brick, no
    pore at all): the device-assembled primitive graph equals the oracle's,
    integers and distances bit for bit."""
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd import pngm
    rng = np.random.default_rng(seed)
    mask = (rng.random(shape) < por).astype(np.uint8)
    g = Graph.from_masks(mask, brick=b)
    part = pngm.partition(g, b)
    ref = po.partition(mask, b)
    assert part.q == ref["q"]
    np.testing.assert_array_equal(part.v.cpu().numpy(), ref["v"])
    np.testing.assert_array_equal(part.row.cpu().numpy(), ref["row"])
    np.testing.assert_array_equal(part.col.cpu().numpy(), ref["col"])
    np.testing.assert_array_equal(part.S, ref["S"])
    np.testing.assert_array_equal(part.d, ref["d"])
    np.testing.assert_array_equal(part.offsets.cpu().numpy(), np.concatenate([[0], np.cumsum(ref["v"])]))
    # the bricks of the primitives, from the oracle's voxel-to-primitive map
    nz, ny, nx = shape
    nbx, nby = -(-nx // b), -(-ny // b)
    zz, yy, xx = np.nonzero(mask)
    brick = (zz // b * nby + yy // b) * nbx + xx // b
    np.testing.assert_array_equal(part.bricks, np.unique(brick))


def test_primitive_masses_equal_oracle(vol):
    from paper_2406_04177_amd import pngm
    mask, g, part, ref = vol
    spec = inputs.init_scenario(mask, 3, frac=0.2)
    x = g.fields_from_specs(spec, torch.float64)
    got = pngm.primitive_masses(part, x[1]).cpu().numpy()
    og = orc.build_graph(mask)
    xo = orc.fields_from_spec(og, spec)
    np.testing.assert_allclose(got, po.primitive_masses(ref, xo[1]), rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("objective", [1, 2])
def test_loss_grad_step_and_update_equal_oracle(vol, objective):
    from paper_2406_04177_amd import pngm
    mask, g, part, ref = vol
    rng = np.random.default_rng(objective)
    X = rng.random((4, ref["q"])) * ref["v"]
    Y = X * (1 + 0.05 * rng.standard_normal(X.shape))
    theta = (ref["S"] / ref["d"]) * (1 + 0.1 * rng.standard_normal(ref["S"].size))
    c = 2.5
    loss_o, grad_o = po.loss_grad(ref, X, Y, theta, c, objective)
    dev = "cuda"
    loss, grad = pngm.loss_grad(part, torch.as_tensor(X, device=dev), torch.as_tensor(Y, device=dev),
                                torch.as_tensor(theta, device=dev), c, objective)
    np.testing.assert_allclose(float(loss), loss_o, rtol=1e-12)
    np.testing.assert_allclose(grad.cpu().numpy(), grad_o, rtol=1e-12, atol=1e-15 * np.abs(grad_o).max())
    m = torch.as_tensor(X[0], device=dev)
    np.testing.assert_allclose(pngm.step(part, m, torch.as_tensor(theta, device=dev), c).cpu().numpy(),
                               po.scheme3_step(ref, X[0], theta, c), rtol=1e-14, atol=1e-14 * X[0].max())
    # one normalised-gradient step, box [0.05, 20] of the start
    t0 = ref["S"] / ref["d"]
    th = torch.as_tensor(theta, device=dev)
    t0d = torch.as_tensor(t0, device=dev)
    pngm.sign_update(th, grad, 0.1, t0d, t0d * 0.05, t0d * 20.0)
    expect = np.clip(theta - 0.1 * t0 * np.sign(grad_o), 0.05 * t0, 20.0 * t0)
    robust = np.abs(grad_o) > 1e-9 * np.abs(grad_o).max()
    np.testing.assert_allclose(th.cpu().numpy()[robust], expect[robust], rtol=1e-15)


def oracle_data(mask, scenarios, records, every_s, dt=0.1):
    from paper_2406_04177_amd import pngm
    og = orc.build_graph(mask)
    ref = po.partition(mask, B)
    p = pngm.pngm_params()
    out = np.zeros((len(scenarios), records + 1, ref["q"]))
    nper = int(round(every_s / dt))
    for k, seed in enumerate(scenarios):
        x = orc.fields_from_spec(og, inputs.init_scenario(mask, seed))
        out[k, 0] = po.primitive_masses(ref, x[1])
        for r in range(records):
            x, _ = orc.run(p, dt, og, x, nper, with_totals=False)
            out[k, r + 1] = po.primitive_masses(ref, x[1])
    return ref, out


def test_data_and_fit_follow_the_oracle(vol):
    """Voxel-method data (4 scenarios, 6 records 2 s apart) equal the oracle's;
    then the GPU fit on objective 2 moves, at every epoch, as the oracle's
    gradient at the GPU's parameters prescribes (robust signs)."""
    from paper_2406_04177_amd import pngm
    mask, g, part, _ = vol
    scen, records, every = [0, 1, 2, 3], 6, 2.0
    data = pngm.generate(g, part, mask, scen, records, every)
    ref, odata = oracle_data(mask, scen, records, every)
    np.testing.assert_allclose(data.cpu().numpy(), odata, rtol=1e-11, atol=1e-14)
    X = data[:, :-1].reshape(-1, part.q)
    Y = data[:, 1:].reshape(-1, part.q)
    Xo = odata[:, :-1].reshape(-1, ref["q"])
    Yo = odata[:, 1:].reshape(-1, ref["q"])
    c = 100950.0 / 86400.0 * every
    epochs = 25
    theta, losses, hist, batches = pngm.fit(part, X, Y, c, epochs, batch=4, objective=2, record=True)
    t0 = ref["S"] / ref["d"]
    for e in range(epochs):
        lo, go = po.loss_grad(ref, Xo[batches[e]], Yo[batches[e]], hist[e], c, 2)
        assert abs(losses[e] - lo) <= 1e-9 * lo, (e, losses[e], lo)
        rate = 0.1 * 0.5 ** (e // 10)
        robust = np.abs(go) > 1e-6 * np.abs(go).max()
        expect = np.clip(hist[e] - rate * t0 * np.sign(go), 0.05 * t0, 20.0 * t0)
        np.testing.assert_allclose(hist[e + 1][robust], expect[robust], rtol=1e-14)
    assert losses[-5:].mean() < losses[:5].mean()


def test_implicit_step_equals_dense_solve(vol):
    """Scheme 4 by Jacobi sweeps on the GPU against the oracle's dense solve,
    at c = D * 10 s (the data spacing) with perturbed, non-symmetric theta;
    the reported residual is the result's own; a sweep cap below what is
    needed is reported as VG_ENOCONV."""
    from paper_2406_04177_amd import _lib, pngm
    mask, g, part, ref = vol
    rng = np.random.default_rng(5)
    m = rng.random(ref["q"]) * ref["v"]
    theta = (ref["S"] / ref["d"]) * (1 + 0.3 * rng.random(ref["S"].size))
    c = 100950.0 / 86400.0 * 10.0
    expect = po.scheme4_step(ref, m, theta, c)
    dev = "cuda"
    th = torch.as_tensor(theta, device=dev)
    y, it, rel = pngm.implicit_step(part, torch.as_tensor(m, device=dev), th, c, rtol=1e-13)
    assert rel <= 1e-13 and it > 0
    y = y.cpu().numpy()
    np.testing.assert_allclose(y, expect, rtol=0, atol=1e-10 * np.abs(expect).max())
    # the residual of the definition, in mass units, from the oracle's side
    A_y = y + c * np.array([sum(theta[e] * (y[i] / ref["v"][i] - y[ref["col"][e]] / ref["v"][ref["col"][e]])
                                for e in range(ref["row"][i], ref["row"][i + 1])) for i in range(ref["q"])])
    assert np.linalg.norm(A_y - m) <= 2e-13 * np.linalg.norm(m)
    with pytest.raises(_lib.VgError) as err:
        pngm.implicit_step(part, torch.as_tensor(m, device=dev), th, c, rtol=1e-13, max_iter=3)
    assert err.value.code == _lib.VG_ENOCONV
