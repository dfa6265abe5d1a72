"""Implicit step (Sec. II.B.3b Scheme 2; Jacobi PCG, Sec. III) on the GPU vs
the oracle.  Several answers are correct (any iterate within rtol), so the
checks are: the GPU iterate's true residual, computed by the oracle's own
matrix, is <= rtol (plus a rounding allowance); the GPU answer is within
kappa(B) * rtol of the oracle's tight solve; the transformation half is
bit-identical; the iteration count is close to the oracle's PCG."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2406_04177_amd import inputs

pytestmark = pytest.mark.gpu


KERNELS = pytest.mark.parametrize("kernel", [1, 3, 4], ids=["table", "offset", "relative"])


def make(shape=(32, 30, 28), seed=1, regions=None, precision="f64", kernel=0):
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    mask = inputs.synthetic_volume(shape, seed=seed)
    spec = inputs.init_random_all(mask, seed)
    g = Graph.from_masks(mask, regions=regions is not None)
    og = orc.build_graph(mask)
    p = inputs.ModelParams(mu=1e-4, rho=5e-5)
    sim = Simulation(g, p, precision=precision, implicit=True, regions=regions)
    sim.set_kernel(kernel)
    sim.set_fields(g.fields_from_specs(spec, torch.float64))
    return sim, og, orc.fields_from_spec(og, spec), p


@KERNELS
@pytest.mark.parametrize("factor", [1.0, 20.0])
def test_implicit_step_fp64(factor, kernel):
    """The SpMV gathers through the explicit step's neighbour source."""
    sim, og, x0, p = make(kernel=kernel)
    dt = factor * inputs.explicit_dt(p, 1.0)
    a = p.D[1] * dt / p.h ** 2
    rtol = 1e-10
    its, rel, rc = sim.implicit_step(dt, rtol=rtol)
    assert rc == 0 and rel[1] <= rtol and its[1] > 0
    got = sim.fields.cpu().numpy()
    # transformation half is exact; only DOM goes through CG
    xt = orc.transform(p, dt, x0)
    for s in (0, 2, 3, 4):
        np.testing.assert_array_equal(got[s], xt[s])
    b = xt[1]
    true_res = np.linalg.norm(b - orc.apply_B(a, og, got[1])) / np.linalg.norm(b)
    assert true_res <= 2 * rtol, true_res
    ref, oits, orel = orc.implicit_step(p, dt, og, x0, rtol=1e-14)
    kappa = 1 + 12 * a
    err = np.abs(got[1] - ref[1]).max() / np.abs(ref[1]).max()
    assert err <= kappa * rtol, (err, kappa * rtol)
    _, oits10, _ = orc.implicit_step(p, dt, og, x0, rtol=rtol)
    assert abs(its[1] - oits10[1]) <= 2, (its, oits10)


@KERNELS
def test_implicit_with_regions_fp32_fields(kernel):
    c = [0.7, 1.0, 0.8, 0.9, 1.1, 0.75, 0.95, 0.85]
    sim, og, x0, p = make(regions=c, precision="f32", kernel=kernel)
    dt = 20 * inputs.explicit_dt(p, 1.0)
    a = p.D[1] * dt / p.h ** 2
    its, rel, rc = sim.implicit_step(dt, rtol=1e-10)
    assert rc == 0
    w = orc.edge_weights(og, orc.octant_regions(og), c)
    ref, _, _ = orc.implicit_step(p, dt, og, x0, rtol=1e-14, w=w)
    got = sim.fields.cpu().numpy().astype(np.float64)
    for s in range(5):
        err = np.abs(got[s] - ref[s]).max() / np.abs(ref[s]).max()
        assert err <= 1e-6, (s, err)


def test_implicit_reports_nonconvergence():
    from paper_2406_04177_amd import _lib
    sim, og, x0, p = make(shape=(20, 20, 20))
    dt = 20 * inputs.explicit_dt(p, 1.0)
    its, rel, rc = sim.implicit_step(dt, rtol=1e-12, max_iter=3, check=False)
    assert rc == _lib.VG_ENOCONV and its[1] == 3 and rel[1] > 1e-12


@pytest.mark.parametrize("k", [1, 2, 3, 7, 20])
def test_implicit_iterate_after_k_iterations(k):
    """Stopped at max_iter = k (VG_ENOCONV), the state holds the k-th PCG
    iterate: the oracle's PCG stopped after k iterations, up to rounding.
    (The GPU applies each iteration's solution update one kernel later and
    the last one on write-back; a lost or doubled update is off by ~|alpha p|.)"""
    from paper_2406_04177_amd import _lib
    sim, og, x0, p = make()
    dt = 20 * inputs.explicit_dt(p, 1.0)
    a = p.D[1] * dt / p.h ** 2
    its, rel, rc = sim.implicit_step(dt, rtol=1e-30, max_iter=k, check=False)
    assert rc == _lib.VG_ENOCONV and its[1] == k
    b = orc.transform(p, dt, x0)[1]
    y, oits, orel, conv = orc.pcg(a, og, b, rtol=1e-30, max_iter=k)
    assert oits == k and not conv
    got = sim.fields.cpu().numpy()[1]
    err = np.abs(got - y).max() / np.abs(y).max()
    assert err <= 1e-11, (k, err)
    assert abs(rel[1] - orel) <= 1e-9 * orel, (rel[1], orel)


@pytest.mark.parametrize("shape", [(3, 4, 5), (11, 13, 17), (24, 40, 40)])
@KERNELS
def test_implicit_unfiltered_masks(shape, kernel):
    """Raw random masks (isolated voxels, every neighbour count 0-6, one to
    hundreds of tiles): converged answer by the oracle's matrix, the 5-th
    iterate against the oracle's, isolated voxels unchanged by the solve."""
    from paper_2406_04177_amd import _lib
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    mask = (np.random.default_rng(sum(shape)).random(shape) < 0.45).astype(np.uint8)
    spec = inputs.init_random_all(mask, 3)
    g = Graph.from_masks(mask)
    og = orc.build_graph(mask)
    p = inputs.ModelParams(mu=1e-4, rho=5e-5)
    dt = 20 * inputs.explicit_dt(p, 1.0)
    a = p.D[1] * dt / p.h ** 2
    deg = (og.nbr >= 0).sum(axis=0)
    assert deg.min() == 0 and deg.max() == 6 or shape == (3, 4, 5)
    b = orc.transform(p, dt, orc.fields_from_spec(og, spec))[1]
    results = {}
    for max_iter, rtol in ((5, 1e-30), (1000, 1e-12)):
        sim = Simulation(g, p, precision="f64", implicit=True)
        sim.set_kernel(kernel)
        sim.set_fields(g.fields_from_specs(spec, torch.float64))
        its, rel, rc = sim.implicit_step(dt, rtol=rtol, max_iter=max_iter, check=False)
        results[max_iter] = (sim.fields.cpu().numpy()[1], its[1], rc)
    got5, its5, rc5 = results[5]
    y5, oits5, _, _ = orc.pcg(a, og, b, rtol=1e-30, max_iter=5)
    if oits5 == 5:
        assert rc5 == _lib.VG_ENOCONV and its5 == 5
    np.testing.assert_allclose(got5, y5, rtol=0, atol=1e-11 * np.abs(y5).max())
    got, its, rc = results[1000]
    assert rc == 0
    true_res = np.linalg.norm(b - orc.apply_B(a, og, got)) / np.linalg.norm(b)
    assert true_res <= 2e-12, true_res
    iso = deg == 0
    np.testing.assert_array_equal(got[iso], b[iso])


def test_implicit_fourier_mode_periodic_channel():
    """Closed form: the channel mode decays by 1 / (1 + a lambda) per step."""
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    W, H, Lz, k = 4, 4, 64, 3
    mask = np.ones((Lz, H, W), np.uint8)
    g = Graph.from_masks(mask, periodic=7)
    p = inputs.ModelParams(D=(0, 1.0, 0, 0, 0), h=1.0, v_dom=0, rho=0, mu=0, v_som=0, v_p4=0)
    sim = Simulation(g, p, precision="f64", implicit=True)
    z = g.vox.cpu().numpy() // (W * H)
    mode = np.cos(2 * np.pi * k * z / Lz)
    x = np.zeros((5, g.n))
    x[1] = 1 + 0.5 * mode
    sim.set_fields(torch.tensor(x))
    a = 2.0
    for _ in range(4):
        sim.implicit_step(a, rtol=1e-13)
    lam = 4 * np.sin(np.pi * k / Lz) ** 2
    np.testing.assert_allclose(sim.fields[1].cpu().numpy(), 1 + 0.5 * mode / (1 + a * lam) ** 4, atol=1e-11)
