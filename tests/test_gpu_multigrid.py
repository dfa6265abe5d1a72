"""The multigrid preconditioner of the implicit step (an addition to the
paper's Jacobi PCG, vg_set_preconditioner) on the GPU.

Its definition is restated here with scipy sparse matrices, independently of
the library: aggregates of 2x2x2 cells by position, level l + 1's operator
the Galerkin product P^T B_l P with the piecewise-constant P (mass vector and
weighted Laplacian), damped Jacobi (0.8) once before and once after each
coarse correction, 8 sweeps from zero on the coarsest level (reached once a
level has at most 1024 cells).  Checks: the hierarchy's cell counts, the
V-cycle against that restatement, its symmetry and positive definiteness,
and solves whose true residual (the oracle's matrix) meets rtol and whose
answer agrees with the oracle's tight Jacobi-PCG solve within kappa * rtol,
in far fewer iterations than Jacobi."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import oracle as orc
from paper_2406_04177_amd import inputs

pytestmark = pytest.mark.gpu

OMEGA, COARSEST, SWEEPS, MAX_LEVELS = 0.8, 1024, 8, 12


def ref_hierarchy(og, w0):
    """[(mass, Laplacian, P to the next level or None)] from the definition."""
    n = og.n
    nz, ny, nx = og.shape
    v = og.vox.astype(np.int64)
    coords = np.stack([v % nx, (v // nx) % ny, v // (nx * ny)], 1)
    rows, cols, vals = [], [], []
    for k in range(6):
        j = og.nbr[k]
        ok = j >= 0
        rows.append(np.nonzero(ok)[0])
        cols.append(j[ok])
        vals.append(w0[k, ok])
    W = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    lap = (sp.diags(np.asarray(W.sum(axis=1)).ravel()) - W).tocsr()
    levels = [[np.ones(n), lap, None]]
    dims = (nx, ny, nz)
    while len(levels) < MAX_LEVELS and max(dims) > 1:
        if len(levels) > 1 and levels[-1][0].size <= COARSEST:
            break
        dims = tuple((d + 1) // 2 for d in dims)
        coords = coords // 2
        key = coords[:, 0] + dims[0] * (coords[:, 1] + dims[1] * coords[:, 2])
        used, agg = np.unique(key, return_inverse=True)
        m = levels[-1][0].size
        P = sp.csr_matrix((np.ones(m), (np.arange(m), agg)), shape=(m, used.size))
        levels[-1][2] = P
        levels.append([P.T @ levels[-1][0], (P.T @ levels[-1][1] @ P).tocsr(), None])
        coords = np.stack([used % dims[0], (used // dims[0]) % dims[1], used // (dims[0] * dims[1])], 1)
    return levels


def ref_vcycle(levels, a, r):
    Bs = [sp.diags(m) + a * lap for m, lap, _ in levels]
    ds = [B.diagonal() for B in Bs]

    def cyc(l, r):
        B, d, P = Bs[l], ds[l], levels[l][2]
        x = OMEGA * r / d
        if P is None:
            for _ in range(SWEEPS - 1):
                x = x + OMEGA * (r - B @ x) / d
            return x
        y = x + P @ cyc(l + 1, P.T @ (r - B @ x))
        return y + OMEGA * (r - B @ y) / d
    return cyc(0, r)


def make(shape, seed=1, regions=None, kernel=0, brick=0, porosity=0.17):
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    mask = inputs.synthetic_volume(shape, porosity=porosity, seed=seed)
    g = Graph.from_masks(mask, brick=brick, regions=regions is not None)
    og = orc.build_graph(mask, brick=brick)
    p = inputs.ModelParams(mu=1e-4, rho=5e-5)
    sim = Simulation(g, p, precision="f64", implicit=True, regions=regions, multigrid=True)
    sim.set_kernel(kernel)
    sim.set_fields(g.fields_from_specs(inputs.init_random_all(mask, seed), torch.float64))
    w0 = (orc.edge_weights(og, orc.octant_regions(og), regions) if regions is not None
          else np.where(og.nbr >= 0, 1.0, 0.0))
    return sim, og, mask, p, w0


@pytest.mark.parametrize("shape", [(40, 36, 44), (33, 17, 50), (8, 8, 8)], ids=["40x36x44", "ragged", "tiny"])
def test_hierarchy_cells(shape):
    sim, og, _, _, w0 = make(shape)
    levels = ref_hierarchy(og, w0)
    assert sim.mg_levels() == [lv[0].size for lv in levels]
    print("levels", sim.mg_levels())


@pytest.mark.parametrize("regions", [None, [0.7, 1.0, 0.8, 0.9, 1.1, 0.75, 0.95, 0.85]], ids=["unit", "regions"])
@pytest.mark.parametrize("kernel", [1, 3, 4], ids=["table", "offset", "relative"])
@pytest.mark.parametrize("a", [0.3, 35.0])
def test_vcycle_equals_definition(regions, kernel, a):
    """The GPU's z = M^-1 r against the scipy restatement: 1e-11 of max |z|
    with unit weights (integer weights, exact in the float storage), 1e-6
    with region weights (the coarse weights are stored as floats)."""
    sim, og, _, _, w0 = make((48, 40, 36), seed=3, regions=regions, kernel=kernel)
    sim.set_preconditioner("mg")
    levels = ref_hierarchy(og, w0)
    rng = np.random.default_rng(5)
    for _ in range(2):
        r = rng.standard_normal(og.n)
        z = sim.precondition(a, torch.from_numpy(r).cuda()).cpu().numpy()
        ref = ref_vcycle(levels, a, r)
        err = np.abs(z - ref).max() / np.abs(ref).max()
        assert err <= (1e-11 if regions is None else 1e-6), err


def test_jacobi_precondition_is_the_diagonal():
    sim, og, _, _, w0 = make((20, 22, 24))
    a = 2.5
    r = np.random.default_rng(0).standard_normal(og.n)
    z = sim.precondition(a, torch.from_numpy(r).cuda()).cpu().numpy()     # default: Jacobi
    d = 1.0 + a * w0.sum(axis=0)
    np.testing.assert_allclose(z, r / d, rtol=1e-15, atol=0)


@pytest.mark.parametrize("regions", [None, [0.7, 1.0, 0.8, 0.9, 1.1, 0.75, 0.95, 0.85]], ids=["unit", "regions"])
def test_vcycle_symmetric_positive_definite(regions):
    sim, og, _, _, _ = make((44, 38, 40), seed=7, regions=regions)
    sim.set_preconditioner("mg")
    rng = np.random.default_rng(11)
    for a in (0.5, 35.0):
        U = [torch.from_numpy(rng.standard_normal(og.n)).cuda() for _ in range(4)]
        Z = [sim.precondition(a, u) for u in U]
        for i in range(4):
            assert float(torch.dot(U[i], Z[i])) > 0
            for j in range(i):
                uv, vu = float(torch.dot(U[i], Z[j])), float(torch.dot(U[j], Z[i]))
                scale = float(torch.linalg.vector_norm(U[i]) * torch.linalg.vector_norm(Z[j]))
                assert abs(uv - vu) <= 1e-12 * scale, (a, uv, vu)


@pytest.mark.parametrize("kernel", [1, 3, 4], ids=["table", "offset", "relative"])
@pytest.mark.parametrize("factor", [1.0, 20.0, 400.0])
def test_mg_solve_meets_rtol(kernel, factor):
    sim, og, mask, p, _ = make((48, 44, 40), seed=2, kernel=kernel)
    x0 = sim.state().cpu().numpy()
    sim.set_preconditioner("mg")
    dt = factor * inputs.explicit_dt(p, 1.0)
    a = p.D[1] * dt / p.h ** 2
    rtol = 1e-10
    its, rel, rc = sim.implicit_step(dt, rtol=rtol)
    assert rc == 0 and rel[1] <= rtol
    got = sim.fields.cpu().numpy()
    xt = orc.transform(p, dt, x0)
    for s in (0, 2, 3, 4):
        np.testing.assert_array_equal(got[s], xt[s])
    b = xt[1]
    true_res = np.linalg.norm(b - orc.apply_B(a, og, got[1])) / np.linalg.norm(b)
    assert true_res <= 2 * rtol, true_res
    ref, _, _ = orc.implicit_step(p, dt, og, x0, rtol=1e-14)
    err = np.abs(got[1] - ref[1]).max() / np.abs(ref[1]).max()
    assert err <= (1 + 12 * a) * rtol, err
    _, jits, _ = orc.implicit_step(p, dt, og, x0, rtol=rtol)
    print("a = %.1f: MG %d iterations, Jacobi %d" % (a, its[1], jits[1]))
    if factor >= 20:
        assert its[1] * 2 <= jits[1], (its, jits)


def test_mg_solve_with_regions_brick_order_and_fp32_fields():
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    c = [0.7, 1.0, 0.8, 0.9, 1.1, 0.75, 0.95, 0.85]
    mask = inputs.synthetic_volume((40, 48, 36), seed=4)
    spec = inputs.init_random_all(mask, 4)
    og = orc.build_graph(mask, brick=8)
    g = Graph.from_masks(mask, brick=8, regions=True)
    p = inputs.ModelParams(mu=1e-4, rho=5e-5)
    sim = Simulation(g, p, precision="f32", implicit=True, regions=c, multigrid=True)
    sim.set_fields(g.fields_from_specs(spec, torch.float64))
    sim.set_preconditioner("mg")
    dt = 50 * inputs.explicit_dt(p, 1.0)
    its, rel, rc = sim.implicit_step(dt, rtol=1e-10)
    assert rc == 0
    w = orc.edge_weights(og, orc.octant_regions(og), c)
    ref, _, _ = orc.implicit_step(p, dt, og, orc.fields_from_spec(og, spec), rtol=1e-14, w=w)
    got = sim.fields.cpu().numpy().astype(np.float64)
    for s in range(5):
        assert np.abs(got[s] - ref[s]).max() / np.abs(ref[s]).max() <= 1e-6, s
    # new region factors: the coarse weights follow
    c2 = [1.2, 0.6, 1.0, 0.9, 1.3, 0.8, 1.1, 0.7]
    sim.set_regions(c2)
    x1 = sim.state().cpu().numpy()
    its2, rel2, rc2 = sim.implicit_step(dt, rtol=1e-10)
    w2 = orc.edge_weights(og, orc.octant_regions(og), c2)
    ref2, _, _ = orc.implicit_step(p, dt, og, x1, rtol=1e-14, w=w2)
    got2 = sim.fields.cpu().numpy().astype(np.float64)
    assert rc2 == 0
    assert np.abs(got2[1] - ref2[1]).max() / np.abs(ref2[1]).max() <= 1e-6


def test_degenerate_volumes():
    """One voxel: no coarser level, MG falls back to Jacobi (same result bit
    for bit); one row and one plane: a few levels, solves meet rtol."""
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    p = inputs.ModelParams(mu=1e-4, rho=5e-5)
    dt = 20 * inputs.explicit_dt(p, 1.0)
    a = p.D[1] * dt / p.h ** 2
    for shape, fill in (((1, 1, 1), None), ((1, 1, 37), None), ((1, 23, 19), 0.6)):
        mask = np.ones(shape, np.uint8) if fill is None else inputs.synthetic_volume(shape, porosity=fill, seed=1)
        spec = inputs.init_random_all(mask, 1)
        g = Graph.from_masks(mask)
        og = orc.build_graph(mask)
        res = []
        for pc in ("jacobi", "mg"):
            sim = Simulation(g, p, precision="f64", implicit=True, multigrid=True)
            sim.set_fields(g.fields_from_specs(spec, torch.float64))
            sim.set_preconditioner(pc)
            its, rel, rc = sim.implicit_step(dt, rtol=1e-10)
            assert rc == 0
            res.append(sim.fields.cpu().numpy())
        if g.n == 1:
            assert sim.mg_levels() == [1]
            np.testing.assert_array_equal(res[0], res[1])
        else:
            assert len(sim.mg_levels()) >= 2
            x0 = orc.fields_from_spec(og, spec)
            b = orc.transform(p, dt, x0)[1]
            assert np.linalg.norm(b - orc.apply_B(a, og, res[1][1])) <= 2e-10 * np.linalg.norm(b)


def test_batch_refused():
    from paper_2406_04177_amd import _lib
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    masks = [inputs.synthetic_volume((16, 16, 16), seed=s) for s in range(2)]
    g = Graph.from_masks(masks)
    with pytest.raises(_lib.VgError):
        Simulation(g, inputs.ModelParams(), precision="f64", implicit=True, multigrid=True)
