"""The diffusion comparison of Sec. IV.B (DOM on the first two z-layers,
D = 100950 voxel^2/day, profile of the mass per layer) on the GPU against the
oracle, on a small synthetic volume; and the range-sum kernel against numpy."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2406_04177_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_range_sums_against_numpy(dtype):
    from paper_2406_04177_amd.graph import range_sums
    rng = np.random.default_rng(0)
    x = rng.standard_normal(100003)
    cuts = np.sort(rng.integers(0, 100003, 300))
    off = np.concatenate([[0], cuts, [100003]]).astype(np.int64)
    off[5] = off[6]                          # an empty range
    got = range_sums(torch.as_tensor(x, dtype=dtype, device="cuda"), torch.as_tensor(off, device="cuda")).cpu().numpy()
    xr = x.astype(np.float32).astype(np.float64) if dtype == torch.float32 else x
    ref = np.array([xr[a:b].sum() for a, b in zip(off[:-1], off[1:])])
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
    assert got[5] == 0.0
    # offsets outside [0, n] are clamped, an inverted range is empty
    bad = torch.as_tensor(np.array([-50, 10, 5, 200000], np.int64), device="cuda")
    g2 = range_sums(torch.as_tensor(x, dtype=dtype, device="cuda"), bad).cpu().numpy()
    np.testing.assert_allclose(g2, [xr[0:10].sum(), 0.0, xr[5:].sum()], rtol=1e-12, atol=1e-12)


def small():
    from paper_2406_04177_amd.graph import Graph
    mask = inputs.synthetic_volume((48, 40, 36), porosity=0.3, seed=5)
    return mask, Graph.from_masks(mask), orc.build_graph(mask)


def oracle_profile(og, mask, x):
    nz, ny, nx = mask.shape
    return np.bincount(og.vox // (nx * ny), weights=x[1], minlength=nz)


def test_explicit_profile_fp64_equals_oracle():
    from paper_2406_04177_amd import diffusion_experiment as de
    mask, g, og = small()
    t_end = 20.0
    sim, nsteps = de.run_explicit(mask, g, dt=0.1, t_end=t_end, precision="f64")
    prof = de.layer_profile(sim, mask)
    x0 = de.initial_fields(mask, g).cpu().numpy()
    np.testing.assert_allclose(oracle_profile(og, mask, x0)[:2].sum(), de.M0, rtol=1e-12)   # k additions of M0/k
    ref, _ = orc.run(de.params(), 0.1, og, x0, nsteps, with_totals=False)
    np.testing.assert_array_equal(sim.fields.cpu().numpy(), ref)           # fields bit for bit
    np.testing.assert_allclose(prof, oracle_profile(og, mask, ref), rtol=1e-12, atol=1e-12 * de.M0)
    np.testing.assert_allclose(prof.sum(), de.M0, rtol=1e-12)              # no flux out of the image


@pytest.mark.parametrize("multigrid", [False, True], ids=["jacobi", "multigrid"])
@pytest.mark.parametrize("t_end", [30.0, 40.0])
def test_implicit_profile_against_oracle(t_end, multigrid):
    """30 s steps (and a 10 s remainder for t_end = 40 s): the GPU iterate is
    within kappa * rtol of the oracle's tight solve, layer by layer (with the
    paper's Jacobi preconditioner and with the multigrid one)."""
    from paper_2406_04177_amd import diffusion_experiment as de
    mask, g, og = small()
    rtol = 1e-11
    sim, its = de.run_implicit(mask, g, dt=30.0, t_end=t_end, precision="f64", rtol=rtol, multigrid=multigrid)
    prof = de.layer_profile(sim, mask)
    x = de.initial_fields(mask, g).cpu().numpy()
    p = de.params()
    steps = [30.0] * int(t_end // 30.0) + ([t_end % 30.0] if t_end % 30.0 else [])
    for dt in steps:
        x, _, _ = orc.implicit_step(p, dt, og, x, rtol=1e-14)
    kappa = 1 + 12 * p.D[1] * 30.0 / p.h ** 2
    ref = oracle_profile(og, mask, x)
    assert np.abs(prof - ref).max() <= len(steps) * kappa * rtol * de.M0, (np.abs(prof - ref).max())
    np.testing.assert_allclose(prof.sum(), de.M0, rtol=1e-9)
    assert len(its) == len(steps)
