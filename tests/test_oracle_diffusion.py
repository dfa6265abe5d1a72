"""Pins of the oracle's diffusion: graph Laplacian (Sec. II.B.2), explicit
Scheme 1 (Sec. II.B.3a) and implicit Scheme 2 with PCG (Sec. II.B.3b, Sec. III).

Expected values come from independent constructions: the 7-point stencil with
mirrored ghost cells, dense matrices built directly from voxel coordinates,
closed-form Fourier modes, scipy's matrix exponential and dense solves.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import oracle as orc
from paper_2406_04177_amd.inputs import ModelParams


def dom_only(D=1e-9, h=1.0):
    return ModelParams(D=(0.0, D, 0.0, 0.0, 0.0), h=h, v_dom=0.0, rho=0.0, mu=0.0,
                       v_som=0.0, v_p4=0.0)


def dense_laplacian_from_mask(mask, periodic=0):
    """Graph Laplacian built from the coordinates of the pore voxels (raster
    order), independently of the oracle's neighbour table."""
    nz, ny, nx = mask.shape
    zz, yy, xx = np.nonzero(mask)  # raster order (z slowest)
    pts = np.stack([xx, yy, zz], 1)
    n = len(pts)
    dims = np.array([nx, ny, nz])
    L = np.zeros((n, n))
    for i in range(n):
        d = np.abs(pts - pts[i])
        for a in range(3):
            if periodic & (1 << a):
                d[:, a] = np.minimum(d[:, a], dims[a] - d[:, a])
        adj = np.flatnonzero(d.sum(1) == 1)
        L[i, adj] -= 1
        L[i, i] += len(adj)
    return L


def test_laplacian_equals_7_point_stencil_on_open_cube():
    """All-pore box, no-flux faces: L x = 6 x - sum of the 6 neighbours with
    ghost cells mirrored at the faces.  Integer inputs make it exact."""
    rng = np.random.default_rng(0)
    shape = (6, 7, 8)
    g = orc.build_graph(np.ones(shape, np.uint8))
    xs = rng.integers(-1000, 1000, size=shape).astype(np.float64)
    pad = np.pad(xs, 1, mode="edge")
    c = pad[1:-1, 1:-1, 1:-1]
    stencil = (6 * c - pad[:-2, 1:-1, 1:-1] - pad[2:, 1:-1, 1:-1] - pad[1:-1, :-2, 1:-1]
               - pad[1:-1, 2:, 1:-1] - pad[1:-1, 1:-1, :-2] - pad[1:-1, 1:-1, 2:])
    got = orc.laplacian(g, xs.ravel())
    np.testing.assert_array_equal(got, stencil.ravel())


@pytest.mark.parametrize("seed,periodic", [(0, 0), (1, 0), (2, 7), (3, 1)])
def test_laplacian_equals_dense_definition(seed, periodic):
    rng = np.random.default_rng(seed)
    mask = (rng.random((5, 6, 5)) < 0.55).astype(np.uint8)
    g = orc.build_graph(mask, periodic=periodic)
    L = dense_laplacian_from_mask(mask, periodic)
    got = np.stack([orc.laplacian(g, e) for e in np.eye(g.n)], 1)
    np.testing.assert_array_equal(got, L)
    assert np.allclose(L, L.T)
    np.testing.assert_array_equal(L.sum(1), 0)
    ev = np.linalg.eigvalsh(L)
    assert ev.min() > -1e-12 and ev.max() <= 12 + 1e-12


def test_scheme1_fourier_mode_periodic_channel():
    """Periodic straight channel: cos(2 pi k z / L) is an eigenvector of L with
    eigenvalue 4 sin^2(pi k / L); Scheme 1 scales it by (1 - a lambda) per step."""
    W, H, Lz, k, steps = 3, 4, 32, 3, 50
    mask = np.ones((Lz, H, W), np.uint8)
    g = orc.build_graph(mask, periodic=7)
    p = dom_only(D=0.2, h=1.0)
    dt = 1.0
    a = 0.2
    z = g.vox // (W * H)
    x = np.zeros((5, g.n))
    # a positive state (the constant is the lambda = 0 mode), so that no clamp
    # of the transformation acts
    mode = np.cos(2 * np.pi * k * z / Lz)
    x[1] = 1.0 + 0.5 * mode
    lam = 4 * np.sin(np.pi * k / Lz) ** 2
    out, _ = orc.run(p, dt, g, x, steps, with_totals=False)
    np.testing.assert_allclose(out[1], 1.0 + 0.5 * (1 - a * lam) ** steps * mode, rtol=0, atol=1e-13)
    for s in (0, 2, 3, 4):
        np.testing.assert_array_equal(out[s], 0)


def test_scheme1_fourier_mode_closed_channel():
    """No-flux ends: cos(pi k (z + 1/2) / L) with eigenvalue 4 sin^2(pi k / (2L))."""
    W, H, Lz, k, steps = 2, 3, 20, 2, 40
    g = orc.build_graph(np.ones((Lz, H, W), np.uint8))
    p = dom_only(D=0.15, h=1.0)
    z = g.vox // (W * H)
    x = np.zeros((5, g.n))
    mode = np.cos(np.pi * k * (z + 0.5) / Lz)
    x[1] = 1.0 + 0.5 * mode
    lam = 4 * np.sin(np.pi * k / (2 * Lz)) ** 2
    out, _ = orc.run(p, 1.0, g, x, steps, with_totals=False)
    np.testing.assert_allclose(out[1], 1.0 + 0.5 * (1 - 0.15 * lam) ** steps * mode, rtol=0, atol=1e-13)


@pytest.mark.parametrize("seed", range(4))
def test_scheme1_equals_dense_matrix_power(seed):
    """Q = I - D dt Delta built densely from voxel coordinates (Scheme 1)."""
    rng = np.random.default_rng(100 + seed)
    mask = (rng.random((6, 6, 5)) < 0.5).astype(np.uint8)
    assert mask.sum() <= 200
    g = orc.build_graph(mask)
    L = dense_laplacian_from_mask(mask)
    a = 0.13
    Q = np.eye(g.n) - a * L
    x = np.zeros((5, g.n))
    x[1] = rng.random(g.n)
    out, _ = orc.run(dom_only(D=a, h=1.0), 1.0, g, x, 25, with_totals=False)
    np.testing.assert_allclose(out[1], np.linalg.matrix_power(Q, 25) @ x[1], rtol=0, atol=1e-13)


def test_scheme1_converges_to_matrix_exponential_first_order():
    """M(t) = exp(-D t Delta) M(0) (Sec. II.B.2): the explicit error halves when
    dt halves."""
    rng = np.random.default_rng(7)
    mask = (rng.random((5, 5, 6)) < 0.6).astype(np.uint8)
    g = orc.build_graph(mask)
    L = dense_laplacian_from_mask(mask)
    D, T = 0.1, 2.0
    x = np.zeros((5, g.n))
    x[1] = rng.random(g.n)
    exact = scipy.linalg.expm(-D * T * L) @ x[1]
    errs = []
    for nsteps in (40, 80, 160):
        out, _ = orc.run(dom_only(D=D, h=1.0), T / nsteps, g, x, nsteps, with_totals=False)
        errs.append(np.abs(out[1] - exact).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 1.8 < r1 < 2.2 and 1.8 < r2 < 2.2, errs


def test_paper_explicit_limit_and_negative_values():
    """Sec. IV.C: with D = 100950 voxel^2/day, dt = 0.1 s keeps masses
    non-negative while larger steps give negative values; a unit spike in an
    interior voxel goes negative once 1 - 6 D dt < 0 (dt > 0.1426 s)."""
    D_vox = 100950.0 / 86400.0                      # voxel^2 / s
    bound = 1.0 / (6.0 * D_vox)
    assert 0.1 <= bound and abs(bound - 0.14264) < 1e-4
    g = orc.build_graph(np.ones((7, 7, 7), np.uint8))
    centre = 3 + 7 * (3 + 7 * 3)
    x = np.zeros((5, g.n))
    x[1, centre] = 1.0
    h = 24e-6
    p = dom_only(D=D_vox * h * h, h=h)
    for steps in (1, 50):
        out, _ = orc.run(p, 0.1, g, x, steps, with_totals=False)
        assert out[1].min() >= 0.0
    out, _ = orc.run(p, 0.15, g, x, 1, with_totals=False)
    assert out[1, centre] < 0.0


@pytest.mark.parametrize("seed", range(3))
def test_pcg_equals_dense_solve(seed):
    """Scheme 2: B = I + D dt Delta; the PCG answer equals numpy's dense solve."""
    rng = np.random.default_rng(200 + seed)
    mask = (rng.random((6, 5, 6)) < 0.55).astype(np.uint8)
    g = orc.build_graph(mask)
    L = dense_laplacian_from_mask(mask)
    a = 3.3
    b = rng.random(g.n)
    y, it, rel, ok = orc.pcg(a, g, b, rtol=1e-14)
    assert ok and rel <= 1e-14
    np.testing.assert_allclose(y, np.linalg.solve(np.eye(g.n) + a * L, b), rtol=0, atol=1e-12)
    np.testing.assert_allclose(orc.apply_B(a, g, y), b, rtol=0, atol=1e-13)


def test_pcg_with_weights_equals_dense_solve():
    rng = np.random.default_rng(300)
    mask = (rng.random((6, 6, 6)) < 0.55).astype(np.uint8)
    g = orc.build_graph(mask)
    reg = orc.octant_regions(g)
    c = rng.uniform(0.5, 1.5, 8)
    w = orc.edge_weights(g, reg, c)
    n = g.n
    B = np.eye(n)
    for k in range(6):
        for i in range(n):
            j = g.nbr[k, i]
            if j >= 0:
                B[i, i] += 2.0 * w[k, i]
                B[i, j] -= 2.0 * w[k, i]
    b = rng.random(n)
    y, it, rel, ok = orc.pcg(2.0, g, b, rtol=1e-14, w=w)
    assert ok
    np.testing.assert_allclose(y, np.linalg.solve(B, b), rtol=0, atol=1e-12)


def test_scheme2_fourier_mode():
    """Implicit step scales the periodic-channel mode by 1 / (1 + a lambda)."""
    W, H, Lz, k = 2, 2, 24, 2
    g = orc.build_graph(np.ones((Lz, H, W), np.uint8), periodic=7)
    z = g.vox // (W * H)
    x = np.zeros((5, g.n))
    mode = np.cos(2 * np.pi * k * z / Lz)
    x[1] = 1.0 + 0.5 * mode
    lam = 4 * np.sin(np.pi * k / Lz) ** 2
    a = 2.5
    p = dom_only(D=a, h=1.0)
    y = x.copy()
    for _ in range(5):
        y, iters, rel = orc.implicit_step(p, 1.0, g, y, rtol=1e-15)
    np.testing.assert_allclose(y[1], 1.0 + 0.5 * mode / (1 + a * lam) ** 5, rtol=0, atol=1e-13)


def test_pcg_zero_rhs_and_zero_iterations():
    g = orc.build_graph(np.ones((3, 3, 3), np.uint8))
    y, it, rel, ok = orc.pcg(1.0, g, np.zeros(g.n))
    assert ok and it == 0 and np.all(y == 0)
    # uniform vector: B 1 = 1, so the start guess is already exact
    y, it, rel, ok = orc.pcg(1.0, g, np.ones(g.n))
    assert ok and it == 0 and np.all(y == 1)


def test_weighted_scheme1_with_unit_weights_is_bitwise_unweighted():
    rng = np.random.default_rng(4)
    mask = (rng.random((8, 8, 8)) < 0.5).astype(np.uint8)
    g = orc.build_graph(mask)
    w = orc.edge_weights(g, orc.octant_regions(g), np.ones(8))
    x = np.zeros((5, g.n))
    x[1] = rng.random(g.n)
    a, _ = orc.run(dom_only(0.1), 1.0, g, x, 10, with_totals=False)
    b, _ = orc.run(dom_only(0.1), 1.0, g, x, 10, w=w, with_totals=False)
    np.testing.assert_array_equal(a, b)
