"""Pins of the oracle's graph construction (Sec. II.A, Fig. 2; Sec. III).

The oracle's C builder is compared with a pure-Python brute force written from
the definition (pore voxels in enumeration order; a neighbour per face), plus
invariants of the 6-connected graph.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as orc

OFFS = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]


def brute_graph(mask, periodic=0, brick=0):
    nz, ny, nx = mask.shape
    if brick <= 0:
        coords = [(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx)]
    else:
        b = brick
        coords = []
        for bz, by, bx in itertools.product(range(0, nz, b), range(0, ny, b), range(0, nx, b)):
            for z in range(bz, min(bz + b, nz)):
                for y in range(by, min(by + b, ny)):
                    for x in range(bx, min(bx + b, nx)):
                        coords.append((x, y, z))
    pores = [c for c in coords if mask[c[2], c[1], c[0]]]
    index = {c: i for i, c in enumerate(pores)}
    vox = np.array([x + nx * (y + ny * z) for (x, y, z) in pores], np.int32)
    nbr = np.full((6, len(pores)), -1, np.int32)
    dims = (nx, ny, nz)
    for i, c in enumerate(pores):
        for k, o in enumerate(OFFS):
            q = list(c)
            ok = True
            for a in range(3):
                q[a] += o[a]
                if not 0 <= q[a] < dims[a]:
                    if periodic & (1 << a):
                        q[a] %= dims[a]
                    else:
                        ok = False
            if ok and tuple(q) in index:
                nbr[k, i] = index[tuple(q)]
    return vox, nbr


@pytest.mark.parametrize("shape,seed,periodic,brick", [
    ((4, 5, 6), 0, 0, 0), ((3, 7, 5), 1, 0, 0), ((6, 6, 6), 2, 7, 0), ((5, 4, 3), 3, 5, 0),
    ((8, 8, 8), 4, 0, 4), ((7, 9, 10), 5, 0, 4), ((6, 5, 7), 6, 3, 2), ((1, 1, 1), 7, 0, 0),
])
def test_graph_matches_brute_force(shape, seed, periodic, brick):
    rng = np.random.default_rng(seed)
    mask = (rng.random(shape) < 0.6).astype(np.uint8)
    g = orc.build_graph(mask, brick=brick, periodic=periodic)
    vox, nbr = brute_graph(mask, periodic, brick)
    assert g.n == int(mask.sum())
    np.testing.assert_array_equal(g.vox, vox)
    np.testing.assert_array_equal(g.nbr, nbr)


def test_graph_empty_mask():
    g = orc.build_graph(np.zeros((3, 4, 5), np.uint8))
    assert g.n == 0 and g.nbr.shape == (6, 0)


def test_neighbour_symmetry():
    rng = np.random.default_rng(11)
    mask = (rng.random((12, 13, 14)) < 0.5).astype(np.uint8)
    for periodic in (0, 7):
        g = orc.build_graph(mask, periodic=periodic)
        for k in range(6):
            i = np.flatnonzero(g.nbr[k] >= 0)
            j = g.nbr[k, i]
            np.testing.assert_array_equal(g.nbr[k ^ 1, j], i)


def test_open_cube_degree_histogram():
    m = 7
    g = orc.build_graph(np.ones((m, m, m), np.uint8))
    deg = (g.nbr >= 0).sum(0)
    hist = np.bincount(deg, minlength=7)
    assert hist[3] == 8
    assert hist[4] == 12 * (m - 2)
    assert hist[5] == 6 * (m - 2) ** 2
    assert hist[6] == (m - 2) ** 3
    assert hist[:3].sum() == 0


def test_brick_order_is_a_relabelling_of_raster():
    rng = np.random.default_rng(5)
    mask = (rng.random((16, 12, 20)) < 0.4).astype(np.uint8)
    gr = orc.build_graph(mask)
    gb = orc.build_graph(mask, brick=4)
    # same voxel set
    np.testing.assert_array_equal(np.sort(gb.vox), gr.vox)
    # neighbour relation identical after mapping brick index -> raster index
    perm = np.searchsorted(gr.vox, gb.vox)          # brick i -> raster perm[i]
    for k in range(6):
        jb = gb.nbr[k]
        expect = gr.nbr[k, perm]
        got = np.where(jb >= 0, perm[np.maximum(jb, 0)], -1)
        np.testing.assert_array_equal(got, expect)
    # brick keys are increasing
    nz, ny, nx = mask.shape
    v = gb.vox
    x, y, z = v % nx, (v // nx) % ny, v // (nx * ny)
    nbx, nby = (nx + 3) // 4, (ny + 3) // 4
    key = (((z // 4) * nby + (y // 4)) * nbx + (x // 4)) * 64 + ((z % 4) * 4 + (y % 4)) * 4 + (x % 4)
    assert np.all(np.diff(key) > 0)


def test_batch_offsets():
    rng = np.random.default_rng(9)
    masks = [(rng.random((5, 6, 7)) < p).astype(np.uint8) for p in (0.3, 0.5, 0.7)]
    g = orc.build_batch(masks)
    off = 0
    for b, m in enumerate(masks):
        gb = orc.build_graph(m)
        assert g.seg_off[b] == off
        np.testing.assert_array_equal(g.vox[off:off + gb.n], gb.vox)
        sub = g.nbr[:, off:off + gb.n]
        np.testing.assert_array_equal(np.where(sub >= 0, sub - off, -1), gb.nbr)
        off += gb.n
    assert g.seg_off[-1] == g.n
