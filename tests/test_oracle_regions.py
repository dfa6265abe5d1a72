"""Pins of the oracle's region rule and edge weights.

The region conductance factors generalise the unit conductance S_ij / d_ij = 1
of Sec. II.B.1-2: voxel i belongs to the octant 4[z >= nz/2] + 2[y >= ny/2] +
[x >= nx/2] of its own volume (integer halves), and the edge between i and j
has weight (c[r(i)] + c[r(j)]) / 2.  Every expected value below is worked out
by hand from that rule (no call of the function under test builds it), on
boxes whose three sizes differ, so a swapped axis, a strict comparison at the
half or a wrong bit weight changes at least one of them.
"""
import numpy as np

from oracle import oracle as orc


def _box(nz, ny, nx):
    g = orc.build_graph(np.ones((nz, ny, nx), np.uint8))
    assert g.n == nx * ny * nz           # all pore: compact index = x + nx (y + ny z)
    return g


def _idx(x, y, z, nx, ny):
    return x + nx * (y + ny * z)


def test_octants_even_box_by_hand():
    nz, ny, nx = 4, 6, 8                 # halves at z = 2, y = 3, x = 4
    r = orc.octant_regions(_box(nz, ny, nx))
    named = {
        (0, 0, 0): 0,
        (3, 2, 1): 0,                    # last voxel below every half
        (4, 0, 0): 1,                    # x = nx/2 is in the upper half
        (7, 0, 0): 1,
        (0, 3, 0): 2,                    # y = ny/2
        (3, 5, 1): 2,
        (4, 3, 0): 3,
        (0, 0, 2): 4,                    # z = nz/2
        (3, 2, 3): 4,
        (4, 0, 2): 5,
        (7, 2, 3): 5,
        (0, 3, 2): 6,
        (4, 3, 2): 7,
        (7, 5, 3): 7,
    }
    for (x, y, z), want in named.items():
        assert r[_idx(x, y, z, nx, ny)] == want, ((x, y, z), r[_idx(x, y, z, nx, ny)], want)
    # every octant of an even box holds (nz/2)(ny/2)(nx/2) = 2 * 3 * 4 voxels
    assert np.bincount(r, minlength=8).tolist() == [24] * 8


def test_octants_odd_box_by_hand():
    nz, ny, nx = 5, 7, 9                 # integer halves: z >= 2, y >= 3, x >= 4
    r = orc.octant_regions(_box(nz, ny, nx))
    assert r[_idx(3, 2, 1, nx, ny)] == 0
    assert r[_idx(4, 2, 1, nx, ny)] == 1
    assert r[_idx(3, 3, 1, nx, ny)] == 2
    assert r[_idx(3, 2, 2, nx, ny)] == 4
    assert r[_idx(8, 6, 4, nx, ny)] == 7
    # lower / upper extents: z 2 / 3, y 3 / 4, x 4 / 5 voxels
    counts = {0: 2 * 3 * 4, 1: 2 * 3 * 5, 2: 2 * 4 * 4, 3: 2 * 4 * 5,
              4: 3 * 3 * 4, 5: 3 * 3 * 5, 6: 3 * 4 * 4, 7: 3 * 4 * 5}
    assert np.bincount(r, minlength=8).tolist() == [counts[o] for o in range(8)]
    assert sum(counts.values()) == nx * ny * nz


def test_octants_batch_offset_by_volume():
    masks = [np.ones((4, 6, 8), np.uint8), np.ones((4, 6, 8), np.uint8)]
    g = orc.build_batch(masks)
    r = orc.octant_regions(g, per_volume=True)
    n0 = 4 * 6 * 8
    assert r[_idx(7, 5, 3, 8, 6)] == 7
    assert r[n0 + _idx(0, 0, 0, 8, 6)] == 8          # volume 1, octant 0
    assert r[n0 + _idx(4, 3, 2, 8, 6)] == 15         # volume 1, octant 7


def test_edge_weights_by_hand():
    nz, ny, nx = 4, 6, 8
    g = _box(nz, ny, nx)
    c = [1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0, 8.0]     # c[r] = r + 1
    w = orc.edge_weights(g, orc.octant_regions(g), c)
    # slots: 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z
    i = _idx(3, 0, 0, nx, ny)            # octant 0
    assert w[1, i] == 1.5                # +x neighbour (4, 0, 0) in octant 1: (1 + 2) / 2
    assert w[0, i] == 1.0                # -x neighbour (2, 0, 0) in octant 0
    assert w[2, i] == 0.0                # y = -1: no neighbour
    assert w[4, i] == 0.0                # z = -1: no neighbour
    i = _idx(0, 2, 1, nx, ny)            # octant 0
    assert w[3, i] == 2.0                # +y neighbour (0, 3, 1) in octant 2: (1 + 3) / 2
    assert w[5, i] == 3.0                # +z neighbour (0, 2, 2) in octant 4: (1 + 5) / 2
    assert w[0, i] == 0.0                # x = -1
    i = _idx(7, 5, 3, nx, ny)            # octant 7
    assert w[4, i] == 8.0                # -z neighbour (7, 5, 2) also octant 7
    assert w[0, i] == 8.0                # -x neighbour (6, 5, 3) also octant 7
    assert w[5, i] == 0.0 and w[1, i] == 0.0 and w[3, i] == 0.0
    i = _idx(4, 3, 2, nx, ny)            # octant 7, corner of the upper octant
    assert w[0, i] == 7.5                # (3, 3, 2) in octant 6: (8 + 7) / 2
    assert w[2, i] == 7.0                # (4, 2, 2) in octant 5: (8 + 6) / 2
    assert w[4, i] == 6.0                # (4, 3, 1) in octant 3: (8 + 4) / 2
    # symmetric: w on slot k of i equals w on the opposite slot of its neighbour
    for k in range(6):
        j = g.nbr[k]
        ok = j >= 0
        assert np.array_equal(w[k, ok], w[k ^ 1, j[ok]])
