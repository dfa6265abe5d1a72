"""Oracle of the pore-network (PNGM) objectives of Sec. V on a coarse
partition of the voxel graph.

TEST INFRASTRUCTURE ONLY (callers: the test suite).  Plain numpy and Python
loops; shares nothing with the HIP path.

Primitives.  The paper's primitives are maximal balls; here they are the
bricks of side b of the image (the ball extraction is out of scope): primitive
k is the set of pore voxels in brick k, numbered in raster order of the
bricks, empty bricks skipped; v_k is its number of pore voxels (voxel volume
units).  Two primitives are adjacent when a face of a pore voxel of one
touches a pore voxel of the other; the contact surface S_ij is the number of
such faces and d_ij the distance between the centres of gravity of the two
primitives (in voxels).  The starting conductances are theta_ij = S_ij / d_ij
(Sec. V.B).

Objectives (Sec. V.A), for data pairs (X^p, Y^p) of primitive masses at t and
t + dt, c = Dc dt, s_i = x_i / v_i (or y_i / v_i):
  r1_i = y_i - x_i + c sum_j theta_ij (x_i/v_i - x_j/v_j),  L1 = mean_p mean_i r1_i^2
  r2_i = x_i - y_i - c sum_j theta_ij (y_i/v_i - y_j/v_j),  L2 = mean_p mean_i r2_i^2
Readings: the inner term is x_j / v_j (the printed x_i / v_j is a slip: with
it the sum would not vanish for equal concentrations); theta_ij is a
parameter per ordered pair, as the paper's derivative treats it (it appears
in row i only); the derivative of L2 carries a minus sign, which the printed
formula drops (d r2_i / d theta_ij = -c (y_i/v_i - y_j/v_j)).
Scheme 3 (explicit PNGM step): m_i <- m_i - c sum_j theta_ij (m_i/v_i - m_j/v_j).
Scheme 4 (implicit PNGM step): the new masses y solve
y_i + c sum_j theta_ij (y_i/v_i - y_j/v_j) = m_i (a dense solve here).
"""
from __future__ import annotations

import numpy as np


def partition(mask: np.ndarray, b: int):
    """Primitives of the pore voxels of `mask` ([nz][ny][nx], nonzero = pore)
    for bricks of side b.  Returns a dict with
      prim  [n]   primitive of each pore voxel, pore voxels in raster order
      v     [q]   pore voxels per primitive
      row   [q+1], col [E]  directed adjacency (CSR, columns ascending)
      S, d  [E]   contact faces and centroid distance per directed edge."""
    mask = np.asarray(mask) != 0
    nz, ny, nx = mask.shape
    nbx, nby, nbz = -(-nx // b), -(-ny // b), -(-nz // b)
    zz, yy, xx = np.nonzero(mask)                       # raster order (z slowest)
    brick = (zz // b * nby + yy // b) * nbx + xx // b
    used, prim = np.unique(brick, return_inverse=True)  # bricks with pore, raster order
    q = used.size
    v = np.bincount(prim, minlength=q).astype(np.float64)
    cx = np.bincount(prim, weights=xx, minlength=q) / v
    cy = np.bincount(prim, weights=yy, minlength=q) / v
    cz = np.bincount(prim, weights=zz, minlength=q) / v
    # primitive of every voxel position (-1: solid)
    pmap = -np.ones(mask.shape, np.int64)
    pmap[zz, yy, xx] = prim
    contacts = {}
    for axis, (dz, dy, dx) in enumerate(((0, 0, 1), (0, 1, 0), (1, 0, 0))):
        a = pmap[:nz - dz, :ny - dy, :nx - dx]
        c = pmap[dz:, dy:, dx:]
        sel = (a >= 0) & (c >= 0) & (a != c)
        for i, j in zip(a[sel].ravel(), c[sel].ravel()):
            contacts[(i, j)] = contacts.get((i, j), 0) + 1
            contacts[(j, i)] = contacts.get((j, i), 0) + 1
    keys = sorted(contacts)
    row = np.zeros(q + 1, np.int64)
    col = np.array([j for _, j in keys], np.int64)
    S = np.array([contacts[k] for k in keys], np.float64)
    for i, _ in keys:
        row[i + 1] += 1
    row = np.cumsum(row)
    src = np.array([i for i, _ in keys], np.int64)
    d = np.sqrt((cx[src] - cx[col]) ** 2 + (cy[src] - cy[col]) ** 2 + (cz[src] - cz[col]) ** 2)
    return dict(prim=prim, v=v, row=row, col=col, S=S, d=d, q=q)


def primitive_masses(part, m_voxels: np.ndarray) -> np.ndarray:
    """Masses per primitive of a voxel field (pore voxels in raster order)."""
    return np.bincount(part["prim"], weights=m_voxels, minlength=part["q"])


def scheme3_step(part, m: np.ndarray, theta: np.ndarray, c: float) -> np.ndarray:
    """One explicit PNGM step (scheme 3)."""
    v, row, col = part["v"], part["row"], part["col"]
    out = m.copy()
    for i in range(part["q"]):
        s = 0.0
        for e in range(row[i], row[i + 1]):
            j = col[e]
            s += theta[e] * (m[i] / v[i] - m[j] / v[j])
        out[i] = m[i] - c * s
    return out


def loss_grad(part, X: np.ndarray, Y: np.ndarray, theta: np.ndarray, c: float, objective: int):
    """L1 or L2 over the data pairs X, Y ([l][q]) and its gradient [E]."""
    v, row, col = part["v"], part["row"], part["col"]
    q = part["q"]
    l = X.shape[0]
    loss = 0.0
    grad = np.zeros(col.size)
    for p in range(l):
        x, y = X[p], Y[p]
        for i in range(q):
            if objective == 1:
                s = sum(theta[e] * (x[i] / v[i] - x[col[e]] / v[col[e]]) for e in range(row[i], row[i + 1]))
                r = y[i] - x[i] + c * s
                for e in range(row[i], row[i + 1]):
                    grad[e] += 2.0 / (l * q) * r * c * (x[i] / v[i] - x[col[e]] / v[col[e]])
            else:
                s = sum(theta[e] * (y[i] / v[i] - y[col[e]] / v[col[e]]) for e in range(row[i], row[i + 1]))
                r = x[i] - y[i] - c * s
                for e in range(row[i], row[i + 1]):
                    grad[e] -= 2.0 / (l * q) * r * c * (y[i] / v[i] - y[col[e]] / v[col[e]])
            loss += r * r / (l * q)
    return loss, grad


def scheme4_step(part, m: np.ndarray, theta: np.ndarray, c: float) -> np.ndarray:
    """One implicit PNGM step (scheme 4): the matrix of the linear system is
    written out densely and solved (small partitions only)."""
    v, row, col, q = part["v"], part["row"], part["col"], part["q"]
    A = np.eye(q)
    for i in range(q):
        for e in range(row[i], row[i + 1]):
            j = col[e]
            A[i, i] += c * theta[e] / v[i]
            A[i, j] -= c * theta[e] / v[j]
    return np.linalg.solve(A, m)
