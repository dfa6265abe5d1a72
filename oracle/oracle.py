"""Plain FP64 CPU oracle of the voxel-graph diffusion-transformation method.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  Nothing here is imported by, or
imports, the HIP path; the only thing the two sides share is the seeded input
description (masks and sparse initial masses), which each side materialises
itself.

The arithmetic lives in ``vg_oracle.c`` (plain loops, FP64, no FMA
contraction); this wrapper builds it with gcc, loads it with ctypes and adds
plain numpy glue (materialising initial masses, octant regions, edge weights).

Every function is "pinned" by the ``-m "not gpu"`` tests against what the
paper and the mathematics fix (closed forms, dense matrices built from the
mask, invariants, brute force); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vg_oracle.c")
# VG_ORACLE_SANITIZE=1 (the sanitizer test, with the runtimes preloaded)
# builds and loads a copy under AddressSanitizer and UndefinedBehaviorSanitizer
_SANITIZE = os.environ.get("VG_ORACLE_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "liboracle_san.so" if _SANITIZE else "liboracle.so")
_SAN_FLAGS = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
_lock = threading.Lock()
_lib = None

NPOOL = 5
NPARAM_BASE = 12
GRAD_NAMES = ("D_MB", "D_DOM", "D_SOM", "D_P4", "D_CO2", "v_dom", "k_dom", "rho", "mu",
              "beta", "v_som", "v_p4")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (``-ffp-contract=off``: no fused multiply-add,
    so every operation rounds exactly as written)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        opt = _SAN_FLAGS if _SANITIZE else ["-O2"]
        cmd = ["gcc"] + opt + ["-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
            L.orc_count.restype = i64
            L.orc_count.argtypes = [P, i64]
            L.orc_build_graph.restype = i32
            L.orc_build_graph.argtypes = [P, i32, i32, i32, i32, i32, P, P, i64]
            L.orc_transform.restype = None
            L.orc_transform.argtypes = [P, dbl, i64, P]
            L.orc_diffuse.restype = None
            L.orc_diffuse.argtypes = [P, dbl, i64, P, P, P, P]
            L.orc_laplacian.restype = None
            L.orc_laplacian.argtypes = [i64, P, P, P, P]
            L.orc_totals.restype = None
            L.orc_totals.argtypes = [i64, P, i32, P, P]
            L.orc_run.restype = i32
            L.orc_run.argtypes = [P, dbl, i32, i64, P, P, P, i64, i32, P, P]
            L.orc_run_subcycled.restype = i32
            L.orc_run_subcycled.argtypes = [P, dbl, dbl, i64, i64, P, P, P]
            L.orc_apply_B.restype = None
            L.orc_apply_B.argtypes = [dbl, i64, P, P, P, P]
            L.orc_pcg.restype = i32
            L.orc_pcg.argtypes = [dbl, i64, P, P, P, P, dbl, i32, P, P]
            L.orc_implicit_step.restype = i32
            L.orc_implicit_step.argtypes = [P, dbl, i64, P, P, P, dbl, i32, P, P]
            L.orc_adjoint.restype = i32
            L.orc_adjoint.argtypes = [P, dbl, i32, i64, P, P, P, i32, i64, P, i32, P, P, P, P, P]
            _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def pack_params(params) -> np.ndarray:
    """prm[15] from any object with attributes D, h, v_dom, k_dom, rho, mu,
    beta, v_som, v_p4, mort_to_p4 (SI units) and optionally sequential
    (Algorithm 2 instead of Algorithm 1)."""
    return np.array(list(map(float, params.D)) + [params.h, params.v_dom, params.k_dom, params.rho,
                    params.mu, params.beta, params.v_som, params.v_p4,
                    1.0 if params.mort_to_p4 else 0.0,
                    1.0 if getattr(params, "sequential", False) else 0.0], dtype=np.float64)


# ---------------------------------------------------------------------------
# graph
# ---------------------------------------------------------------------------
class OracleGraph:
    """Compacted pore-voxel graph, possibly several volumes back to back.

    vox[i]: linear index of voxel i inside its own volume; nbr[6][n]: global
    compact neighbour indices (-1 absent); seg_off[nseg+1]: volume offsets.
    """

    def __init__(self, shape, vox, nbr, seg_off):
        self.shape = tuple(shape)
        self.vox = vox
        self.nbr = nbr
        self.seg_off = np.ascontiguousarray(seg_off, np.int64)   # handed to C as a pointer

    @property
    def n(self) -> int:
        return int(self.vox.size)

    @property
    def nseg(self) -> int:
        return int(self.seg_off.size - 1)


def build_graph(mask: np.ndarray, brick: int = 0, periodic: int = 0) -> OracleGraph:
    """Sec. II.A / Sec. III graph construction (see ``orc_build_graph``)."""
    return build_batch([mask], brick=brick, periodic=periodic)


def build_batch(masks, brick: int = 0, periodic: int = 0) -> OracleGraph:
    L = lib()
    shape = masks[0].shape
    voxs, nbrs, offs = [], [], [0]
    for m in masks:
        m = np.ascontiguousarray(m, dtype=np.uint8)
        if m.shape != shape:
            raise ValueError("all volumes of a batch must share one shape")
        nz, ny, nx = m.shape
        n = int(L.orc_count(_p(m), m.size))
        vox = np.empty(n, np.int32)
        nbr = np.empty((6, n), np.int32)
        rc = L.orc_build_graph(_p(m), nx, ny, nz, int(brick), int(periodic), _p(vox), _p(nbr), n)
        if rc != 0:
            raise RuntimeError("orc_build_graph failed (%d)" % rc)
        base = offs[-1]
        nbrs.append(np.where(nbr >= 0, nbr + base, -1).astype(np.int32))
        voxs.append(vox)
        offs.append(base + n)
    return OracleGraph(shape, np.concatenate(voxs), np.ascontiguousarray(np.concatenate(nbrs, axis=1)),
                       np.array(offs, np.int64))


def fields_from_spec(graph: OracleGraph, specs) -> np.ndarray:
    """Materialise sparse initial masses (one spec per volume) as x[5][n]."""
    if isinstance(specs, dict):
        specs = [specs]
    x = np.zeros((NPOOL, graph.n), np.float64)
    nvox = int(np.prod(graph.shape))
    for g, spec in enumerate(specs):
        lo, hi = int(graph.seg_off[g]), int(graph.seg_off[g + 1])
        where = np.full(nvox, -1, np.int64)
        where[graph.vox[lo:hi]] = np.arange(lo, hi)
        for s, (idx, val) in spec.items():
            pos = where[np.asarray(idx, np.int64)]
            if (pos < 0).any():
                raise ValueError("initial mass on a solid voxel")
            x[s, pos] = np.asarray(val, np.float64)
    return x


def octant_regions(graph: OracleGraph, per_volume: bool = False) -> np.ndarray:
    """Region of voxel i: octant 4[z >= nz/2] + 2[y >= ny/2] + [x >= nx/2]
    (plus 8 * volume when ``per_volume``)."""
    nz, ny, nx = graph.shape
    v = graph.vox.astype(np.int64)
    x, y, z = v % nx, (v // nx) % ny, v // (nx * ny)
    r = 4 * (z >= nz // 2) + 2 * (y >= ny // 2) + (x >= nx // 2)
    if per_volume:
        seg = np.repeat(np.arange(graph.nseg), np.diff(graph.seg_off))
        r = r + 8 * seg
    return r.astype(np.int32)


def edge_weights(graph: OracleGraph, region: np.ndarray, c) -> np.ndarray:
    """w[k][i] = (c[r(i)] + c[r(j)]) / 2 for present neighbours j, else 0."""
    c = np.asarray(c, np.float64)
    w = np.zeros((6, graph.n), np.float64)
    for k in range(6):
        j = graph.nbr[k]
        ok = j >= 0
        w[k, ok] = (c[region[ok]] + c[region[j[ok]]]) / 2.0
    return w


# ---------------------------------------------------------------------------
# time stepping
# ---------------------------------------------------------------------------
def transform(params, dt: float, x: np.ndarray) -> np.ndarray:
    """Eq. (3) / Algorithm 1 on every voxel (returns a new array)."""
    x = np.array(x, np.float64, order="C", copy=True)
    lib().orc_transform(_p(pack_params(params)), float(dt), x.shape[1], _p(x))
    return x


def diffuse(params, dt: float, graph: OracleGraph, x: np.ndarray, w=None) -> np.ndarray:
    """Scheme 1 for every pool with D_s > 0 (returns a new array)."""
    x = np.array(x, np.float64, order="C", copy=True)
    n = x.shape[1]
    tmp = np.empty(max(n, 1), np.float64)
    lib().orc_diffuse(_p(pack_params(params)), float(dt), n, _p(graph.nbr), _p(_c(w, np.float64)),
                      _p(x), _p(tmp))
    return x


def laplacian(graph: OracleGraph, m: np.ndarray, w=None) -> np.ndarray:
    m = np.ascontiguousarray(m, np.float64)
    out = np.empty_like(m)
    lib().orc_laplacian(m.size, _p(graph.nbr), _p(_c(w, np.float64)), _p(m), _p(out))
    return out


def totals(graph: OracleGraph, x: np.ndarray) -> np.ndarray:
    """[nseg][6]: Neumaier sums of the five pools and of total carbon."""
    x = np.ascontiguousarray(x, np.float64)
    out = np.empty((graph.nseg, 6), np.float64)
    lib().orc_totals(x.shape[1], _p(x), graph.nseg, _p(graph.seg_off), _p(out))
    return out


def run(params, dt: float, graph: OracleGraph, x: np.ndarray, nsteps: int, order: int = 0,
        w=None, with_totals: bool = True):
    """Advance ``nsteps`` steps (order 0: transformation then diffusion, as in
    the paper).  Returns (x, totals[nsteps+1][nseg][6] or None)."""
    x = np.array(x, np.float64, order="C", copy=True)
    tot = np.empty((nsteps + 1, graph.nseg, 6), np.float64) if with_totals else None
    rc = lib().orc_run(_p(pack_params(params)), float(dt), int(order), x.shape[1], _p(graph.nbr),
                       _p(_c(w, np.float64)), _p(x), int(nsteps), graph.nseg, _p(graph.seg_off),
                       _p(tot))
    if rc != 0:
        raise RuntimeError("orc_run failed")
    return x, tot


def run_subcycled(params, dt_t: float, dt_d: float, graph: OracleGraph, x: np.ndarray, nt: int, w=None):
    """Unequal transformation / diffusion steps over nt * dt_t (see
    ``orc_run_subcycled``).  Returns the final state."""
    x = np.array(x, np.float64, order="C", copy=True)
    rc = lib().orc_run_subcycled(_p(pack_params(params)), float(dt_t), float(dt_d), int(nt), x.shape[1],
                                 _p(graph.nbr), _p(_c(w, np.float64)), _p(x))
    if rc != 0:
        raise RuntimeError("orc_run_subcycled failed")
    return x


def run_states(params, dt: float, graph: OracleGraph, x: np.ndarray, nsteps: int, order: int = 0,
               w=None) -> np.ndarray:
    """All states x^0..x^nsteps as [nsteps+1][5][n]."""
    st = np.empty((nsteps + 1,) + x.shape, np.float64)
    st[0] = x
    for t in range(nsteps):
        st[t + 1], _ = run(params, dt, graph, st[t], 1, order=order, w=w, with_totals=False)
    return st


def apply_B(a: float, graph: OracleGraph, p: np.ndarray, w=None) -> np.ndarray:
    """(I + a L_w) p (Scheme 2's matrix)."""
    p = np.ascontiguousarray(p, np.float64)
    q = np.empty_like(p)
    lib().orc_apply_B(float(a), p.size, _p(graph.nbr), _p(_c(w, np.float64)), _p(p), _p(q))
    return q


def pcg(a: float, graph: OracleGraph, b: np.ndarray, rtol: float = 1e-14, max_iter: int = 10000,
        w=None):
    """Jacobi-preconditioned CG on (I + a L_w) y = b.  Returns (y, iters, relres, converged)."""
    b = np.ascontiguousarray(b, np.float64)
    y = np.empty_like(b)
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    rc = lib().orc_pcg(float(a), b.size, _p(graph.nbr), _p(_c(w, np.float64)), _p(b), _p(y),
                       float(rtol), int(max_iter), ctypes.byref(it), ctypes.byref(rr))
    if rc < 0:
        raise RuntimeError("orc_pcg failed")
    return y, it.value, rr.value, rc == 0


def implicit_step(params, dt: float, graph: OracleGraph, x: np.ndarray, rtol: float = 1e-14,
                  max_iter: int = 10000, w=None):
    """Transformation, then Scheme 2 by PCG for each pool with D_s > 0."""
    x = np.array(x, np.float64, order="C", copy=True)
    iters = np.zeros(NPOOL, np.int32)
    rel = np.zeros(NPOOL, np.float64)
    rc = lib().orc_implicit_step(_p(pack_params(params)), float(dt), x.shape[1], _p(graph.nbr),
                                 _p(_c(w, np.float64)), _p(x), float(rtol), int(max_iter),
                                 _p(iters), _p(rel))
    if rc < 0:
        raise RuntimeError("orc_implicit_step failed")
    return x, iters, rel


def adjoint(params, dt: float, graph: OracleGraph, states: np.ndarray, seeds: np.ndarray,
            order: int = 0, w=None, region=None, nreg: int = 0, lam_final=None):
    """Discrete adjoint: seeds[t][g][s] = dL/dTotal_{g,s}(t), t = 0..nsteps;
    ``lam_final`` ([5][n]) is an optional adjoint of the last state.
    Returns (dL/dx^0 [5][n], grad[12 + nreg])."""
    states = np.ascontiguousarray(states, np.float64)
    seeds = np.ascontiguousarray(seeds, np.float64)
    nsteps = states.shape[0] - 1
    n = states.shape[2]
    if seeds.shape != (nsteps + 1, graph.nseg, NPOOL):
        raise ValueError("seeds must be [nsteps+1][nseg][5]")
    lam0 = np.empty((NPOOL, n), np.float64)
    grad = np.empty(NPARAM_BASE + nreg, np.float64)
    if getattr(params, "sequential", False):
        raise ValueError("the adjoint follows Algorithm 1 only")
    rc = lib().orc_adjoint(_p(pack_params(params)), float(dt), int(order), n, _p(graph.nbr),
                           _p(_c(w, np.float64)), _p(_c(region, np.int32)), int(nreg), int(nsteps),
                           _p(states), graph.nseg, _p(graph.seg_off), _p(seeds),
                           _p(_c(lam_final, np.float64)), _p(lam0), _p(grad))
    if rc != 0:
        raise RuntimeError("orc_adjoint failed")
    return lam0, grad
