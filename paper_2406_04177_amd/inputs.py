"""Seeded synthetic inputs: pore masks, initial masses and workload presets.

This module only *describes* inputs.  It holds none of the method's
arithmetic (no graph, no transformation, no diffusion): both the HIP path and
the CPU oracle receive what it returns and build everything else themselves.

Stand-in for the paper's data (Sec. IV.A): the authors' 512^3 micro-CT image
of a sandy-loam soil at 24 um with 17 % visible porosity is not available, so
volumes are drawn as seeded uniform noise, smoothed with a Gaussian of sigma = 2
voxels, thresholded so that exactly round(porosity * N) voxels are pore, and
reduced to the largest 6-connected pore component.

Conventions
-----------
* Masks are ``uint8`` arrays of shape ``(nz, ny, nx)``; nonzero marks a pore
  voxel.  The paper tags pore voxels with 0 (Sec. II.A); ``mask = (I == 0)``
  converts.
* The linear index of voxel ``(x, y, z)`` is ``x + nx * (y + ny * z)``, i.e. the
  C-order ravel of the ``(nz, ny, nx)`` array.
* Pools are numbered in the paper's order (Sec. II.A): 0 = MB, 1 = DOM,
  2 = SOM, 3 = FOM (called P4 here), 4 = CO2.
* Initial masses are returned sparsely, as ``{pool: (linear_indices, values)}``;
  every pool not listed, and every voxel not listed, starts at 0.
"""
from __future__ import annotations

import dataclasses

import numpy as np

MB, DOM, SOM, P4, CO2 = range(5)
POOL_NAMES = ("MB", "DOM", "SOM", "P4", "CO2")


# ---------------------------------------------------------------------------
# volumes
# ---------------------------------------------------------------------------
def synthetic_volume(shape, porosity: float = 0.17, sigma: float = 2.0,
                     seed: int = 0, largest_component: bool = True) -> np.ndarray:
    """Seeded pore mask of ``shape = (nz, ny, nx)`` (or an int for a cube).

    Noise ``default_rng(seed).random(shape, float32)`` is smoothed by a separable
    Gaussian (sigma voxels, truncated at 4 sigma, reflecting borders).  The
    ``round(porosity * N)`` smallest smoothed values become pore; ties at the
    threshold go to the lowest linear indices, so the count is exact.  With
    ``largest_component`` only the largest 6-connected pore component is kept
    (ties: the component holding the lowest linear index).
    """
    import scipy.ndimage as ndi

    if isinstance(shape, (int, np.integer)):
        shape = (int(shape),) * 3
    shape = tuple(int(s) for s in shape)
    rng = np.random.default_rng(seed)
    noise = rng.random(shape, dtype=np.float32)
    g = ndi.gaussian_filter(noise, sigma, mode="reflect", truncate=4.0)
    flat = g.ravel()
    k = int(round(porosity * flat.size))
    pore = np.zeros(flat.size, dtype=bool)
    if k > 0:
        t = np.partition(flat, k - 1)[k - 1]
        pore = flat < t
        need = k - int(pore.sum())
        if need > 0:
            pore[np.flatnonzero(flat == t)[:need]] = True
    pore = pore.reshape(shape)
    if largest_component and pore.any():
        lab, nlab = ndi.label(pore)  # default structure = 6-connectivity
        counts = np.bincount(lab.ravel())
        counts[0] = 0
        keep = int(np.argmax(counts))  # first maximum = lowest label = lowest index
        pore = lab == keep
    return pore.astype(np.uint8)


# ---------------------------------------------------------------------------
# initial masses
# ---------------------------------------------------------------------------
def init_spots(mask: np.ndarray, seed: int = 0, n_dom: int = 50, dom_value: float = 1.0,
               n_mb: int = 100, mb_value: float = 0.5) -> dict:
    """DOM = ``dom_value`` in ``n_dom`` random pore voxels and MB = ``mb_value`` in
    ``n_mb`` random pore voxels (two independent draws without replacement from
    ``default_rng(seed + 1)``; the two sets may overlap)."""
    lin = np.flatnonzero(mask.ravel())
    rng = np.random.default_rng(seed + 1)
    d = rng.choice(lin.size, size=min(n_dom, lin.size), replace=False)
    m = rng.choice(lin.size, size=min(n_mb, lin.size), replace=False)
    return {DOM: (lin[np.sort(d)], np.full(d.size, float(dom_value))),
            MB: (lin[np.sort(m)], np.full(m.size, float(mb_value)))}


def init_uniform(mask: np.ndarray, seed: int = 0, frac_dom: float = 0.005,
                 n_mb: int = 100, mb_value: float = 0.5) -> dict:
    """DOM ~ U(0,1) in ``round(frac_dom * n)`` random pore voxels and MB =
    ``mb_value`` in ``n_mb`` random pore voxels (``default_rng(seed + 1)``)."""
    lin = np.flatnonzero(mask.ravel())
    rng = np.random.default_rng(seed + 1)
    nd = min(int(round(frac_dom * lin.size)), lin.size)
    d = np.sort(rng.choice(lin.size, size=nd, replace=False))
    vals = rng.random(nd)
    m = np.sort(rng.choice(lin.size, size=min(n_mb, lin.size), replace=False))
    return {DOM: (lin[d], vals), MB: (lin[m], np.full(m.size, float(mb_value)))}


def init_random_all(mask: np.ndarray, seed: int = 0, scale=(0.5, 1.0, 0.3, 0.2, 0.1)) -> dict:
    """Every pool U(0, scale[s]) in every pore voxel (dense test states)."""
    lin = np.flatnonzero(mask.ravel())
    rng = np.random.default_rng(seed + 7)
    return {s: (lin, scale[s] * rng.random(lin.size)) for s in range(5)}


# ---------------------------------------------------------------------------
# parameters and workloads
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class ModelParams:
    """Physical parameters in SI units (m, s).  ``D`` is per pool.

    Mortality routing: ``mort_to_p4 = False`` is the paper's (a fraction ``beta``
    of dead biomass to DOM, the rest to SOM, Sec. II.C); ``True`` sends it all
    to pool 3 (the "dead microbial biomass" reading of that pool).
    """
    D: tuple = (0.0, 1e-9, 0.0, 0.0, 0.0)
    h: float = 24e-6
    v_dom: float = 1e-4
    k_dom: float = 0.5
    rho: float = 2e-6
    mu: float = 5e-7
    beta: float = 0.55
    v_som: float = 1e-7
    v_p4: float = 1e-7
    mort_to_p4: bool = False
    sequential: bool = False       # Appendix A Algorithm 2 instead of Algorithm 1

    def replace(self, **kw) -> "ModelParams":
        return dataclasses.replace(self, **kw)


def explicit_dt(params: ModelParams, factor: float = 0.9, max_weight_sum: float = 6.0) -> float:
    """``factor * h^2 / (max_s D_s * max_weight_sum)`` as a plain number."""
    dmax = max(params.D)
    return factor * params.h * params.h / (dmax * max_weight_sum)


@dataclasses.dataclass
class Workload:
    name: str
    shape: tuple
    seeds: tuple
    porosities: tuple
    init: str
    steps: int
    dt_factor: float


# The five workloads: 48^3 FP64 parity; 256^3 FP32 vs FP64; 512^3 full size
# (explicit + implicit at 20x the bound); 16 x 128^3 batch for gradients;
# 1024^3 brick-ordered.
WORKLOADS = {
    "w48": Workload("48^3 spots FP64", (48, 48, 48), (0,), (0.17,), "spots", 2000, 0.9),
    "w256": Workload("256^3 FP32 vs FP64", (256, 256, 256), (0,), (0.17,), "uniform", 10000, 0.9),
    "w512": Workload("512^3 17% explicit FP32", (512, 512, 512), (0,), (0.17,), "uniform", 100000, 0.9),
    "b16x128": Workload("16 x 128^3 batch gradients", (128, 128, 128), tuple(range(16)),
                        tuple(float(np.random.default_rng(b).uniform(0.12, 0.25)) for b in range(16)),
                        "uniform", 2000, 0.8),
    "w1024": Workload("1024^3 brick-ordered", (1024, 1024, 1024), (0,), (0.17,), "uniform", 2000, 0.9),
}


def workload_inputs(key: str, shape=None):
    """Masks and sparse initial masses for a workload (``shape`` overrides size)."""
    w = WORKLOADS[key]
    shp = tuple(shape) if shape is not None else w.shape
    masks, inits = [], []
    for seed, por in zip(w.seeds, w.porosities):
        m = synthetic_volume(shp, porosity=por, seed=seed)
        masks.append(m)
        inits.append(init_spots(m, seed) if w.init == "spots" else init_uniform(m, seed))
    return masks, inits



# Parameters the gradient workload perturbs to make its target curve: the
# diffusing pool's D, the uptake rate, the respiration rate and the eight region
# factors, as indices into the 20-entry parameter vector
# [D_0..D_4, v_DOM, K_DOM, rho, mu, beta, v_SOM, v_P4, c_0..c_7].
PERTURBED = (1, 5, 7) + tuple(range(12, 20))


def target_factors(seed: int = 1000, spread: float = 0.1) -> dict:
    """Multipliers 1 + U(-spread, spread) for the PERTURBED entries, in order."""
    d = np.random.default_rng(seed).uniform(-spread, spread, len(PERTURBED))
    return {q: 1.0 + float(v) for q, v in zip(PERTURBED, d)}


def epoch_subsets(nvol: int, size: int, epochs: int, seed: int = 0) -> list:
    """Volumes used by each epoch of a stochastic fit: `size` distinct volumes
    per epoch, sorted, from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return [np.sort(rng.choice(nvol, size=size, replace=False)) for _ in range(epochs)]


def init_scenario(mask: np.ndarray, seed: int, frac: float = 0.01, mass_range=(0.5, 1.5)) -> dict:
    """A random DOM distribution for the pore-network data (Sec. V.B): a total
    mass M0 ~ U(mass_range) spread over round(frac * n) random pore voxels with
    U(0, 1) weights (``default_rng(seed + 11)``)."""
    lin = np.flatnonzero(mask.ravel())
    rng = np.random.default_rng(seed + 11)
    k = max(1, min(int(round(frac * lin.size)), lin.size))
    idx = np.sort(rng.choice(lin.size, size=k, replace=False))
    w = rng.random(k)
    m0 = rng.uniform(*mass_range)
    return {DOM: (lin[idx], m0 * w / w.sum())}
