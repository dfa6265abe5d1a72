"""Simulation state on the GPU: explicit and implicit time steps, mass totals,
forward recording and the adjoint sweep (thin wrapper over the C ABI).

Pools are numbered in the paper's order (Sec. II.A): 0 MB, 1 DOM, 2 SOM,
3 FOM (called P4), 4 CO2.  Fields are a ``[5, n]`` tensor of the field type;
torch allocates every buffer and supplies the stream, the library's kernels do
all the arithmetic.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from .graph import Graph
from .inputs import ModelParams

_DTYPES = {"f32": torch.float32, "f64": torch.float64, "f32c": torch.float32}
_PREC = {"f32": _lib.VG_F32, "f64": _lib.VG_F64, "f32c": _lib.VG_F32C}


def to_vg_params(p: ModelParams, step_order: int = _lib.VG_ORDER_TD) -> _lib.VgParams:
    vp = _lib.VgParams()
    for s in range(5):
        vp.D[s] = float(p.D[s])
    vp.h, vp.v_dom, vp.k_dom, vp.rho, vp.mu = float(p.h), float(p.v_dom), float(p.k_dom), float(p.rho), float(p.mu)
    vp.beta, vp.v_som, vp.v_p4 = float(p.beta), float(p.v_som), float(p.v_p4)
    vp.mort_to_p4 = 1 if p.mort_to_p4 else 0
    vp.step_order = int(step_order)
    vp.sequential = 1 if getattr(p, "sequential", False) else 0
    return vp


class Simulation:
    """Binds a graph, parameters and GPU buffers to a library handle."""

    def __init__(self, graph: Graph, params: ModelParams, precision: str = "f32",
                 implicit: bool = True, adjoint: bool = False, mobile_all=None,
                 step_order: int = _lib.VG_ORDER_TD, regions=None, stream=None, rank_neighbours: bool = True,
                 band: bool = True, segments=None, multigrid: bool = False):
        self.L = _lib.load()
        self.graph = graph
        self.precision = precision
        self.dtype = _DTYPES[precision]
        self.step_order = step_order
        self.stream = stream
        if mobile_all is None:
            mobile_all = any(float(d) != 0.0 for s, d in enumerate(params.D) if s != 1)
        self.mobile_all = bool(mobile_all)
        self._adj_skip = self._adj_tape_dom = False
        features = ((_lib.VG_FEAT_CG if implicit else 0) | (_lib.VG_FEAT_ADJ if adjoint else 0)
                    | (_lib.VG_FEAT_BAND if band else 0) | (_lib.VG_FEAT_MG if multigrid else 0))
        # segments of the totals (and of the adjoint's seeds): the volumes, or
        # a finer split of the compacted list given by the caller
        self._seg = np.ascontiguousarray(graph.seg_off if segments is None else segments, np.int64)
        self.nseg = int(self._seg.size - 1)
        use_regions = regions is not None or graph.rcode is not None
        if use_regions and graph.rcode is None:
            graph.make_region_codes(stream)
        desc = _lib.VgDesc()
        desc.n = graph.n
        desc.nseg = self.nseg
        desc.precision = _PREC[precision]
        desc.seg_off = self._seg.ctypes.data
        desc.nbr_d = graph.nbr.data_ptr() if graph.n else None
        desc.rcode_d = graph.rcode.data_ptr() if (use_regions and graph.n) else None
        desc.mobile_all = 1 if mobile_all else 0
        desc.features = features
        if self.nseg == 1 and graph.n and rank_neighbours:
            nz, ny, nx = graph.shape
            desc.rank_d = graph.ranks[0].data_ptr()
            desc.vox_d = graph.vox.data_ptr()
            desc.nx, desc.ny, desc.nz = nx, ny, nz
            desc.brick, desc.periodic = graph.brick, graph.periodic
        h = ctypes.c_void_p()
        _lib.check(self.L.vg_create(ctypes.byref(desc), ctypes.byref(h)), "vg_create")
        self.h = h
        self.set_params(params)
        if regions is not None:
            self.set_regions(regions)
        dev = graph.vox.device
        alt = ctypes.c_int64(0)
        _lib.check(self.L.vg_alt_elems(h, ctypes.byref(alt)), "vg_alt_elems")
        wsb = ctypes.c_size_t(0)
        _lib.check(self.L.vg_workspace_bytes(h, ctypes.byref(wsb)), "vg_workspace_bytes")
        self.fields = torch.zeros((5, graph.n), dtype=self.dtype, device=dev)
        self.alt = torch.empty(max(alt.value, 1), dtype=self.dtype, device=dev)
        self.work = torch.empty(wsb.value, dtype=torch.uint8, device=dev)
        _lib.check(self.L.vg_init_state(h, self.fields.data_ptr(), self.alt.data_ptr(), self.work.data_ptr(),
                                        wsb.value, self._sp()), "vg_init_state")

    # ------------------------------------------------------------------ setup
    def _sp(self):
        return _lib.stream_ptr(self.stream)

    def set_kernel(self, variant: int):
        """Neighbour source of the explicit step: _lib.VG_KERNEL_AUTO / TABLE / RANK / OFFSET / RELATIVE /
        BAND (relative codes, pass pairs in one launch)."""
        _lib.check(self.L.vg_set_kernel(self.h, int(variant)), "vg_set_kernel")

    def set_launch_options(self, graphs: str = "auto"):
        """Replay runs of fused passes from captured HIP graphs: "auto" (small
        volumes), "on" or "off"; results are bit-identical either way."""
        flags = {"auto": _lib.VG_LAUNCH_GRAPHS_AUTO, "on": _lib.VG_LAUNCH_GRAPHS_ON, "off": _lib.VG_LAUNCH_GRAPHS_OFF}
        _lib.check(self.L.vg_set_launch_options(self.h, flags[graphs]), "vg_set_launch_options")

    def kernel_in_use(self) -> int:
        """The kernel the next explicit passes use (TABLE, RANK, OFFSET, RELATIVE or BAND)."""
        v = ctypes.c_int(-1)
        _lib.check(self.L.vg_get_kernel(self.h, ctypes.byref(v)), "vg_get_kernel")
        return v.value

    def set_params(self, params: ModelParams):
        self.params = params
        vp = to_vg_params(params, self.step_order)
        _lib.check(self.L.vg_set_params(self.h, ctypes.byref(vp)), "vg_set_params")

    def set_regions(self, c):
        arr = (ctypes.c_double * 8)(*[float(v) for v in c])
        _lib.check(self.L.vg_set_regions(self.h, arr), "vg_set_regions")
        self.regions = list(map(float, c))

    def set_fields(self, x: torch.Tensor):
        """Copy a [5, n] tensor into the bound fields.  Compensated fields
        ("f32c") take a float64 state at their full precision (vg_load_state)."""
        if self.precision == "f32c":
            src = x.to(device=self.fields.device)
            if src.dtype != torch.float32:
                src = src.to(torch.float64)
            src = src.contiguous()
            prec = _lib.VG_F64 if src.dtype == torch.float64 else _lib.VG_F32
            _lib.check(self.L.vg_load_state(self.h, src.data_ptr(), prec, self._sp()), "vg_load_state")
            if self.stream is not None:     # src belongs to the current stream
                self.stream.synchronize()
            return
        self.fields.copy_(x.to(device=self.fields.device, dtype=self.dtype))

    def state(self, dtype=torch.float64) -> torch.Tensor:
        """The bound state as a new [5, n] tensor (float64: for compensated
        fields the full-precision value, vg_store_state)."""
        out = torch.empty((5, self.graph.n), dtype=dtype, device=self.fields.device)
        prec = _lib.VG_F64 if dtype == torch.float64 else _lib.VG_F32
        _lib.check(self.L.vg_store_state(self.h, out.data_ptr(), prec, self._sp()), "vg_store_state")
        return out

    def close(self):
        if getattr(self, "h", None) is not None:
            self.L.vg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ stepping
    def step(self, nsteps: int, dt: float, log_every: int = 0, force: bool = False,
             totals_out: torch.Tensor = None):
        """Advance ``nsteps`` explicit steps.  Returns the FP64 totals log
        [nsteps // log_every, nseg, 6] (cuda) when ``log_every > 0``."""
        nlog = nsteps // log_every if log_every > 0 else 0
        log = totals_out
        if nlog and log is None:
            log = torch.empty((nlog, self.nseg, 6), dtype=torch.float64, device=self.fields.device)
        _lib.check(self.L.vg_step_explicit(self.h, int(nsteps), float(dt), int(log_every),
                                           log.data_ptr() if nlog else None,
                                           _lib.VG_FORCE if force else 0, self._sp()), "vg_step_explicit")
        return log if nlog else None

    def step_subcycled(self, n_t: int, dt_t: float, dt_d: float, force: bool = False):
        """Unequal steps: n_t transformation steps of dt_t and diffusion steps of
        dt_d (the last shortened) over n_t * dt_t, ordered by start time."""
        _lib.check(self.L.vg_step_subcycled(self.h, int(n_t), float(dt_t), float(dt_d),
                                            _lib.VG_FORCE if force else 0, self._sp()), "vg_step_subcycled")

    def implicit_step(self, dt: float, rtol: float = 1e-10, max_iter: int = 1000, check: bool = True):
        """One implicit step (transformation + Scheme 2 by PCG).  Returns
        (iterations[5], relative residuals[5], status)."""
        it = (ctypes.c_int * 5)()
        rr = (ctypes.c_double * 5)()
        rc = self.L.vg_solve_implicit_step(self.h, float(dt), float(rtol), int(max_iter), it, rr, self._sp())
        if check:
            _lib.check(rc, "vg_solve_implicit_step")
        return list(it), list(rr), rc

    def set_preconditioner(self, which: str = "jacobi"):
        """Preconditioner of the implicit step's CG: "jacobi" (the paper's) or
        "mg" (the multigrid V-cycle; needs multigrid=True at construction)."""
        v = {"jacobi": _lib.VG_PRECOND_JACOBI, "mg": _lib.VG_PRECOND_MG}[which]
        _lib.check(self.L.vg_set_preconditioner(self.h, v), "vg_set_preconditioner")

    def mg_levels(self) -> list:
        """Cells of each level of the multigrid hierarchy (empty without one)."""
        lv = ctypes.c_int(0)
        cells = (ctypes.c_int64 * _lib.VG_MG_MAX_LEVELS)()
        _lib.check(self.L.vg_mg_levels(self.h, ctypes.byref(lv), cells), "vg_mg_levels")
        return [int(cells[l]) for l in range(lv.value)]

    def precondition(self, a: float, r: torch.Tensor) -> torch.Tensor:
        """z = M^-1 r for the system I + a L_w with the current preconditioner
        (r: [n] float64 on the device)."""
        r = r.contiguous()
        if r.dtype != torch.float64 or r.numel() != self.graph.n:
            raise ValueError("r must be a float64 vector of n entries")
        z = torch.empty_like(r)
        _lib.check(self.L.vg_precondition(self.h, float(a), r.data_ptr(), z.data_ptr(), self._sp()),
                   "vg_precondition")
        return z

    def totals(self) -> np.ndarray:
        """[nseg, 6] FP64 totals (pools 0-4, total carbon) of the current state."""
        out = np.zeros((self.nseg, 6), np.float64)
        _lib.check(self.L.vg_mass_totals(self.h, out.ctypes.data_as(ctypes.c_void_p), self._sp()),
                   "vg_mass_totals")
        return out

    # ------------------------------------------------------------------ adjoint
    @property
    def tape_rows(self) -> int:
        """Rows per recorded state (5, or 4 with the kept DOM)."""
        return _lib.check(self.L.vg_tape_rows(self.h), "vg_tape_rows")

    def _check_states(self, nsteps: int, states: torch.Tensor):
        rows = self.tape_rows
        if states.dtype != self.dtype or not states.is_contiguous() or \
                states.numel() < int(nsteps) * rows * self.graph.n or \
                (states.dim() == 3 and states.shape[1:] != (rows, self.graph.n)):
            raise ValueError("states must be a contiguous [nsteps, %d, n] tensor of the field type (the row count "
                             "follows the adjoint option tape_dom)" % rows)

    def record(self, nsteps: int, dt: float, states: torch.Tensor):
        """Record nsteps steps from the bound fields into states
        ([nsteps, tape_rows, n], field type) for adjoint()."""
        self._check_states(nsteps, states)
        _lib.check(self.L.vg_record(self.h, int(nsteps), float(dt), states.data_ptr(), self._sp()), "vg_record")

    def step_record(self, nsteps: int, dt: float, states: torch.Tensor, totals_out: torch.Tensor,
                    force: bool = False):
        """Advance nsteps steps, recording the adjoint's states ([nsteps,
        tape_rows, n] field type, as record()) and the totals after every
        step into totals_out ([nsteps, nseg, 6] FP64 on the device)."""
        if totals_out.dtype != torch.float64 or not totals_out.is_contiguous() or \
                totals_out.numel() < nsteps * self.nseg * 6:
            raise ValueError("totals_out must be a contiguous float64 tensor of nsteps * nseg * 6 entries")
        self._check_states(nsteps, states)
        _lib.check(self.L.vg_step_record(self.h, int(nsteps), float(dt), states.data_ptr(), totals_out.data_ptr(),
                                         _lib.VG_FORCE if force else 0, self._sp()), "vg_step_record")

    def adjoint(self, nsteps: int, dt: float, states: torch.Tensor, seeds: torch.Tensor, lam: torch.Tensor,
                grad: torch.Tensor):
        self._check_states(nsteps, states)
        _lib.check(self.L.vg_adjoint(self.h, int(nsteps), float(dt), states.data_ptr(), seeds.data_ptr(),
                                     lam.data_ptr(), grad.data_ptr(), self._sp()), "vg_adjoint")

    def set_adjoint_options(self, skip_static_d=None, tape_dom=None):
        """skip_static_d: do not compute dL/dD_s for the pools that do not
        diffuse (their gradient entries come back NaN); faster reverse sweep.
        tape_dom: recordings keep each state's diffused DOM, four rows per
        state instead of five (see tape_rows), and the reverse sweep reads it
        (bit-identical results; such recorded states hold no CO2).  An option
        given as None keeps its current value."""
        skip = self._adj_skip if skip_static_d is None else bool(skip_static_d)
        tape = self._adj_tape_dom if tape_dom is None else bool(tape_dom)
        flags = (_lib.VG_ADJ_SKIP_STATIC_D if skip else 0) | (_lib.VG_ADJ_TAPE_DOM if tape else 0)
        _lib.check(self.L.vg_set_adjoint_options(self.h, flags), "vg_set_adjoint_options")
        self._adj_skip, self._adj_tape_dom = skip, tape

    @property
    def adjoint_options(self) -> dict:
        return {"skip_static_d": self._adj_skip, "tape_dom": self._adj_tape_dom}

    def seed_lambda(self, seed: torch.Tensor, lam: torch.Tensor, zero: bool):
        _lib.check(self.L.vg_seed_lambda(self.h, seed.data_ptr(), lam.data_ptr(), 1 if zero else 0, self._sp()),
                   "vg_seed_lambda")
