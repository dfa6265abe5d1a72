"""Pore-voxel graph on the GPU (Sec. II.A, Fig. 2; Sec. III).

``Graph.from_masks`` uploads binary masks and calls ``vg_count_pores`` /
``vg_build_graph`` per volume: the compacted pore list ``vox`` and the 6-slot
neighbour table ``nbr`` ([6][n], slots -x, +x, -y, +y, -z, +z; -1 absent) of
all volumes share one index space, volume b owning ``[seg_off[b],
seg_off[b+1])``.  Tensors live on the GPU; torch only allocates them.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib


class Graph:
    def __init__(self, shape, n, seg_off, vox, nbr, ranks, brick, periodic, rcode=None):
        self.shape = tuple(int(v) for v in shape)   # (nz, ny, nx) of every volume
        self.n = int(n)
        self.seg_off = np.asarray(seg_off, np.int64)
        self.vox = vox          # int32 [n] cuda
        self.nbr = nbr          # int32 [6, n] cuda
        self.ranks = ranks      # per-volume rank index (uint8 cuda tensors)
        self.brick = int(brick)
        self.periodic = int(periodic)
        self.rcode = rcode      # int16 [n] cuda (bit pattern of uint16 codes) or None

    @property
    def nseg(self) -> int:
        return int(self.seg_off.size - 1)

    @classmethod
    def from_masks(cls, masks, brick: int = 0, periodic: int = 0, regions: bool = False,
                   device="cuda", stream=None) -> "Graph":
        """Build the graph of one mask ([nz, ny, nx]) or of a batch of equally
        shaped masks (sequence or [B, nz, ny, nx]); nonzero = pore."""
        L = _lib.load()
        if isinstance(masks, np.ndarray) and masks.ndim == 3:
            masks = [masks]
        masks = [np.ascontiguousarray(m, dtype=np.uint8) for m in masks]
        shape = masks[0].shape
        if any(m.shape != shape for m in masks):
            raise ValueError("all volumes of a batch must share one shape")
        nz, ny, nx = shape
        dev = torch.device(device)
        sp = _lib.stream_ptr(stream)
        nbytes = ctypes.c_size_t(0)
        _lib.check(L.vg_rank_bytes(nx, ny, nz, brick, ctypes.byref(nbytes)), "vg_rank_bytes")
        ranks, counts = [], []
        for m in masks:
            md = torch.from_numpy(m).to(dev)
            rank = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
            cnt = ctypes.c_int64(0)
            _lib.check(L.vg_count_pores(md.data_ptr(), nx, ny, nz, brick, rank.data_ptr(),
                                        ctypes.byref(cnt), sp), "vg_count_pores")
            ranks.append(rank)
            counts.append(cnt.value)
            del md
        seg_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        n = int(seg_off[-1])
        if n > 2**31 - 1:
            raise ValueError("more than 2^31-1 pore voxels")
        vox = torch.empty(n, dtype=torch.int32, device=dev)
        nbr = torch.empty((6, n), dtype=torch.int32, device=dev)
        for b, rank in enumerate(ranks):
            lo = int(seg_off[b])
            nb = counts[b]
            if nb == 0:
                continue
            _lib.check(L.vg_build_graph(rank.data_ptr(), nx, ny, nz, brick, periodic, lo, nb, n,
                                        vox.data_ptr() + 4 * lo, nbr.data_ptr() + 4 * lo, sp),
                       "vg_build_graph")
        g = cls(shape, n, seg_off, vox, nbr, ranks, brick, periodic)
        if regions:
            g.make_region_codes(stream)
        return g

    def make_region_codes(self, stream=None):
        """Octant region codes for the region conductance factors."""
        L = _lib.load()
        nz, ny, nx = self.shape
        self.rcode = torch.empty(self.n, dtype=torch.int16, device=self.vox.device)
        if self.n:
            _lib.check(L.vg_region_codes(self.vox.data_ptr(), self.n, nx, ny, nz, self.periodic,
                                         self.rcode.data_ptr(), _lib.stream_ptr(stream)), "vg_region_codes")
        return self.rcode

    def lookup(self, volume: int, lin, stream=None) -> torch.Tensor:
        """Compact indices (int32, -1 for solid) of linear voxel indices of a volume."""
        L = _lib.load()
        nz, ny, nx = self.shape
        lin_d = torch.as_tensor(np.asarray(lin, np.int64)).to(self.vox.device)
        out = torch.empty(lin_d.numel(), dtype=torch.int32, device=self.vox.device)
        if lin_d.numel():
            _lib.check(L.vg_lookup(self.ranks[volume].data_ptr(), nx, ny, nz, self.brick, lin_d.data_ptr(),
                                   lin_d.numel(), int(self.seg_off[volume]), out.data_ptr(),
                                   _lib.stream_ptr(stream)), "vg_lookup")
        return out

    def fields_from_specs(self, specs, dtype=torch.float32) -> torch.Tensor:
        """[5, n] tensor of initial masses from sparse specs (one per volume,
        ``{pool: (linear_indices, values)}``)."""
        if isinstance(specs, dict):
            specs = [specs]
        x = torch.zeros((5, self.n), dtype=dtype, device=self.vox.device)
        for b, spec in enumerate(specs):
            for s, (idx, val) in spec.items():
                pos = self.lookup(b, idx).long()
                if bool((pos < 0).any()):
                    raise ValueError("initial mass on a solid voxel")
                x[s, pos] = torch.as_tensor(np.asarray(val, np.float64), device=x.device).to(dtype)
        return x


def layer_offsets(mask: np.ndarray) -> np.ndarray:
    """[nz + 1] start of every z-layer in the raster-ordered compacted list of
    one volume (its pore voxels in layers < z), from the mask."""
    counts = (np.asarray(mask).reshape(mask.shape[0], -1) != 0).sum(axis=1)
    return np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)


def range_sums(x: torch.Tensor, offsets: torch.Tensor) -> torch.Tensor:
    """FP64 sums of a 1-D float/double CUDA tensor over contiguous ranges
    (``offsets``: int64 CUDA tensor of nranges + 1 starts), by vg_range_sums."""
    L = _lib.load()
    if x.dim() != 1 or x.dtype not in (torch.float32, torch.float64) or offsets.dtype != torch.int64:
        raise ValueError("x must be 1-D float32/float64, offsets int64")
    x = x.contiguous()
    offsets = offsets.contiguous()
    nr = offsets.numel() - 1
    out = torch.empty(max(nr, 0), dtype=torch.float64, device=x.device)
    prec = _lib.VG_F64 if x.dtype == torch.float64 else _lib.VG_F32
    _lib.check(L.vg_range_sums(x.data_ptr(), prec, x.numel(), offsets.data_ptr(), max(nr, 0),
                               out.data_ptr() if nr > 0 else None, _lib.stream_ptr(None)), "vg_range_sums")
    return out

