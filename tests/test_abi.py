"""The C ABI loads, exports every entry point that include/vgsim.h declares,
and its host-side validation rejects bad arguments (no GPU needed: none of
these calls reaches the device)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2406_04177_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "vgsim.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(vg_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(_lib.EXPORTS)


def declared_arity():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for m in re.finditer(r"^\s*(?:const\s+)?\w+\s*\*?\s*(vg_\w+)\s*\(([^)]*)\)\s*;", text, flags=re.M):
        params = m.group(2).strip()
        out[m.group(1)] = 0 if params in ("", "void") else len(params.split(","))
    return out


def test_binding_argument_counts_match_the_header():
    L = _lib.load()
    arity = declared_arity()
    assert sorted(arity) == declared_functions()
    for name, count in arity.items():
        assert len(getattr(L, name).argtypes) == count, name


def test_every_declared_symbol_is_exported():
    L = _lib.load()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert L.vg_version() >= 100


def test_error_strings():
    L = _lib.load()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert len(L.vg_strerror(code)) > 0


def test_rank_bytes_validation():
    L = _lib.load()
    n = ctypes.c_size_t(0)
    assert L.vg_rank_bytes(48, 48, 48, 0, ctypes.byref(n)) == 0
    assert n.value >= 48 ** 3 // 32 * 8
    assert L.vg_rank_bytes(0, 4, 4, 0, ctypes.byref(n)) == _lib.VG_EINVAL
    assert L.vg_rank_bytes(4, 4, 4, -1, ctypes.byref(n)) == _lib.VG_EINVAL
    assert L.vg_rank_bytes(2048, 2048, 1024, 0, ctypes.byref(n)) == _lib.VG_EINVAL   # > 2^31 voxels
    assert b"2^31" in L.vg_last_error()
    assert L.vg_count_pores(None, 4, 4, 4, 0, None, None, None) == _lib.VG_EINVAL


def make_handle(n=1000, nseg=1, mobile_all=0, features=3):
    L = _lib.load()
    seg = np.linspace(0, n, nseg + 1).astype(np.int64)
    desc = _lib.VgDesc()
    desc.n, desc.nseg, desc.precision = n, nseg, _lib.VG_F32
    desc.seg_off = seg.ctypes.data
    desc.nbr_d = 0x1000          # never dereferenced by host-side calls
    desc.rcode_d = None
    desc.mobile_all, desc.features = mobile_all, features
    h = ctypes.c_void_p()
    rc = L.vg_create(ctypes.byref(desc), ctypes.byref(h))
    return rc, h, seg


def test_create_validates_descriptor():
    L = _lib.load()
    rc, h, seg = make_handle()
    assert rc == 0 and h.value
    L.vg_destroy(h)
    desc = _lib.VgDesc()
    seg = np.array([0, 5, 3], np.int64)
    desc.n, desc.nseg, desc.precision, desc.seg_off, desc.nbr_d = 3, 2, 0, seg.ctypes.data, 0x1000
    assert L.vg_create(ctypes.byref(desc), ctypes.byref(ctypes.c_void_p())) == _lib.VG_EINVAL
    desc.precision = 7
    assert L.vg_create(ctypes.byref(desc), ctypes.byref(ctypes.c_void_p())) == _lib.VG_EINVAL


def test_params_validation():
    from paper_2406_04177_amd.inputs import ModelParams
    from paper_2406_04177_amd.sim import to_vg_params
    L = _lib.load()
    rc, h, _ = make_handle()
    ok = to_vg_params(ModelParams())
    assert L.vg_set_params(h, ctypes.byref(ok)) == 0
    for bad in (ModelParams(k_dom=0.0), ModelParams(rho=-1.0), ModelParams(beta=1.5), ModelParams(h=0.0),
                ModelParams(D=(1e-9, 1e-9, 0, 0, 0)), ModelParams(mu=float("nan"))):
        assert L.vg_set_params(h, ctypes.byref(to_vg_params(bad))) == _lib.VG_EINVAL
    # another pool may diffuse when the handle allows it
    rc, h2, _ = make_handle(mobile_all=1)
    assert L.vg_set_params(h2, ctypes.byref(to_vg_params(ModelParams(D=(1e-9, 1e-9, 0, 0, 0))))) == 0
    c_bad = (ctypes.c_double * 8)(1, 1, 1, 0, 1, 1, 1, 1)
    assert L.vg_set_regions(h, c_bad) == _lib.VG_EINVAL
    L.vg_destroy(h)
    L.vg_destroy(h2)


def test_explicit_stability_bound_is_checked_before_any_device_work():
    """Sec. IV.C: beyond dt = h^2 / (6 D) the explicit scheme gives negative
    masses; the library refuses such a step unless forced."""
    from paper_2406_04177_amd.inputs import ModelParams, explicit_dt
    from paper_2406_04177_amd.sim import to_vg_params
    L = _lib.load()
    rc, h, _ = make_handle()
    p = ModelParams()
    L.vg_set_params(h, ctypes.byref(to_vg_params(p)))
    bound = explicit_dt(p, factor=1.0)
    assert L.vg_step_explicit(h, 10, bound * 1.01, 0, None, 0, None) == _lib.VG_EUNSTABLE
    # below the bound (or forced) the call gets as far as the state check
    assert L.vg_step_explicit(h, 10, bound * 0.99, 0, None, 0, None) == _lib.VG_ESTATE
    assert L.vg_step_explicit(h, 10, bound * 1.01, 0, None, _lib.VG_FORCE, None) == _lib.VG_ESTATE
    assert L.vg_step_explicit(h, -1, bound, 0, None, 0, None) == _lib.VG_EINVAL
    assert L.vg_step_explicit(h, 10, 0.0, 0, None, 0, None) == _lib.VG_EINVAL
    assert L.vg_step_explicit(h, 10, bound * 0.5, 1, None, 0, None) == _lib.VG_EINVAL  # log without buffer
    L.vg_destroy(h)


def test_subcycled_step_validation():
    """Unequal steps: arguments checked, the diffusion step held to the
    stability bound before any device work; Algorithm 2 is a parameter."""
    from paper_2406_04177_amd.inputs import ModelParams, explicit_dt
    from paper_2406_04177_amd.sim import to_vg_params
    L = _lib.load()
    rc, h, _ = make_handle()
    p = ModelParams(sequential=True)
    assert L.vg_set_params(h, ctypes.byref(to_vg_params(p))) == 0
    vp = to_vg_params(p)
    vp.sequential = 2
    assert L.vg_set_params(h, ctypes.byref(vp)) == _lib.VG_EINVAL
    bound = explicit_dt(p, factor=1.0)
    assert L.vg_step_subcycled(None, 1, 1.0, bound, 0, None) == _lib.VG_EINVAL
    assert L.vg_step_subcycled(h, -1, 1.0, bound, 0, None) == _lib.VG_EINVAL
    assert L.vg_step_subcycled(h, 1, 0.0, bound, 0, None) == _lib.VG_EINVAL
    assert L.vg_step_subcycled(h, 1, 1.0, float("inf"), 0, None) == _lib.VG_EINVAL
    assert L.vg_step_subcycled(h, 1, 1.0, bound, 4, None) == _lib.VG_EINVAL          # unknown flag
    # the transformation step may be anything; the diffusion step is bounded
    assert L.vg_step_subcycled(h, 1, 50 * bound, bound * 1.01, 0, None) == _lib.VG_EUNSTABLE
    assert L.vg_step_subcycled(h, 1, 50 * bound, bound * 0.99, 0, None) == _lib.VG_ESTATE
    assert L.vg_step_subcycled(h, 1, 50 * bound, bound * 1.01, _lib.VG_FORCE, None) == _lib.VG_ESTATE
    L.vg_destroy(h)


def test_calls_out_of_sequence():
    L = _lib.load()
    rc, h, _ = make_handle(features=0)
    out = np.zeros(6)
    assert L.vg_mass_totals(h, out.ctypes.data, None) == _lib.VG_ESTATE
    assert L.vg_solve_implicit_step(h, 1.0, 1e-10, 10, None, None, None) == _lib.VG_ESTATE
    assert L.vg_record(h, 1, 1.0, None, None) == _lib.VG_ESTATE
    assert L.vg_step_record(h, 1, 1.0, None, None, 0, None) == _lib.VG_ESTATE
    assert L.vg_step_record(None, 1, 1.0, None, None, 0, None) == _lib.VG_EINVAL
    assert L.vg_precondition(h, 1.0, None, None, None) == _lib.VG_ESTATE
    ws = ctypes.c_size_t(0)
    assert L.vg_workspace_bytes(h, ctypes.byref(ws)) == 0 and ws.value > 0
    assert L.vg_init_state(h, 0x1000, 0x1000, 0x1000, 0, None) == _lib.VG_EINVAL   # workspace too small
    L.vg_destroy(h)


def test_workspace_grows_with_features():
    L = _lib.load()
    sizes = []
    for feat in (0, 1, 2, 3):
        rc, h, _ = make_handle(n=100000, features=feat)
        ws = ctypes.c_size_t(0)
        L.vg_workspace_bytes(h, ctypes.byref(ws))
        sizes.append(ws.value)
        L.vg_destroy(h)
    assert sizes[0] < sizes[1] < sizes[3] and sizes[0] < sizes[2] < sizes[3]
    assert sizes[1] >= 7 * 8 * 100000          # seven FP64 CG vectors


def test_workspace_counts_geometry_words_of_the_rank_index():
    """With a rank index the workspace holds a 4-byte geometry word per voxel
    (regression: it was laid out but not counted)."""
    L = _lib.load()
    n = 1 << 20
    sizes = []
    for with_rank in (False, True):
        seg = np.array([0, n], np.int64)
        desc = _lib.VgDesc()
        desc.n, desc.nseg, desc.precision = n, 1, _lib.VG_F32
        desc.seg_off = seg.ctypes.data
        desc.nbr_d = 0x1000
        desc.features = 0
        if with_rank:
            desc.rank_d, desc.vox_d = 0x2000, 0x3000    # never dereferenced here
            desc.nx = desc.ny = desc.nz = 128
        h = ctypes.c_void_p()
        assert L.vg_create(ctypes.byref(desc), ctypes.byref(h)) == 0
        ws = ctypes.c_size_t(0)
        assert L.vg_workspace_bytes(h, ctypes.byref(ws)) == 0
        sizes.append(ws.value)
        L.vg_destroy(h)
    assert sizes[1] - sizes[0] >= 4 * n


def test_range_sums_validation():
    L = _lib.load()
    assert L.vg_range_sums(None, 0, 10, None, 0, None, None) == 0            # nothing to do
    assert L.vg_range_sums(None, 0, -1, None, 0, None, None) == _lib.VG_EINVAL
    assert L.vg_range_sums(None, 7, 10, None, 0, None, None) == _lib.VG_EINVAL  # precision
    assert L.vg_range_sums(None, 0, 10, None, 3, None, None) == _lib.VG_EINVAL  # null pointers


def test_pngm_entry_points_validate_before_device_work():
    import ctypes
    L = _lib.load()
    E = _lib.VG_EINVAL
    assert L.vg_brick_stats(None, None, 10, 8, 8, 8, 4, None, None, None) == E
    assert L.vg_brick_stats(None, None, 0, 8, 8, 0, 4, None, None, None) == E
    assert L.vg_pngm_loss_grad(None, None, 1, 1, None, None, None, None, 1.0, 1, None, None, None, None) == E
    assert L.vg_pngm_step(None, None, -1, None, None, None, None, 1.0, None) == E
    assert L.vg_pngm_step(None, None, 0, None, None, None, None, 1.0, None) == 0
    assert L.vg_sign_update(None, None, 0, -0.1, None, None, None, None) == E
    it, rel = ctypes.c_int(-1), ctypes.c_double(-1.0)
    ok = dict(iters_out=ctypes.byref(it), relres_out=ctypes.byref(rel))

    def implicit(q, m, out, c, rtol, max_iter, work, iters_out=ok["iters_out"], relres_out=ok["relres_out"]):
        one = 0x1000                      # never dereferenced: every call below is rejected or has q = 0
        return L.vg_pngm_implicit_step(m, out, q, one, one, one, one, c, rtol, max_iter, work, iters_out,
                                       relres_out, None)
    assert implicit(0, None, None, 1.0, 1e-10, 10, None) == 0 and it.value == 0 and rel.value == 0.0
    assert implicit(4, 0x2000, 0x2000, 1.0, 1e-10, 10, 0x9000) == E             # out aliases m
    assert implicit(4, 0x2000, 0x9008, 1.0, 1e-10, 10, 0x9000) == E             # out inside the work area
    assert implicit(4, 0x2000, 0x3000, 1.0, 0.0, 10, 0x9000) == E               # rtol
    assert implicit(4, 0x2000, 0x3000, 1.0, 1e-10, 0, 0x9000) == E              # max_iter
    assert implicit(4, 0x2000, 0x3000, -1.0, 1e-10, 10, 0x9000) == E            # c < 0
    assert implicit(4, 0x2000, 0x3000, 1.0, 1e-10, 10, None) == E               # no work area
    assert implicit(4, 0x2000, 0x3000, 1.0, 1e-10, 10, 0x9000, iters_out=None) == E


def test_band_feature_workspace():
    """VG_FEAT_BAND is accepted (unknown bits are not) and, for a single raster
    volume with a rank index and no periodic axis, adds the row index
    ((nz * ny + 1) int32) and a second set of the five fields to the
    workspace; brick order, periodic axes or no rank index add nothing."""
    L = _lib.load()
    rc, h, _ = make_handle(features=_lib.VG_FEAT_BAND)
    assert rc == 0
    L.vg_destroy(h)
    rc, h, _ = make_handle(features=16)
    assert rc == _lib.VG_EINVAL
    n = 1 << 20

    def ws(features, rank=True, brick=0, periodic=0):
        seg = np.array([0, n], np.int64)
        desc = _lib.VgDesc()
        desc.n, desc.nseg, desc.precision = n, 1, _lib.VG_F32
        desc.seg_off = seg.ctypes.data
        desc.nbr_d = 0x1000
        desc.features = features
        if rank:
            desc.rank_d, desc.vox_d = 0x2000, 0x3000    # never dereferenced here
            desc.nx = desc.ny = desc.nz = 128
            desc.brick, desc.periodic = brick, periodic
        h = ctypes.c_void_p()
        assert L.vg_create(ctypes.byref(desc), ctypes.byref(h)) == 0
        out = ctypes.c_size_t(0)
        assert L.vg_workspace_bytes(h, ctypes.byref(out)) == 0
        L.vg_destroy(h)
        return out.value
    base = ws(0)
    assert ws(_lib.VG_FEAT_BAND) - base >= 5 * 4 * n + 4 * (128 * 128 + 1)
    assert ws(_lib.VG_FEAT_BAND, brick=8) == ws(0, brick=8)
    assert ws(_lib.VG_FEAT_BAND, periodic=1) == ws(0, periodic=1)
    assert ws(_lib.VG_FEAT_BAND, rank=False) == ws(0, rank=False)


def test_batches_with_empty_volumes_every_precision():
    """Descriptors of batches whose volumes are empty, smaller than a tile or
    span several tiles, for every precision and feature set: the piece tables
    and workspace layout are built on the host (exercised under the
    sanitizers too); compensated fields add 12 B per voxel of compensation
    words (2 B per pool, 2 B for the diffusing pool's ping-pong) and refuse
    the adjoint."""
    L = _lib.load()
    layouts = ([0, 0, 300, 300, 1000, 70000], [0, 1], [0, 256, 512, 768], [0, 0, 0, 5, 5, 100001])
    for offs in layouts:
        seg = np.array(offs, np.int64)
        sizes = {}
        for prec in (_lib.VG_F32, _lib.VG_F64, _lib.VG_F32C):
            for feat in (0, _lib.VG_FEAT_CG, _lib.VG_FEAT_ADJ, _lib.VG_FEAT_CG | _lib.VG_FEAT_ADJ):
                for mob in (0, 1):
                    desc = _lib.VgDesc()
                    desc.n, desc.nseg, desc.precision = int(seg[-1]), len(seg) - 1, prec
                    desc.seg_off = seg.ctypes.data
                    desc.nbr_d = 0x1000
                    desc.mobile_all, desc.features = mob, feat
                    h = ctypes.c_void_p()
                    rc = L.vg_create(ctypes.byref(desc), ctypes.byref(h))
                    if prec == _lib.VG_F32C and feat & _lib.VG_FEAT_ADJ:
                        assert rc == _lib.VG_EINVAL and not h.value
                        continue
                    assert rc == 0, (offs, prec, feat, L.vg_last_error())
                    ws = ctypes.c_size_t(0)
                    assert L.vg_workspace_bytes(h, ctypes.byref(ws)) == 0
                    sizes[(prec, feat, mob)] = ws.value
                    for k in (2, 5):       # rank index and band kernel need what this handle lacks
                        assert L.vg_set_kernel(h, k) == _lib.VG_EINVAL
                    x = np.zeros(5)
                    assert L.vg_load_state(h, x.ctypes.data, _lib.VG_F64, None) == _lib.VG_ESTATE
                    assert L.vg_store_state(h, x.ctypes.data, _lib.VG_F64, None) == _lib.VG_ESTATE
                    L.vg_destroy(h)
        n = int(seg[-1])
        for feat in (0, _lib.VG_FEAT_CG):
            for mob in (0, 1):
                extra = sizes[(_lib.VG_F32C, feat, mob)] - sizes[(_lib.VG_F32, feat, mob)]
                assert 2 * (5 + (5 if mob else 1)) * n <= extra <= 2 * (5 + (5 if mob else 1)) * n + 512, (offs, extra)


def test_pngm_noalloc_validates_before_device_work():
    L = _lib.load()
    it, rel = ctypes.c_int(0), ctypes.c_double(0.0)
    p = 0x1000
    q = _lib.VG_PNGM_NOALLOC_MAX_Q + 1
    assert L.vg_pngm_implicit_step_noalloc(p, p + 8, q, p, p, p, p, 1.0, 1e-12, 10, ctypes.byref(it),
                                           ctypes.byref(rel), None) == _lib.VG_EINVAL
    for bad in ((p, p, 10, 1.0, 1e-12, 10), (p, p + 8, 10, -1.0, 1e-12, 10), (p, p + 8, 10, 1.0, 0.0, 10),
                (p, p + 8, 10, 1.0, 1e-12, 0), (0, p + 8, 10, 1.0, 1e-12, 10)):
        m, o, qq, c, rtol, mi = bad
        assert L.vg_pngm_implicit_step_noalloc(m, o, qq, p, p, p, p, c, rtol, mi, ctypes.byref(it),
                                               ctypes.byref(rel), None) == _lib.VG_EINVAL


def test_pngm_partition_sizes_and_validation():
    L = _lib.load()
    wb, mp, me = ctypes.c_size_t(0), ctypes.c_int64(0), ctypes.c_int64(0)
    # 36 x 40 x 44 (nz, ny, nx) in bricks of 8: 6 x 5 x 5 bricks, 2 (5*5*5 + 6*4*5 + 6*5*4) directed pairs
    assert L.vg_pngm_partition_bytes(44, 40, 36, 8, ctypes.byref(wb), ctypes.byref(mp), ctypes.byref(me)) == 0
    assert mp.value == 150 and me.value == 730 and wb.value >= 150 * (12 + 32 + 4)
    assert L.vg_pngm_partition_bytes(44, 40, 36, 0, ctypes.byref(wb), ctypes.byref(mp), ctypes.byref(me)) == _lib.VG_EINVAL
    assert L.vg_pngm_partition_bytes(1, 1, 1, 4, ctypes.byref(wb), ctypes.byref(mp), ctypes.byref(me)) == 0
    assert mp.value == 1 and me.value == 0
    q, e = ctypes.c_int64(0), ctypes.c_int64(0)
    p = 0x1000
    args = [p, p, 10, 44, 40, 36, 8, p, 10, p, p, p, p, p, p, p, ctypes.byref(q), ctypes.byref(e), None]
    assert L.vg_pngm_partition(*args) == _lib.VG_EINVAL            # workspace too small
    args[8] = 1 << 20
    for k in (0, 9, 13):
        bad = list(args)
        bad[k] = None
        assert L.vg_pngm_partition(*bad) == _lib.VG_EINVAL


def test_multigrid_feature_validation_and_workspace():
    """VG_FEAT_MG needs VG_FEAT_CG and a single volume with a rank index and
    no periodic axis; it reserves the hierarchy at its bound (level l + 1:
    min(cells of level l, cells of the half-resolution grid), about 92 B per
    cell plus the grid's rank index), a parent index and an FP64 scratch
    entry per voxel.  The
    preconditioner choice and the level query validate on the host."""
    L = _lib.load()
    n = 1 << 18
    CG, MG = _lib.VG_FEAT_CG, _lib.VG_FEAT_MG

    def create(features, rank=True, periodic=0, side=64):
        seg = np.array([0, n], np.int64)
        desc = _lib.VgDesc()
        desc.n, desc.nseg, desc.precision = n, 1, _lib.VG_F64
        desc.seg_off = seg.ctypes.data
        desc.nbr_d = 0x1000
        desc.features = features
        if rank:
            desc.rank_d, desc.vox_d = 0x2000, 0x3000    # never dereferenced here
            desc.nx = desc.ny = desc.nz = side
            desc.periodic = periodic
        h = ctypes.c_void_p()
        return L.vg_create(ctypes.byref(desc), ctypes.byref(h)), h

    for bad in (dict(features=MG), dict(features=CG | MG, rank=False), dict(features=CG | MG, periodic=1)):
        rc, _ = create(**bad)
        assert rc == _lib.VG_EINVAL, bad
        assert b"VG_FEAT_MG" in L.vg_last_error()
    rc, h0 = create(CG)
    rc1, h1 = create(CG | MG)
    assert rc == 0 and rc1 == 0
    w0, w1 = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert L.vg_workspace_bytes(h0, ctypes.byref(w0)) == 0 and L.vg_workspace_bytes(h1, ctypes.byref(w1)) == 0
    caps = [32 ** 3, 16 ** 3, 8 ** 3, 4 ** 3, 2 ** 3, 1]    # levels 1.. of a 64^3 grid (n > 32^3)
    assert w1.value - w0.value >= 12 * n + 92 * sum(caps)
    assert w1.value - w0.value <= 12 * n + 92 * sum(caps) + 64 * 1024 + 32 ** 3 + 256 * 40
    # preconditioner choice
    assert L.vg_set_preconditioner(h0, _lib.VG_PRECOND_MG) == _lib.VG_EINVAL
    assert b"VG_FEAT_MG" in L.vg_last_error()
    assert L.vg_set_preconditioner(h1, 7) == _lib.VG_EINVAL
    assert L.vg_set_preconditioner(h1, _lib.VG_PRECOND_MG) == 0
    assert L.vg_set_preconditioner(h0, _lib.VG_PRECOND_JACOBI) == 0
    lv = ctypes.c_int(-1)
    cells = (ctypes.c_int64 * _lib.VG_MG_MAX_LEVELS)()
    assert L.vg_mg_levels(h1, ctypes.byref(lv), cells) == 0 and lv.value == 0    # built by vg_init_state
    assert L.vg_mg_levels(h1, None, None) == _lib.VG_EINVAL
    assert L.vg_precondition(h1, 1.0, 0x1000, 0x2000, None) == _lib.VG_ESTATE   # nothing bound yet
    for h in (h0, h1):
        L.vg_destroy(h)


def test_adjoint_options_and_tape_rows():
    """Adjoint options: the two flags and their combination accepted, any
    other bit refused; a kept-DOM recording has four rows per state, five
    otherwise and whenever every pool diffuses (host side only)."""
    L = _lib.load()
    assert L.vg_tape_rows(None) == _lib.VG_EINVAL
    assert L.vg_set_adjoint_options(None, 0) == _lib.VG_EINVAL
    rc, h, _ = make_handle()
    rc2, h2, _ = make_handle(mobile_all=1)
    for flags in range(4):
        assert L.vg_set_adjoint_options(h, flags) == 0
        assert L.vg_tape_rows(h) == (4 if flags & _lib.VG_ADJ_TAPE_DOM else 5)
        assert L.vg_set_adjoint_options(h2, flags) == 0
        assert L.vg_tape_rows(h2) == 5
    assert L.vg_set_adjoint_options(h, 4) == _lib.VG_EINVAL
    assert L.vg_set_adjoint_options(h, 0x80000000) == _lib.VG_EINVAL
    L.vg_destroy(h)
    L.vg_destroy(h2)
