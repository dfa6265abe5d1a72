"""The no-allocation variant of the implicit pore-network step
(vg_pngm_implicit_step_noalloc, scratch in a static device array) against the
entry point with a caller-owned scratch buffer (vg_pngm_implicit_step), both
called through the C ABI: bit-identical masses, sweep counts and residuals,
on two calls in a row, the second with fewer primitives (the static array
still holds the first call's values), and refusal of sizes beyond it."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _network(q, seed):
    """A connected random network of q primitives: a chain plus random chords,
    every edge in both directions (CSR by row), v_i > 0 pore-voxel counts,
    theta > 0 per directed edge, masses m = v * U(0, 1)."""
    rng = np.random.default_rng(seed)
    pairs = {(i, i + 1) for i in range(q - 1)}
    for a, b in rng.integers(0, q, size=(2 * q, 2)):
        if a != b:
            pairs.add((min(a, b), max(a, b)))
    rows = [[] for _ in range(q)]
    for a, b in sorted(pairs):
        rows[a].append(b)
        rows[b].append(a)
    row = np.zeros(q + 1, np.int64)
    row[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([j for r in rows for j in sorted(r)], np.int32)
    v = rng.integers(1, 60, size=q).astype(np.float64)
    theta = rng.uniform(0.2, 3.0, size=col.size)
    m = v * rng.random(q)
    dev = "cuda"
    t = lambda a: torch.as_tensor(a, device=dev)
    return t(m), t(v), t(row), t(col), t(theta)


def _call_both(L, q, seed, c=2.5, rtol=1e-12, max_iter=20000):
    m, v, row, col, theta = _network(q, seed)
    s = torch.cuda.current_stream().cuda_stream
    out_w = torch.full((q,), np.nan, dtype=torch.float64, device="cuda")
    out_s = torch.full((q,), np.nan, dtype=torch.float64, device="cuda")
    work = torch.empty(3 * q + 2, dtype=torch.float64, device="cuda")
    it_w, rel_w = ctypes.c_int(-1), ctypes.c_double(-1.0)
    it_s, rel_s = ctypes.c_int(-1), ctypes.c_double(-1.0)
    rc_w = L.vg_pngm_implicit_step(m.data_ptr(), out_w.data_ptr(), q, v.data_ptr(), row.data_ptr(),
                                   col.data_ptr(), theta.data_ptr(), c, rtol, max_iter, work.data_ptr(),
                                   ctypes.byref(it_w), ctypes.byref(rel_w), s)
    rc_s = L.vg_pngm_implicit_step_noalloc(m.data_ptr(), out_s.data_ptr(), q, v.data_ptr(), row.data_ptr(),
                                           col.data_ptr(), theta.data_ptr(), c, rtol, max_iter,
                                           ctypes.byref(it_s), ctypes.byref(rel_s), s)
    torch.cuda.synchronize()
    assert rc_w == 0 and rc_s == 0, (rc_w, rc_s, L.vg_last_error())
    return (out_w.cpu().numpy(), it_w.value, rel_w.value), (out_s.cpu().numpy(), it_s.value, rel_s.value), \
        (m.cpu().numpy(), v.cpu().numpy(), row.cpu().numpy(), col.cpu().numpy(), theta.cpu().numpy())


def test_noalloc_equals_workspace_entry_point_twice():
    from paper_2406_04177_amd import _lib
    L = _lib.load()
    for q, seed in ((40_000, 1), (3_001, 2)):          # the second call is smaller
        print("no-alloc PNGM implicit step: q =", q, flush=True)
        (yw, iw, rw), (ys, is_, rs), (m, v, row, col, theta) = _call_both(L, q, seed)
        np.testing.assert_array_equal(ys, yw)
        assert is_ == iw and rs == rw, (is_, iw, rs, rw)
        assert rw <= 1e-12 and iw > 0
        # the result solves y_i + c sum_j theta_ij (y_i/v_i - y_j/v_j) = m_i
        y = ys
        r = y.copy()
        for i in range(q):
            js = col[row[i]:row[i + 1]]
            r[i] += 2.5 * np.sum(theta[row[i]:row[i + 1]] * (y[i] / v[i] - y[js] / v[js]))
        assert np.linalg.norm(r - m) <= 1e-11 * np.linalg.norm(m)


def test_noalloc_refuses_sizes_beyond_the_static_array():
    from paper_2406_04177_amd import _lib
    L = _lib.load()
    q = _lib.VG_PNGM_NOALLOC_MAX_Q + 1
    dummy = torch.zeros(8, dtype=torch.float64, device="cuda")
    it, rel = ctypes.c_int(0), ctypes.c_double(0.0)
    p = dummy.data_ptr()
    rc = L.vg_pngm_implicit_step_noalloc(p, p + 8, q, p, p, p, p, 1.0, 1e-12, 10, ctypes.byref(it),
                                         ctypes.byref(rel), None)
    assert rc == _lib.VG_EINVAL
    assert b"static scratch" in L.vg_last_error()
    rc = L.vg_pngm_implicit_step_noalloc(None, p, 10, p, p, p, p, 1.0, 1e-12, 10, ctypes.byref(it),
                                         ctypes.byref(rel), None)
    assert rc == _lib.VG_EINVAL
