"""Benchmark: explicit diffusion-transformation steps on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]

Workload: a 512^3 synthetic volume at 17 % porosity (largest 6-connected pore
component of Gaussian-smoothed seeded noise, the stand-in for the paper's
512^3 sandy-loam CT image), five pools with DOM the only diffusing one, FP32
fields, explicit dt = 0.9 h^2 / (6 D), FP64 totals every 100 steps.  One
"step" is one time step of the method (transformation + Scheme 1 diffusion +
totals when logged) over every pore voxel.  Inputs are resident in HBM before
the timed region; K steps are timed with HIP events on the stream the kernels
run on, bracketed by device synchronisation.

Prints one JSON line.  Besides the headline it reports the fused step's
roofline (algorithmic bytes per launch / average launch time against 8 TB/s),
the oracle's CPU rate on a bounded sample of the same workload, and timings of
the other parts of the path: graph build, the plain FP64 step, the implicit
step (PCG at 20x the explicit bound) and the adjoint / forward time ratio.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "pore-voxel species updates/s + HBM GB/s (% peak); adjoint/forward time ratio"
# algorithmic bytes per pore voxel and launch (read 5 pools, write 5 pools,
# read the 6-slot int32 neighbour table)
BYTES_FUSED_F32 = 5 * 4 + 5 * 4 + 6 * 4
BYTES_FUSED_F64 = 5 * 8 + 5 * 8 + 6 * 4
# rank-index kernel: the pools, a 4-byte geometry word per voxel and the
# pore-bitmap words (8 B per 32 positions, 8 / (32 * 0.17) ~ 1.5 B per pore voxel)
BYTES_RANK_F32 = 5 * 4 + 5 * 4 + 4 + 8.0 / (32 * 0.17)
# packed-offset kernel: the pools and two 4-byte offset words per voxel
BYTES_OFFSET_F32 = 5 * 4 + 5 * 4 + 8
# relative-code kernel: the pools, one 4-byte code word per voxel and 32 B of
# base distances per 64 voxels
BYTES_RELATIVE_F32 = 5 * 4 + 5 * 4 + 4 + 32.0 / 64
# band kernel (two fused passes per launch): per voxel and pass pair the
# first pass reads four pools and the code word of the band and its two
# neighbour rows (band of 8 rows: 10/8 of the voxels), the second pass reads
# four pools and the code word again and writes the five pools; per step half
BYTES_BAND_F32 = (10.0 / 8 * (4 * 4 + 4 + 32.0 / 64) + (4 * 4 + 4 + 32.0 / 64) + 5 * 4) / 2
# compensated FP32 fields: the method's algorithmic count with 6-byte values
BYTES_FUSED_F32C = 5 * 6 + 5 * 6 + 6 * 4
# compensated FP32 fields (float + 16-bit word per value), relative codes:
# six bytes per pool read and written, the code word and the group bases
BYTES_COMP_RELATIVE = 5 * 6 + 5 * 6 + 4 + 32.0 / 64
BYTES_F64_RELATIVE = 5 * 8 + 5 * 8 + 4 + 32.0 / 64
KERNEL_NAMES = {1: "table", 2: "rank", 3: "offset", 4: "relative", 5: "band"}
KERNEL_FUNCS = {1: "k_step (6-slot table)", 2: "k_step_geo (rank index)", 3: "k_step_off (packed offsets)",
                4: "k_step_off (relative codes)",
                5: "k_band2 (relative codes, two fused passes per launch, rows of a band marching along z)"}
OWN_BYTES = {1: BYTES_FUSED_F32, 2: BYTES_RANK_F32, 3: BYTES_OFFSET_F32, 4: BYTES_RELATIVE_F32, 5: BYTES_BAND_F32}
PASSES_PER_LAUNCH = {1: 1, 2: 1, 3: 1, 4: 1, 5: 2}

# HBM bytes per launch of the headline kernel read from hardware counters
# (FETCH_SIZE x 2 + WRITE_SIZE, the factors of a plain 1 GiB device copy on the
# same GPU), valid only for the kernel sources they were taken on: the sha256
# of KERNEL_SOURCES must match, else the roofline reports traffic = null.
KERNEL_SOURCES = ("paper_2406_04177_amd/csrc/vg_step.hip", "paper_2406_04177_amd/csrc/vg_internal.h",
                  "paper_2406_04177_amd/build.py")
MEASURED_TRAFFIC = {
    # (kernel, size): (bytes per launch, sha256 of KERNEL_SOURCES); from
    # profiles/k_band2_f32_512cube.md: FETCH_SIZE 593521.3 KiB x 2 +
    # WRITE_SIZE 412398.7 KiB x 1 per launch (two fused passes), and
    # profiles/k_step_c_f32c_512cube.md: FETCH_SIZE 479815.7 KiB x 2 +
    # WRITE_SIZE 614750.5 KiB per launch (one pass, compensated FP32)
    ("band", 512): (593521.3 * 1024 * 2 + 412398.7 * 1024, "69b7e38df9ad0daa574489029c012a67ae0251ed2b47373b68c9c967b88515e5"),
    ("relative_f32c", 512): (479815.7 * 1024 * 2 + 614750.5 * 1024, "69b7e38df9ad0daa574489029c012a67ae0251ed2b47373b68c9c967b88515e5"),
}


def sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def timed(fn, stream=None):
    import torch
    s = stream or torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    out = fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_threads(k=None):
    """OpenMP threads of this process's runtime (the oracle's): read, or set
    to k (the oracle is built with -fopenmp and runs its loops on the calling
    thread's team)."""
    import ctypes
    gomp = ctypes.CDLL("libgomp.so.1")
    if k is not None:
        gomp.omp_set_num_threads(int(k))
    return int(gomp.omp_get_max_threads())


def oracle_gradient_seconds(steps=200, K=20):
    """The oracle's FP64 discrete-adjoint gradient of a CO2-curve loss on the
    16 x 128^3 gradient workload (region factors, seeds on every step's CO2
    totals), checkpointed every K steps: forward to every checkpoint, then per
    segment (last first) its states and the reverse sweep."""
    import numpy as np
    from oracle import oracle as orc
    from paper_2406_04177_amd import inputs
    masks, specs = inputs.workload_inputs("b16x128")
    params = inputs.ModelParams()
    dt = inputs.explicit_dt(params, 0.8)
    og = orc.build_batch(masks)
    reg = orc.octant_regions(og)
    w = orc.edge_weights(og, reg, [1.0] * 8)
    x0 = orc.fields_from_spec(og, specs)
    seeds = np.zeros((steps + 1, og.nseg, 5))
    seeds[:, :, 4] = 1.0 / ((steps + 1) * og.nseg)       # d(mean CO2 total) / d(CO2 total)
    t0 = time.perf_counter()
    ckpts, x = [], x0
    for k0 in range(0, steps, K):
        k = min(K, steps - k0)
        ckpts.append((k0, k, x))
        x, _ = orc.run(params, dt, og, x, k, w=w, with_totals=False)
    lam, grad = None, np.zeros(20)
    for k0, k, xc in reversed(ckpts):
        st = orc.run_states(params, dt, og, xc, k, w=w)
        sd = seeds[k0:k0 + k + 1].copy()
        if k0 + k != steps:
            sd[-1] = 0.0
        lam, gr = orc.adjoint(params, dt, og, st, sd, w=w, region=reg, nreg=8, lam_final=lam)
        grad += gr
        del st
    return time.perf_counter() - t0, og.n


def cpu_baseline(mask, spec, params, dt, steps, steps_1t, grad_steps):
    """The FP64 oracle on the host cores: the first `steps` steps of the
    workload on all threads and `steps_1t` on one, and its checkpointed
    discrete-adjoint gradient of the gradient workload over `grad_steps`
    steps (checkpoints every 20; its reverse sweep is a plain serial loop:
    200 steps take about two minutes, so the default sample is 40)."""
    from oracle import oracle as orc
    og = orc.build_graph(mask)
    n = og.n
    x0 = orc.fields_from_spec(og, spec)
    threads = _omp_threads()
    t0 = time.perf_counter()
    orc.run(params, dt, og, x0, steps, with_totals=False)
    sec = time.perf_counter() - t0
    _omp_threads(1)
    t0 = time.perf_counter()
    orc.run(params, dt, og, x0, steps_1t, with_totals=False)
    sec1 = time.perf_counter() - t0
    _omp_threads(threads)
    del x0, og
    gsec, gn = oracle_gradient_seconds(grad_steps)
    return {"value": 5.0 * n * steps / sec,
            "unit": "pore-voxel species updates/s", "cores": threads, "kind": "oracle",
            "sample": "%d explicit steps of the same 512^3 workload, FP64, %.1f s on %d threads"
                      % (steps, sec, threads),
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "one_thread": {"value": 5.0 * n * steps_1t / sec1, "unit": "pore-voxel species updates/s",
                           "sample": "%d explicit steps, FP64, %.1f s on 1 thread" % (steps_1t, sec1)},
            "gradient_16x128": {"seconds": gsec, "steps": grad_steps, "checkpoint_every": 20, "n_pore_voxels": gn,
                                "seconds_per_step": gsec / grad_steps,
                                "threads": threads,
                                "what": "FP64 discrete-adjoint gradient of a CO2-curve loss (20 parameters), "
                                        "checkpointed forward + reverse sweep"}}


def step_1024(steps=101):
    """The 1024^3 volume at 17 % porosity (about 1.7e8 pore voxels): FP32 step
    time with the relative-code single passes and with the band kernel
    (totals every 100 steps), and the kernel AUTO takes; the same for one
    z-slab of eight (1024 x 1024 x 128)."""
    import numpy as np
    import torch
    from paper_2406_04177_amd import inputs
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    t0 = time.perf_counter()
    mask = inputs.synthetic_volume((1024, 1024, 1024), porosity=0.17, seed=0)
    spec = inputs.init_uniform(mask, seed=0)
    g = Graph.from_masks(mask)
    slab = np.ascontiguousarray(mask[:128])
    mask_full, spec_full = mask, spec
    log("1024^3 volume and graph in %.1f s (n = %d)" % (time.perf_counter() - t0, g.n))
    p = inputs.ModelParams()
    dt = inputs.explicit_dt(p, 0.9)
    x0 = g.fields_from_specs(spec, torch.float32)
    sim = Simulation(g, p, precision="f32", implicit=False)
    res = {"workload": "1024^3 17% porosity explicit step, FP32 fields, FP64 totals every 100 steps",
           "n_pore_voxels": g.n}
    for kern, name in ((4, "relative"), (5, "band")):
        sim.set_kernel(kern)
        sim.set_fields(x0)
        sim.step(9, dt)
        sim.set_fields(x0)
        ms, _ = timed(lambda: sim.step(steps, dt, log_every=100))
        res["ms_per_step_" + name] = ms / steps
        res["achieved_GBs_64B_" + name] = BYTES_FUSED_F32 * g.n / (ms / steps / 1e3) / 1e9
    sim.set_kernel(0)
    res["auto_kernel"] = KERNEL_NAMES[sim.kernel_in_use()]
    log("1024^3: %.3f ms/step single passes, %.3f ms/step band kernel"
        % (res["ms_per_step_relative"], res["ms_per_step_band"]))
    del sim, x0, g
    torch.cuda.empty_cache()
    # the brick-ordered compacted list (8^3 bricks): no packed source fits its
    # cross-brick distances, so AUTO takes the rank index (a neighbour's
    # compact index from the pore bitmap); the table kernel for comparison
    gb = Graph.from_masks(mask_full, brick=8)
    x0 = gb.fields_from_specs(spec_full, torch.float32)
    sim = Simulation(gb, p, precision="f32", implicit=False)
    br = {"workload": "1024^3 17% porosity, brick-ordered compacted list (8^3 bricks), FP32 fields, "
                      "FP64 totals every 100 steps", "auto_kernel": KERNEL_NAMES[sim.kernel_in_use()]}
    for kern, name in ((2, "rank"), (1, "table")):
        sim.set_kernel(kern)
        sim.set_fields(x0)
        sim.step(9, dt)
        sim.set_fields(x0)
        ms, _ = timed(lambda: sim.step(steps, dt, log_every=100))
        br["ms_per_step_" + name] = ms / steps
        br["achieved_GBs_64B_" + name] = BYTES_FUSED_F32 * gb.n / (ms / steps / 1e3) / 1e9
    br["achieved_GBs_own_rank"] = BYTES_RANK_F32 * gb.n / (br["ms_per_step_rank"] / 1e3) / 1e9
    res["brick_order"] = br
    log("1024^3 brick order: %.3f ms/step rank index, %.3f ms/step table (AUTO %s)"
        % (br["ms_per_step_rank"], br["ms_per_step_table"], br["auto_kernel"]))
    del sim, x0
    torch.cuda.empty_cache()
    # the gradient at this size: the first 200 steps, checkpoints every 20,
    # region weights, CO2 totals every step, static pools' D gradients skipped
    from paper_2406_04177_amd.autograd import co2_mse, simulate_totals, theta_of
    gb.make_region_codes()
    sima = Simulation(gb, p, precision="f32", implicit=False, adjoint=True, regions=[1.0] * 8)
    sima.set_adjoint_options(skip_static_d=True)
    dta = inputs.explicit_dt(p, 0.8)
    xa = gb.fields_from_specs(spec_full, torch.float32)
    theta = theta_of(p, [1.0] * 8)
    gsteps, gk = 200, 20
    target = torch.zeros((gsteps + 1, gb.nseg), dtype=torch.float64, device="cuda")
    with torch.no_grad():
        simulate_totals(sima, theta, xa, gsteps, dta, gk)
    ms_f, _ = timed(lambda: simulate_totals(sima, theta, xa, gsteps, dta, gk))

    def grad1024():
        th = theta.clone().requires_grad_(True)
        co2_mse(simulate_totals(sima, th, xa, gsteps, dta, gk), target).backward()
    grad1024()
    ms_g, _ = timed(grad1024)
    br["gradient_200_steps"] = {
        "workload": "first 200 FP32 steps, checkpoints every 20, region weights, CO2 totals every step, "
                    "static pools' D gradients skipped (table neighbours: brick order)",
        "forward_ms": ms_f, "gradient_ms": ms_g, "gradient_forward_ratio": ms_g / ms_f,
        "taped_segments": "%d of %d" % (sima.last_taped_segments, gsteps // gk)}
    log("1024^3 brick order, gradient of 200 steps: forward %.0f ms, gradient %.0f ms (ratio %.2f, %s segments "
        "recorded in the forward)" % (ms_f, ms_g, ms_g / ms_f, br["gradient_200_steps"]["taped_segments"]))
    del sima, xa, gb
    torch.cuda.empty_cache()
    # one GPU's share of the 1024^3 volume split into 8 z-slabs: its first 128
    # planes as a volume of their own (closed faces: no halo exchange)
    spec = inputs.init_uniform(slab, seed=0)
    g = Graph.from_masks(slab)
    x0 = g.fields_from_specs(spec, torch.float32)
    sim = Simulation(g, p, precision="f32", implicit=False)
    sl = {"workload": "1024x1024x128 slab (first 128 planes of the 1024^3 volume), one of 8 z-slabs; no halo",
          "n_pore_voxels": g.n}
    for kern, name in ((4, "relative"), (5, "band")):
        sim.set_kernel(kern)
        sim.set_fields(x0)
        sim.step(9, dt)
        sim.set_fields(x0)
        ms, _ = timed(lambda: sim.step(steps, dt, log_every=100))
        sl["ms_per_step_" + name] = ms / steps
        sl["achieved_GBs_64B_" + name] = BYTES_FUSED_F32 * g.n / (ms / steps / 1e3) / 1e9
    sim.set_kernel(0)
    sl["auto_kernel"] = KERNEL_NAMES[sim.kernel_in_use()]
    res["slab_of_8"] = sl
    log("1024x1024x128 slab (n = %d): %.4f ms/step single passes, %.4f ms/step band kernel, AUTO %s"
        % (g.n, sl["ms_per_step_relative"], sl["ms_per_step_band"], sl["auto_kernel"]))
    del sim, x0, g
    torch.cuda.empty_cache()
    return res


def copy_1gib():
    """A plain 1 GiB device-to-device copy (the HIP runtime's copy kernel):
    bytes read + written per second, a reference for the attainable rate."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    ms, _ = timed(lambda: [b.copy_(a) for _ in range(10)])
    return {"bytes_per_copy": 2 * 4 * (1 << 28), "GBs": 2 * 4 * (1 << 28) * 10 / (ms / 1e3) / 1e9}


def _errors_vs(ref_x, ref_t, x, t):
    """Per-pool field errors (relative to each pool's max) and per-curve
    totals errors (relative per logged point) against a reference run."""
    import numpy as np
    names = ("MB", "DOM", "SOM", "P4", "CO2")
    fe = {names[s]: float(np.abs(x[s] - ref_x[s]).max() / max(np.abs(ref_x[s]).max(), 1e-300)) for s in range(5)}
    curves = names + ("total",)
    te = {curves[s]: float((np.abs(t[:, s] - ref_t[:, s]) / np.maximum(np.abs(ref_t[:, s]), 1e-300)).max())
          for s in range(6)}
    return fe, te


def precision_runs(N, steps, log_every=100, precs=("f32", "f32c", "f64")):
    """The same explicit run in each precision on the N^3 workload: time per
    step and the final state (FP64) with the totals log.  Each run is timed
    as one call of `steps` steps (totals every `log_every`)."""
    import torch
    from paper_2406_04177_amd import inputs
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    mask = inputs.synthetic_volume((N, N, N), porosity=0.17, seed=0)
    spec = inputs.init_uniform(mask, seed=0)
    params = inputs.ModelParams()
    dt = inputs.explicit_dt(params, 0.9)
    g = Graph.from_masks(mask)
    x0 = g.fields_from_specs(spec, torch.float64)
    out = {}
    for prec in precs:
        sim = Simulation(g, params, precision=prec, implicit=False)
        sim.set_fields(x0)
        sim.step(20, dt)
        sim.set_fields(x0)
        c0 = sim.totals()[0, 5]
        ms, logt = timed(lambda: sim.step(steps, dt, log_every=log_every))
        out[prec] = {"ms_per_step": ms / steps, "x": sim.state().cpu().numpy(), "log": logt[:, 0, :].cpu().numpy(),
                     "c0": c0, "kernel": KERNEL_NAMES[sim.kernel_in_use()]}
        log("%d^3 %s: %d steps in %.1f s (%.4f ms/step, %s kernel)" % (N, prec, steps, ms / 1e3, ms / steps,
                                                                     out[prec]["kernel"]))
        del sim
        torch.cuda.empty_cache()
    return g.n, out


def accuracy_runs(N, steps, label):
    """FP32 and compensated-FP32 fields against the FP64 step (itself
    bit-identical to the FP64 oracle) on the N^3 workload: error per species
    (fields) and per totals curve, carbon drift, time per step."""
    import numpy as np
    n, out = precision_runs(N, steps)
    ref = out["f64"]
    res = {"workload": "%d^3 17%% porosity, %d explicit steps, totals every 100 (%s)" % (N, steps, label),
           "n_pore_voxels": n, "reference": "the FP64 GPU step (bit-identical to the FP64 oracle)"}
    for prec in ("f32", "f32c", "f64"):
        r = out[prec]
        res["%s_ms_per_step" % prec] = r["ms_per_step"]
        res["%s_kernel" % prec] = r["kernel"]
        res["total_carbon_drift_%s" % prec] = float(np.abs(r["log"][:, 5] - r["c0"]).max() / r["c0"])
        if prec != "f64":
            fe, te = _errors_vs(ref["x"], ref["log"], r["x"], r["log"])
            res["%s_field_rel_err" % prec] = fe
            res["%s_totals_curve_rel_err" % prec] = te
            res["%s_max_err" % prec] = max(max(fe.values()), max(te.values()))
            res["%s_meets_1e-5" % prec] = res["%s_max_err" % prec] <= 1e-5
    res["f32c_own_bytes_per_voxel_step"] = BYTES_COMP_RELATIVE
    res["f32c_achieved_GBs_own"] = BYTES_COMP_RELATIVE * n / (res["f32c_ms_per_step"] / 1e3) / 1e9
    res["f64_achieved_GBs_own"] = BYTES_F64_RELATIVE * n / (res["f64_ms_per_step"] / 1e3) / 1e9
    res["fp32_speedup_over_fp64"] = res["f64_ms_per_step"] / res["f32_ms_per_step"]
    res["f32c_speedup_over_fp64"] = res["f64_ms_per_step"] / res["f32c_ms_per_step"]
    log("%d^3 x %d accuracy: FP32 %.4f ms/step max err %.1e, compensated %.4f ms/step max err %.1e, FP64 %.4f ms/step"
        % (N, steps, res["f32_ms_per_step"], res["f32_max_err"], res["f32c_ms_per_step"], res["f32c_max_err"],
           res["f64_ms_per_step"]))
    return res


def implicit_run(mask, nsteps, every=5):
    """The 512^3 workload's implicit run: nsteps implicit steps at 20x the
    explicit bound (1.92 s; 4500 of them cover the 8640 s of the explicit
    run's 10^5 steps of 0.0864 s), FP64 fields, multigrid-preconditioned CG
    at rtol 1e-10, totals every `every` steps; against the explicit FP64 run
    over the same simulated time: final totals per pool and carbon drift."""
    import numpy as np
    import torch
    from paper_2406_04177_amd import inputs
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    g = Graph.from_masks(mask)
    spec = inputs.init_uniform(mask, seed=0)
    p = inputs.ModelParams()
    dti, dte = 20.0 * inputs.explicit_dt(p, 1.0), inputs.explicit_dt(p, 0.9)
    x0 = g.fields_from_specs(spec, torch.float64)
    sim = Simulation(g, p, precision="f64", implicit=True, multigrid=True)
    sim.set_preconditioner("mg")
    sim.set_fields(x0)
    c0 = float(sim.totals()[:, 5].sum())
    its, drift = [], 0.0
    t0 = time.perf_counter()
    for k in range(1, nsteps + 1):
        its.append(sim.implicit_step(dti, rtol=1e-10)[0][1])
        if k % every == 0 or k == nsteps:
            drift = max(drift, abs(float(sim.totals()[:, 5].sum()) / c0 - 1))
    sec_i = time.perf_counter() - t0
    tot_i = sim.totals()[0]
    del sim
    torch.cuda.empty_cache()
    ne = int(round(nsteps * dti / dte))
    sim = Simulation(g, p, precision="f64", implicit=False)
    sim.set_fields(x0)
    ms_e, _ = timed(lambda: sim.step(ne, dte, log_every=100, totals_out=torch.empty(
        (ne // 100, g.nseg, 6), dtype=torch.float64, device="cuda")))
    tot_e = sim.totals()[0]
    rel = np.abs(tot_i[:5] - tot_e[:5]) / np.maximum(np.abs(tot_e[:5]), 1e-300)
    res = {"workload": "512^3, %d implicit steps of %.3f s (FP64 fields, multigrid CG, rtol 1e-10, totals every %d) "
                       "vs %d explicit FP64 steps of %.4f s" % (nsteps, dti, every, ne, dte),
           "simulated_s": nsteps * dti, "implicit_s": sec_i, "cg_iterations": int(sum(its)),
           "cg_iterations_per_step": float(np.mean(its)), "explicit_s": ms_e / 1e3,
           "carbon_drift_implicit": drift,
           "final_totals_rel_diff_vs_explicit": dict(zip(("MB", "DOM", "SOM", "P4", "CO2"), map(float, rel)))}
    log("implicit run: %d steps in %.1f s (%.1f CG iterations per step), explicit %d steps in %.1f s; final totals "
        "differ by %s" % (nsteps, sec_i, np.mean(its), ne, ms_e / 1e3, " ".join("%.1e" % v for v in rel)))
    return res


def gradient_batch(steps, K=100):
    """The gradient workload: 16 x 128^3 volumes (porosities U(0.12, 0.25)),
    FP32 fields, CO2 totals every step, loss = MSE against the curve of the
    perturbed parameters, checkpoints every K steps.  Times a plain forward
    run and a full gradient (checkpointed forward + reverse sweep)."""
    import torch
    from paper_2406_04177_amd import inputs
    from paper_2406_04177_amd.autograd import co2_mse, simulate_totals, theta_of
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    masks, specs = inputs.workload_inputs("b16x128")
    params = inputs.ModelParams()
    dt = inputs.explicit_dt(params, 0.8)
    g = Graph.from_masks(masks, regions=True)
    c = [1.0] * 8
    sim = Simulation(g, params, precision="f32", implicit=False, adjoint=True, regions=c)
    x0 = g.fields_from_specs(specs, torch.float32)
    theta = theta_of(params, c)
    tgt_theta = theta.clone()
    for q, f in inputs.target_factors().items():
        tgt_theta[q] *= f
    with torch.no_grad():
        target = simulate_totals(sim, tgt_theta, x0, steps, dt, K)[:, :, 4].clone()
    sim.set_fields(x0)
    sim.set_params(params)
    sim.set_regions(c)
    sim.step(100, dt, log_every=1)
    sim.set_fields(x0)
    ms_fwd, _ = timed(lambda: sim.step(steps, dt, log_every=1))
    res = {"workload": "16 x 128^3 batch (n = %d), %d FP32 steps, CO2 totals every step, checkpoints every %d"
                       % (g.n, steps, K), "forward_ms": ms_fwd}

    # the forward records as many segments as fit 85 % of the free device
    # memory (at this size all 20: 226 GB of FP32 states), the backward
    # runs the others again
    tape = int(0.85 * torch.cuda.mem_get_info()[0])

    def grad():
        th = theta.clone().requires_grad_(True)
        loss = co2_mse(simulate_totals(sim, th, x0, steps, dt, K, tape_bytes=tape), target)
        loss.backward()
        return th.grad
    for skip in (False, True):
        sim.set_adjoint_options(skip_static_d=skip)
        grad()
        ms_g, gr = timed(grad)
        key = "skip_static_d" if skip else "all_d"
        res["gradient_ms_" + key] = ms_g
        res["gradient_forward_ratio_" + key] = ms_g / ms_fwd
        res["backward_forward_ratio_" + key] = (ms_g - ms_fwd) / ms_fwd
    log("16 x 128^3 gradient: forward %.1f ms, gradient %.1f ms (ratio %.2f), skipping static D %.1f ms (%.2f)"
        % (ms_fwd, res["gradient_ms_all_d"], res["gradient_forward_ratio_all_d"], res["gradient_ms_skip_static_d"],
           res["gradient_forward_ratio_skip_static_d"]))
    # without the forward's recorded segments (every segment run again in the backward)
    sim.set_adjoint_options(skip_static_d=False)

    def grad_no_tape():
        th = theta.clone().requires_grad_(True)
        loss = co2_mse(simulate_totals(sim, th, x0, steps, dt, K, tape_bytes=0), target)
        loss.backward()
    res["taped_segments"] = "%d of %d" % (sim.last_taped_segments, (steps + K - 1) // K)
    ms_nt, _ = timed(grad_no_tape)
    res["gradient_ms_all_d_no_tape"] = ms_nt
    res["tape"] = ("segments the forward records itself (vg_step_record): the last ones whose states fit 85 % of "
                   "the free device memory; the others are recorded again in the backward")
    del sim, x0
    torch.cuda.empty_cache()
    return res


def fit_batch(epochs, steps=2000, K=100, subset=4, lr=0.01):
    """Sec. V's normalised-gradient SGD on the gradient workload, twice.

    (1) The configured loss, the CO2 total curve of every volume: recover
    the perturbed parameters (D_DOM, v_DOM, rho, the eight region factors)
    from the unperturbed start.  (2) Per-octant DOM and CO2 curves (each
    volume enumerated in bricks of 64, its octants, one totals segment per
    octant), each curve divided by its largest value.  D_DOM and the region
    factors enter only as the products D_DOM c_r, so the second fit holds
    D_DOM (the gauge) and the recovered quantities are the products, v_DOM
    and rho.  Before fitting, the sensitivity of both losses' curves to the
    eleven log-parameters at the truth (central differences of the FP64
    forward) gives their singular values: the combinations each loss
    identifies.  `subset` volumes per epoch, learning rate halved every 10
    epochs.  The paper starts at 0.1 for O(1) conductances; here steps are
    fractions of each parameter and the perturbations are ~10 %, where 0.1
    overshoots and 0.01 works.  (3) A Gauss-Newton refinement (outside the
    paper) of the second fit's end point on the same curves with the FP64
    forward: the loss is nearly flat along the weakest identifiable
    combination, which the sign steps barely move and a least-squares solve
    recovers."""
    import numpy as np
    import torch
    from paper_2406_04177_amd import inputs
    from paper_2406_04177_amd.autograd import THETA_NAMES, simulate_totals, theta_of
    from paper_2406_04177_amd.fit import fit, gauss_newton, identifiability, octant_segments, sensitivity
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation
    masks, specs = inputs.workload_inputs("b16x128")
    params = inputs.ModelParams()
    # the fit holds every parameter within [0.5, 1.5] of its start, so D and
    # the region factors may both reach 1.5x: dt = 0.9 / 1.5^2 of the bound
    dt = inputs.explicit_dt(params, 0.9 / 1.5 ** 2)
    theta0 = theta_of(params, [1.0] * 8)
    truth = theta0.clone()
    for q, f in inputs.target_factors().items():
        truth[q] *= f
    which = list(inputs.PERTURBED)
    names = [THETA_NAMES[q] for q in which]
    subsets = inputs.epoch_subsets(len(masks), subset, epochs, seed=0)
    res = {"workload": "16 x 128^3, %d FP32 steps per epoch, %d volumes per epoch, %d epochs, lr %g halved every 10"
                       % (steps, subset, epochs, lr)}

    # (1) CO2 curve per volume
    g = Graph.from_masks(masks, regions=True)
    sim = Simulation(g, params, precision="f32", implicit=False, adjoint=True, regions=[1.0] * 8)
    sim.set_adjoint_options(skip_static_d=True)
    x0 = g.fields_from_specs(specs, torch.float32)
    with torch.no_grad():
        target = simulate_totals(sim, truth, x0, steps, dt, K)[:, :, 4].clone()
    sim64 = Simulation(g, params, precision="f64", implicit=False, adjoint=False, regions=[1.0] * 8)
    x64 = g.fields_from_specs(specs, torch.float64)
    scale1 = [float(target.abs().max())]
    sv1, weak1 = identifiability(sensitivity(sim64, truth, x64, steps, dt, which, (4,), scale1, checkpoint_every=K),
                                 names)
    del sim64
    ms, (hist, losses) = timed(lambda: fit(sim, x0, target, theta0, steps, dt, which, epochs=epochs,
                                           checkpoint_every=K, subsets=subsets, lr=lr))
    t0, tr = theta0.numpy(), truth.numpy()
    err0 = np.abs(t0[which] / tr[which] - 1)
    err = np.abs(hist[-1][which] / tr[which] - 1)
    res["co2_per_volume"] = {
        "ms_per_epoch": ms / epochs, "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
        "param_rel_err_start": dict(zip(names, map(float, err0))),
        "param_rel_err_end": dict(zip(names, map(float, err))),
        "singular_values_rel": [float(v) for v in sv1], "weakest_direction": weak1}
    log("fit, CO2 per volume (16 x 128^3): %.0f ms/epoch, loss %.3e -> %.3e, max parameter error %.3f -> %.3f; "
        "sensitivity singular values %s" % (ms / epochs, losses[0], losses[-1], err0.max(), err.max(),
                                           " ".join("%.1e" % v for v in sv1)))
    del sim, x0, g
    torch.cuda.empty_cache()

    # (2) DOM and CO2 per octant, D_DOM held
    g = Graph.from_masks(masks, brick=64, regions=True)
    seg = octant_segments(g)
    sim = Simulation(g, params, precision="f32", implicit=False, adjoint=True, regions=[1.0] * 8, segments=seg)
    sim.set_adjoint_options(skip_static_d=True)
    x0 = g.fields_from_specs(specs, torch.float32)
    with torch.no_grad():
        target = simulate_totals(sim, truth, x0, steps, dt, K)[:, :, [1, 4]].clone()
    scale2 = [float(v) for v in target.abs().amax(dim=(0, 1))]
    sim64 = Simulation(g, params, precision="f64", implicit=False, adjoint=False, regions=[1.0] * 8, segments=seg)
    x64 = g.fields_from_specs(specs, torch.float64)
    sv2, weak2 = identifiability(sensitivity(sim64, truth, x64, steps, dt, which, (1, 4), scale2, checkpoint_every=K),
                                 names)
    del sim64
    which2 = [q for q in which if q != 1]
    ms2, (hist2, losses2) = timed(lambda: fit(sim, x0, target, theta0, steps, dt, which2, epochs=epochs,
                                              checkpoint_every=K, subsets=subsets, lr=lr, curves=(1, 4),
                                              curve_scale=scale2, segs_per_vol=8))
    th = hist2[-1]

    def combos(t):
        return np.array([t[1] * t[12 + r] for r in range(8)] + [t[5], t[7]])
    cnames = ["D_DOM*c%d" % r for r in range(8)] + ["v_dom", "rho"]
    ce0 = np.abs(combos(t0) / combos(tr) - 1)
    ce = np.abs(combos(th) / combos(tr) - 1)
    res["dom_co2_per_octant"] = {
        "kernel": KERNEL_NAMES[sim.kernel_in_use()], "segments": int(seg.size - 1),
        "ms_per_epoch": ms2 / epochs, "loss_first": float(losses2[0]), "loss_last": float(losses2[-1]),
        "fitted": [THETA_NAMES[q] for q in which2], "held": "D_DOM (gauge of the D_DOM c_r products)",
        "identifiable_rel_err_start": dict(zip(cnames, map(float, ce0))),
        "identifiable_rel_err_end": dict(zip(cnames, map(float, ce))),
        "singular_values_rel": [float(v) for v in sv2], "weakest_direction": weak2}
    log("fit, DOM and CO2 per octant: %.0f ms/epoch, loss %.3e -> %.3e, max error of D c_r, v_DOM, rho %.3f -> %.4f; "
        "sensitivity singular values %s" % (ms2 / epochs, losses2[0], losses2[-1], ce0.max(), ce.max(),
                                           " ".join("%.1e" % v for v in sv2)))
    del sim, x0
    torch.cuda.empty_cache()

    # (3) Gauss-Newton refinement (not the paper's method) from the SGD's
    # end point: the same per-octant curves with the FP64 forward and an
    # FP64 target, the Jacobian by central differences, a truncated SVD solve
    sim64 = Simulation(g, params, precision="f64", implicit=False, adjoint=False, regions=[1.0] * 8, segments=seg)
    x64 = g.fields_from_specs(specs, torch.float64)
    with torch.no_grad():
        target64 = simulate_totals(sim64, truth, x64, steps, dt, K)[:, :, [1, 4]].clone()
    scale3 = [float(v) for v in target64.abs().amax(dim=(0, 1))]
    ms3, (hist3, norms3) = timed(lambda: gauss_newton(sim64, torch.as_tensor(th), x64, target64, steps, dt, which2,
                                                      curves=(1, 4), scale=scale3, iters=3, checkpoint_every=K))
    ce3 = [np.abs(combos(h) / combos(tr) - 1) for h in hist3]
    res["gauss_newton_fp64"] = {
        "start": "the per-octant SGD's end point", "iterations": len(hist3) - 1,
        "forward_runs": (len(hist3) - 1) * (2 * len(which2) + 1) + 1, "ms": ms3,
        "squared_misfit": [float(v) for v in norms3],
        "identifiable_max_rel_err": [float(e.max()) for e in ce3],
        "identifiable_rel_err_end": dict(zip(cnames, map(float, ce3[-1])))}
    log("fit, Gauss-Newton refinement (FP64, per-octant DOM and CO2): %.1f s, max error of D c_r, v_DOM, rho %s"
        % (ms3 / 1e3, " -> ".join("%.2e" % e.max() for e in ce3)))
    del sim64, x64, g
    torch.cuda.empty_cache()
    return res


def zlayer_experiment(mask):
    """Sec. IV.B's diffusion comparison on the 512^3 volume: DOM on layers 0-1,
    1.76 h of diffusion, explicit 0.1 s steps vs implicit 30 s steps, the DOM
    mass per z-layer."""
    import numpy as np
    import torch
    from paper_2406_04177_amd import diffusion_experiment as de
    from paper_2406_04177_amd.graph import Graph
    g = Graph.from_masks(mask)
    ms_e, (sim_e, nsteps) = timed(lambda: de.run_explicit(mask, g, dt=0.1, precision="f32"))
    pe = de.layer_profile(sim_e, mask)
    del sim_e
    ms_i, (sim_i, its) = timed(lambda: de.run_implicit(mask, g, dt=30.0, precision="f32", rtol=1e-10))
    pi = de.layer_profile(sim_i, mask)
    del sim_i
    torch.cuda.empty_cache()
    ms_m, (sim_m, its_m) = timed(lambda: de.run_implicit(mask, g, dt=30.0, precision="f32", rtol=1e-10,
                                                           multigrid=True))
    pm = de.layer_profile(sim_m, mask)
    del sim_m
    res = {"workload": "512^3, M0 = %.4f mg on layers 0-1, D = 100950 voxel^2/day, %.0f s" % (de.M0, de.T_END),
           "explicit": {"dt_s": 0.1, "steps": nsteps, "ms": ms_e, "mass_rel_err": float(abs(pe.sum() / de.M0 - 1))},
           "implicit": {"dt_s": 30.0, "steps": len(its), "cg_iterations": int(sum(its)), "ms": ms_i,
                        "mass_rel_err": float(abs(pi.sum() / de.M0 - 1)), "preconditioner": "Jacobi (the paper's)"},
           "implicit_multigrid": {"dt_s": 30.0, "steps": len(its_m), "cg_iterations": int(sum(its_m)), "ms": ms_m,
                                  "mass_rel_err": float(abs(pm.sum() / de.M0 - 1)),
                                  "profile_max_abs_diff_vs_jacobi_rel_to_peak": float(np.abs(pm - pi).max() / pi.max()),
                                  "note": "ms includes building the hierarchy"},
           "profile_max_abs_diff_rel_to_peak": float(np.abs(pe - pi).max() / pe.max()),
           "profile_layers_0_4_explicit": [float(v) for v in pe[:5]],
           "profile_layers_0_4_implicit": [float(v) for v in pi[:5]],
           "layer_of_half_mass_explicit": int(np.searchsorted(np.cumsum(pe), de.M0 / 2)),
           "layer_of_half_mass_implicit": int(np.searchsorted(np.cumsum(pi), de.M0 / 2))}
    log("z-layer experiment: explicit %d steps %.1f s, implicit %d steps (%d CG iterations) %.1f s, with "
        "multigrid %d CG iterations %.1f s; profiles differ by %.2e of the peak"
        % (nsteps, ms_e / 1e3, len(its), sum(its), ms_i / 1e3, sum(its_m), ms_m / 1e3,
           res["profile_max_abs_diff_rel_to_peak"]))
    return res


def pngm_row(mask, b=16, scenarios=8, records=30, every_s=10.0, epochs=1000):
    """Sec. V on the 512^3 volume: primitives = bricks of side b; data pairs =
    primitive masses of voxel-method diffusion runs (D = 100950 voxel^2/day,
    explicit 0.1 s steps) recorded every 10 s from random DOM scenarios;
    objective L2, normalised-gradient SGD for `epochs` epochs of 4 pairs (lr 0.1
    halved every 10 epochs) from theta = S / d; then the explicit pore-network
    scheme with 0.1 s steps and the implicit one with 10 s steps from a held-out
    scenario, against the voxel method (mean relative L2 error of the primitive
    masses over the 10 s records), and objective 2 on the held-out pairs."""
    import numpy as np
    import torch
    from paper_2406_04177_amd import pngm
    from paper_2406_04177_amd.graph import Graph
    ms_setup, (g, part) = timed(lambda: (lambda gg: (gg, pngm.partition(gg, b)))(Graph.from_masks(mask, brick=b)))
    scen = list(range(scenarios))
    ms_data, data = timed(lambda: pngm.generate(g, part, mask, scen + [1000], records, every_s))
    train, held = data[:-1], data[-1]
    X = train[:, :-1].reshape(-1, part.q)
    Y = train[:, 1:].reshape(-1, part.q)
    c = 100950.0 / 86400.0 * every_s
    ms_fit, (theta, losses) = timed(lambda: pngm.fit(part, X, Y, c, epochs, batch=4, objective=2))
    theta0 = torch.as_tensor(part.S / part.d, dtype=torch.float64, device=X.device)

    # the networks run from a held-out scenario: scheme 3 at the voxel method's
    # 0.1 s step and scheme 4 at the data spacing (the scheme objective 2
    # encodes), from t = 0 and from t = 30 s (after the sub-brick transient)
    c_sub = 100950.0 / 86400.0 * 0.1
    nsub = int(round(every_s / 0.1))
    work = torch.empty(3 * part.q + 2, dtype=torch.float64, device=X.device)
    sweeps = []

    def rollout(th, scheme, start):
        m = held[start].clone()
        errs = []
        for r in range(start, records):
            if scheme == 3:
                for _ in range(nsub):
                    m = pngm.step(part, m, th, c_sub)
            else:
                m, it, _ = pngm.implicit_step(part, m, th, c, rtol=1e-12, work=work)
                sweeps.append(it)
            errs.append(float(torch.linalg.norm(m - held[r + 1]) / torch.linalg.norm(held[r + 1])))
        return float(np.mean(errs))
    err = {}
    for scheme in (3, 4):
        for start in (0, 3):
            for name, th in (("start", theta0), ("fitted", theta)):
                err["scheme%d_from_%ds_%s_theta" % (scheme, int(start * every_s), name)] = rollout(th, scheme, start)
    ms_r4, _ = timed(lambda: rollout(theta, 4, 0))
    # objective 2 on the held-out pairs, one pair at a time
    per0 = np.array([float(pngm.loss_grad(part, held[r:r + 1], held[r + 1:r + 2], theta0, c, 2)[0])
                     for r in range(records)])
    per1 = np.array([float(pngm.loss_grad(part, held[r:r + 1], held[r + 1:r + 2], theta, c, 2)[0])
                     for r in range(records)])
    full0 = float(pngm.loss_grad(part, X, Y, theta0, c, 2)[0])
    full1 = float(pngm.loss_grad(part, X, Y, theta, c, 2)[0])
    ratio = (theta / theta0).cpu().numpy()
    res = {"workload": "512^3 in %d^3 bricks (q = %d primitives, %d directed edges), %d scenarios x %d pairs "
                       "10 s apart, 1 held-out scenario" % (b, part.q, int(part.col.numel()), scenarios, records),
           "ms_partition": ms_setup, "ms_data": ms_data, "ms_fit": ms_fit, "epochs": epochs,
           "L2_train_start": full0, "L2_train_end": full1,
           "L2_heldout_start": float(per0.mean()), "L2_heldout_end": float(per1.mean()),
           "L2_heldout_pair_ratio_median": float(np.median(per1 / per0)),
           "theta_over_theta0_percentiles_10_50_90": np.percentile(ratio, [10, 50, 90]).tolist(),
           "rollout_mean_rel_err": err, "scheme4_sweeps_max": int(max(sweeps)),
           "ms_scheme4_step": ms_r4 / records}
    log("PNGM (q = %d): data %.1f s, fit %d epochs %.2f s; L2 train %.3e -> %.3e, held-out %.3e -> %.3e (median pair "
        "ratio %.3f); mean held-out error from 30 s, scheme 3 at 0.1 s %.3f -> %.3f, scheme 4 at 10 s %.3f -> %.3f "
        "(%.2f ms/step)" % (part.q, ms_data / 1e3, epochs, ms_fit / 1e3, full0, full1, per0.mean(), per1.mean(),
                            np.median(per1 / per0), err["scheme3_from_30s_start_theta"],
                            err["scheme3_from_30s_fitted_theta"], err["scheme4_from_30s_start_theta"],
                            err["scheme4_from_30s_fitted_theta"], ms_r4 / records))
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--quick", action="store_true", help="headline only (no extra rows, no CPU baseline)")
    ap.add_argument("--cpu-steps", type=int, default=450,
                    help="steps of the oracle CPU baseline (about 10-15 s on 16 cores)")
    ap.add_argument("--acc-steps", type=int, default=10000, help="steps of the 256^3 precision row")
    ap.add_argument("--long-steps", type=int, default=100000,
                    help="steps of the 512^3 precision row (FP32, compensated FP32, FP64; 0: skip)")
    ap.add_argument("--cpu-steps-1t", type=int, default=20, help="steps of the one-thread oracle sample")
    ap.add_argument("--cpu-grad-steps", type=int, default=40,
                    help="steps of the oracle's gradient sample on the 16 x 128^3 workload (200 take ~2 min)")
    ap.add_argument("--grad-steps", type=int, default=2000, help="steps of the 16 x 128^3 gradient row")
    ap.add_argument("--fit-epochs", type=int, default=30, help="epochs of the 16 x 128^3 fitting row (0: skip)")
    ap.add_argument("--zlayer", type=int, default=1, help="run the 512^3 z-layer diffusion comparison (0: skip)")
    ap.add_argument("--pngm", type=int, default=1, help="run the 512^3 pore-network fitting row (0: skip)")
    ap.add_argument("--big", type=int, default=1, help="run the 1024^3 explicit-step row (0: skip)")
    ap.add_argument("--implicit-run", type=int, default=0,
                    help="implicit steps of the 512^3 implicit run (4500 cover the explicit run's 8640 s; "
                         "0: skip; about 2.5 min for 4500)")
    ap.add_argument("--kernel", choices=("auto", "table", "rank", "offset", "relative", "band"), default="auto",
                    help="neighbour source of the explicit-step kernel")
    ap.add_argument("--precision", choices=("f32", "f32c", "f64"), default="f32",
                    help="fields of the headline step: FP32, compensated FP32 or FP64 (totals FP64 in every case)")
    ap.add_argument("--rows", default=None,
                    help="comma-separated rows to run after the headline (default: all unless --quick): " + ",".join(
                        ("sources", "alg2", "fp64", "implicit", "adjoint", "zlayer", "pngm", "gradient", "fit",
                         "precision", "copy", "big", "cpu")))
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="finish with three plain 1 GiB device copies (scale for HBM byte counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (the z-slab sharding is a design, not code)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2406_04177_amd import inputs
    from paper_2406_04177_amd.graph import Graph
    from paper_2406_04177_amd.sim import Simulation

    torch.cuda.set_device(0)
    N = args.size
    t0 = time.perf_counter()
    mask = inputs.synthetic_volume((N, N, N), porosity=0.17, seed=0)
    spec = inputs.init_uniform(mask, seed=0)
    log("generated %d^3 volume in %.1f s" % (N, time.perf_counter() - t0))
    params = inputs.ModelParams()
    dt = inputs.explicit_dt(params, 0.9)

    # a1: graph build (mask already on the device)
    Graph.from_masks(mask)       # warm-up (kernel loading)
    ms_graph, g = timed(lambda: Graph.from_masks(mask))
    n = g.n
    log("n = %d pore voxels; graph build %.2f ms (incl. mask upload and host sync)" % (n, ms_graph))

    prec = args.precision
    sim = Simulation(g, params, precision=prec, implicit=False, adjoint=False)
    sim.set_kernel({"auto": 0, "table": 1, "rank": 2, "offset": 3, "relative": 4, "band": 5}[args.kernel])
    kernel = sim.kernel_in_use()
    x0 = g.fields_from_specs(spec, torch.float32)
    sim.set_fields(x0 if prec == "f32" else g.fields_from_specs(spec, torch.float64))
    sim.step(args.warmup, dt, log_every=100)
    K = args.steps
    # FP64 totals every 100 steps, or once at the end of a shorter timed run
    every = min(100, K)
    tot_log = torch.empty((K // every, g.nseg, 6), dtype=torch.float64, device="cuda")
    ms, _ = timed(lambda: sim.step(K, dt, log_every=every, totals_out=tot_log))
    ms_step = ms / K
    vps = n * K / (ms / 1e3)
    # the dominant kernel's own average launch time: K2 = 4 m + 1 paper steps
    # launch a transformation-only pass, 4 m fused passes (m runs of four: 2 m
    # band launches, or 4 m single passes) and a diffusion-only pass, one step
    # launches the two end passes only; no totals in either
    ppl = PASSES_PER_LAUNCH[kernel]
    K2 = (K - 1) // 4 * 4 + 1
    ms_k, _ = timed(lambda: sim.step(K2, dt))
    ms_1, _ = timed(lambda: sim.step(1, dt))
    us_launch = (ms_k - ms_1) / ((K2 - 1) / ppl) * 1e3
    # the roofline counts the method's algorithmic bytes per voxel and step
    # (five pools read and written plus the 6-slot neighbour table: 64 B for
    # FP32 fields) whichever neighbour source the kernel uses, times the
    # passes one launch applies; own_bytes_per_voxel is what the kernel
    # itself moves per step
    if prec == "f32":
        own_bpv, bpv = OWN_BYTES[kernel], BYTES_FUSED_F32
    elif prec == "f32c":
        own_bpv, bpv = BYTES_COMP_RELATIVE if kernel == 4 else BYTES_FUSED_F32C, BYTES_FUSED_F32C
    else:
        own_bpv, bpv = BYTES_F64_RELATIVE if kernel == 4 else BYTES_FUSED_F64, BYTES_FUSED_F64
    achieved = bpv * ppl * n / (us_launch / 1e6) / 1e9
    kname = KERNEL_FUNCS[kernel] if prec != "f32c" else "k_step_c (compensated FP32, relative codes)"
    traffic = None
    rec = MEASURED_TRAFFIC.get((KERNEL_NAMES[kernel] + ("" if prec == "f32" else "_" + prec), N))
    if rec is not None and rec[1] == sources_sha():
        traffic = rec[0]
    log("explicit %s: %.4f ms/step, %.3e voxel-steps/s; %s kernel %.2f us/launch (%d pass(es)), %.0f GB/s "
        "algorithmic" % (prec.upper(), ms_step, vps, KERNEL_NAMES[kernel], us_launch, ppl, achieved))
    out = {
        "metric": METRIC,
        "value": 5.0 * vps,
        "unit": "pore-voxel species updates/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": "%d^3 17%% porosity explicit step, %s fields, FP64 totals every %d steps"
                               % (N, {"f32": "FP32", "f32c": "compensated FP32", "f64": "FP64"}[prec], every),
                   "shape": [N, N, N], "n_pore_voxels": n, "dt_s": dt, "order": "transformation then diffusion",
                   "voxel_steps_per_s": vps},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_GBs": None if traffic is None else traffic / (us_launch / 1e6) / 1e9,
                     "traffic_frac": None if traffic is None else traffic / (us_launch / 1e6) / 1e9 / HBM_PEAK_GBS,
                     "kernel": "%s, %s, DOM-only diffusion (fused transformation + diffusion)" % (kname, prec.upper()),
                     "neighbour_source": KERNEL_NAMES[kernel],
                     "launch_us": us_launch, "passes_per_launch": ppl, "bytes_per_voxel_step": bpv,
                     "bytes_per_launch": bpv * ppl * n, "own_bytes_per_voxel_step": own_bpv,
                     "own_frac": own_bpv * ppl * n / (us_launch / 1e6) / 1e9 / HBM_PEAK_GBS},
    }
    del tot_log

    selected = None if args.rows is None else set(r.strip() for r in args.rows.split(",") if r.strip())

    def want(name):
        return (selected is None and not args.quick) or (selected is not None and name in selected)

    have_rows = selected is not None or not args.quick or args.implicit_run > 0
    if have_rows:
        rows = {}
        rows["a1_graph_build_ms"] = ms_graph
    sim32 = sim
    if prec != "f32" and (want("sources") or want("alg2")):
        sim32 = Simulation(g, params, precision="f32", implicit=False, adjoint=False)
        sim32.set_fields(x0)
        sim32.step(20, dt)
        kernel = sim32.kernel_in_use()
    if want("sources"):
        # the other neighbour sources on the same state, for comparison
        for other in (1, 2, 3, 4, 5):
            if other == kernel and prec == "f32":
                continue
            sim32.set_kernel(other)
            sim32.step(20, dt)
            mso, _ = timed(lambda: sim32.step(K // 2, dt, log_every=100))
            rows["fp32_step_%s_kernel" % KERNEL_NAMES[other]] = {
                "ms_per_step": mso / (K // 2), "own_bytes_per_voxel": OWN_BYTES[other],
                "achieved_GBs_64B": BYTES_FUSED_F32 * n / (mso / (K // 2) / 1e3) / 1e9,
                "achieved_GBs_own": OWN_BYTES[other] * n / (mso / (K // 2) / 1e3) / 1e9}
            log("explicit FP32, %s kernel: %.4f ms/step" % (KERNEL_NAMES[other], mso / (K // 2)))
        sim32.set_kernel(0)
    if want("alg2"):
        # Algorithm 2 (sequential transformation) and unequal steps (the
        # paper's test 3 ratio: transformation 4.3x the diffusion step)
        sim2 = Simulation(g, params.replace(sequential=True), precision="f32", implicit=False, adjoint=False)
        sim2.set_fields(x0)
        sim2.step(20, dt)
        ms2, _ = timed(lambda: sim2.step(K // 2, dt))
        sim2.set_params(params)
        sim2.set_fields(x0)
        nt = max(K // 8, 10)
        sim2.step_subcycled(5, 4.3 * dt, dt)
        mss, _ = timed(lambda: sim2.step_subcycled(nt, 4.3 * dt, dt))
        ndiff = int(np.ceil(nt * 4.3 - 1e-9))
        rows["f2_algorithm2_and_subcycling"] = {
            "algorithm2_ms_per_step": ms2 / (K // 2),
            "subcycled": {"transformation_steps": nt, "dt_t_over_dt_d": 4.3, "diffusion_steps": ndiff,
                          "ms_total": mss, "ms_per_diffusion_step": mss / ndiff}}
        log("Algorithm 2: %.4f ms/step; sub-cycled (dt_t = 4.3 dt_d): %.4f ms per diffusion step"
            % (ms2 / (K // 2), mss / ndiff))
        del sim2
    if want("fp64") or want("implicit"):
        # plain FP64 step on the same input
        t_mg = time.perf_counter()
        sim64 = Simulation(g, params, precision="f64", implicit=True, adjoint=False, multigrid=want("implicit"))
        ms_mg_setup = (time.perf_counter() - t_mg) * 1e3
        sim64.set_fields(x0.double())
        sim64.step(20, dt)
        k64 = max(K // 4, 50)
        ms64, _ = timed(lambda: sim64.step(k64, dt, log_every=100))
        rows["fp64_step"] = {"ms_per_step": ms64 / k64, "voxel_steps_per_s": n * k64 / (ms64 / 1e3),
                             "achieved_GBs": BYTES_FUSED_F64 * n / (ms64 / k64 / 1e3) / 1e9,
                             "fp32_speedup": (ms64 / k64) / ms_step}
        log("explicit FP64: %.4f ms/step (FP32 speed-up %.2fx)" % (ms64 / k64, (ms64 / k64) / ms_step))
    if want("implicit"):
        # a5: implicit step at 20x the explicit bound (FP64 CG vectors, rtol 1e-10)
        dti = 20.0 * inputs.explicit_dt(params, 1.0)
        sim64.set_fields(x0.double())
        sim64.implicit_step(dti)
        its = []
        nimp = 3
        def imp():
            for _ in range(nimp):
                its.append(sim64.implicit_step(dti, rtol=1e-10)[0][1])
        msi, _ = timed(imp)
        rows["a5_implicit_step"] = {"dt_s": dti, "rtol": 1e-10, "ms_per_step": msi / nimp,
                                    "cg_iterations": its, "ms_per_cg_iteration": msi / max(sum(its), 1),
                                    "precision": "f64 fields, f64 CG", "preconditioner": "Jacobi (the paper's)"}
        log("implicit: %.2f ms/step, CG iterations %s" % (msi / nimp, its))
        # the same steps with the multigrid V-cycle as preconditioner
        sim64.set_preconditioner("mg")
        sim64.set_fields(x0.double())
        sim64.implicit_step(dti)
        its_mg = []
        def imp_mg():
            for _ in range(nimp):
                its_mg.append(sim64.implicit_step(dti, rtol=1e-10)[0][1])
        msm, _ = timed(imp_mg)
        rows["a5_implicit_step"]["multigrid"] = {
            "ms_per_step": msm / nimp, "cg_iterations": its_mg, "ms_per_cg_iteration": msm / max(sum(its_mg), 1),
            "levels": sim64.mg_levels(), "ms_handle_with_hierarchy": ms_mg_setup,
            "speedup_vs_jacobi": (msi / nimp) / (msm / nimp)}
        log("implicit, multigrid: %.2f ms/step, CG iterations %s, levels %s" % (msm / nimp, its_mg,
                                                                              sim64.mg_levels()))
    if want("fp64") or want("implicit"):
        del sim64
        torch.cuda.empty_cache()
    if want("adjoint"):
        # a6: adjoint / forward time ratio over a 20-step segment; the
        # recording keeps each step's diffused DOM (as the gradient does)
        sima = Simulation(g, params, precision="f32", implicit=False, adjoint=True)
        sima.set_adjoint_options(tape_dom=True)
        sima.set_fields(x0)
        KA = 20
        states = torch.empty((KA, sima.tape_rows, n), dtype=torch.float32, device="cuda")
        seeds = torch.zeros((KA, g.nseg, 5), dtype=torch.float64, device="cuda")
        seeds[:, :, 4] = 1.0
        lam = torch.zeros((5, n), dtype=torch.float32, device="cuda")
        grad = torch.zeros(20, dtype=torch.float64, device="cuda")
        sima.step(KA, dt, log_every=1)
        sima.set_fields(x0)
        msf, _ = timed(lambda: sima.step(KA, dt, log_every=1))
        sima.set_fields(x0)
        sima.record(KA, dt, states)
        sima.adjoint(KA, dt, states, seeds, lam, grad)
        msr, _ = timed(lambda: sima.record(KA, dt, states))
        msa, _ = timed(lambda: sima.adjoint(KA, dt, states, seeds, lam, grad))
        sima.set_adjoint_options(skip_static_d=True)
        sima.adjoint(KA, dt, states, seeds, lam, grad)
        msa_s, _ = timed(lambda: sima.adjoint(KA, dt, states, seeds, lam, grad))
        rows["a6_adjoint"] = {"workload": "512^3, one %d-step checkpoint segment, CO2 seeds every step, diffused "
                                          "DOM kept by the recording" % KA,
                              "segment_steps": KA, "forward_ms": msf, "record_ms": msr, "adjoint_ms": msa,
                              "adjoint_forward_ratio": (msr + msa) / msf,
                              "adjoint_only_ratio": msa / msf,
                              "adjoint_ms_skip_static_d": msa_s,
                              "adjoint_forward_ratio_skip_static_d": (msr + msa_s) / msf}
        log("adjoint/forward ratio %.2f (record %.2f ms, adjoint %.2f ms, forward %.2f ms); "
            "static-pool D gradients skipped: adjoint %.2f ms, ratio %.2f"
            % ((msr + msa) / msf, msr, msa, msf, msa_s, (msr + msa_s) / msf))
        del sima, states, lam
        torch.cuda.empty_cache()
    if want("zlayer") and args.zlayer:
        rows["f3_zlayer_diffusion"] = zlayer_experiment(mask)
    if want("pngm") and args.pngm:
        rows["f4_pngm_512"] = pngm_row(mask)
    if want("gradient"):
        rows["a6_gradient_16x128"] = gradient_batch(args.grad_steps)
        out["adjoint_forward_ratio"] = rows["a6_gradient_16x128"]["gradient_forward_ratio_all_d"]
    if want("fit") and args.fit_epochs > 0:
        rows["f1_fit_16x128"] = fit_batch(args.fit_epochs, steps=args.grad_steps)
    if have_rows:
        out["rows"] = rows
        # FP32 and compensated FP32 fields (FP64 totals) against the plain
        # FP64 step: the 256^3 workload at its length (10^4 steps) and the
        # 512^3 one at its (10^5 steps), totals every 100, error per species
        # (fields, relative to each pool's max) and per totals curve
    if args.implicit_run > 0:
        rows["implicit_run_512"] = implicit_run(mask, args.implicit_run)
    if want("precision"):
        rows["precision_256"] = accuracy_runs(256, args.acc_steps, "FP32 vs FP64 workload")
        if args.long_steps > 0:
            rows["precision_512_long"] = accuracy_runs(N, args.long_steps, "full-size decomposition run")
    if want("copy"):
        rows["copy_1GiB"] = copy_1gib()
        log("plain 1 GiB device copy: %.0f GB/s (read + written)" % rows["copy_1GiB"]["GBs"])
    if want("big") and args.big:
        rows["explicit_1024"] = step_1024()
    if want("cpu"):
        # CPU baseline: the oracle on the host cores
        cb = cpu_baseline(mask, spec, params, dt, args.cpu_steps, args.cpu_steps_1t, args.cpu_grad_steps)
        out["cpu_baseline"] = cb
        log("cpu baseline (%s): %.3e species updates/s on %d threads, %.3e on 1; oracle gradient "
            "(16 x 128^3, %d steps) %.1f s" % (cb["cpu_model"], cb["value"], cb["cores"], cb["one_thread"]["value"],
                                              args.cpu_grad_steps, cb["gradient_16x128"]["seconds"]))
    # the paper's own timing, other hardware (context only, not a target):
    # Table 1 test 2, explicit 0.1 s steps for 5 days on the 512^3 image
    # (about 0.17 x 512^3 pore voxels) in 7.9 days on a laptop CPU
    paper_vps = 5 * 86400 / 0.1 * 0.17 * 512 ** 3 / (7.9 * 86400)
    out["paper_context"] = {"value": 5.0 * paper_vps, "unit": "pore-voxel species updates/s",
                            "hardware": "AMD Ryzen 7 PRO 6850H laptop CPU (the paper's C code)",
                            "source": "Table 1, test 2 (explicit 0.1 s, 5 simulated days, 7.9 days wall time)",
                            "gpu_over_paper": 5.0 * vps / (5.0 * paper_vps)}
    print(json.dumps(out), flush=True)
    try:   # nothing here starts processes; report any that would outlive the run
        import psutil
        kids = psutil.Process().children(recursive=True)
        if kids:
            log("child processes at exit: %s" % [(k.pid, k.name()) for k in kids])
    except Exception:
        pass
    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("calibration copies done (3 x 1 GiB)")
    return 0


if __name__ == "__main__":
    sys.exit(main())
