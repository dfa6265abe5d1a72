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


def cpu_baseline(mask, spec, params, dt, steps):
    """The FP64 oracle on the host cores, on the first `steps` steps."""
    from oracle import oracle as orc
    og = orc.build_graph(mask)
    x0 = orc.fields_from_spec(og, spec)
    t0 = time.perf_counter()
    orc.run(params, dt, og, x0, steps, with_totals=False)
    sec = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", 0)) or os.cpu_count()
    return {"value": 5.0 * og.n * steps / sec, "unit": "pore-voxel species updates/s", "cores": cores,
            "kind": "oracle",
            "sample": "%d explicit steps of the same 512^3 workload (n = %d), FP64, %.1f s" % (steps, og.n, sec)}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--quick", action="store_true", help="headline only (no extra rows, no CPU baseline)")
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--kernel", choices=("auto", "table", "rank"), default="auto",
                    help="neighbour source of the explicit-step kernel")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (see DESIGN.md, sharding)",
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

    sim = Simulation(g, params, precision="f32", implicit=False, adjoint=False)
    kernel = {"auto": 0, "table": 1, "rank": 2}[args.kernel]
    sim.set_kernel(kernel)
    x0 = g.fields_from_specs(spec, torch.float32)
    sim.set_fields(x0)
    sim.step(args.warmup, dt, log_every=100)
    K = args.steps
    tot_log = torch.empty((max(K // 100, 1), g.nseg, 6), dtype=torch.float64, device="cuda")
    ms, _ = timed(lambda: sim.step(K, dt, log_every=100, totals_out=tot_log if K >= 100 else None))
    ms_step = ms / K
    vps = n * K / (ms / 1e3)
    rank_used = kernel == 2 or (kernel == 0 and g.nseg == 1)
    own_bpv = BYTES_RANK_F32 if rank_used else BYTES_FUSED_F32
    # the roofline counts the method's algorithmic bytes per voxel and step
    # (five pools read and written plus the 6-slot neighbour table, 64 B)
    # whichever neighbour source the kernel uses; own_bytes_per_voxel is what
    # the rank-index kernel itself has to move
    bpv = BYTES_FUSED_F32
    achieved = bpv * n / (ms_step / 1e3) / 1e9
    log("explicit FP32: %.4f ms/step, %.3e voxel-steps/s, %.0f GB/s algorithmic" % (ms_step, vps, achieved))
    out = {
        "metric": METRIC,
        "value": 5.0 * vps,
        "unit": "pore-voxel species updates/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "%d^3 17%% porosity explicit step, FP32 fields, FP64 totals every 100 steps" % N,
                   "shape": [N, N, N], "n_pore_voxels": n, "dt_s": dt, "order": "transformation then diffusion",
                   "voxel_steps_per_s": vps},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "%s<float, DT, DOM-only> (fused transformation + diffusion)"
                               % ("k_step_geo" if rank_used else "k_step"),
                     "bytes_per_voxel": bpv, "own_bytes_per_voxel": own_bpv,
                     "own_frac": own_bpv * n / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS},
    }
    del tot_log

    if not args.quick:
        rows = {}
        rows["a1_graph_build_ms"] = ms_graph
        # the other neighbour source on the same state, for comparison
        other = 1 if kernel != 1 else 2
        sim.set_kernel(other)
        sim.step(20, dt)
        mso, _ = timed(lambda: sim.step(K // 2, dt, log_every=100))
        rows["fp32_step_%s_kernel" % ("table" if other == 1 else "rank")] = {
            "ms_per_step": mso / (K // 2), "bytes_per_voxel": BYTES_FUSED_F32 if other == 1 else BYTES_RANK_F32,
            "achieved_GBs": (BYTES_FUSED_F32 if other == 1 else BYTES_RANK_F32) * n / (mso / (K // 2) / 1e3) / 1e9}
        log("explicit FP32, %s kernel: %.4f ms/step" % ("table" if other == 1 else "rank", mso / (K // 2)))
        sim.set_kernel(kernel)
        # plain FP64 step on the same input
        sim64 = Simulation(g, params, precision="f64", implicit=True, adjoint=False)
        sim64.set_fields(x0.double())
        sim64.step(20, dt)
        k64 = max(K // 4, 50)
        ms64, _ = timed(lambda: sim64.step(k64, dt, log_every=100))
        rows["fp64_step"] = {"ms_per_step": ms64 / k64, "voxel_steps_per_s": n * k64 / (ms64 / 1e3),
                             "achieved_GBs": BYTES_FUSED_F64 * n / (ms64 / k64 / 1e3) / 1e9,
                             "fp32_speedup": (ms64 / k64) / ms_step}
        log("explicit FP64: %.4f ms/step (FP32 speed-up %.2fx)" % (ms64 / k64, (ms64 / k64) / ms_step))
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
                                    "precision": "f64 fields, f64 CG"}
        log("implicit: %.2f ms/step, CG iterations %s" % (msi / nimp, its))
        del sim64
        torch.cuda.empty_cache()
        # a6: adjoint / forward time ratio over a 20-step segment
        sima = Simulation(g, params, precision="f32", implicit=False, adjoint=True)
        sima.set_fields(x0)
        KA = 20
        states = torch.empty((KA, 5, n), dtype=torch.float32, device="cuda")
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
        rows["a6_adjoint"] = {"segment_steps": KA, "forward_ms": msf, "record_ms": msr, "adjoint_ms": msa,
                              "adjoint_forward_ratio": (msr + msa) / msf,
                              "adjoint_only_ratio": msa / msf}
        log("adjoint/forward ratio %.2f (record %.2f ms, adjoint %.2f ms, forward %.2f ms)"
            % ((msr + msa) / msf, msr, msa, msf))
        out["rows"] = rows
        out["adjoint_forward_ratio"] = (msr + msa) / msf
        del sima, states, lam
        torch.cuda.empty_cache()
        # CPU baseline: the oracle on the host cores
        cb = cpu_baseline(mask, spec, params, dt, args.cpu_steps)
        out["cpu_baseline"] = cb
        log("cpu baseline: %.3e species updates/s on %d cores" % (cb["value"], cb["cores"]))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
