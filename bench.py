"""Benchmark: RK4 grid-point updates/s of the fused FP64 stage kernels.

Workload: 256^3 interior points on [-16,16]^3 (h = 0.125), mu^2 = 2,
lambda = 1, phi0 = 8 seeded Gaussians (seed 0), phi1 = 0, dt = 0.005 (the
2000-step single-solve configuration).  A "step" is one full RK4 step (4 fused
stage kernels + the step-counter tick) over the whole grid; inputs are
resident in HBM before timing starts.

Prints ONE JSON line.  Extra objects:
  roofline      -- dominant kernel (stage 4: 7 field passes = 56 B/point FP64)
                   algorithmic bytes / its average duration, from HIP events
                   on the solver's stream, against 8 TB/s;
  cpu_baseline  -- the FP64 CPU oracle on a bounded number of steps of the
                   same grid, on this host's cores;
  forms         -- the same step rate for the FP32c form (same grid) when
                   --forms is given.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per point per stage (field passes x element size)
PASSES = {1: 3, 2: 4, 3: 5, 4: 7}


def stage_bytes(stage, precision):
    if precision == 0:
        return PASSES[stage] * 8
    return PASSES[stage] * 4 + (16 if stage == 4 else 0)


def run_gpu(w, precision, steps, warmup, timed_stage_steps):
    import numpy as np
    import torch
    from paper_1803_01291_amd import hb

    p0, p1 = w.initial()
    h = hb.hb_create(hb.config_from_workload(w, precision))
    try:
        hb.hb_set_initial(h, p0, p1)
        hb.hb_step(h, warmup)
        hb.hb_sync(h)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hb.hb_step(h, steps)
        hb.hb_sync(h)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        stage_ms = hb.hb_step_timed(h, timed_stage_steps)
        d = hb.hb_diagnostics(h, allow_nonfinite=True)
    finally:
        hb.hb_destroy(h)
    return elapsed, [m / timed_stage_steps for m in stage_ms], d


def cpu_baseline(w, steps):
    import oracle
    p0, p1 = w.initial()
    t0 = time.perf_counter()
    oracle.solve(p0, p1, w.h, w.mu2, w.lam, w.dt, steps, t0=w.t0, inv_L2=w.inv_L2)
    dt = time.perf_counter() - t0
    return {"value": w.points * steps / dt, "unit": "grid-point-updates/s",
            "cores": oracle.get_threads(), "kind": "oracle",
            "sample": f"{steps} RK4 steps of the same {w.n[0]}^3 grid (FP64 C oracle, OpenMP), "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--stage-steps", type=int, default=50)
    ap.add_argument("--cpu-steps", type=int, default=24)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--forms", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solver has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import synth_inputs as si
    w = si.config2(n=args.n)
    N = w.points
    elapsed, stage_ms, diag = run_gpu(w, 0, args.steps, args.warmup, args.stage_steps)
    rate = N * args.steps / elapsed
    dom = max(range(4), key=lambda s: stage_ms[s])
    dom_bytes = stage_bytes(dom + 1, 0) * N
    achieved = dom_bytes / (stage_ms[dom] * 1e-3) / 1e9
    step_alg = sum(stage_bytes(s, 0) for s in range(1, 5)) * N
    out = {
        "metric": "RK4 grid-point updates/s (FP64, fused 13-point stencil stages)",
        "value": rate,
        "unit": "grid-point-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"single solve {args.n}^3 on [-16,16]^3, mu^2=2, lambda=1, "
                               f"8 seeded Gaussians, dt=0.005, FP64",
                   "grid": [args.n] * 3, "dt": w.dt, "precision": "f64"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": f"stage {dom + 1}",
                     "stage_ms": stage_ms,
                     "step_alg_GBps": step_alg / (elapsed / args.steps) / 1e9,
                     "step_frac": step_alg / (elapsed / args.steps) / 1e9 / HBM_PEAK_GBS},
        "state_check": {"linf_phi": diag["linf_phi"], "nonfinite": diag["nonfinite"]},
    }
    if args.forms:
        e32, ms32, _ = run_gpu(w, 1, args.steps, args.warmup, args.stage_steps)
        out["forms"] = {"f32c": {"value": N * args.steps / e32, "speedup_vs_f64": elapsed / e32,
                                 "stage_ms": ms32}}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
