"""Benchmark: RK4 grid-point updates/s of the fused FP64 stage kernels.

Workload: 256^3 interior points on [-16,16]^3 (h = 0.125), mu^2 = 2,
lambda = 1, phi0 = 8 seeded Gaussians (seed 0), phi1 = 0, dt = 0.005 (the
2000-step single-solve configuration).  A "step" is one full RK4 step (2 fused
stage-pair kernels + the step-counter tick) over the whole grid; inputs are
resident in HBM before timing starts.

Prints ONE JSON line.  Extra objects:
  roofline      -- dominant kernel (stage pair 3+4: 6 field passes = 48 B/point
                   FP64) algorithmic bytes / its average duration, from HIP
                   events on the solver's stream, against 8 TB/s;
  cpu_baseline  -- the FP64 CPU oracle on a bounded number of steps of the
                   same grid, on this host's cores;
  forms         -- the same step rate for the FP32c form (same grid) when
                   --forms is given;
  hbm_probe     -- with --probe, the streamed-bandwidth ceiling measured by
                   the library's copy and 5-read/2-write probe kernels.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per interior point for each kernel of one RK4 step
# (field passes x element size).  Stage-pair scheme: kernel A (stages 1+2)
# reads Y_phi, Y_psi and writes G1, G2 (4 passes); kernel B (stages 3+4)
# reads Y_phi, Y_psi, G1, G2 and writes Y'_phi, Y'_psi (6 passes); FP32c adds
# the read and write of the two FP32 low parts in kernel B (16 B).
KERNEL_BYTES = {0: [32, 48], 1: [16, 40]}
# the per-stage (19-pass) scheme: 3, 4, 5, 7 passes; FP32c + 16 B in stage 4
STAGEWISE_BYTES = {0: [24, 32, 40, 56], 1: [12, 16, 20, 44]}


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
    ap.add_argument("--probe", action="store_true",
                    help="also measure the streamed-HBM ceiling (copy and 5-read/2-write probes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solver has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import synth_inputs as si
    w = si.config2(n=args.n)
    N = w.points
    elapsed, stage_ms, diag = run_gpu(w, 0, args.steps, args.warmup, args.stage_steps)
    stage_ms = stage_ms[:2]
    rate = N * args.steps / elapsed
    dom = max(range(2), key=lambda s: stage_ms[s])
    dom_bytes = KERNEL_BYTES[0][dom] * N
    achieved = dom_bytes / (stage_ms[dom] * 1e-3) / 1e9
    step_alg = sum(KERNEL_BYTES[0]) * N
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
                     "kernel": ["pair_kernel stages 1+2", "pair_kernel stages 3+4"][dom],
                     "kernel_ms": stage_ms,
                     "bytes_per_point": KERNEL_BYTES[0],
                     "step_alg_GBps": step_alg / (elapsed / args.steps) / 1e9,
                     "step_frac": step_alg / (elapsed / args.steps) / 1e9 / HBM_PEAK_GBS},
        "state_check": {"linf_phi": diag["linf_phi"], "nonfinite": diag["nonfinite"]},
    }
    if args.forms:
        e32, ms32, _ = run_gpu(w, 1, args.steps, args.warmup, args.stage_steps)
        out["forms"] = {"f32c": {"value": N * args.steps / e32, "speedup_vs_f64": elapsed / e32,
                                 "kernel_ms": ms32[:2],
                                 "step_alg_GBps": sum(KERNEL_BYTES[1]) * N / (e32 / args.steps) / 1e9}}
    if args.probe:
        from paper_1803_01291_amd import hb
        gib = 1 << 30
        out["hbm_probe"] = {"copy_GBps": hb.hb_probe_bandwidth(0, gib, 20),
                            "read5_write2_GBps": hb.hb_probe_bandwidth(2, gib // 2, 20),
                            "bytes_per_array": [gib, gib // 2]}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
