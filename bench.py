"""Benchmark: right-hand-side evaluations per second of the BS5-stepped
pseudo-spectral Navier--Stokes solver on one MI355X.

Workload: 3D Taylor--Green vortex at 256^3, nu = 1/1600, FFTs and nonlinear
term in FP32, state / stage combinations / error norm in FP64.  One step is
one BS5 attempt through the C ABI (seven right-hand sides, the stage
combinations, the fused error-norm + diagnostics reduction, the controller's
accept test and the commit), with the inputs already resident in HBM.
value = right-hand-side evaluations per second over the whole timed region.

The dominant kernel's roofline figure divides its algorithmic bytes per launch
(reads + writes of the pruned pass model) by its average
launch duration, measured with HIP events recorded on the solver's stream
inside the timed region.  The CPU baseline times the FP64 NumPy oracle's
right-hand side at the same size on the host, on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rhs256_fp32_hbm_traffic.txt")
TRAFFIC_SOURCES = ["fft_core.hpp", "pass_common.hpp", "rhs3d.hip"]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE /
    WRITE_SIZE summary (copy-calibrated), or None when the kernel sources have
    changed since the counters were taken."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1810_10197_amd", "csrc", f), "rb").read())
    text = open(TRAFFIC_FILE).read().splitlines()
    sha = [l.split()[1] for l in text if l.startswith("source_sha256:")]
    if not sha or sha[0] != h.hexdigest()[:16]:
        return None
    for l in text:
        parts = l.split()
        if len(parts) == 3 and parts[0] == "traffic_bytes" and parts[1] == kernel:
            return float(parts[2])
    return None


def pass_bytes(n, fp64=False):
    """Algorithmic HBM bytes per launch of each right-hand-side pass (one
    member): reads + writes of the retained-mode pencil model.  cb = bytes per
    complex value in the rhs precision, 16 bytes per FP64 state value."""
    K = (n - 1) // 3
    Kf, Kx = 2 * K + 1, K + 1
    mr = Kf * Kf * Kx
    c1 = Kx * Kf * n
    c2 = Kx * n * n
    cb = 16 if fp64 else 8
    return {
        "zinv": 3 * mr * 16 + 6 * c1 * cb,
        "yinv": 6 * c1 * cb + 6 * c2 * cb,
        "xpass": 6 * c2 * cb + 3 * c2 * cb,
        "yfwd": 3 * c2 * cb + 3 * c1 * cb,
        "zfwd": 3 * c1 * cb + 3 * mr * 16 + 3 * mr * 16,
    }


def cpu_baseline(n, nu, budget_s):
    """Oracle RHS/s on the host: repeat the FP64 NumPy right-hand side until
    the time budget is used (at least one evaluation)."""
    import numpy as np
    from oracle import spectral
    from paper_1810_10197_amd import inputs
    u = inputs.tgv3d(n)
    t0 = time.perf_counter()
    count = 0
    while True:
        spectral.rhs_ns3d(u, nu)
        count += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": count / dt, "unit": "RHS evals/s", "cores": 1, "kind": "oracle",
            "sample": "%d FP64 NumPy right-hand sides of the %d^3 Taylor-Green field "
                      "(%.1f s; numpy.fft is single-threaded)" % (count, n, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--dt", type=float, default=0.005)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--variants", default=None,
                    help="comma-separated launch variants of the 5 passes (skips the autotuner)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (HBM counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how the solver would shard)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        nbytes = args.calibrate_copy * 1024 * 1024
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "copies": 3}))
        return
    from paper_1810_10197_amd import inputs, ns

    n, nu = args.n, 1.0 / 1600
    atol = rtol = 1e-6
    s = ns.Solver(dim=3, n=n, batch=1, nu=nu, rhs_precision=args.prec)
    s.set_state(inputs.tgv3d(n)[None])
    if args.variants:
        tune_variants = s.tune([int(v) for v in args.variants.split(",")])
        tune_ms = __import__("numpy").zeros((5, 4))
    else:
        tune_variants, tune_ms = s.autotune(reps=3)
    for _ in range(args.warmup):
        s.step_bs5(args.dt, atol, rtol)
    # pure right-hand-side rate (context): f(u_n) into the cached stage
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nr = 20
    for _ in range(nr):
        s.refresh_rhs()
    torch.cuda.synchronize()
    rhs_only = nr / (time.perf_counter() - t0)

    torch.cuda.synchronize()
    s.profile_start()
    t0 = time.perf_counter()
    rejected = 0
    for _ in range(args.steps):
        st, _ = s.step_bs5(args.dt, atol, rtol)
        rejected += int(st == ns.NS_STEP_REJECTED)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = s.profile_stop()
    s.close()

    rhs_evals = 7 * args.steps
    value = rhs_evals / elapsed
    fp64 = args.prec == "fp64"
    pb = pass_bytes(n, fp64)
    per_kernel = {}
    for name in ["zinv", "yinv", "xpass", "yfwd", "zfwd", "combine", "reduce"]:
        ms, cnt = prof[name]
        if cnt:
            per_kernel[name] = {"avg_us": 1000.0 * ms / cnt, "launches": cnt}
            if name in pb:
                per_kernel[name]["gbs"] = pb[name] / (ms / cnt * 1e-3) / 1e9
    rhs_passes = ["zinv", "yinv", "xpass", "yfwd", "zfwd"]
    dom = max(rhs_passes, key=lambda k: per_kernel[k]["avg_us"])
    achieved = per_kernel[dom]["gbs"]
    rhs_ms = sum(per_kernel[k]["avg_us"] for k in rhs_passes) / 1000.0
    model_bytes = sum(pb.values())
    out = {
        "metric": "RHS evals/s at 256^3 (BS5 step, FP32 RHS / FP64 state)",
        "value": value,
        "unit": "RHS evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if not fp64 else "f64",
        "data": "synthetic",
        "config": {"workload": "3D Taylor-Green vortex %d^3, nu=1/1600, BS5 attempts at "
                               "h=%g, atol=rtol=1e-6, %s FFTs, FP64 state" % (n, args.dt, args.prec),
                   "n": n, "batch": 1},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom) if (n == 256 and not fp64) else None,
                     "kernel": dom},
        "rhs_model_gb": model_bytes / 1e9,
        "rhs_passes_ms": rhs_ms,
        "rhs_model_gbs": model_bytes / (rhs_ms * 1e-3) / 1e9,
        "rhs_only_per_s": rhs_only,
        "rejected_steps": rejected,
        "autotune": {"variants": tune_variants,
                     "ms": [[round(x, 4) for x in row] for row in tune_ms.tolist()]},
        "kernels": per_kernel,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n, nu, args.cpu_budget)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
