"""Benchmark: right-hand-side evaluations per second of the BS5-stepped
pseudo-spectral Navier--Stokes solver on one MI355X.

Default workload: 3D Taylor--Green vortex at 256^3, nu = 1/1600, FFTs and
nonlinear term in FP32, state / stage combinations / error norm in FP64.  One
step is one BS5 attempt through the C ABI (seven right-hand sides, the stage
combinations, the fused error-norm + diagnostics reduction, the controller's
accept test and the commit), with the inputs already resident in HBM.
value = right-hand-side evaluations per second over the whole timed region
(member evaluations for an ensemble).  --workload ensemble runs 128 members at
64^3 (Taylor--Green and random-phase fields, nu log-uniform), --workload rt2d
the 2D Boussinesq Rayleigh--Taylor problem at 1024^2.

The dominant kernel's roofline figure divides its algorithmic bytes per launch
(reads + writes of the pruned pass model in pass_bytes) by its average launch
duration, from HIP events recorded around every launch on the launch's stream
in a separate run of the same steps (the events themselves cost about a tenth
of the step time, so the timed region that gives value runs without them; a
second events run brackets the y/x/y phase as a whole for the right-hand
side's wall time).  The CPU baseline times the FP64 NumPy oracle's
right-hand side at the same size on the host, on a bounded sample, and the
oracle's time to solution of the 32^3 Taylor-Green runs.  The default
workload also reports the time to a 1e-6 relative energy error at T = 10
(FP64 RK4 against BS5 with an FP32 right-hand side, with and without the
trained proposer; about a minute, --no-tts skips it).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rhs256_fp32_hbm_traffic.txt")
TRAFFIC_SOURCES = ["fft_core.hpp", "pass_common.hpp", "rhs3d_kernels.hpp", "rhs3d.hip"]


def measured_traffic(kernel, launches_per_rhs=1.0):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE /
    WRITE_SIZE summary (copy-calibrated bytes per right-hand side, divided by
    this run's launches per right-hand side), or None when the kernel sources
    have changed since the counters were taken."""
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
        if len(parts) == 3 and parts[0] == "traffic_per_rhs" and parts[1] == kernel:
            return float(parts[2]) / launches_per_rhs
    return None


# slab schedule variants that alternate two streams -> the same slab size on one stream
ONE_STREAM_SLAB = {5: 1, 6: 2, 7: 3, 8: 4, 11: 9, 12: 10}


def pass_bytes(n, fp64=False, stage32=False):
    """Algorithmic HBM bytes of each right-hand-side pass per evaluation (one
    member): reads + writes of the retained-mode pencil model.  cb = bytes per
    complex value in the rhs precision; the state is read in FP64 (16 bytes),
    or (stage32: a stage of an FP32 step, whose input is written in FP32) in
    FP32, and f is written in FP64 -- in a BS5 step 6 of the 7 stage
    evaluations also write f's FP32 copy, counted here on average.  The y/x/y
    passes run in slabs of z planes; one launch covers its slab's share."""
    K = (n - 1) // 3
    Kf, Kx = 2 * K + 1, K + 1
    mr = Kf * Kf * Kx
    c1 = Kx * Kf * n
    c2 = Kx * n * n
    cb = 16 if fp64 else 8
    sb = 8 if stage32 else 16
    return {
        "zinv": 3 * mr * sb + 6 * c1 * cb,
        "yinv": 6 * c1 * cb + 6 * c2 * cb,
        "xpass": 6 * c2 * cb + 3 * c2 * cb,
        "yfwd": 3 * c2 * cb + 3 * c1 * cb,
        "zfwd": 3 * c1 * cb + 3 * mr * sb + 3 * mr * 16 + (3 * mr * 8 * 6 // 7 if stage32 else 0),
    }


def pass_bytes_2d(n, fp64=False, stage32=False):
    """Same for the 2D Boussinesq passes (state u, v, rho; four transformed
    fields): Q1 y-inverse, Q2 x-pass, Q3 y-forward + epilogue; stage32 as in
    pass_bytes (the stage input read in FP32 by Q1 and Q3, f's FP32 copy
    written by Q3 in 6 of 7 evaluations)."""
    K = (n - 1) // 3
    Kf, Kx = 2 * K + 1, K + 1
    mr = Kf * Kx
    cb = 16 if fp64 else 8
    sb = 8 if stage32 else 16
    col = 4 * n * Kx * cb
    return {"zinv": 3 * mr * sb + col, "xpass": 2 * col,
            "zfwd": col + 3 * mr * sb + 3 * mr * 16 + (3 * mr * 8 * 6 // 7 if stage32 else 0)}


def hbm_copy_gbs(nbytes=1 << 30, reps=10):
    """What a plain device-to-device copy streams on this GPU: bytes read plus
    bytes written per second over `reps` copies of a 1 GiB buffer (torch's
    copy kernel, timed with events on torch's stream)."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    del a, b
    return 2.0 * nbytes * reps / (ms * 1e-3) / 1e9


def host_cpu():
    """CPU model name and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "nproc": usable, "logical_cpus": os.cpu_count()}


def c1_oracle_time_to_solution():
    """The oracle on the 32^3 Taylor-Green vortex (nu = 1/1600) to T = 1:
    RK4 at dt = 0.01 and BS5 with the Sec. 2.2.1 controller at
    atol = rtol = 1e-8 (h0 = 0.01); wall time and right-hand sides."""
    from oracle import control, spectral
    from paper_1810_10197_amd import inputs
    n, nu = 32, 1.0 / 1600
    u0 = inputs.tgv3d(n)
    rhs = lambda u: spectral.rhs_ns3d(u, nu)
    t0 = time.perf_counter()
    _, steps = control.rk4_fixed(rhs, u0, 1.0, 0.01)
    rk4 = {"wall_s": time.perf_counter() - t0, "n_rhs": 4 * steps}
    t0 = time.perf_counter()
    ref = control.integrate(rhs, u0, 1.0, 0.01, 1e-8, 1e-8)
    bs5 = {"wall_s": time.perf_counter() - t0, "n_rhs": ref["n_rhs"], "n_accept": ref["n_accept"],
           "n_reject": ref["n_reject"]}
    return {"rk4_dt0.01": rk4, "bs5_tol1e-8": bs5}


def c1_gpu_time_to_solution(ns, inputs):
    """The same two C1 runs on the GPU (FP64 right-hand side and state)."""
    import torch
    n, nu = 32, 1.0 / 1600
    u0 = inputs.tgv3d(n)[None]
    s = ns.Solver(dim=3, n=n, nu=nu, rhs_precision="fp64")
    s.set_state(u0)
    s.step_rk4(0.01)                          # first-launch costs outside the timing
    s.set_state(u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(100):
        s.step_rk4(0.01)
    torch.cuda.synchronize()
    rk4 = {"wall_s": time.perf_counter() - t0, "n_rhs": 400}
    s.set_state(u0)
    s.set_time(0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = s.integrate(1.0, 0.01, 1e-8, 1e-8)[0]
    torch.cuda.synchronize()
    bs5 = {"wall_s": time.perf_counter() - t0, "n_rhs": st["n_rhs"], "n_accept": st["n_accept"],
           "n_reject": st["n_reject"]}
    s.close()
    return {"rk4_dt0.01": rk4, "bs5_tol1e-8": bs5}


def cpu_baseline(n, nu, budget_s, padded=False):
    """Oracle RHS/s on the host: repeat the FP64 NumPy right-hand side (2/3
    rule, or padded: 3/2 rule) until the time budget is used (at least one
    evaluation); and the oracle's time to solution of the 32^3 Taylor-Green
    runs (RK4 at dt = 0.01 and adaptive BS5 at 1e-8, to T = 1)."""
    from oracle import spectral
    from paper_1810_10197_amd import inputs
    u = inputs.tgv3d(n)
    rhs = spectral.rhs_ns3d_padded if padded else spectral.rhs_ns3d
    t0 = time.perf_counter()
    count = 0
    while True:
        rhs(u, nu)
        count += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    rate = count / dt
    # the small grids of the workload family (a second of work each)
    small = {}
    for m in (32, 64):
        um = inputs.tgv3d(m)
        t1, c = time.perf_counter(), 0
        while c < 3 or time.perf_counter() - t1 < 1.0:
            rhs(um, nu)
            c += 1
        small["%d^3" % m] = c / (time.perf_counter() - t1)
    return {"value": rate, "unit": "RHS evals/s", "cores": 1, "kind": "oracle",
            "sample": "%d FP64 NumPy right-hand sides (%s rule) of the %d^3 Taylor-Green field "
                      "(%.1f s; numpy.fft is single-threaded, so one core)"
                      % (count, "3/2" if padded else "2/3", n, dt),
            "host": host_cpu(),
            "rhs_per_s_small_grids": small,
            "c1_time_to_solution": c1_oracle_time_to_solution(),
            "c2_to_t1_rk4_dt0.01_estimate_s": 400 / rate,
            "c2_note": "the %d^3 run to T = 1 (RK4, dt = 0.01: 400 right-hand sides) estimated from the "
                       "measured rate, not run" % n}


def quadratic_interpolant(tref, yref):
    """Reference curve of the Re = 280 test (Sec. 3.1): between samples
    (tref, yref) of the reference run, the quadratic through the three samples
    nearest to t (Lagrange form)."""
    import numpy as np
    tref = np.asarray(tref, dtype=float)
    yref = np.asarray(yref, dtype=float)
    if len(tref) < 3:
        raise ValueError("a quadratic needs three samples")

    def at(t):
        j = int(np.clip(np.searchsorted(tref, t) - 1, 1, len(tref) - 2))
        x, y = tref[j - 1:j + 2], yref[j - 1:j + 2]
        return (y[0] * (t - x[1]) * (t - x[2]) / ((x[0] - x[1]) * (x[0] - x[2]))
                + y[1] * (t - x[0]) * (t - x[2]) / ((x[1] - x[0]) * (x[1] - x[2]))
                + y[2] * (t - x[0]) * (t - x[1]) / ((x[2] - x[0]) * (x[2] - x[1])))
    return at


def max_deviation(ts, ys, ref):
    """An arm's error in the Re = 280 test: max |y(t) - ref(t)| over the arm's
    own output times (inf if any value is not finite)."""
    d = [abs(y - ref(t)) for t, y in zip(ts, ys)]
    return float(max(d)) if d and all(math.isfinite(x) for x in d) else float("inf")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def _initial_weights(ns, seed):
    import numpy as np
    rng = np.random.default_rng(seed)
    w0 = np.zeros(ns.NS_MLP_NWEIGHTS, dtype=np.float32)
    lim1, lim2, lim3 = np.sqrt(6.0 / 84), np.sqrt(6.0 / 128), np.sqrt(6.0 / 65)
    w0[:1280] = rng.uniform(-lim1, lim1, 1280)                 # W1 (64 x 20)
    w0[1344:1344 + 4096] = rng.uniform(-lim2, lim2, 4096)      # W2 (64 x 64)
    w0[5504:5568] = rng.uniform(-lim3, lim3, 64)               # W3 (1 x 64)
    w0[ns.NS_MLP_NPARAM + 20:] = 1.0                           # feature scale
    return w0


def collect_rows(ns, fields, nus, n, t_end, tols, h0=1e-3, chunks=1):
    """(features, label) rows of accepted steps of Sec. 2.2.1-controlled
    runs of the given members (FP32 right-hand side)."""
    import numpy as np
    import torch
    B = len(nus)
    s = ns.Solver(dim=3, n=n, batch=B, nu=nus, rhs_precision="fp32")
    s.mlp_set_weights(np.zeros(ns.NS_MLP_NWEIGHTS, dtype=np.float32))
    s.mlp_collect(True)
    nrhs = 0
    t0 = time.perf_counter()
    for tol in tols:
        s.set_state(fields)
        s.set_time(np.zeros(B))
        torch.cuda.synchronize()
        h = h0
        for c in range(chunks):
            st = s.integrate(t_end * (c + 1) / chunks, h, tol, tol, resume=c > 0)
            h = float(np.min([x["h_next"] for x in st]))
            nrhs += sum(x["n_rhs"] for x in st)
        log("collect n=%d B=%d tol=%g: %d rows" % (n, B, tol, s.mlp_rows(0)[2]))
    x, y, _ = s.mlp_rows()
    s.close()
    return x, y, nrhs, time.perf_counter() - t0


def train_proposer(ns, inputs, members=128, n=64, t_end=2.0, tols=(1e-5, 1e-7, 1e-9),
                   iters=3000, batch=256, seed=1810, target=None):
    """Proposer training: rows from the mixed ensemble (Taylor-Green and
    random-phase fields, nu log-uniform in [1e-3, 1e-2]) integrated with the
    Sec. 2.2.1 controller at several tolerances, plus (target = (n_list,
    nu, T, tols)) runs of the target problem at reduced resolution; then Adam
    on the GPU.  Returns (weights, info)."""
    import numpy as np
    fields, nus = inputs.ensemble_members(members, n)
    xs, ys, nrhs, secs = collect_rows(ns, fields, nus, n, t_end, tols)
    info = {"ensemble": {"members": members, "n": n, "t_end": t_end, "tolerances": list(tols),
                         "rows": int(len(ys)), "member_rhs_evals": nrhs, "collect_s": secs,
                         "member_rhs_per_s": nrhs / secs}}
    X, Y = [xs], [ys]
    if target:
        tn, tnu, tT, ttols = target
        for nn in tn:
            x2, y2, r2, s2 = collect_rows(ns, inputs.tgv3d(nn)[None], [tnu], nn, tT, ttols,
                                          chunks=int(math.ceil(tT)))
            X.append(x2)
            Y.append(y2)
            info["target_n%d" % nn] = {"rows": int(len(y2)), "collect_s": s2}
    X = np.concatenate(X)
    Y = np.concatenate(Y)
    s = ns.Solver(dim=3, n=8, nu=0.01, rhs_precision="fp32")
    s.mlp_set_weights(_initial_weights(ns, seed))
    s.mlp_push_rows(X, Y)
    s.mlp_fit_stats()
    t1 = time.perf_counter()
    loss0 = s.mlp_train(1, batch, 1e-3, seed)
    loss = loss0
    for k in range(iters // 500):
        loss = s.mlp_train(500, batch, 1e-3, seed + 1 + k)
        log("train iter %d loss %.5f" % ((k + 1) * 500, loss))
    w = s.mlp_get_weights()
    s.close()
    info.update({"rows": int(len(Y)), "train_iters": iters, "train_s": time.perf_counter() - t1,
                 "loss_first": loss0, "loss_last": loss})
    return w, info


def study_mlp(args):
    """What the trained proposer gains: held-out ensemble members integrated
    with the Sec. 2.2.1 controller and with the proposer, same tolerance;
    rejections, right-hand sides, wall time and final-state error against a
    tight-tolerance run."""
    import numpy as np
    import torch
    from paper_1810_10197_amd import inputs, ns
    w, info = train_proposer(ns, inputs, members=args.members, n=64, iters=args.iters)
    n, B = 64, 32
    fields, nus = inputs.ensemble_members(B + args.members, n)
    fields, nus = fields[args.members:], nus[args.members:]       # held out
    res = {"training": info}
    ref = ns.Solver(dim=3, n=n, batch=B, nu=nus, rhs_precision="fp64")
    ref.set_state(fields)
    ref.integrate(2.0, 1e-3, 1e-12, 1e-12)
    uref = ref.get_state().cpu().numpy()
    ref.close()
    for tol in (1e-5, 1e-7):
        for ctl in ("pi", "mlp"):
            s = ns.Solver(dim=3, n=n, batch=B, nu=nus, rhs_precision="fp32")
            s.mlp_set_weights(w)
            s.set_state(fields)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = s.integrate(2.0, 1e-3, tol, tol, controller=ctl)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            u = s.get_state().cpu().numpy()
            s.close()
            err = float(np.max(np.linalg.norm((u - uref).reshape(B, -1), axis=1) /
                               np.linalg.norm(uref.reshape(B, -1), axis=1)))
            res["%s_tol%g" % (ctl, tol)] = {
                "n_rhs": int(sum(x["n_rhs"] for x in st)),
                "n_accept": int(sum(x["n_accept"] for x in st)),
                "n_reject": int(sum(x["n_reject"] for x in st)),
                "wall_s": dt, "max_rel_l2_err": err}
            log("%s tol=%g: %s" % (ctl, tol, res["%s_tol%g" % (ctl, tol)]))
    if args.weights:
        np.save(args.weights, w)
    print(json.dumps({"study": "proposer_gain", "results": res}))


def study_e1(args):
    """Sec. 3.1 first test: Taylor-Green vortex at Re = 280 (nu = 1/280), 64^3,
    T = 9.4, FP64 throughout.  Reference eps(t) from RK4 at dt = 1e-4 (sampled
    every 5 steps, piecewise-quadratic interpolation between samples); each
    arm's error is max |eps - eps_ref| over its step times, its cost the number
    of right-hand sides.  Arms: RK4 and BS5 at fixed steps, BS5 and DP5 with
    the Sec. 2.2.1 controller (the attempt loop runs on the host here so that
    eps is read after every accepted step)."""
    import numpy as np
    import torch
    from paper_1810_10197_amd import inputs, ns
    n, nu, T = args.n if args.n != 256 else 64, 1.0 / 280, 9.4
    u0 = inputs.tgv3d(n)[None]
    out = {"study": "tgv_re280", "n": n, "T": T, "nu": nu, "precision": "fp64", "dealias": args.dealias}

    def solver():
        s = ns.Solver(dim=3, n=n, nu=nu, rhs_precision="fp64", dealias=args.dealias)
        s.set_state(u0)
        return s

    def eps_now(s):
        return float(s.diagnostics()[1][0])

    def rk4_run(dt, every=1):
        s = solver()
        steps = max(1, int(math.ceil(T / dt - 1e-9)))
        ts, es = [0.0], [eps_now(s)]
        for i in range(steps):
            h = dt if i < steps - 1 else T - (steps - 1) * dt
            s.step_rk4(h)
            if (i + 1) % every == 0 or i == steps - 1:
                ts.append(min(T, (i + 1) * dt))
                es.append(eps_now(s))
            if (i + 1) % 20000 == 0:
                log("rk4 dt=%g step %d/%d" % (dt, i + 1, steps))
        s.close()
        return np.array(ts), np.array(es), 4 * steps

    t0 = time.perf_counter()
    tref, eref, _ = rk4_run(1e-4, every=5)
    out["ref_wall_s"] = time.perf_counter() - t0
    log("reference: %d samples, %.1f s" % (len(tref), out["ref_wall_s"]))

    eps_ref = quadratic_interpolant(tref, eref)

    def err_of(ts, es):
        return max_deviation(ts, es, eps_ref)

    out["rk4"] = []
    for dt in args.e1_dts:
        ts, es, nr = rk4_run(dt)
        out["rk4"].append({"dt": dt, "n_rhs": nr, "max_eps_err": err_of(ts, es)})
        log("rk4 dt=%g rhs %d err %.3e" % (dt, nr, out["rk4"][-1]["max_eps_err"]))

    out["bs5_fixed"] = []
    for dt in args.e1_dts:
        s = solver()
        steps = max(1, int(math.ceil(T / dt - 1e-9)))
        ts, es = [0.0], [eps_now(s)]
        for i in range(steps):
            h = dt if i < steps - 1 else T - (steps - 1) * dt
            s.step_bs5(h, 1.0, 1.0, force=True)
            ts.append(min(T, (i + 1) * dt))
            es.append(eps_now(s))
        s.close()
        out["bs5_fixed"].append({"dt": dt, "n_rhs": 7 * steps + 1, "max_eps_err": err_of(ts, es)})
        log("bs5 fixed dt=%g err %.3e" % (dt, out["bs5_fixed"][-1]["max_eps_err"]))

    def adaptive(method, tol, h0=0.01):
        # Sec. 2.2.1: fac = 0.8 err^(-1/5) clamped to [0.01, 2] (1 for the step
        # accepted right after a rejection), accept iff err <= 1, last step
        # clipped to T
        s = solver()
        step = s.step_bs5 if method == "bs5" else s.step_dp5
        per = 7 if method == "bs5" else 6
        t, h, prev_rej = 0.0, h0, False
        ts, es = [0.0], [eps_now(s)]
        att = rej = consec = 0
        while t < T and consec < 50:
            last = h >= T - t
            hc = T - t if last else h
            _, errs = step(hc, tol, tol)
            err = float(errs[0])
            att += 1
            ok = math.isfinite(err) and err <= 1.0
            fmax = 1.0 if (ok and prev_rej) else 2.0
            fac = 0.01 if not math.isfinite(err) else (fmax if err == 0.0 else
                                                       min(fmax, max(0.01, 0.8 * err ** -0.2)))
            if ok:
                t = T if last else t + hc
                ts.append(t)
                es.append(eps_now(s))
                prev_rej = False
                consec = 0
            else:
                rej += 1
                consec += 1
                prev_rej = True
            h = hc * fac
        s.close()
        return {"tol": tol, "n_rhs": per * att + 1, "attempts": att, "rejected": rej,
                "max_eps_err": err_of(ts, es) if t >= T else float("inf")}

    for method in ("bs5", "dp5"):
        key = "%s_adaptive" % method
        out[key] = []
        for tol in args.e1_tols:
            r = adaptive(method, tol)
            out[key].append(r)
            log("%s tol=%g rhs %d rej %d err %.3e" % (method, tol, r["n_rhs"], r["rejected"],
                                                       r["max_eps_err"]))

    # RHS of RK4 needed for the error each adaptive run reached (log-log
    # interpolation along the RK4 sweep), and the ratio to the adaptive count
    rk = sorted(out["rk4"], key=lambda r: r["max_eps_err"])
    le = np.log([r["max_eps_err"] for r in rk])
    lr = np.log([r["n_rhs"] for r in rk])
    for key in ("bs5_adaptive", "dp5_adaptive", "bs5_fixed"):
        for r in out[key]:
            e = r["max_eps_err"]
            if le[0] <= math.log(e) <= le[-1]:
                r["rk4_rhs_same_err"] = float(np.exp(np.interp(math.log(e), le, lr)))
                r["rk4_over_this"] = r["rk4_rhs_same_err"] / r["n_rhs"]
    print(json.dumps(out))


def study_problem(args):
    """Time to solution on the other workloads, FP32 right-hand side, FP64
    state.  rt2d: the 2D Boussinesq Rayleigh-Taylor problem at 1024^2 to
    T = 4 (Ri = 0.5, nu = kappa = 1e-4): fixed-step RK4 against BS5 with the
    Sec. 2.2.1 controller and with the proposer.  hit512: forced isotropic
    turbulence at 512^3 (nu = 0.005, energy held at 0.125 by the rescale of
    0 < |k| <= 2) to T = 5: BS5 with the controller against BS5 with the
    proposer.  The error is the relative L2 of the final state against an
    FP64 reference (RK4 at dt = 1e-4 for rt2d, BS5 at tol 1e-10 for hit512),
    and the relative error of the kinetic energy.  An FP64-RHS BS5 arm shows
    the method's own error: the Rayleigh-Taylor flow is unstable, so FP32
    rounding in the right-hand side grows with the instability.  The proposer
    is trained on the ensemble rows plus the problem itself at reduced
    resolution (weighted ten times)."""
    import numpy as np
    import torch
    from paper_1810_10197_amd import inputs, ns
    pr = args.problem
    if pr == "rt2d":
        n, T, nu, dim = 1024, 4.0, 1e-4, 2
        kw = dict(dim=2, scalar=1, ri=0.5, kappa=1e-4)
        state = lambda nn: inputs.rayleigh_taylor2d(nn)[None]
        train_ns, train_T, h0 = (256, 512), 4.0, 1e-3
    else:
        n, T, nu, dim = 512, 5.0, 0.005, 3
        kw = dict(dim=3, force_kf=2.0, force_e0=0.125)
        state = lambda nn: inputs.random_isotropic(nn, 1810)[None]
        train_ns, train_T, h0 = (64, 128), 5.0, 1e-3
    out = {"study": "time_to_solution", "problem": pr, "n": n, "T": T, "nu": nu}

    def solver(prec, nn=n):
        s = ns.Solver(n=nn, nu=nu, rhs_precision=prec, **kw)
        s.set_state(state(nn))
        return s

    def rel_l2(a, b):
        return float(np.sqrt(np.sum(np.abs(a - b) ** 2) / np.sum(np.abs(b) ** 2)))

    def energy(u):
        # kinetic energy of the velocity components (half-spectrum weights)
        w = np.full(u.shape[1:], 2.0)
        w[..., 0] = 1.0
        return 0.5 * float(np.sum(w * np.abs(u[:dim]) ** 2))

    def errs(u, uref):
        return {"rel_l2_err": rel_l2(u, uref), "rel_energy_err": abs(energy(u) - energy(uref)) / energy(uref)}

    def rk4_run(dt, prec):
        s = solver(prec)
        steps = max(1, int(math.ceil(T / dt - 1e-9)))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            s.step_rk4(dt if i < steps - 1 else T - (steps - 1) * dt)
            if (i + 1) % 5000 == 0:
                log("rk4 %s dt=%g step %d/%d" % (prec, dt, i + 1, steps))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        u = s.get_state().cpu().numpy()[0]
        s.close()
        return u, wall, 4 * steps

    def bs5_run(tol, prec, ctl, w=None, budget_s=150.0):
        # quarter-unit chunks (progress lines between them); a run that
        # exceeds its wall budget stops early and is reported as such
        s = solver(prec)
        if w is not None:
            s.mlp_set_weights(w)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h, tot = h0, {"n_rhs": 0, "n_accept": 0, "n_reject": 0}
        nch = int(math.ceil(4 * T - 1e-9))
        for c in range(nch):
            st = s.integrate(min(T, 0.25 * (c + 1)), h, tol, tol, controller=ctl, resume=c > 0)[0]
            h = st["h_next"]
            for k in tot:
                tot[k] += st[k]
            log("%s %s tol=%g t=%g rhs %d rej %d" % (ctl, prec, tol, st["t"], tot["n_rhs"], tot["n_reject"]))
            if time.perf_counter() - t0 > budget_s and c < nch - 1:
                tot["stopped_at_t"] = st["t"]
                break
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        u = s.get_state().cpu().numpy()[0]
        s.close()
        return u, wall, tot

    t0 = time.perf_counter()
    if pr == "rt2d":
        uref, _, _ = rk4_run(1e-4, "fp64")
    else:
        uref, _, _ = bs5_run(1e-10, "fp64", "pi")
    out["ref_wall_s"] = time.perf_counter() - t0
    log("reference done (%.1f s)" % out["ref_wall_s"])
    if pr == "rt2d":
        out["rk4_fp64"] = []
        for dt in args.rk4_dts:
            u, wall, nr = rk4_run(dt, "fp64")
            out["rk4_fp64"].append({"dt": dt, "wall_s": wall, "n_rhs": nr, **errs(u, uref)})
            log("rk4 fp64 dt=%g err %.3e / energy %.3e wall %.2f s" % (dt, out["rk4_fp64"][-1]["rel_l2_err"],
                                                                     out["rk4_fp64"][-1]["rel_energy_err"], wall))
    # proposer: ensemble rows plus the problem at reduced resolution
    fields, nus = inputs.ensemble_members(args.members, 64)
    xs, ys, _, _ = collect_rows(ns, fields, nus, 64, 2.0, (1e-5, 1e-7, 1e-9))
    X, Y = [xs], [ys]
    for nn in train_ns:
        s = solver("fp32", nn)
        s.mlp_set_weights(np.zeros(ns.NS_MLP_NWEIGHTS, dtype=np.float32))
        s.mlp_collect(True)
        for tol in (1e-6, 1e-7, 1e-8):
            s.set_state(state(nn))
            s.set_time(np.zeros(1))
            h = h0
            for c in range(int(math.ceil(train_T - 1e-12))):
                st = s.integrate(min(train_T, c + 1.0), h, tol, tol, resume=c > 0)[0]
                h = st["h_next"]
        x2, y2, _ = s.mlp_rows()
        s.close()
        # the problem's own rows are few next to the ensemble's: weight them
        X += [x2] * 10
        Y += [y2] * 10
        log("collect %s n=%d: %d rows" % (pr, nn, len(y2)))
    X, Y = np.concatenate(X), np.concatenate(Y)
    s = ns.Solver(dim=3, n=8, nu=0.01, rhs_precision="fp32")
    s.mlp_set_weights(_initial_weights(ns, 1810))
    s.mlp_push_rows(X, Y)
    s.mlp_fit_stats()
    loss = s.mlp_train(1, 256, 1e-3, 1810)
    for k in range(args.iters // 500):
        loss = s.mlp_train(500, 256, 1e-3, 1811 + k)
    w = s.mlp_get_weights()
    s.close()
    out["proposer_training"] = {"rows": int(len(Y)), "loss_last": loss}
    for ctl, prec in (("pi", "fp32"), ("mlp", "fp32"), ("pi", "fp64")):
        key = "bs5_%s_%s" % (ctl, prec)
        out[key] = []
        for tol in args.tols:
            u, wall, tot = bs5_run(tol, prec, ctl, w if ctl == "mlp" else None)
            out[key].append({"tol": tol, "wall_s": wall, **tot, **errs(u, uref)})
            r = out[key][-1]
            log("%s tol=%g err %.3e / energy %.3e wall %.2f s rhs %d rej %d" % (
                key, tol, r["rel_l2_err"], r["rel_energy_err"], wall, tot["n_rhs"], tot["n_reject"]))
    print(json.dumps(out))


def rel_l2_fields(u, uref):
    """Per-component relative L2 error of a device state (torch) against a
    device reference."""
    import torch
    out = []
    for c in range(u.shape[1]):
        d = torch.linalg.vector_norm(u[:, c] - uref[:, c]).item()
        r = torch.linalg.vector_norm(uref[:, c]).item()
        out.append(d / max(r, 1e-300))
    return out


def time_to_solution(ns, inputs, n=256, T=10.0, target=1e-6):
    """Metric 2 of the workload: wall time to a relative energy error of
    `target` at T on the Taylor-Green vortex (nu = 1/1600).  Reference: FP64
    RK4 at dt = 1e-3 (E_ref and the state).  Arms: FP64 RK4 at dt = 0.01 and
    0.008 (and, as context, RK4 with an FP32 right-hand side at 0.01); BS5
    with an FP32 right-hand side (FP64 state) at tol 1e-10 with the Sec. 2.2.1
    controller and with the trained proposer; the BS5 FP32 tolerance sweep
    1e-4, 1e-6, 1e-8 with per-field errors against the FP64 reference; and the
    FP32 right-hand side's energy-error floor (BS5 at 1e-11 and 1e-12).  Each
    run is timed from set-state to the final diagnostics."""
    import numpy as np
    import torch
    nu = 1.0 / 1600
    u0 = inputs.tgv3d(n)[None]
    out = {"workload": "3D Taylor-Green vortex %d^3, nu=1/1600, T=%g" % (n, T), "target": target}

    def rk4(dt, prec, keep=False):
        s = ns.Solver(dim=3, n=n, nu=nu, rhs_precision=prec)
        s.set_state(u0)
        steps = max(1, int(math.ceil(T / dt - 1e-9)))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            s.step_rk4(dt if i < steps - 1 else T - (steps - 1) * dt)
        e, _, _ = s.diagnostics()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        u = s.get_state() if keep else None
        s.close()
        return float(e[0]), wall, 4 * steps, u

    t0 = time.perf_counter()
    eref, wref, _, uref = rk4(1e-3, "fp64", keep=True)
    out["E_ref"] = eref
    out["reference"] = "FP64 RK4 dt=1e-3 (%.1f s)" % wref
    log("tts: E_ref(T=%g) = %.15e (%.1f s)" % (T, eref, wref))
    for dt in (0.01, 0.008):
        e, wall, nr, _ = rk4(dt, "fp64")
        out["rk4_fp64_dt%g" % dt] = {"rel_energy_err": abs(e - eref) / eref, "wall_s": wall, "n_rhs": nr}
        log("tts: rk4 fp64 dt=%g err %.2e wall %.2f s" % (dt, abs(e - eref) / eref, wall))
    # context arm: RK4 with the FP32 right-hand side
    e, wall, nr, _ = rk4(0.01, "fp32")
    out["rk4_fp32_dt0.01"] = {"rel_energy_err": abs(e - eref) / eref, "wall_s": wall, "n_rhs": nr}
    log("tts: rk4 fp32 dt=0.01 err %.2e wall %.2f s" % (abs(e - eref) / eref, wall))
    w, info = train_proposer(ns, inputs, iters=3000, members=128,
                             target=((64, 128), nu, T, (1e-7, 1e-8, 1e-9, 1e-10)))
    out["proposer_training"] = {k: info[k] for k in ("rows", "train_iters", "train_s", "loss_first",
                                                      "loss_last")}

    def bs5(tol, ctl, budget_s=60.0, chunk=0.5):
        # chunks of `chunk` time units, each continuing the controller of the
        # previous one (a progress line between); a run whose steps collapse
        # (the unstable loose tolerances of an FP32 right-hand side) is
        # abandoned after budget_s and reported as such
        s = ns.Solver(dim=3, n=n, nu=nu, rhs_precision="fp32")
        s.mlp_set_weights(w)
        s.set_state(u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h, tot, ok = 1e-3, {"n_rhs": 0, "n_accept": 0, "n_reject": 0}, True
        t_now = 0.0
        try:
            for c in range(int(math.ceil(T / chunk - 1e-12))):
                st = s.integrate(min(T, (c + 1) * chunk), h, tol, tol, controller=ctl, resume=c > 0)[0]
                h, t_now = st["h_next"], st["t"]
                for k in tot:
                    tot[k] += st[k]
                log("tts: bs5 %s tol=%g t=%g rhs %d rej %d" % (ctl, tol, t_now, tot["n_rhs"], tot["n_reject"]))
                if time.perf_counter() - t0 > budget_s and t_now < T:
                    ok = False
                    tot["abandoned"] = "after %.0f s at t = %g (step %.2e)" % (time.perf_counter() - t0, t_now, h)
                    break
        except ns.NsError as e:
            ok = False
            tot["failed"] = str(e)
        e, _, _ = s.diagnostics()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        r = {"tol": tol, "wall_s": wall, **tot}
        if ok:
            r["rel_energy_err"] = abs(float(e[0]) - eref) / eref
            r["per_field_rel_l2"] = rel_l2_fields(s.get_state(), uref)
        s.close()
        log("tts: bs5 %s tol=%g %s" % (ctl, tol, r))
        return r

    out["bs5_pi_fp32"] = bs5(1e-10, "pi")
    out["bs5_mlp_fp32"] = bs5(1e-10, "mlp")
    # (chunks of 0.1 time units: at the loose tolerances the steps collapse, and
    # the budget is checked between chunks)
    out["bs5_pi_fp32_rtol_sweep"] = [bs5(tol, "pi", budget_s=15.0, chunk=0.1) for tol in (1e-4, 1e-6, 1e-8)]
    # the FP32 right-hand side's floor on this metric: BS5 at tight tolerances
    floor = [bs5(tol, "pi") for tol in (1e-11, 1e-12)]
    out["fp32_energy_error_floor"] = {
        "runs": floor,
        "floor": min(r.get("rel_energy_err", 1.0) for r in floor),
        "note": "above 3e-7 the 1e-6 target leaves little room for the FP32 right-hand side"}
    fp64 = out["rk4_fp64_dt0.008"]
    best = out["bs5_mlp_fp32"]
    if best.get("rel_energy_err", 1.0) <= target and fp64["rel_energy_err"] <= target:
        out["speedup_bs5_mlp_over_rk4_fp64"] = fp64["wall_s"] / best["wall_s"]
    out["total_s"] = time.perf_counter() - t0
    del uref
    return out


def study_tts(args):
    """Wall time to a fixed relative energy error at T on the Taylor-Green
    vortex (nu = 1/1600): plain FP64 RK4 at fixed steps (the last one clipped
    to land on T) versus BS5 (FP64 state; FP32 and FP64 right-hand sides) with
    the Sec. 2.2.1 controller and with the trained proposer.  E_ref(T) from
    FP64 RK4 at dt = 1e-3."""
    import numpy as np
    import torch
    from paper_1810_10197_amd import inputs, ns
    n, T, nu = args.n, args.t_end, 1.0 / 1600
    u0 = inputs.tgv3d(n)[None]
    out = {"study": "time_to_solution", "n": n, "T": T, "nu": nu}

    def rk4_run(dt, prec):
        s = ns.Solver(dim=3, n=n, nu=nu, rhs_precision=prec)
        s.set_state(u0)
        steps = max(1, int(math.ceil(T / dt - 1e-9)))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            s.step_rk4(dt if i < steps - 1 else T - (steps - 1) * dt)
            if (i + 1) % 1000 == 0:
                log("rk4 %s dt=%g step %d/%d" % (prec, dt, i + 1, steps))
        e, _, _ = s.diagnostics()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        s.close()
        return float(e[0]), wall, 4 * steps

    eref, wref, _ = rk4_run(1e-3, "fp64")
    out["E_ref"] = eref
    out["ref_wall_s"] = wref
    log("E_ref(T=%g) = %.15e (%.1f s)" % (T, eref, wref))
    out["rk4_fp64"] = []
    for dt in args.rk4_dts:
        e, wall, nr = rk4_run(dt, "fp64")
        rel = abs(e - eref) / eref
        out["rk4_fp64"].append({"dt": dt, "rel_energy_err": rel, "wall_s": wall, "n_rhs": nr})
        log("rk4 fp64 dt=%g err %.3e wall %.2f s" % (dt, rel, wall))
    w = None
    if args.weights and os.path.exists(args.weights):
        w = np.load(args.weights)
    if w is None:
        w, info = train_proposer(ns, inputs, iters=args.iters, members=args.members,
                                 target=((64, 128), nu, T, (1e-7, 1e-8, 1e-9, 1e-10)))
        out["proposer_training"] = info
        if args.weights:
            np.save(args.weights, w)
    arms = [(c, p) for p in args.bs5_precs for c in ("pi", "mlp")]
    for ctl, prec in arms:
        key = "bs5_%s_%s" % (ctl, prec)
        out[key] = []
        for tol in args.tols:
            s = ns.Solver(dim=3, n=n, nu=nu, rhs_precision=prec)
            s.mlp_set_weights(w)
            s.set_state(u0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            # unit-time chunks, each continuing the controller of the previous
            # one (progress lines between)
            h, tot = 1e-3, {"n_rhs": 0, "n_accept": 0, "n_reject": 0}
            nchunk = int(math.ceil(T - 1e-12))
            for c in range(nchunk):
                st = s.integrate(min(T, c + 1.0), h, tol, tol, controller=ctl, resume=c > 0)[0]
                h = st["h_next"]
                for k in tot:
                    tot[k] += st[k]
                log("%s tol=%g t=%g rhs %d rej %d" % (ctl, tol, st["t"], tot["n_rhs"], tot["n_reject"]))
            e, _, _ = s.diagnostics()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            s.close()
            rel = abs(float(e[0]) - eref) / eref
            out[key].append({"tol": tol, "rel_energy_err": rel, "wall_s": wall, **tot})
            log("%s tol=%g err %.3e wall %.2f s rhs %d rej %d" % (key, tol, rel, wall, tot["n_rhs"],
                                                                 tot["n_reject"]))

    def cheapest(runs, target):
        ok = [r for r in runs if r["rel_energy_err"] <= target]
        return min(ok, key=lambda r: r["wall_s"]) if ok else None
    out["target"] = args.target
    out["best"] = {k: cheapest(out[k], args.target) for k in ["rk4_fp64"] + ["bs5_%s_%s" % a for a in arms]}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--dt", type=float, default=0.005)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tts", action="store_true",
                    help="skip the time-to-solution runs of the default workload (about a minute)")
    ap.add_argument("--variants", default=None,
                    help="comma-separated launch variants of the 5 passes and the slab (skips the autotuner)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (HBM counter scale)")
    ap.add_argument("--study", choices=["tts", "mlp", "e1", "problem"], default=None,
                    help="tts: wall time to a fixed energy error, BS5 (+proposer) vs FP64 RK4; "
                         "mlp: what the trained proposer gains on held-out ensemble members; "
                         "e1: Taylor-Green at Re=280, 64^3, RHS counts at equal dissipation error; "
                         "problem: time to solution on --problem (rt2d or hit512)")
    ap.add_argument("--t-end", type=float, default=10.0)
    ap.add_argument("--target", type=float, default=1e-6)
    ap.add_argument("--rk4-dts", type=float, nargs="*", default=[0.02, 0.01, 0.005, 0.0025])
    ap.add_argument("--tols", type=float, nargs="*", default=[1e-4, 1e-5, 1e-6, 1e-7, 1e-8])
    ap.add_argument("--weights", default=None,
                    help="proposer weights (.npy): read (or written after training) by --study tts, written by --study mlp")
    ap.add_argument("--bs5-precs", nargs="*", default=["fp32", "fp64"])
    ap.add_argument("--e1-dts", type=float, nargs="*", default=[0.1, 0.05, 0.02, 0.01, 0.005, 0.0025])
    ap.add_argument("--e1-tols", type=float, nargs="*",
                    default=[1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8, 1e-9, 1e-10])
    ap.add_argument("--members", type=int, default=128)
    ap.add_argument("--problem", choices=["rt2d", "hit512"], default="rt2d",
                    help="--study problem: which workload")
    ap.add_argument("--dealias", choices=["2/3", "3/2"], default="2/3",
                    help="3/2: products on the zero-padded 3n/2 grid (Sec. 2.1.1)")
    ap.add_argument("--workload", choices=["tgv", "ensemble", "rt2d"], default="tgv",
                    help="tgv: 3D Taylor-Green at --n; ensemble: --members x 64^3; rt2d: 2D "
                         "Boussinesq at 1024^2")
    ap.add_argument("--iters", type=int, default=3000)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.study == "tts":
        return study_tts(args)
    if args.study == "mlp":
        return study_mlp(args)
    if args.study == "e1":
        return study_e1(args)
    if args.study == "problem":
        return study_problem(args)
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
    return bench_throughput(args)


def bench_throughput(args):
    import numpy as np
    import torch
    from paper_1810_10197_amd import inputs, ns

    wl = args.workload
    fp64 = args.prec == "fp64"
    padded = args.dealias == "3/2"
    if padded and wl == "ensemble":
        raise SystemExit("--dealias 3/2 applies to the Taylor-Green and Rayleigh-Taylor workloads "
                         "(and to --study e1)")
    if wl == "tgv":
        n, batch, dim = args.n, 1, 3
        nu = 1.0 / 1600
        s = ns.Solver(dim=3, n=n, batch=1, nu=nu, rhs_precision=args.prec, dealias=args.dealias)
        s.set_state(inputs.tgv3d(n)[None])
        cfg = {"workload": "3D Taylor-Green vortex %d^3, nu=1/1600, BS5 attempts at h=%g, "
                           "atol=rtol=1e-6, %s FFTs, FP64 state, %s" %
                           (n, args.dt, args.prec,
                            "3/2-rule dealiasing (products on %d^3)" % (3 * n // 2) if padded
                            else "2/3-rule dealiasing"),
               "n": n, "batch": 1, "dealias": args.dealias}
        h = args.dt
    elif wl == "ensemble":
        n, batch, dim = 64, args.members, 3
        fields, nus = inputs.ensemble_members(batch, n)
        nu = float(np.min(nus))
        s = ns.Solver(dim=3, n=n, batch=batch, nu=nus, rhs_precision=args.prec)
        s.set_state(fields)
        cfg = {"workload": "ensemble of %d independent 64^3 runs (Taylor-Green and random-phase "
                           "fields, nu log-uniform in [1e-3, 1e-2]), BS5 attempts at h=%g, "
                           "atol=rtol=1e-6, %s FFTs, FP64 state" % (batch, args.dt, args.prec),
               "n": n, "batch": batch}
        h = args.dt
    else:
        n, batch, dim = 1024, 1, 2
        nu = 1e-4
        s = ns.Solver(dim=2, n=n, batch=1, nu=nu, rhs_precision=args.prec, scalar=True, ri=0.5,
                      kappa=1e-4, dealias=args.dealias)
        s.set_state(inputs.rayleigh_taylor2d(n)[None])
        cfg = {"workload": "2D Boussinesq Rayleigh-Taylor 1024^2 (tanh interface, Ri=0.5, "
                           "nu=kappa=1e-4), BS5 attempts at h=%g, atol=rtol=1e-6, %s FFTs, "
                           "FP64 state, %s" % (args.dt, args.prec,
                                               "3/2-rule dealiasing (products on 1536^2)" if padded
                                               else "2/3-rule dealiasing"),
               "n": n, "batch": 1, "dealias": args.dealias}
        h = args.dt
    atol = rtol = 1e-6
    if args.variants:
        tune_variants = s.tune([int(v) for v in args.variants.split(",")])
        tune_ms = np.zeros((ns.NS_NTUNE, ns.NS_TUNE_MAXV))
    else:
        tune_variants, tune_ms = s.autotune(reps=3)
    for _ in range(args.warmup):
        s.step_bs5(h, atol, rtol)
    # pure right-hand-side rate (context): f(u_n) into the cached stage
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nr = 20
    for _ in range(nr):
        s.refresh_rhs()
    torch.cuda.synchronize()
    rhs_only = nr * batch / (time.perf_counter() - t0)

    # timed region: BS5 attempts, no events
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rejected = 0
    for _ in range(args.steps):
        st, _ = s.step_bs5(h, atol, rtol)
        rejected += int(st == ns.NS_STEP_REJECTED)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # the same steps again with HIP events around every launch (the y/x/y
    # slab phase as one unit): per-pass durations for the right-hand side
    torch.cuda.synchronize()
    s.profile_start()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        s.step_bs5(h, atol, rtol)
    torch.cuda.synchronize()
    elapsed_ev = time.perf_counter() - t1
    prof = s.profile_stop()
    # and once more with every y/x/y launch bracketed on its own stream: the
    # duration of each kernel, for the dominant kernel's roofline
    # (with a two-stream slab schedule the launches of one stream overlap those
    # of the other and their brackets would hold both; this run then takes the
    # same slab size on one stream, which runs the same kernels one at a time)
    prof_fine = None
    fine_variants = list(tune_variants)
    if dim == 3:
        fine_variants[5] = ONE_STREAM_SLAB.get(fine_variants[5], fine_variants[5])
        s.tune(fine_variants)
        s.profile_mode(1)
        s.profile_start()
        for _ in range(args.steps):
            s.step_bs5(h, atol, rtol)
        torch.cuda.synchronize()
        prof_fine = s.profile_stop()
        s.profile_mode(0)
        s.tune(list(tune_variants))
    # and once more with one event pair around each whole right-hand side (no
    # events between its passes): the evaluation's wall time
    s.profile_mode(2)
    s.profile_start()
    for _ in range(args.steps):
        s.step_bs5(h, atol, rtol)
    torch.cuda.synchronize()
    prof_whole = s.profile_stop()
    s.profile_mode(0)
    s.close()
    copy_gbs = hbm_copy_gbs()

    rhs_evals = 7 * args.steps * batch
    value = rhs_evals / elapsed
    # inside the BS5 steps an FP32 right-hand side reads FP32 stage inputs (3D and 2D)
    # the 3/2 rule runs the same passes on the padded grid 3n/2
    pb = (pass_bytes(3 * n // 2 if padded else n, fp64, stage32=not fp64) if dim == 3
          else pass_bytes_2d(3 * n // 2 if padded else n, fp64, stage32=not fp64))
    pb = {k: v * batch for k, v in pb.items()}
    n_rhs = prof["zinv"][1]                       # one first-pass launch per evaluation
    per_kernel = {}
    for name in ["zinv", "yinv", "xpass", "yfwd", "zfwd", "combine", "reduce"]:
        ms, cnt = prof[name]
        if cnt:
            per_kernel[name] = {"avg_us": 1000.0 * ms / cnt, "launches": cnt}
            if name in pb:
                per_launch_bytes = pb[name] * n_rhs / cnt
                per_kernel[name]["us_per_rhs"] = 1000.0 * ms / n_rhs
                per_kernel[name]["bytes_per_launch"] = per_launch_bytes
                per_kernel[name]["gbs"] = per_launch_bytes / (ms / cnt * 1e-3) / 1e9
    rhs_passes = [k for k in ["zinv", "yinv", "xpass", "yfwd", "zfwd"] if k in pb]
    if dim == 3:
        # wall time per evaluation: z passes plus the y/x/y slab phase (its
        # passes may overlap on two streams, so the phase is timed as a unit)
        slab_ms, slab_cnt = prof["slab"]
        slab_us = 1000.0 * slab_ms / max(slab_cnt, 1)
        ph_bytes = pb["yinv"] + pb["xpass"] + pb["yfwd"]
        per_kernel["yxy_phase"] = {"us_per_rhs": slab_us, "bytes_per_rhs": ph_bytes,
                                   "gbs": ph_bytes / (slab_us * 1e-6) / 1e9}
        phase_sum_ms = (per_kernel["zinv"]["us_per_rhs"] + slab_us + per_kernel["zfwd"]["us_per_rhs"]) / 1000.0
        # single kernels from the run with every launch bracketed
        for name in ["yinv", "xpass", "yfwd"]:
            ms, cnt = prof_fine[name]
            nr = prof_fine["zinv"][1]
            if cnt and nr:
                bpl = pb[name] * nr / cnt
                per_kernel[name] = {"avg_us": 1000.0 * ms / cnt, "launches": cnt,
                                    "us_per_rhs": 1000.0 * ms / nr, "bytes_per_launch": bpl,
                                    "gbs": bpl / (ms / cnt * 1e-3) / 1e9,
                                    "timing": "every launch bracketed on its stream"
                                    + ("" if fine_variants == list(tune_variants) else
                                       ", the slab schedule's launches on one stream (variants %s)"
                                       % ",".join(map(str, fine_variants)))}
        units = ["zinv", "yinv", "xpass", "yfwd", "zfwd"]
    else:
        phase_sum_ms = sum(per_kernel[k]["us_per_rhs"] for k in rhs_passes) / 1000.0
        units = rhs_passes
    whole_ms, whole_cnt = prof_whole["rhs"]
    rhs_ms = whole_ms / whole_cnt if whole_cnt else phase_sum_ms
    dom = max([k for k in units if k in per_kernel], key=lambda k: per_kernel[k]["us_per_rhs"])
    achieved = per_kernel[dom]["gbs"]
    model_bytes = sum(pb.values())
    unit = "RHS evals/s" if batch == 1 else "member RHS evals/s"
    out = {
        "metric": "RHS evals/s at 256^3 (BS5 step, FP32 RHS / FP64 state)"
        if wl == "tgv" and n == 256 and not padded
        else "RHS evals/s (BS5 step, %s RHS / FP64 state%s)" % (args.prec.upper(),
                                                              ", 3/2 rule" if padded else ""),
        "value": value,
        "unit": unit,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if fp64 else "f32",
        "data": "synthetic",
        "config": cfg,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom, per_kernel[dom].get("launches", n_rhs) / n_rhs)
                     if (wl == "tgv" and n == 256 and not fp64 and not padded) else None,
                     "kernel": dom},
        "rhs_model_gb": model_bytes / 1e9,
        "rhs_passes_ms": rhs_ms,
        "rhs_phase_brackets_ms": phase_sum_ms,
        "rhs_model_gbs": model_bytes / (rhs_ms * 1e-3) / 1e9,
        "rhs_model_frac": model_bytes / (rhs_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "rhs_only_per_s": rhs_only,
        "hbm_copy_gbs": copy_gbs,
        "value_with_events": rhs_evals / elapsed_ev,
        "rejected_steps": rejected,
        "autotune": {"variants": tune_variants,
                     "ms": [[round(x, 4) for x in row] for row in np.asarray(tune_ms).tolist()]},
        "kernels": per_kernel,
    }
    if not args.no_cpu and wl == "tgv":
        out["cpu_baseline"] = cpu_baseline(n, nu, args.cpu_budget, padded)
        out["c1_gpu_time_to_solution"] = c1_gpu_time_to_solution(ns, inputs)
    if not args.no_tts and wl == "tgv" and n == 256 and not padded and not fp64:
        out["time_to_solution"] = time_to_solution(ns, inputs)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
