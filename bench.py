"""Benchmark: trajectories/s of one ensemble solve on one MI355X.

Default workload (the headline): 2^24 Lorenz trajectories, rho ~ U[0,28],
u0 = (1,0,0) + N(0, 0.01^2), FP32 state with FP64 compensated time, adaptive
Tsit5 at reltol = abstol = 1e-6, 16 evenly spaced saves on t in [0, 1].
One "step" = one ens_solve over the whole ensemble (inputs resident in HBM).

    python bench.py [--steps K] [--warmup W] [--workload lorenz_fp32|lorenz_fp64|
                     robertson|gbm] [--form plain|persistent|auto] [--no-cpu-baseline]

Prints one JSON line.  The roofline object reports the solver kernel's
algorithmic FP32 (or FP64) flop rate -- flops per attempted step of the
method x attempted steps, over the kernel time measured with events on the
launch stream -- against the non-packed VALU peak.  The cpu_baseline leg times
the FP64 C oracle on a bounded sample on the host cores and reports the max
normwise relative error of the GPU result against the oracle.
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

METRIC = "trajectories/sec at stated tolerance (FP32 vs FP64, plain vs persistent vs surrogate)"

# Algorithmic flops per attempted step (FMA = 2), counted from the method:
#  Tsit5, Lorenz (n = 3): stage combinations 144, 6 RHS x 8 = 48, error
#    estimate 42, error norm 19, step-size control 7  -> 260.
#  Rodas4, Robertson (n = 3): Jacobian 6, W 12, LU 26, 6 stages x (combination
#    + RHS + solve-rhs + triangular solves) = 6 x 69 = 414 minus the
#    empty first-stage combinations 18 -> 396, u_new 3, error norm 19,
#    control 7  -> 466.
#  EM, GBM4: per step 4 x (2 flops for the increment + 2 for the update) +
#    Box-Muller 2 x 8  -> 32 (Philox is integer work, counted separately).
FLOPS = {("tsit5", "lorenz"): 260, ("rodas4", "robertson"): 466, ("em", "gbm4"): 32}

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.  A non-packed FMA retires
# 2 flops per lane per cycle in FP32 and in FP64: 78.6 TFLOP/s for both.
# (The published 157.3 TFLOP/s FP32 figure counts packed dual-FP32 FMAs,
# which this library does not emit.)
PEAK_FP32_NONPACKED = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PEAK_FP32_PUBLISHED = 157.3
PEAK_FP64 = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="lorenz_fp32",
                    choices=["lorenz_fp32", "lorenz_fp64", "robertson", "gbm"])
    ap.add_argument("--n", type=int, default=0, help="override the ensemble size")
    ap.add_argument("--form", default="plain", choices=["plain", "persistent", "auto"])
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target wall time of the CPU-baseline sample")
    return ap.parse_args()


def make_workload(name, n):
    from paper_2304_06835_amd import workloads as W
    f = {"lorenz_fp32": W.lorenz_fp32, "lorenz_fp64": W.lorenz_fp64,
         "robertson": W.robertson, "gbm": W.gbm}[name]
    return f(N=n) if n else f()


def describe(e):
    if e.name == "lorenz_fp32":
        return ("Lorenz 2^24-ensemble, rho~U[0,28], u0=(1,0,0)+N(0,0.01^2), FP32 state + FP64 "
                "compensated time, Tsit5 rtol=atol=1e-6, 16 saves on [0,1]")
    if e.name == "lorenz_fp64":
        return "Lorenz 8192-ensemble, rho~U[0,21], FP64, Tsit5 rtol=atol=1e-8, final state"
    if e.name == "robertson":
        return ("Robertson 2^20-ensemble, rates x logU[0.5,2], tf~logU[1,1e5], FP32 state + "
                "FP64 W/LU, Rodas4 rtol=1e-6 atol=1e-8, final state")
    return "GBM 4-component 2^22-ensemble, Euler-Maruyama dt=1/256, Philox4x32-10, FP32"


class Runner:
    """Device copies of one workload and a configured solver context."""

    def __init__(self, e, precision, **opts):
        import numpy as np
        import torch

        import paper_2304_06835_amd as ens
        self.e = e
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
        self.params, self.u0, self.tspan = dev(e.params), dev(e.u0), dev(e.tspan)
        self.s = ens.Solver(0, precision=precision)
        if e.h0:
            self.s.set(h0=e.h0)
        if e.alg == "em":
            self.s.set(dt=e.dt, seed=e.seed)
        if opts:
            self.s.set(**opts)
        n, _ = ens.system_dims(e.system)
        dt = torch.float64 if precision == 64 else torch.float32
        self.out = torch.empty((len(e.theta), n, e.n), dtype=dt, device="cuda")

    def solve(self, status=None, stats=None):
        e = self.e
        return self.s.solve(e.system, self.params, self.u0, self.tspan, e.alg, e.abstol,
                            e.reltol, e.theta, out=self.out, status=status, stats=stats)

    def attempts(self):
        import torch
        st = torch.empty((2, self.e.n), dtype=torch.int32, device="cuda")
        self.solve(stats=st)
        torch.cuda.synchronize()
        return int(st.to(torch.int64).sum().item()), st

    def time(self, steps, warmup):
        import torch
        for _ in range(warmup):
            self.solve()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        t0 = time.perf_counter()
        for a, b in evs:
            a.record()
            self.solve()
            b.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ker = [a.elapsed_time(b) for a, b in evs]
        return wall, sum(ker) / len(ker), min(ker)


def cpu_baseline(e, gpu_out, seconds):
    """The oracle timed on the host cores on a bounded sample of the same
    workload, plus the max normwise error of the GPU result against the FP64
    oracle (truth at tol 1e-12 for adaptive solvers) on a 4096 subsample."""
    import numpy as np

    import oracle
    from paper_2304_06835_amd import workloads as W
    nth = oracle.default_threads()
    sysid = {"lorenz": oracle.LORENZ, "robertson": oracle.ROBERTSON}.get(e.system)

    def sub(idx):
        return (np.ascontiguousarray(e.params[:, idx]), np.ascontiguousarray(e.u0[:, idx]),
                np.ascontiguousarray(e.tspan[:, idx]))

    def run(idx, tol=None):
        p, u, ts = sub(idx)
        if e.alg == "em":
            return oracle.em(p, u, e.dt, e.n_steps, e.seed, ids=idx, nthreads=nth)[None]
        alg = oracle.TSIT5 if e.alg == "tsit5" else oracle.RODAS4
        at = e.abstol if tol is None else tol
        rt = e.reltol if tol is None else tol
        return oracle.solve(sysid, alg, p, u, ts, at, rt, e.theta, h0=e.h0, nthreads=nth)[0]

    # calibrate on 1024, then size the sample to about `seconds` of wall time
    idx = W.sample_indices(e.n, 1024)
    t0 = time.perf_counter()
    run(idx)
    rate = len(idx) / max(time.perf_counter() - t0, 1e-6)
    k = int(min(e.n, max(1024, rate * seconds)))
    idx = W.sample_indices(e.n, k)
    t0 = time.perf_counter()
    run(idx)
    dt = time.perf_counter() - t0
    res = {"value": len(idx) / dt, "unit": "trajectories/s", "cores": nth, "kind": "oracle",
           "sample": f"{len(idx)} of {e.n} trajectories (every {e.n // len(idx)}-th), "
                     f"FP64 C oracle, OpenMP over trajectories, {dt:.1f} s"}
    # accuracy of the GPU result on the fixed 4096 subsample
    idx = W.sample_indices(e.n, 4096)
    g = gpu_out[:, :, idx].astype(np.float64)
    if e.alg == "em":
        ref = run(idx)
        err = float((np.abs(g - ref) / np.abs(ref)).max())
        kind = "pathwise relative error vs FP64 oracle on the same Philox stream"
    else:
        truth = run(idx, tol=1e-12)
        err = float((np.abs(g - truth).max(axis=1) / np.abs(truth).max(axis=1)).max())
        kind = "max normwise relative error vs FP64 oracle at tol 1e-12"
    return res, {"max_rel_err": err, "subsample": len(idx), "kind": kind}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(trajectories are independent: N GPUs would each solve their own slice)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    e = make_workload(args.workload, args.n)
    precision = 64 if args.workload == "lorenz_fp64" else 32
    opts = {}
    if args.block:
        opts["block"] = args.block
    if args.form == "persistent":
        opts["form"] = 1
    r = Runner(e, precision, **opts)
    tuned = None
    if args.form == "auto":
        from paper_2304_06835_amd import workloads as W
        k = min(e.n, 1 << 18)
        idx = W.sample_indices(e.n, k)
        pe = make_workload(args.workload, 0)
        pe.params, pe.u0, pe.tspan = (e.params[:, idx].copy(), e.u0[:, idx].copy(),
                                      e.tspan[:, idx].copy())
        probe = Runner(pe, precision)
        ms, cfg = probe.s.autotune(pe.system, probe.params, probe.u0, probe.tspan, pe.alg,
                                   pe.abstol, pe.reltol, pe.theta)
        tuned = cfg
        r.s.set(**{k2: v for k2, v in cfg.items()})
    print(f"[bench] {e.name} N={e.n} precision={precision} form={args.form}", file=sys.stderr,
          flush=True)

    attempts, stats = r.attempts()
    wall, ker_ms, ker_min = r.time(args.steps, args.warmup)
    out_host = r.out.cpu().numpy()
    value = e.n * args.steps / wall
    ms_per_step = wall / args.steps * 1e3
    flops = FLOPS[(e.alg, e.system)] * attempts
    peak = PEAK_FP64 if precision == 64 else PEAK_FP32_NONPACKED
    achieved = flops / (ker_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": None,
            "kernel_ms_avg": ker_ms, "kernel_ms_min": ker_min,
            "flops_per_launch": flops, "attempted_steps": attempts,
            "flops_per_attempt": FLOPS[(e.alg, e.system)]}
    if precision == 32:
        roof["frac_of_published_fp32_peak_157.3"] = achieved / PEAK_FP32_PUBLISHED
    st = stats.cpu().numpy()
    steps_per = st.sum(axis=0)
    config = {"workload": describe(e), "name": e.name, "n_traj": e.n, "alg": e.alg,
              "abstol": e.abstol, "reltol": e.reltol, "n_save": len(e.theta),
              "form": args.form, "block": int(r.s.get("block")) or 256,
              "tuned": tuned,
              "steps_per_traj_mean": float(steps_per.mean()),
              "steps_per_traj_max": int(steps_per.max()),
              "rejected_frac": float(st[1].sum() / max(1, st.sum()))}

    variants = {}
    if not args.no_variants and e.name == "lorenz_fp32":
        rp = Runner(e, 32, form=1)
        w2, k2, _ = rp.time(max(3, args.steps // 2), 1)
        p_out = rp.out.cpu().numpy()
        variants["fp32_persistent"] = {
            "traj_per_s": e.n * max(3, args.steps // 2) / w2, "kernel_ms": k2,
            "speedup_vs_plain": ker_ms / k2,
            "bitwise_equal_to_plain": bool((p_out.view("u1") == out_host.view("u1")).all())}
        del rp
        r64 = Runner(make_workload("lorenz_fp32", args.n), 64)
        r64.e = e  # same draws, promoted to FP64
        import numpy as np
        import torch as _t
        r64.params = _t.from_numpy(e.params.astype(np.float64)).cuda()
        r64.u0 = _t.from_numpy(e.u0.astype(np.float64)).cuda()
        r64.out = _t.empty((len(e.theta), 3, e.n), dtype=_t.float64, device="cuda")
        w3, k3, _ = r64.time(max(3, args.steps // 2), 1)
        variants["fp64_plain"] = {"traj_per_s": e.n * max(3, args.steps // 2) / w3,
                                  "kernel_ms": k3, "fp32_speedup": k3 / ker_ms}
        del r64

    res = {"metric": METRIC, "value": value, "unit": "trajectories/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if precision == 64 else "f32", "data": "synthetic",
           "config": config, "roofline": roof}
    if variants:
        res["variants"] = variants
    if not args.no_cpu_baseline:
        cb, acc = cpu_baseline(e, out_host, args.cpu_seconds)
        res["cpu_baseline"] = cb
        res["accuracy"] = acc
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
