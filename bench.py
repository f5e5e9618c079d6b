"""Benchmark: trajectories/s of one ensemble solve on one MI355X.

Default workload (the headline): 2^24 Lorenz trajectories, rho ~ U[0,28],
u0 = (1,0,0) + N(0, 0.01^2), FP32 state with FP64 compensated time, adaptive
Tsit5 at reltol = abstol = 1e-6, 16 evenly spaced saves on t in [0, 1].
One "step" = one ens_solve over the whole ensemble (inputs resident in HBM).

    python bench.py [--steps K] [--warmup W] [--workload lorenz_fp32|lorenz_fp64|
                     robertson|gbm] [--alg rodas4|rodas5p|ros23]
                    [--form plain|persistent|persistent_sorted_chunks|sorted|sorted_b512_r2|
                     sorted_staged|auto]
                    [--save-mode landing|dense]
                    [--no-cpu-baseline] [--no-variants] [--no-surrogate]

Prints one JSON line.  `roofline` reports the solver kernel's algorithmic
flop rate -- flops per attempted step of the method x attempted steps, over
the kernel time measured with events on the launch stream -- against the
MI355X vector peak of the arithmetic type.  `variants` times the other
work-assignment forms on the same inputs (bitwise-identical answers), the
stiff Robertson ensemble's forms, and the learned surrogate's audited solve
against the plain solver.  `cpu_baseline` times the FP64 C oracle on a
bounded sample on the host cores; `accuracy` is the GPU result's max
normwise relative error against the FP64 oracle on a 4096 subsample.
"""
from __future__ import annotations

import argparse
import hashlib
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
#  Stiffly accurate Rosenbrock (RODAS4: 6 stages, Rodas5P: 8), Robertson
#    (n = 3): Jacobian 6, W 12, LU 26; stage s = 0..S-1: stage point 6s, RHS 8,
#    C-combination 6s + 6, triangular solves 15  -> 12s + 29 per stage, so
#    12 S(S-1)/2 + 29 S over the stages (354 for S = 6, 568 for S = 8); u_new
#    3, error norm 19, control 7  -> 427 (RODAS4), 641 (Rodas5P).
#  Rosenbrock23, Robertson (n = 3): Jacobian 6, W 12, LU 26, three solves
#    3 x 15, two RHS 2 x 8, stage right-hand sides and points 3 + 3 + 18 + 7
#    + 6, error estimate 13, error norm 19, control 7  -> 181.
#  EM, GBM4: per step 4 x (2 flops for the increment + 2 for the update) +
#    Box-Muller 2 x 8  -> 32 (Philox is integer work, counted separately).
#  Weak order-2 scheme, GBM4: per step 4 x 29 (drift and diffusion at four
#    points, the three combinations) + Box-Muller 16 -> 132.
#  EM, CRN: per step drift 14 + Hill term 10 (two powers as exp2/log2 counted
#    as 1 each) + 8 noise terms 24 + updates 8, + Box-Muller 4 x 8 -> 88.
FLOPS = {("tsit5", "lorenz"): 260, ("rodas4", "robertson"): 427, ("rodas5p", "robertson"): 641,
         ("ros23", "robertson"): 181,
         ("em", "gbm4"): 32, ("siea", "gbm4"): 132, ("em", "crn"): 88}
# Tsit5 dense output, per save time read off a step (save mode 1; every save
# but the last, which a step lands on): theta 2; h b_0(theta) by Horner 8;
# h theta^2 2; the six other weights have no linear term, b_i = theta^2 q_i,
# q_i by Horner 6 x 4; u + (h b_0) k_0 + (h theta^2) sum_{i>0} q_i k_i for
# n = 3: 3 x 15 -> 81.
DENSE_FLOPS_PER_SAVE = 81
MLP_FLOPS_PER_QUERY = 2 * (4 * 256 + 256 * 256 + 256 * 256 + 256 * 48)  # 288,768
# one training sample: the forward pass, the weight gradients (the same
# products) and the input gradients of every layer but the first
MLP_TRAIN_FLOPS_PER_SAMPLE = 2 * MLP_FLOPS_PER_QUERY + 2 * (256 * 256 + 256 * 256 + 256 * 48)

# MI355X published vector peaks (256 CUs, 2.4 GHz): FP32 157.3 TFLOP/s, FP64
# 78.6 TFLOP/s; dense bf16 MFMA 2.5 PFLOP/s.  The FP32 figure counts 32 FMA
# lanes per SIMD clock; ordinary (non-packed) FP32 instructions issue fewer
# (the probe, issue_rates(), measures about 23 lane-ops per SIMD per rated
# clock), which the issue roofline accounts for.
PEAK = {32: 157.3, 64: 78.6}
PEAK_BF16_MFMA = 2500.0

FORMS = {"plain": {"form": 0}, "persistent": {"form": 1},
         "persistent_sorted_chunks": {"form": 3, "block": 256},
         "sorted": {"form": 2, "block": 256}}
# the stiff ensemble also at a sort over 1024 items in 512-thread blocks
STIFF_FORMS = dict(FORMS, sorted_b512_r2={"form": 2, "block": 512, "tpl": 2})
# Tsit5 also with the sorted form's saves staged in LDS (whole-row writes)
TSIT5_FORMS = dict(FORMS, sorted_staged={"form": 2, "block": 256, "stage_saves": 1})
LAUNCH_FORMS = dict(STIFF_FORMS, **TSIT5_FORMS)
DEFAULT_FORM = {"lorenz_fp32": "sorted", "lorenz_fp64": "plain", "robertson": "sorted",
                "gbm": "plain", "orego": "sorted", "hires": "sorted", "pollu": "plain",
                "crn": "plain"}
# save times: "landing" (steps end on every save time) or "dense" (Tsit5's
# dense output between steps that land only on the last save time)
DEFAULT_SAVE = {"lorenz_fp32": "dense"}  # every other workload: "landing"
SAVE_MODES = {"landing": 0, "dense": 1}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="lorenz_fp32",
                    choices=["lorenz_fp32", "lorenz_fp64", "robertson", "gbm", "orego", "hires",
                             "pollu", "crn"])
    ap.add_argument("--n", type=int, default=0, help="override the ensemble size")
    ap.add_argument("--alg", default="", choices=["", "rodas4", "rodas5p", "ros23", "siea"],
                    help="stiff method of the Robertson and appendix-B.1 workloads (default "
                         "rodas4), or siea for the GBM workload")
    ap.add_argument("--form", default="",
                    choices=["", "plain", "persistent", "persistent_sorted_chunks", "sorted",
                             "sorted_b512_r2", "sorted_staged", "auto"])
    ap.add_argument("--save-mode", default="", choices=["", "landing", "dense"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--surrogate-epochs", type=int, default=160)
    ap.add_argument("--surrogate-only", action="store_true",
                    help="only train the surrogate for --surrogate-epochs epochs on 2^20 solver "
                         "trajectories and run its inference on 2^24 queries (for profiling)")
    ap.add_argument("--surrogate-scaling", action="store_true",
                    help="with --surrogate-only: also time training at several batch sizes")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target wall time of the CPU-baseline sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy five times (the "
                         "reference kernel that scales rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--record-counters", metavar="DIR", default="",
                    help="no GPU: write profiles/valu_mix.json and profiles/traffic.json from "
                         "the rocprofv3 --pmc output directories under DIR (the commands in "
                         "profiles/valu_issue_rates.md and tsit5_sorted_f32_lorenz_2p24.md)")
    return ap.parse_args()


def copy_calibration():
    """Two copies of known size: the runtime's blit copy (16-byte accesses)
    and an index_select gather (4-byte element accesses, like the solver's
    loads and save stores): 2^28 floats = 1 GiB written; the gather also
    reads a 2 GiB int64 index."""
    import torch
    n = 1 << 28
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    idx = torch.arange(n, dtype=torch.int64, device="cuda")
    for _ in range(3):
        y.copy_(x)
    for _ in range(3):
        torch.index_select(x, 0, idx, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {
        "blit": {"bytes_read": 4 * n, "bytes_written": 4 * n, "launches": 3},
        "index_select": {"bytes_read": 12 * n, "bytes_written": 4 * n, "launches": 3}}}),
        flush=True)


def make_workload(name, n, alg=""):
    from paper_2304_06835_amd import workloads as W
    if name in W.STIFF:
        return W.stiff(name, N=n, alg=alg or "rodas4")
    if name == "crn":
        return W.crn()
    if name == "gbm" and alg:
        return W.gbm(N=n, alg=alg) if n else W.gbm(alg=alg)
    f = {"lorenz_fp32": W.lorenz_fp32, "lorenz_fp64": W.lorenz_fp64,
         "robertson": W.robertson, "gbm": W.gbm}[name]
    kw = {"alg": alg} if (alg and name == "robertson") else {}
    return f(N=n, **kw) if n else f(**kw)


def describe(e):
    if e.name == "lorenz_fp32":
        return ("Lorenz 2^24-ensemble, rho~U[0,28], u0=(1,0,0)+N(0,0.01^2), FP32 state + FP64 "
                "compensated time, Tsit5 rtol=atol=1e-6, 16 saves on [0,1]")
    if e.name == "lorenz_fp64":
        return "Lorenz 8192-ensemble, rho~U[0,21], FP64, Tsit5 rtol=atol=1e-8, final state"
    method = {"ros23": "Rosenbrock23", "rodas5p": "Rodas5P"}.get(e.alg, "Rodas4")
    if e.name in ("orego", "hires", "pollu"):
        return (f"{e.name.upper()} 8192-ensemble (appendix B.1), rate constants x logU[0.5,2], "
                f"{method} rtol=1e-6 atol=1e-8, 4 saves")
    if e.name == "robertson":
        return ("Robertson 2^20-ensemble, rates x logU[0.5,2], tf~logU[1,1e5], FP32 state + "
                f"FP64 W/LU, {method} rtol=1e-6 atol=1e-8, final state")
    if e.name == "crn":
        return ("sigma-factor CRN SDE (appendix), 10^6-trajectory Cartesian parameter sweep, "
                "Euler-Maruyama dt=0.1 on [0,1000] (10^4 steps), 8 Wiener processes, FP32")
    return ("GBM 4-component 2^22-ensemble, "
            f"{'weak order-2 scheme' if e.alg == 'siea' else 'Euler-Maruyama'} dt=1/256, "
            "Philox4x32-10, FP32")


def dev(a):
    import numpy as np
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def event_time(fn, steps, warmup):
    """Run fn warmup + steps times; (wall s, mean event ms, min event ms) of the
    timed steps, events recorded on torch's current stream (the launch stream)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ker = [a.elapsed_time(b) for a, b in evs]
    return wall, sum(ker) / len(ker), min(ker)


class Runner:
    """Device copies of one workload and a configured solver context."""

    def __init__(self, e, precision, **opts):
        import torch

        import paper_2304_06835_amd as ens
        self.e = e
        self.params, self.u0, self.tspan = dev(e.params), dev(e.u0), dev(e.tspan)
        self.s = ens.Solver(0, precision=precision)
        if e.h0:
            self.s.set(h0=e.h0)
        if e.alg in ("em", "siea"):
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
        return event_time(self.solve, steps, warmup)

    def host_out(self):
        return self.out.cpu().numpy()


def kernel_name(e, form, precision):
    """The solver kernel a launch of workload e in `form` runs."""
    prec = "double" if precision == 64 else "float"
    if e.alg in ("em", "siea"):
        return "em_gbm4" if (e.alg == "em" and e.system == "gbm4") else f"sde_fixed<{prec}>"
    if e.system == "pollu":
        return f"ros_grouped<{prec}>"
    base = "tsit5" if e.alg == "tsit5" else "ros"
    suffix = {"plain": "_plain", "persistent": "_persistent",
              "persistent_sorted_chunks": "_chunked", "sorted": "_sorted",
              "sorted_b512_r2": "_sorted", "sorted_staged": "_sorted", "auto": ""}[form]
    return f"{base}{suffix}<{prec}>"


def kernel_source_hash(files=None):
    """Hash of the sources a recorded traffic measurement refers to: the
    named files of the kernel's translation unit, or every solver source."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2304_06835_amd", "csrc")
    names = sorted(files) if files else sorted(
        f for f in os.listdir(csrc) if f.endswith((".hip", ".h")))
    for f in names:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(name, form, launches_units):
    """HBM bytes per launch from a committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    record (profiles/traffic.json), if it was taken on the current sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    r = rec.get(f"{name}/{form}")
    if not r or r.get("source_hash") != kernel_source_hash(r.get("sources")):
        return None
    return r.get("hbm_bytes_per_launch")


# ---- counter records (rocprofv3 --pmc output -> profiles/*.json) ----------
TSIT5_SOURCES = ["tsit5.hip", "driver.h", "systems.h", "ens_internal.h"]
SDE_SOURCES = ["em.hip", "driver.h", "philox.h", "ens_internal.h"]
ROS_SOURCES = ["rodas4.hip", "rodas.h", "rosenbrock.h", "pollu.h", "systems.h", "driver.h",
               "ens_internal.h"]
# record key: (directory suffix of the mixA_/mixC_ passes, kernel-name match,
# sources, description)
MIX_RUNS = {
    "lorenz_fp32/tsit5/sorted/dense": (
        "lorenz_fp32", "tsit5_sorted<float, ens::Lorenz, 256, 1, false>", TSIT5_SOURCES,
        "tsit5_sorted<float, Lorenz, 256, 1, false>, save mode 1 (dense output), 2^24 trajectories"),
    "gbm/em/plain": ("gbm", "em_gbm4", SDE_SOURCES, "em_gbm4, 2^22 trajectories x 256 steps"),
    "gbm/siea/plain": ("gbm_siea", "Gbm4Siea", SDE_SOURCES,
                       "sde_fixed<Gbm4Siea>, 2^22 trajectories x 256 steps"),
    "crn/em/plain": ("crn", "Crn>", SDE_SOURCES, "sde_fixed<Crn>, 10^6 trajectories x 10^4 steps"),
    "robertson/rodas4/sorted": (
        "robertson", "ros_sorted<float, ens::Robertson", ROS_SOURCES,
        "ros_sorted<float, Robertson, Rodas4, 256, 1>, 2^20 trajectories"),
}
# record key: (directory tag of the pmc_<tag>_FETCH / _WRITE passes, description)
TRAFFIC_RUNS = {
    "lorenz_fp32/sorted/dense": (
        "h", "tsit5_sorted<float, Lorenz, 256, 1, false>, save mode 1 (dense output), saves "
             "stored directly"),
    "lorenz_fp32/sorted_staged/dense": (
        "st", "tsit5_sorted<float, Lorenz, 256, 1, true>, save mode 1 (dense output), saves "
              "staged in LDS"),
}
HEADLINE_ALG_BYTES = (40 + 192) * (1 << 24)  # inputs + 16 saves of 3 FP32, per trajectory


def pmc_dispatches(path, match):
    """Per-dispatch counter sums {counter: value} of the kernels whose name
    contains `match`, in dispatch order, from a rocprofv3 counter CSV."""
    import collections
    import csv
    agg = collections.OrderedDict()
    with open(os.path.join(path, "run_counter_collection.csv")) as fh:
        for r in csv.DictReader(fh):
            if match in r["Kernel_Name"]:
                e = agg.setdefault(r["Dispatch_Id"], collections.Counter())
                e[r["Counter_Name"]] += float(r["Counter_Value"])
    return list(agg.values())


def record_counters(root, out_dir=None):
    """Write the VALU-mix and HBM-traffic records that bench.py replays (by
    source hash) from the --pmc output directories under `root`."""
    out_dir = out_dir or os.path.join(ROOT, "profiles")

    def mean(ds, k):
        return sum(d[k] for d in ds) / len(ds)

    mix = {"_doc": (
        "Wave-level VALU instructions per launch by class, from two rocprofv3 --pmc passes "
        "(SQ_INSTS_VALU and its FMA/MUL/ADD/TRANS_F32, INT32, INT64, CVT classes; the F64 "
        "classes with SQ_ACTIVE_INST_VALU and SQ_THREAD_CYCLES_VALU), written by bench.py "
        "--record-counters. OTHER = SQ_INSTS_VALU minus the counted classes (moves, compares, "
        "selects, logic, permutes). bench.py prices each class at the issue rate the VALU probe "
        "measures in the same run; source_hash identifies the kernel's sources and bench.py "
        "ignores a record taken on other sources.")}
    for key, (tag, match, src, kern) in MIX_RUNS.items():
        A = pmc_dispatches(os.path.join(root, f"mixA_{tag}"), match)
        C = pmc_dispatches(os.path.join(root, f"mixC_{tag}"), match)
        if not A or not C:
            raise ValueError(f"{key}: no '{match}' dispatches under {root}/mix[AC]_{tag}")
        tot = mean(A, "SQ_INSTS_VALU")
        cls = {c: mean(A, f"SQ_INSTS_VALU_{c}") for c in
               ("FMA_F32", "MUL_F32", "ADD_F32", "TRANS_F32", "INT32", "INT64", "CVT")}
        cls["F64"] = sum(mean(C, f"SQ_INSTS_VALU_{k}_F64") for k in ("FMA", "ADD", "MUL", "TRANS"))
        cls["OTHER"] = max(0.0, tot - sum(cls.values()))
        mix[key] = {"kernel": kern, "sources": src, "source_hash": kernel_source_hash(src),
                    "dispatches": [len(A), len(C)], "per_launch": cls,
                    "sq_insts_valu_raw": [d["SQ_INSTS_VALU"] for d in A],
                    "lanes_active_per_instr": (mean(C, "SQ_THREAD_CYCLES_VALU")
                                               / (64 * mean(C, "SQ_ACTIVE_INST_VALU"))),
                    "sq_waves": mean(C, "SQ_WAVES"),
                    "sq_busy_cycles": [d["SQ_BUSY_CYCLES"] for d in C]}

    def sums(d, match):
        return [sum(c.values()) for c in pmc_dispatches(os.path.join(root, d), match)]

    # the runtime's blit copy of 1 GiB (--copy-calibration); smaller
    # dispatches of the same kernel are torch's own set-up copies
    cf = [v for v in sums("pmc_copy_FETCH", "copyBuffer") if v > 1e5]
    cw = [v for v in sums("pmc_copy_WRITE", "copyBuffer") if v > 1e5]
    if not cf or not cw:
        raise ValueError(f"no 1 GiB copy dispatches under {root}/pmc_copy_*")
    fs, ws = 1048576 / (sum(cf) / len(cf)), 1048576 / (sum(cw) / len(cw))
    tr = {"_doc": (
        "HBM bytes per launch from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB per dispatch), "
        f"each scaled by the ratio the same counter reads for a 1 GiB device copy (bench.py "
        f"--copy-calibration): fetch x{fs:.3f}, write x{ws:.3f}; written by bench.py "
        "--record-counters. source_hash identifies the kernel's translation-unit sources "
        "(bench.kernel_source_hash over `sources`); bench.py reports null once they change.")}
    for key, (tag, kern) in TRAFFIC_RUNS.items():
        f = sums(f"pmc_{tag}_FETCH", "tsit5_sorted")
        w = sums(f"pmc_{tag}_WRITE", "tsit5_sorted")
        if not f or len(w) < 2:
            raise ValueError(f"{key}: need the kernel's dispatches under {root}/pmc_{tag}_*")
        rd = sum(f) / len(f) * 1024 * fs
        wr = sum(w[1:]) / len(w[1:]) * 1024 * ws  # the first dispatch is cold
        tr[key] = {"kernel": kern, "sources": TSIT5_SOURCES,
                   "source_hash": kernel_source_hash(TSIT5_SOURCES),
                   "fetch_kib_raw": [round(v) for v in f], "write_kib_raw": [round(v) for v in w],
                   "hbm_read_bytes_per_launch": rd, "hbm_write_bytes_per_launch": wr,
                   "hbm_bytes_per_launch": rd + wr,
                   "algorithmic_bytes_per_launch": HEADLINE_ALG_BYTES,
                   "traffic_over_algorithmic": (rd + wr) / HEADLINE_ALG_BYTES}
    for name, rec in (("valu_mix.json", mix), ("traffic.json", tr)):
        with open(os.path.join(out_dir, name), "w") as fh:
            json.dump(rec, fh, indent=1)
    return mix, tr


# Vector-ALU instruction classes of the rocprofv3 SQ_INSTS_VALU_* counters and
# the issue-rate probe kind (paper_2304_06835_amd/probe/valu_probe.hip) each
# class is priced at; VALU instructions in no counted class (moves, compares,
# selects, logic, lane permutes) are priced as 32-bit logic.
PROBE_KINDS = {"fma_f32": 0, "add_f32": 1, "mul_f32": 2, "fma_f64": 3, "exp_f32": 4,
               "mad_u64_u32": 5, "xor_b32": 6, "fma_f32_literal": 7, "fma_f32_sgpr": 8}
VALU_CLASS_PROBE = {"FMA_F32": "fma_f32", "MUL_F32": "mul_f32", "ADD_F32": "add_f32",
                    "TRANS_F32": "exp_f32", "F64": "fma_f64", "INT64": "mad_u64_u32",
                    "INT32": "xor_b32", "CVT": "xor_b32", "OTHER": "xor_b32"}


def issue_rates(device=0, iters=16384):
    """Lane-operations per second of each probe kind, measured now on this GPU
    (register-only dependency chains, 16 per lane, 2048 x 256 lanes)."""
    import ctypes
    path = os.path.join(ROOT, "paper_2304_06835_amd", "libvaluprobe.so")
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2304_06835_amd.build`")
    L = ctypes.CDLL(path)
    L.valu_probe_rate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_double)]
    out = {}
    for name, kind in PROBE_KINDS.items():
        r = ctypes.c_double(0.0)
        rc = L.valu_probe_rate(device, kind, iters, ctypes.byref(r))
        if rc != 0:
            raise RuntimeError(f"valu_probe_rate({name}) failed with {rc}")
        out[name] = r.value
    return out


def recorded_valu_mix(key, path=None):
    """Wave-level VALU instruction counts per launch by class, from a committed
    rocprofv3 record (profiles/valu_mix.json) taken on the current sources."""
    path = path or os.path.join(ROOT, "profiles", "valu_mix.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    r = rec.get(key)
    if not r or r.get("source_hash") != kernel_source_hash(r.get("sources")):
        return None
    return r


def mfma_mix_rates(device=0, iters=4096):
    """Wave-iterations per second over the device of the matrix-core probe's
    three kinds, measured now: 24 bf16 products, 12 SiLU rows, and both one
    after the other in a wave (two waves per SIMD)."""
    import ctypes
    path = os.path.join(ROOT, "paper_2304_06835_amd", "libvaluprobe.so")
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2304_06835_amd.build`")
    L = ctypes.CDLL(path)
    L.mfma_mix_rate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.POINTER(ctypes.c_double)]
    out = {}
    for name, kind in (("mfma", 0), ("silu", 1), ("mfma_then_silu", 2)):
        r = ctypes.c_double(0.0)
        rc = L.mfma_mix_rate(device, kind, iters, ctypes.byref(r))
        if rc != 0:
            raise RuntimeError(f"mfma_mix_rate({name}) failed with {rc}")
        out[name] = r.value
    return out


# One 16-query subtile of the fused inference kernel in the probe's units:
# layers 2 and 3 together are 256 products and 128 SiLU rows (the 2 : 1 of
# the mixed kind), layer 1 16 products (K = 4 padded to one k-block) and 64
# SiLU rows, layer 4 24 products (48 outputs padded to 3 row blocks) and no
# activation: 296 products and 192 rows in all.
MIX_PRODUCTS, MIX_ROWS = 24, 12
INFER_SUBTILE = {"mfma_then_silu": 256 / MIX_PRODUCTS, "mfma": (16 + 24) / MIX_PRODUCTS,
                 "silu": 64 / MIX_ROWS}


def coissue_ceiling(queries, kernel_ms, rates):
    """The inference kernel against what its instruction stream can reach on
    this chip: the device time the probe needs for the kernel's products and
    SiLU rows (each layer priced by the probe kind with its mix), over the
    measured kernel time.  Products alone run near the matrix-core peak, but
    a wave's activation rows barely overlap its products, so this, not the
    2.5 PFLOP/s, bounds a kernel whose every product is followed by SiLU."""
    subtiles = queries / 16.0
    ceil_s = subtiles * sum(n / rates[k] for k, n in INFER_SUBTILE.items())
    mfma_frac = rates["mfma"] * MIX_PRODUCTS * 16 * 16 * 32 * 2 / (PEAK_BF16_MFMA * 1e12)
    mix_frac = rates["mfma_then_silu"] * MIX_PRODUCTS * 16 * 16 * 32 * 2 / (PEAK_BF16_MFMA * 1e12)
    return {"ceiling_ms": ceil_s * 1e3, "frac": ceil_s * 1e3 / kernel_ms,
            "probe_products_frac_of_peak": mfma_frac,
            "probe_products_then_silu_frac_of_peak": mix_frac,
            "probe_wave_iters_per_s": rates}


_RATES = {}


def probed_rates():
    """issue_rates() once per process."""
    if "r" not in _RATES:
        _RATES["r"] = issue_rates()
    return _RATES["r"]


def issue_roofline(mix, rates, kernel_ms):
    """The launch's VALU instruction stream against the issue ceiling: the
    time the counted instructions need at the probed per-class rates (each
    wave instruction is 64 lane-operations) over the measured kernel time."""
    if mix is None or rates is None:
        return None
    classes = mix["per_launch"]
    need_s = sum(classes[c] * 64.0 / rates[VALU_CLASS_PROBE[c]] for c in classes)
    simd_clocks = 1024 * 2.4e9 * kernel_ms * 1e-3  # 256 CUs x 4 SIMDs at the rated clock
    total = sum(classes.values())
    return {"valu_wave_instr_per_launch": total,
            "achieved_wave_instr_per_simd_clock": total / simd_clocks,
            "ceiling_wave_instr_per_simd_clock": total / (1024 * 2.4e9 * need_s),
            "frac": need_s / (kernel_ms * 1e-3),
            "lanes_active_per_instr": mix.get("lanes_active_per_instr"),
            "class_mix": {c: classes[c] / total for c in classes},
            "probe_lane_ops_per_simd_clock": {k: v / (1024 * 2.4e9) for k, v in rates.items()}}


def output_checks(e, out):
    """Checks on the whole GPU output that need no oracle: Robertson's
    conserved sum y1 + y2 + y3 = 1 (every Rosenbrock step preserves it up to
    rounding), and for the GBM Euler-Maruyama ensemble the exact discrete
    moments of the scheme: Z = X_N / (1 + mu h)^N has mean 1 and variance
    ((1 + mu h)^2 + sigma^2 h)^N / (1 + mu h)^(2N) - 1 per path, so the
    standardised sum of Z - 1 over all paths and components is N(0, 1)."""
    import numpy as np
    if e.system == "robertson":
        return {"invariant_max_abs_sum_minus_1":
                float(np.abs(out[-1].astype(np.float64).sum(axis=0) - 1.0).max())}
    if e.system == "gbm4" and e.alg == "em":
        mu = e.params[0].astype(np.float64)
        sg = e.params[1].astype(np.float64)
        h, n = e.dt, e.n_steps
        a = 1.0 + mu * h
        var = ((a * a + sg * sg * h) / (a * a)) ** n - 1.0
        z = out[-1].astype(np.float64) / (e.u0.astype(np.float64) * a ** n) - 1.0
        zs = float(z.sum() / np.sqrt(z.shape[0] * var.sum()))
        zv = z * z - var          # second moment of Z - 1, per path
        return {"em_mean_z_score": zs,
                "em_second_moment_rel_dev": float(zv.sum() / (z.shape[0] * var.sum()))}
    return {}


def cpu_model():
    """The host CPU's model name (lscpu, else /proc/cpuinfo) and the cores it offers."""
    import os
    import subprocess
    name = None
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            if line.startswith("Model name:"):
                name = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    if name is None:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    return {"model": name, "logical_cpus": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0))}


def cpu_baseline(e, gpu_out, seconds):
    """The oracle timed on the host cores on a bounded sample of the same
    workload, plus the max normwise error of the GPU result against the FP64
    oracle (truth at tol 1e-12 for adaptive solvers) on a 4096 subsample."""
    import numpy as np

    import oracle
    from paper_2304_06835_amd import workloads as W
    nth = oracle.default_threads()
    sysid = {"lorenz": oracle.LORENZ, "robertson": oracle.ROBERTSON, "orego": oracle.OREGO,
             "hires": oracle.HIRES, "pollu": oracle.POLLU}.get(e.system)

    def sub(idx):
        return (np.ascontiguousarray(e.params[:, idx]), np.ascontiguousarray(e.u0[:, idx]),
                np.ascontiguousarray(e.tspan[:, idx]))

    def run(idx, tol=None):
        p, u, ts = sub(idx)
        if e.alg in ("em", "siea"):
            sid = {"gbm4": oracle.GBM4, "crn": oracle.CRN}[e.system]
            oalg = oracle.EM if e.alg == "em" else oracle.SIEA
            return oracle.sde(sid, oalg, p, u, e.dt, e.n_steps, e.seed, ids=idx,
                              nthreads=nth)[None]
        alg = {"tsit5": oracle.TSIT5, "rodas4": oracle.RODAS4, "ros23": oracle.ROS23,
               "rodas5p": oracle.RODAS5P}[e.alg]
        if tol is not None and alg == oracle.ROS23:  # the truth comes from the 4th-order method
            alg = oracle.RODAS4
        at = e.abstol if tol is None else tol
        rt = e.reltol if tol is None else tol
        return oracle.solve(sysid, alg, p, u, ts, at, rt, e.theta, h0=e.h0, nthreads=nth)[0]

    # pilot runs of growing size until one takes >= 0.5 s, then size the
    # sample for about `seconds` of wall time
    k = 4096
    while True:
        idx = W.sample_indices(e.n, min(k, e.n))
        t0 = time.perf_counter()
        run(idx)
        dt = time.perf_counter() - t0
        if dt >= 0.5 or k >= e.n:
            break
        k *= 4
    rate = len(idx) / max(dt, 1e-6)
    k = int(min(e.n, max(1024, rate * seconds)))
    idx = W.sample_indices(e.n, k)
    t0 = time.perf_counter()
    run(idx)
    dt = time.perf_counter() - t0
    res = {"value": len(idx) / dt, "unit": "trajectories/s", "cores": nth, "kind": "oracle",
           "sample": f"{len(idx)} of {e.n} trajectories (every {e.n // len(idx)}-th), "
                     f"FP64 C oracle, OpenMP over trajectories, {dt:.1f} s",
           "cpu_model": cpu_model()}
    idx = W.sample_indices(e.n, 4096)
    g = gpu_out[:, :, idx].astype(np.float64)
    if e.alg in ("em", "siea"):
        ref = run(idx)
        g = g[-1:]  # the final state
        err = float((np.abs(g - ref) / np.abs(ref)).max())
        kind = "pathwise relative error vs FP64 oracle on the same Philox stream"
    else:
        truth = run(idx, tol=1e-12)
        err = float((np.abs(g - truth).max(axis=1) / np.abs(truth).max(axis=1)).max())
        kind = "max normwise relative error vs FP64 oracle at tol 1e-12"
    return res, {"max_rel_err": err, "subsample": len(idx), "kind": kind}


def form_variants(e, precision, steps, base_out, plain_ms, save_mode=0, forms=None):
    """Every work-assignment form on the same inputs: time and bitwise check."""
    out = {}
    for name, opts in (forms or FORMS).items():
        r = Runner(e, precision, save_mode=save_mode, **opts)
        _, ms, _ = r.time(max(3, steps // 2), 1)
        same = bool((r.host_out().view("u1") == base_out.view("u1")).all())
        out[name] = {"kernel_ms": ms, "traj_per_s": e.n / (ms * 1e-3),
                     "speedup_vs_plain": plain_ms / ms if plain_ms else None,
                     "bitwise_equal_to_headline": same}
        del r
    return out


def stiff_method_variant(alg, steps, rodas4_forms):
    """The Robertson ensemble with another stiff method (Rosenbrock23 or
    Rodas5P) instead of Rodas4: every form (bitwise check against its own
    plain form), attempts, the algorithmic rate of the fastest form, its
    speedup over the fastest Rodas4 form, and the error of a 4096 subsample
    against the FP64 truth (Rodas4 oracle at tol 1e-12)."""
    import numpy as np

    import oracle
    from paper_2304_06835_amd import workloads as W
    e = W.robertson(alg=alg)
    base = _plain_out(e)
    fv = form_variants(e, 32, steps, base, None, forms=STIFF_FORMS)
    pm = fv["plain"]["kernel_ms"]
    for v in fv.values():
        v["speedup_vs_plain"] = pm / v["kernel_ms"]
    best = min(fv, key=lambda k: fv[k]["kernel_ms"])
    r = Runner(e, 32, **STIFF_FORMS[best])
    attempts, stats = r.attempts()
    del r
    ms = fv[best]["kernel_ms"]
    fl = FLOPS[(alg, "robertson")] * attempts / (ms * 1e-3) / 1e12
    idx = W.sample_indices(e.n, 4096)
    truth = oracle.solve(oracle.ROBERTSON, oracle.RODAS4, np.ascontiguousarray(e.params[:, idx]),
                         np.ascontiguousarray(e.u0[:, idx]), np.ascontiguousarray(e.tspan[:, idx]),
                         1e-12, 1e-12, e.theta, h0=e.h0)[0]
    got = base[:, :, idx].astype(np.float64)
    err = np.abs(got - truth).max(axis=1) / np.abs(truth).max(axis=1)
    r4 = min(v["kernel_ms"] for v in rodas4_forms.values())
    st = stats.cpu().numpy().sum(axis=0)
    return {"forms": fv, "fastest_form": best, "attempts_per_traj_mean": float(st.mean()),
            "attempts_per_traj_max": int(st.max()), "achieved_tflops": fl,
            "frac_of_fp32_peak": fl / PEAK[32], "speedup_vs_fastest_rodas4": r4 / ms,
            "max_rel_err_vs_truth_4096": float(err.max())}


def stiff_variant(steps):
    """The stiff test problems of appendix B.1 at the paper's 8192
    trajectories: Rodas4 and Rosenbrock23 in FP32 and FP64 (fastest of the
    plain and sorted forms for the one-lane-per-trajectory OREGO and HIRES;
    POLLU runs one trajectory per 32-lane group), against the FP64 oracle
    solving all 8192 on the host cores with the same method and tolerance."""
    import numpy as np

    import oracle
    from paper_2304_06835_amd import workloads as W
    res = {}
    for name in ("orego", "hires", "pollu"):
        for alg in ("rodas4", "rodas5p", "ros23"):
            e = W.stiff(name, alg=alg)
            sid = {"orego": oracle.OREGO, "hires": oracle.HIRES, "pollu": oracle.POLLU}[name]
            oalg = {"rodas4": oracle.RODAS4, "rodas5p": oracle.RODAS5P,
                    "ros23": oracle.ROS23}[alg]
            t0 = time.perf_counter()
            oracle.solve(sid, oalg, e.params, e.u0, e.tspan, e.abstol, e.reltol, e.theta)
            cpu_s = time.perf_counter() - t0
            row = {"cpu_oracle_ms": cpu_s * 1e3, "cpu_cores": oracle.default_threads()}
            for prec in (32, 64):
                ep = e if prec == 32 else W.stiff(name, alg=alg, dtype=np.float64)
                forms = {"plain": {"form": 0}} if name == "pollu" else {
                    "plain": {"form": 0}, "sorted": {"form": 2, "block": 256}}
                best = None
                for fname, opts in forms.items():
                    r = Runner(ep, prec, **opts)
                    _, ms, _ = r.time(max(3, steps // 3), 1)
                    if best is None or ms < best[1]:
                        attempts, _ = r.attempts()
                        best = (fname, ms, attempts)
                    del r
                fname, ms, attempts = best
                row[f"fp{prec}"] = {"form": fname, "kernel_ms": ms, "traj_per_s": e.n / (ms * 1e-3),
                                    "attempts_per_traj": attempts / e.n,
                                    "speedup_vs_cpu_oracle": cpu_s * 1e3 / ms}
            res[f"{name}_{alg}"] = row
    return res


def mixed_variant(steps):
    """Mixed systems in one launch (ens_solve_mixed) against the same groups
    solved by separate launches one after another on the stream (each in
    the sorted form with block 256), Rodas4 FP32: the appendix-B.1 OREGO
    ensemble and a Robertson ensemble at the paper's 8192 trajectories each
    (small ensembles whose single launches cannot fill the GPU), and at
    2^20 Robertson + 2^16 OREGO.  The answers are bitwise the same."""
    import numpy as np
    import torch

    import paper_2304_06835_amd as ens
    from paper_2304_06835_amd import workloads as W
    res = {}
    for label, n_rob, n_or in (("robertson_8192+orego_8192", 8192, 8192),
                               ("robertson_2p20+orego_2p16", 1 << 20, 1 << 16)):
        gs = [W.robertson(N=n_rob), W.stiff("orego", N=n_or)]
        dev_g = [{"system": e.system, "params": dev(e.params), "u0": dev(e.u0),
                  "tspan": dev(e.tspan)} for e in gs]
        theta = [1.0]
        outs = [torch.empty((1, 3, e.n), dtype=torch.float32, device="cuda") for e in gs]
        for g, o in zip(dev_g, outs):
            g["out"] = o
        # one block per chunk (default) and the persistent queue (form 3)
        mixed = ens.Solver(0, precision=32, h0=1e-4)
        _, b_ms, _ = event_time(lambda: mixed.solve_mixed(dev_g, "rodas4", 1e-8, 1e-6, theta),
                                max(3, steps), 2)
        block_h = [o.cpu().numpy() for o in outs]
        mixed.set(form=3)
        _, m_ms, _ = event_time(lambda: mixed.solve_mixed(dev_g, "rodas4", 1e-8, 1e-6, theta),
                                max(3, steps), 2)
        mixed_h = [o.cpu().numpy() for o in outs]
        sep = ens.Solver(0, precision=32, h0=1e-4, form=2, block=256)

        def separate():
            for g, o in zip(dev_g, outs):
                sep.solve(g["system"], g["params"], g["u0"], g["tspan"], "rodas4", 1e-8, 1e-6,
                          theta, out=o)
        _, s_ms, _ = event_time(separate, max(3, steps), 2)
        same = all(np.array_equal(a.view(np.uint8), o.cpu().numpy().view(np.uint8)) and
                   np.array_equal(b.view(np.uint8), a.view(np.uint8))
                   for a, b, o in zip(mixed_h, block_h, outs))
        n = sum(e.n for e in gs)
        res[label] = {"mixed_persistent_ms": m_ms, "mixed_block_per_chunk_ms": b_ms,
                      "separate_launches_ms": s_ms,
                      "speedup_vs_separate_persistent": s_ms / m_ms,
                      "speedup_vs_separate_block_per_chunk": s_ms / b_ms,
                      "traj_per_s_mixed_best": n / (min(m_ms, b_ms) * 1e-3),
                      "bitwise_equal_to_separate": same}
        mixed.close()
        sep.close()
    return res


def config_variant(name, precision, steps, alg=""):
    """Another configuration of the path at its own size: time, throughput,
    algorithmic rate and the error against the FP64 oracle.  Lorenz FP64 is
    compared on all 8192 trajectories with the oracle at the same method and
    tolerance; GBM pathwise on 4096 trajectories with the oracle drawing the
    same Philox words, plus the standardised mean of X(1) / E[X(1)] over the
    whole ensemble (exact discrete mean of Euler-Maruyama: (1 + mu h)^N)."""
    import numpy as np

    import oracle
    from paper_2304_06835_amd import workloads as W
    e = make_workload(name, 0, alg)
    r = Runner(e, precision, **FORMS["plain"])
    attempts, _ = r.attempts()
    _, ms, _ = r.time(max(3, steps), 2)
    out = r.host_out()
    fl = FLOPS[(e.alg, e.system)] * attempts / (ms * 1e-3) / 1e12
    res = {"workload": describe(e), "kernel_ms": ms, "traj_per_s": e.n / (ms * 1e-3),
           "achieved_tflops": fl, "frac_of_peak": fl / PEAK[precision]}
    mix = recorded_valu_mix(f"{e.name}/{e.alg}/plain")
    if mix is not None:
        res["issue"] = issue_roofline(mix, probed_rates(), ms)
    if e.alg in ("em", "siea"):
        sid = {"gbm4": oracle.GBM4, "crn": oracle.CRN}[e.system]
        oalg = oracle.EM if e.alg == "em" else oracle.SIEA
        k = 4096 if e.system == "gbm4" else 2048
        idx = W.sample_indices(e.n, k)
        P, U = np.ascontiguousarray(e.params[:, idx]), np.ascontiguousarray(e.u0[:, idx])
        t0 = time.perf_counter()
        ref = oracle.sde(sid, oalg, P, U, e.dt, e.n_steps, e.seed, ids=idx)
        cpu_s = time.perf_counter() - t0
        got = out[-1][:, idx].astype(np.float64)
        rel = np.abs(got - ref).max(axis=0) / np.abs(ref).max(axis=0)
        res["pathwise_rel_err_max"] = float(rel.max())
        res["pathwise_rel_err_median"] = float(np.median(rel))
        res["cpu_oracle"] = {"traj_per_s": k / cpu_s, "cores": oracle.default_threads(),
                             "sample": f"{k} of {e.n} trajectories"}
        res["speedup_vs_cpu_oracle"] = (e.n / (ms * 1e-3)) / (k / cpu_s)
        if e.system == "gbm4" and e.alg == "em":
            mu = e.params[0].astype(np.float64)
            z = out[0].astype(np.float64) / ((1.0 + mu * e.dt) ** e.n_steps)[None, :]
            res["standardised_mean_of_X1"] = float(z.mean())
    else:
        ref = oracle.solve(oracle.LORENZ, oracle.TSIT5, e.params, e.u0, e.tspan, e.abstol,
                           e.reltol, e.theta)[0]
        res["max_rel_err_vs_oracle_same_tol"] = float(
            (np.abs(out - ref).max(axis=1) / np.abs(ref).max(axis=1)).max())
    del r
    return res


def surrogate_variant(epochs, plain_ms_2p24, headline_ms_2p24=None):
    """Learned surrogate (4 -> 256 -> 256 -> 256 -> 48, bf16 MFMA): trained on
    2^20 solver trajectories, then the audited solve of 2^24 fresh queries
    (1% audit by the FP32 solver, fallback where audited error > 1e-3) timed
    against the plain solver on the same queries."""
    import numpy as np
    import torch

    import oracle
    import paper_2304_06835_amd as ens
    from paper_2304_06835_amd import workloads as W
    s = ens.Solver(0, precision=32)
    tr = W.lorenz_fp32(N=1 << 20, seed=W.SEEDS["surr_train"])
    P, U, T = dev(tr.params), dev(tr.u0), dev(tr.tspan)
    y = s.solve("lorenz", P, U, T, "tsit5", tr.abstol, tr.reltol, tr.theta)
    m = ens.Surrogate(s, seed=1)
    m.fit_norm(P, U, y.view(48, -1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = m.train(P, U, y.view(48, -1), epochs=epochs, batch=4096, lr_max=3e-3, lr_min=3e-5,
                     seed=11)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    scaling = train_batch_scaling(s, P, U, y)
    del P, U, T, y
    s.set(save_mode=1)  # the audited solve's solver part saves as the headline does
    q = W.lorenz_fp32(seed=W.SEEDS["surr_query"])
    Pq, Uq, Tq = dev(q.params), dev(q.u0), dev(q.tspan)
    out = torch.empty((16, 3, q.n), dtype=torch.float32, device="cuda")
    used = torch.empty(q.n, dtype=torch.uint8, device="cuda")
    rep = torch.zeros(4, dtype=torch.float32, device="cuda")
    _, pred_ms, _ = event_time(lambda: m.predict(Pq, Uq, out=out), 5, 2)
    mfma = MLP_FLOPS_PER_QUERY * q.n / (pred_ms * 1e-3) / 1e12
    train_tf = MLP_TRAIN_FLOPS_PER_SAMPLE * (1 << 20) * epochs / train_s / 1e12
    res = {
        "training": {"samples": 1 << 20, "epochs": epochs, "batch": 4096, "seconds": train_s,
                     "final_loss": float(losses[-1].item()),
                     "mfma": {"achieved": train_tf, "peak": PEAK_BF16_MFMA, "unit": "TFLOP/s",
                              "frac": train_tf / PEAK_BF16_MFMA},
                     "batch_scaling": scaling},
        "predict_ms": pred_ms,
        "predict_mfma": {"achieved": mfma, "peak": PEAK_BF16_MFMA, "unit": "TFLOP/s",
                         "frac": mfma / PEAK_BF16_MFMA,
                         "coissue": coissue_ceiling(q.n, pred_ms, mfma_mix_rates())},
        "queries": q.n, "plain_solver_ms": plain_ms_2p24,
        "predict_only_speedup_vs_plain": plain_ms_2p24 / pred_ms,
    }
    idx = W.sample_indices(q.n, 4096)
    truth = oracle.solve(oracle.LORENZ, oracle.TSIT5, np.ascontiguousarray(q.params[:, idx]),
                         np.ascontiguousarray(q.u0[:, idx]), np.ascontiguousarray(q.tspan[:, idx]),
                         1e-12, 1e-12, q.theta)[0]
    # the configured audit tolerance (1e-3), and a looser one for context
    for tol in (1e-3, 1e-2):
        _, solve_ms, _ = event_time(
            lambda: m.solve(Pq, Uq, Tq, q.abstol, q.reltol, q.theta, audit_frac=0.01,
                            fallback_tol=tol, audit_seed=W.SEEDS["surr_audit"], out=out,
                            used=used, report=rep), 3, 1)
        rep_h = rep.cpu().numpy()
        used_h = used.cpu().numpy()
        g = out.cpu().numpy()[:, :, idx].astype(np.float64)
        err = (np.abs(g - truth).max(axis=1) / np.abs(truth).max(axis=1)).max(axis=0)
        res[f"audited_solve_tol_{tol:g}"] = {
            "ms": solve_ms, "traj_per_s": q.n / (solve_ms * 1e-3),
            "speedup_vs_plain": plain_ms_2p24 / solve_ms,
            "speedup_vs_headline_solver": (headline_ms_2p24 / solve_ms
                                           if headline_ms_2p24 else None),
            "audited": int(rep_h[0]), "fallback": int(rep_h[1]), "flagged_bins": int(rep_h[2]),
            "max_audit_err": float(rep_h[3]),
            "network_answered_frac": float((used_h == 0).mean()),
            "max_rel_err_vs_oracle": float(err.max()),
            "median_rel_err_vs_oracle": float(np.median(err))}
    return res


def surrogate_only(epochs, scaling=False):
    """Training and inference of the surrogate and one audited solve at
    tolerance 1e-3: the workload of the MFMA counter and kernel profiles."""
    import torch

    import paper_2304_06835_amd as ens
    from paper_2304_06835_amd import workloads as W
    s = ens.Solver(0, precision=32)
    tr = W.lorenz_fp32(N=1 << 20, seed=W.SEEDS["surr_train"])
    P, U, T = dev(tr.params), dev(tr.u0), dev(tr.tspan)
    y = s.solve("lorenz", P, U, T, "tsit5", tr.abstol, tr.reltol, tr.theta)
    m = ens.Surrogate(s, seed=1)
    m.fit_norm(P, U, y.view(48, -1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.train(P, U, y.view(48, -1), epochs=epochs, batch=4096, lr_max=3e-3, lr_min=3e-5, seed=11)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    q = W.lorenz_fp32(seed=W.SEEDS["surr_query"])
    Pq, Uq = dev(q.params), dev(q.u0)
    out = torch.empty((16, 3, q.n), dtype=torch.float32, device="cuda")
    _, pred_ms, _ = event_time(lambda: m.predict(Pq, Uq, out=out), 5, 2)
    # the audited solve at tolerance 1e-3 (every bin fails its audit there)
    s.set(save_mode=1)
    Tq = dev(q.tspan)
    _, audit_ms, _ = event_time(
        lambda: m.solve(Pq, Uq, Tq, q.abstol, q.reltol, q.theta, audit_frac=0.01,
                        fallback_tol=1e-3, audit_seed=W.SEEDS["surr_audit"], out=out), 3, 1)
    train_tf = MLP_TRAIN_FLOPS_PER_SAMPLE * (1 << 20) * epochs / train_s / 1e12
    print(json.dumps({"surrogate_only": {
        "audited_solve_tol_0.001_ms": audit_ms,
        "train_epochs": epochs, "train_samples": 1 << 20, "train_seconds": train_s,
        "train_tflops": train_tf, "predict_ms": pred_ms, "queries": q.n,
        "predict_tflops": MLP_FLOPS_PER_QUERY * q.n / (pred_ms * 1e-3) / 1e12,
        "predict_coissue": coissue_ceiling(q.n, pred_ms, mfma_mix_rates()),
        "train_batch_scaling": train_batch_scaling(s, P, U, y) if scaling else None}}),
        flush=True)


def train_batch_scaling(s, P, U, y, batches=(4096, 16384, 65536), epochs=2):
    """Training throughput of a fresh model at several minibatch sizes (the
    same kernels; per-step launch and latency costs amortised over more
    samples): MFMA TFLOP/s over `epochs` epochs of the 2^20 training set."""
    import torch

    import paper_2304_06835_amd as ens
    out = {}
    for b in batches:
        m = ens.Surrogate(s, seed=1)
        m.fit_norm(P, U, y.view(48, -1))
        m.train(P, U, y.view(48, -1), epochs=1, batch=b, seed=3)  # warm-up, workspace
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses = m.train(P, U, y.view(48, -1), epochs=epochs, batch=b, lr_max=3e-3, lr_min=3e-5,
                         seed=11)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        steps = ((1 << 20) // b) * epochs
        tf = MLP_TRAIN_FLOPS_PER_SAMPLE * steps * b / dt / 1e12
        out[str(b)] = {"step_us": dt / steps * 1e6, "tflops": tf, "frac": tf / PEAK_BF16_MFMA,
                       "loss_after": float(losses[-1].item())}
        del m
    return out


def main():
    args = parse()
    if args.record_counters:
        mix, tr = record_counters(args.record_counters)
        print(json.dumps({"recorded": {
            "valu_mix": {k: v["per_launch"] for k, v in mix.items() if k != "_doc"},
            "traffic": {k: v["traffic_over_algorithmic"] for k, v in tr.items() if k != "_doc"}}}))
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.surrogate_only:
        surrogate_only(args.surrogate_epochs, args.surrogate_scaling)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(trajectories are independent: N GPUs would each solve their own slice)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    e = make_workload(args.workload, args.n, args.alg)
    precision = 64 if args.workload == "lorenz_fp64" else 32
    form = args.form or DEFAULT_FORM[args.workload]
    save = args.save_mode or DEFAULT_SAVE.get(args.workload, "landing")
    if e.alg != "tsit5":
        save = "landing"
    tuned = None
    if e.alg in ("em", "siea"):
        form = "plain"
    if form == "auto":
        from paper_2304_06835_amd import workloads as W
        k = min(e.n, 1 << 18)
        idx = W.sample_indices(e.n, k)
        pe = make_workload(args.workload, 0, args.alg)
        pe.params, pe.u0, pe.tspan = (e.params[:, idx].copy(), e.u0[:, idx].copy(),
                                      e.tspan[:, idx].copy())
        probe = Runner(pe, precision)
        _, tuned = probe.s.autotune(pe.system, probe.params, probe.u0, probe.tspan, pe.alg,
                                    pe.abstol, pe.reltol, pe.theta)
        opts = dict(tuned)
    else:
        opts = dict(LAUNCH_FORMS[form])
    opts["save_mode"] = SAVE_MODES[save]
    r = Runner(e, precision, **opts)
    print(f"[bench] {e.name} N={e.n} precision={precision} form={form} save={save}",
          file=sys.stderr, flush=True)

    attempts, stats = r.attempts()
    wall, ker_ms, ker_min = r.time(args.steps, args.warmup)
    out_host = r.host_out()
    value = e.n * args.steps / wall
    ms_per_step = wall / args.steps * 1e3
    fpa = FLOPS.get((e.alg, e.system))  # not counted for the appendix-B.1 problems
    dense_saves = e.n * (len(e.theta) - 1) if save == "dense" else 0
    flops = fpa * attempts + DENSE_FLOPS_PER_SAVE * dense_saves if fpa else None
    peak = PEAK[precision]
    achieved = flops / (ker_ms * 1e-3) / 1e12 if flops else None
    roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak if achieved else None,
            "traffic": recorded_traffic(e.name, form + ("/dense" if save == "dense" else ""), 1),
            "kernel": kernel_name(e, form, precision),
            "kernel_ms_avg": ker_ms, "kernel_ms_min": ker_min,
            "flops_per_launch": flops, "attempted_steps": attempts, "flops_per_attempt": fpa,
            "dense_output_saves": dense_saves, "flops_per_dense_save": DENSE_FLOPS_PER_SAVE}
    mix = recorded_valu_mix(f"{e.name}/{e.alg}/{form}" + ("/dense" if save == "dense" else ""))
    roof["issue"] = issue_roofline(mix, probed_rates(), ker_ms) if mix is not None else None
    st = stats.cpu().numpy()
    steps_per = st.sum(axis=0)
    config = {"workload": describe(e), "name": e.name, "n_traj": e.n, "alg": e.alg,
              "abstol": e.abstol, "reltol": e.reltol, "n_save": len(e.theta),
              "form": form, "save_times": save,
              "launch": {k2: int(r.s.get(k2)) for k2 in ("form", "block", "tpl", "save_mode", "stage_saves")},
              "tuned": tuned,
              "steps_per_traj_mean": float(steps_per.mean()),
              "steps_per_traj_max": int(steps_per.max()),
              "rejected_frac": float(st[1].sum() / max(1, st.sum()))}
    if e.alg not in ("em", "siea"):
        import numpy as np
        config["steps_per_traj_cv"] = float(steps_per.std() / max(1e-30, steps_per.mean()))
        config["steps_per_traj_quantiles"] = {
            q: float(np.quantile(steps_per, float(q))) for q in ("0.5", "0.9", "0.99")}
    config.update(output_checks(e, out_host))
    del r

    variants = {}
    if not args.no_variants and e.alg not in ("em", "siea"):
        fv = form_variants(e, precision, args.steps, out_host, None, SAVE_MODES[save],
                           forms=TSIT5_FORMS if e.alg == "tsit5" else None)
        plain_ms = fv["plain"]["kernel_ms"]
        for v in fv.values():
            v["speedup_vs_plain"] = plain_ms / v["kernel_ms"]
        variants["forms"] = fv
        if e.alg == "tsit5":
            other = "landing" if save == "dense" else "dense"
            ov = form_variants(e, precision, args.steps, _plain_out(e, SAVE_MODES[other]), None,
                               SAVE_MODES[other], forms=TSIT5_FORMS)
            for v in ov.values():
                v["speedup_vs_plain_headline_save_mode"] = plain_ms / v["kernel_ms"]
            variants[f"forms_{other}_saves"] = ov
        if e.name == "lorenz_fp32":
            import numpy as np
            r64 = Runner(e, 64)
            r64.params = dev(e.params.astype(np.float64))
            r64.u0 = dev(e.u0.astype(np.float64))
            r64.out = torch.empty((len(e.theta), 3, e.n), dtype=torch.float64, device="cuda")
            _, k3, _ = r64.time(max(3, args.steps // 2), 1)
            variants["fp64_plain"] = {"kernel_ms": k3, "traj_per_s": e.n / (k3 * 1e-3),
                                      "fp32_headline_speedup": k3 / ker_ms}
            del r64
            rob = make_workload("robertson", 0)
            rv = form_variants(rob, 32, args.steps, _plain_out(rob), None, forms=STIFF_FORMS)
            rp = rv["plain"]["kernel_ms"]
            for v in rv.values():
                v["speedup_vs_plain"] = rp / v["kernel_ms"]
            variants["robertson_2p20_forms"] = rv
            variants["robertson_2p20_ros23"] = stiff_method_variant("ros23", args.steps, rv)
            r5 = stiff_method_variant("rodas5p", args.steps, rv)
            variants["robertson_2p20_rodas5p"] = r5
            # the paper's stiff table gives times relative to Rodas5P (section 6.4)
            t5 = r5["forms"][r5["fastest_form"]]["kernel_ms"]
            r23 = variants["robertson_2p20_ros23"]
            variants["robertson_2p20_time_relative_to_rodas5p"] = {
                "rodas5p": 1.0,
                "rodas4": min(v["kernel_ms"] for v in rv.values()) / t5,
                "ros23": r23["forms"][r23["fastest_form"]]["kernel_ms"] / t5}
            variants["lorenz_fp64_8192"] = config_variant("lorenz_fp64", 64, args.steps)
            variants["gbm_em_2p22"] = config_variant("gbm", 32, args.steps)
            variants["gbm_siea_2p22"] = config_variant("gbm", 32, args.steps, alg="siea")
            variants["crn_em_1e6"] = config_variant("crn", 32, 3)
            variants["stiff_appendix_b1_8192"] = stiff_variant(args.steps)
            variants["mixed_systems_one_launch"] = mixed_variant(args.steps)
            if not args.no_surrogate:
                variants["surrogate"] = surrogate_variant(args.surrogate_epochs, plain_ms,
                                                          ker_ms)

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


def _plain_out(e, save_mode=0):
    """Host copy of the plain form's answer (the reference of the bitwise checks)."""
    r = Runner(e, 32, save_mode=save_mode, **FORMS["plain"])
    r.solve()
    out = r.host_out()
    del r
    return out


if __name__ == "__main__":
    main()
