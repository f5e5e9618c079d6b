"""GPU parity of the adaptive ODE kernels against the FP64 oracle.

Inputs come from the seeded workload generators; the oracle receives the
same (FP32-rounded where the GPU runs FP32) values promoted to FP64.
"""
import numpy as np
import pytest

from paper_2304_06835_amd import workloads as W
from tests.gpu_util import banner, normwise, to_dev, to_host

pytestmark = pytest.mark.gpu

# Bars (derivations in the design notes):
#  - FP32 state at reltol = abstol = 1e-6 vs the 1e-12 oracle: 1e-4 normwise
#    (the accuracy target of the FP32 precision form).
#  - FP64 kernel vs the oracle run with the same method, controller and
#    tolerance: same algorithm, rounding-order differences only, so most
#    trajectories agree to ~1e-12; a flipped accept/reject decision can move
#    one by at most the tolerance-level global error, bounded by 1e-6 at
#    tol 1e-8 on t in [0, 1].
FP32_BAR = 1e-4
FP64_SAME_ALG_BAR = 1e-6


@pytest.fixture(scope="module")
def ens():
    import torch
    import paper_2304_06835_amd as e
    assert torch.cuda.is_available()
    return e


def run(ens, e: W.Ensemble, precision, **opts):
    import torch
    s = ens.Solver(0, precision=precision, **opts)
    if e.h0:
        s.set(h0=e.h0)
    N = e.n
    status = torch.empty(N, dtype=torch.uint8, device="cuda")
    stats = torch.empty((2, N), dtype=torch.int32, device="cuda")
    out = s.solve(e.system, to_dev(e.params), to_dev(e.u0), to_dev(e.tspan), e.alg,
                  e.abstol, e.reltol, e.theta, status=status, stats=stats)
    res = to_host(out), to_host(status), to_host(stats)
    s.close()
    return res


def oracle_solve(orc, e: W.Ensemble, tol=None):
    sysid = {"lorenz": orc.LORENZ, "robertson": orc.ROBERTSON, "linear": orc.LINEAR}[e.system]
    alg = {"tsit5": orc.TSIT5, "rodas4": orc.RODAS4}[e.alg]
    at = e.abstol if tol is None else tol
    rt = e.reltol if tol is None else tol
    return orc.solve(sysid, alg, e.params, e.u0, e.tspan, at, rt, e.theta, h0=e.h0)


def test_lorenz_fp64_matches_oracle(ens, orc):
    e = W.lorenz_fp64(N=3001)          # ragged: 11 full blocks of 256 + 185
    banner(f"lorenz fp64 tsit5 N={e.n}")
    out, st, stats = run(ens, e, 64)
    assert (st == 0).all()
    ref, rst, na, nr = oracle_solve(orc, e)
    err = normwise(out, ref)
    print("fp64 vs same-settings oracle: max %.3e median %.3e" % (err.max(), np.median(err)))
    assert err.max() <= FP64_SAME_ALG_BAR
    assert np.median(err) <= 1e-12
    # step counts agree with the oracle's for almost every trajectory
    assert np.mean((stats[0] == na) & (stats[1] == nr)) > 0.95
    truth, *_ = oracle_solve(orc, e, tol=1e-12)
    et = normwise(out, truth)
    eo = normwise(ref, truth)
    print("fp64 vs truth: gpu %.3e oracle %.3e" % (et.max(), eo.max()))
    assert et.max() <= 2 * eo.max() + 1e-12


def test_lorenz_fp32_precision_form(ens, orc):
    e = W.lorenz_fp32(N=4099)
    banner(f"lorenz fp32 tsit5 N={e.n} n_save=16")
    out, st, stats = run(ens, e, 32)
    assert (st == 0).all()
    truth, *_ = oracle_solve(orc, e, tol=1e-12)
    err = normwise(out, truth)
    same, *_ = oracle_solve(orc, e)
    eo = normwise(same, truth)
    print("fp32 vs truth: max %.3e (oracle at same tol: %.3e), mean steps %.1f"
          % (err.max(), eo.max(), stats.sum(0).mean()))
    assert err.max() <= FP32_BAR


@pytest.mark.parametrize("precision", [32, 64])
def test_tsit5_forms_and_launch_shapes_bitwise_equal(ens, precision):
    e = W.lorenz_fp32(N=5003) if precision == 32 else W.lorenz_fp64(N=5003)
    if precision == 32:
        e.theta = e.theta[::3]
    banner(f"tsit5 forms fp{precision}")
    base, st0, s0 = run(ens, e, precision)
    for opts in ({"block": 64}, {"block": 128, "tpl": 2}, {"tpl": 4},
                 {"form": 1}, {"form": 1, "block": 64, "refill": 1},
                 {"form": 1, "block": 128, "refill": 32}, {"form": 1, "grid": 3},
                 {"form": 2}, {"form": 2, "block": 256}, {"form": 2, "block": 512, "tpl": 2},
                 {"form": 2, "block": 256, "tpl": 4}, {"form": 3}, {"form": 3, "block": 64},
                 {"form": 3, "block": 128, "grid": 5}):
        out, st, s = run(ens, e, precision, **opts)
        assert np.array_equal(out.view(np.uint8), base.view(np.uint8)), opts
        assert np.array_equal(st, st0) and np.array_equal(s, s0), opts


@pytest.mark.parametrize("precision,n_save", [(32, 1), (32, 21), (32, 22), (64, 10), (64, 11)])
def test_sorted_staged_saves_bitwise_equal(ens, precision, n_save):
    """With stage_saves, the sorted form with block 256 and one round keeps a
    block's saves in LDS when n_save x 3 x 256 values fit in 64 KiB (FP32:
    n_save <= 21, FP64: <= 10) and copies them out when the block is done.  On both sides
    of that limit, in both save modes, with a ragged tail, a span with
    tf == t0, an invalid span and a non-finite parameter, it gives the plain
    form's bits, statuses and step counts."""
    e = W.lorenz_fp32(N=1000, seed=31)
    if precision == 64:
        e.params, e.u0 = e.params.astype(np.float64), e.u0.astype(np.float64)
    e.theta = (np.arange(n_save, dtype=np.float64) + 1.0) / n_save
    e.tspan = np.ascontiguousarray(e.tspan.copy())
    e.tspan[1, 300] = e.tspan[0, 300]          # tf == t0: every save is u0
    e.tspan[1, 301] = e.tspan[0, 301] - 1.0    # inverted span: status 3, NaN saves
    e.params[1, 302] = np.nan                  # non-finite error estimate
    banner(f"sorted staged saves fp{precision} n_save={n_save}")
    for mode in (0, 1):
        base, st0, s0 = run(ens, e, precision, save_mode=mode)
        out, st, s = run(ens, e, precision, save_mode=mode, form=2, block=256, stage_saves=1)
        assert st0[300] == 0 and st0[301] == 3 and st0[302] == 3
        assert (np.delete(st0, [301, 302]) == 0).all(), mode
        assert np.isnan(base[:, :, 301]).all() and np.array_equal(base[-1, :, 300], e.u0[:, 300])
        assert np.array_equal(out.view(np.uint8), base.view(np.uint8)), mode
        assert np.array_equal(st, st0) and np.array_equal(s, s0), mode


@pytest.mark.parametrize("mode", [0, 1])
def test_fp32_landing_on_non_dyadic_times(ens, orc, mode):
    """FP32 lanes keep time in FP64 with a compensation term.  Spans and save
    times that no binary fraction holds exactly (per-trajectory t0 in
    [-0.7, 0.7], tf - t0 in [0.31, 0.97], save fractions j/7) must still be
    landed on and written:
    every status 0, the oracle's accuracy and step counts, and the same bits
    in the plain and sorted forms."""
    e = W.lorenz_fp32(N=2051, seed=32)
    rng = np.random.default_rng(33)
    t0 = rng.uniform(-0.7, 0.7, e.n)
    e.tspan = np.ascontiguousarray(np.stack([t0, t0 + rng.uniform(0.31, 0.97, e.n)]))
    e.theta = (np.arange(7, dtype=np.float64) + 1.0) / 7.0
    banner(f"lorenz fp32 non-dyadic times, save mode {mode}")
    out, st, stats = run(ens, e, 32, save_mode=mode)
    assert (st == 0).all(), np.unique(st, return_counts=True)
    truth, _, na, nr = oracle_solve(orc, e, tol=1e-12)
    err = normwise(out, truth)
    same, _, na, nr = orc.solve(orc.LORENZ, orc.TSIT5, e.params, e.u0, e.tspan, e.abstol,
                                e.reltol, e.theta, save_mode=mode)
    print("fp32 non-dyadic vs truth: max %.3e; attempts gpu %.1f oracle %.1f"
          % (err.max(), stats.sum(0).mean(), (na + nr).mean()))
    assert err.max() <= FP32_BAR
    assert abs(stats.sum(0).mean() / (na + nr).mean() - 1.0) < 0.03
    srt, st2, s2 = run(ens, e, 32, save_mode=mode, form=2, block=256)
    assert np.array_equal(srt.view(np.uint8), out.view(np.uint8)) and np.array_equal(s2, stats)


def test_robertson_fp32_rodas4(ens, orc):
    e = W.robertson(N=2053)
    banner(f"robertson fp32 rodas4 N={e.n}")
    out, st, stats = run(ens, e, 32)
    assert (st == 0).all()
    truth, *_ = oracle_solve(orc, e, tol=1e-12)
    same, *_ = oracle_solve(orc, e)
    err = normwise(out, truth)
    eo = normwise(same, truth)
    print("robertson fp32 vs truth: max %.3e (oracle at same tol %.3e); steps mean %.1f max %d"
          % (err.max(), eo.max(), stats.sum(0).mean(), stats.sum(0).max()))
    assert err.max() <= FP32_BAR
    # y1 + y2 + y3 = 1 is preserved by every Rosenbrock step up to FP32 rounding
    assert np.abs(out.sum(axis=1) - 1.0).max() < 1e-5


def test_robertson_fp64_matches_oracle(ens, orc):
    e = W.robertson(N=1500, dtype=np.float64)
    banner(f"robertson fp64 rodas4 N={e.n}")
    out, st, stats = run(ens, e, 64)
    assert (st == 0).all()
    ref, rst, na, nr = oracle_solve(orc, e)
    err = normwise(out, ref)
    print("robertson fp64 vs oracle: max %.3e median %.3e" % (err.max(), np.median(err)))
    assert err.max() <= FP64_SAME_ALG_BAR
    assert np.median(err) <= 1e-11
    assert np.abs(out.sum(axis=1) - 1.0).max() < 1e-12


@pytest.mark.parametrize("precision", [32, 64])
def test_rodas4_forms_bitwise_equal(ens, precision):
    e = W.robertson(N=3001, dtype=np.float32 if precision == 32 else np.float64)
    banner(f"rodas4 forms fp{precision}")
    base, st0, s0 = run(ens, e, precision)
    for opts in ({"block": 64, "tpl": 3}, {"form": 1}, {"form": 1, "refill": 4, "block": 128},
                 {"form": 2}, {"form": 2, "block": 256, "tpl": 2}, {"form": 3},
                 {"form": 3, "block": 64, "grid": 7}):
        out, st, s = run(ens, e, precision, **opts)
        assert np.array_equal(out.view(np.uint8), base.view(np.uint8)), opts
        assert np.array_equal(s, s0), opts


@pytest.mark.parametrize("alg", ["tsit5", "rodas4"])
def test_linear_closed_form_on_gpu(ens, alg):
    """du = A u with a rotation-decay block: e^{-t}(cos 2t, -sin 2t), 2 e^{-t/2}."""
    N = 130
    A = np.array([[-1.0, 2.0, 0.0], [-2.0, -1.0, 0.0], [0.0, 0.0, -0.5]])
    params = np.repeat(A.reshape(9, 1), N, axis=1)
    u0 = np.repeat(np.array([[1.0], [0.0], [2.0]]), N, axis=1)
    tf = np.linspace(0.5, 3.0, N)
    tspan = np.stack([np.zeros(N), tf])
    theta = np.array([0.25, 0.5, 1.0])
    e = W.Ensemble("lin", "linear", alg, params, u0, tspan, theta, abstol=1e-10, reltol=1e-10)
    out, st, _ = run(ens, e, 64)
    assert (st == 0).all()
    t = theta[:, None] * tf[None, :]
    ex = np.stack([np.exp(-t) * np.cos(2 * t), -np.exp(-t) * np.sin(2 * t), 2 * np.exp(-0.5 * t)],
                  axis=1)
    assert np.abs(out - ex).max() < 1e-8


def test_status_codes_and_degenerate_inputs(ens, orc):
    import torch
    N = 70
    e = W.lorenz_fp64(N=N)
    e.params[1, 5] = np.nan                # non-finite error estimate
    e.tspan[1, 7] = e.tspan[0, 7]          # tf == t0: every save is u0
    banner("status codes")
    out, st, stats = run(ens, e, 64)
    assert st[5] == 3 and np.isnan(out[:, :, 5]).all()
    assert st[7] == 0 and np.array_equal(out[0, :, 7], e.u0[:, 7]) and stats[0, 7] == 0
    assert (np.delete(st, [5]) == 0).all()
    out, st, stats = run(ens, W.lorenz_fp64(N=N), 64, maxiters=2)
    assert (st == 1).all() and (stats.sum(0) == 2).all() and np.isnan(out).all()
    # empty ensemble is a no-op
    s = ens.Solver(0, precision=64)
    z = torch.empty((3, 0), dtype=torch.float64, device="cuda")
    o = s.solve("lorenz", z, z, torch.tensor([0.0, 1.0], dtype=torch.float64, device="cuda"),
                "tsit5", 1e-6, 1e-6, [1.0])
    assert o.shape == (1, 3, 0)


def test_argument_errors_are_reported(ens):
    import torch
    s = ens.Solver(0, precision=32)
    N = 8
    p = torch.zeros((3, N), device="cuda")
    u = torch.zeros((3, N), device="cuda")
    ts = torch.tensor([0.0, 1.0], dtype=torch.float64, device="cuda")
    with pytest.raises(ens.EnsError, match="strictly increasing"):
        s.solve("lorenz", p, u, ts, "tsit5", 1e-6, 1e-6, [0.5, 0.5])
    with pytest.raises(ens.EnsError, match="abstol"):
        s.solve("lorenz", p, u, ts, "tsit5", -1.0, 1e-6, [1.0])
    with pytest.raises(ens.EnsError, match="no kernel"):
        s.solve("lorenz", p, u, ts, "em", 1e-6, 1e-6, [1.0])
    with pytest.raises(ens.EnsError, match="n_save"):
        s.solve("lorenz", p, u, ts, "tsit5", 1e-6, 1e-6, list(np.linspace(0.01, 1, 65)))
    with pytest.raises(ens.EnsError, match="refill"):
        s.set(refill=0)
    with pytest.raises(ens.EnsError, match="block"):
        s.set(block=96)
    with pytest.raises(ens.EnsError, match="stage_saves"):
        s.set(stage_saves=2)


def test_autotune_picks_a_valid_config_with_identical_results(ens):
    import torch
    e = W.lorenz_fp32(N=1 << 14)
    s = ens.Solver(0, precision=32)
    args = (to_dev(e.params), to_dev(e.u0), to_dev(e.tspan), "tsit5", 1e-6, 1e-6, e.theta)
    ref = to_host(s.solve("lorenz", *args))
    ms, cfg = s.autotune("lorenz", *args)
    print("autotune:", ms, cfg)
    assert ms > 0 and cfg["form"] in (0, 1, 2, 3)
    if cfg["form"] == 2:   # sorted: one or two blocks' worth of trajectories per sort
        assert (cfg["block"], cfg["tpl"]) in {(256, 1), (512, 1), (1024, 1), (256, 2), (512, 2)}
    elif cfg["form"] == 3:
        assert cfg["block"] in (128, 256)
    else:
        assert cfg["block"] in (64, 128, 256)
    out = to_host(s.solve("lorenz", *args))
    assert np.array_equal(out.view(np.uint8), ref.view(np.uint8))
    torch.cuda.synchronize()


def test_autotune_cache_and_file_round_trip(ens, tmp_path):
    """The autotuner's results are cached per (system, algorithm, precision,
    save mode, log2 n): a second call on the same key sets the recorded
    configuration without timing and reports the recorded time; the JSON
    file carries the entries to a new context; another size bucket is tuned
    anew and added; a malformed file is refused; clearing the cache tunes
    again."""
    import json
    import time
    e = W.lorenz_fp32(N=1 << 14)
    path = tmp_path / "tune.json"
    s = ens.Solver(0, precision=32, save_mode=1)
    s.set_autotune_file(path)
    args = (to_dev(e.params), to_dev(e.u0), to_dev(e.tspan), "tsit5", 1e-6, 1e-6, e.theta)
    ms1, cfg1 = s.autotune("lorenz", *args)
    assert not cfg1["cached"]
    rec = json.loads(path.read_text())["entries"]
    assert len(rec) == 1 and rec[0]["sys"] == 1 and rec[0]["save_mode"] == 1
    assert rec[0]["log2n"] == 14 and rec[0]["form"] == cfg1["form"]
    s.set(form=0, block=64, tpl=1)
    t0 = time.perf_counter()
    ms2, cfg2 = s.autotune("lorenz", *args)
    hit_s = time.perf_counter() - t0
    assert cfg2["cached"] and ms2 == pytest.approx(ms1, rel=1e-5)
    assert {k: cfg2[k] for k in ("form", "block", "tpl")} == \
        {k: cfg1[k] for k in ("form", "block", "tpl")}
    assert hit_s < 0.05, hit_s
    s2 = ens.Solver(0, precision=32, save_mode=1)
    s2.set_autotune_file(path)
    ms3, cfg3 = s2.autotune("lorenz", *args)
    assert cfg3["cached"] and cfg3["form"] == cfg1["form"] and cfg3["block"] == cfg1["block"]
    small = W.lorenz_fp32(N=1 << 12)
    _, cfg4 = s2.autotune("lorenz", to_dev(small.params), to_dev(small.u0), to_dev(small.tspan),
                          "tsit5", 1e-6, 1e-6, small.theta)
    assert not cfg4["cached"]
    assert sorted(r["log2n"] for r in json.loads(path.read_text())["entries"]) == [12, 14]
    bad = tmp_path / "bad.json"
    bad.write_text('{"version": 1, "entries": [{"sys": 1}]}')
    with pytest.raises(ens.EnsError, match="malformed"):
        s2.set_autotune_file(bad)
    s.set_autotune_file(None)
    _, cfg5 = s.autotune("lorenz", *args)
    assert not cfg5["cached"]
    s.close()
    s2.close()


@pytest.mark.parametrize("name", ["orego", "hires", "pollu", "gbm"])
def test_autotune_on_the_other_systems(ens, name):
    """The autotuner on the appendix problems (POLLU's grouped kernel runs its
    plain form whatever is asked) and on an SDE (plain form only): a valid
    configuration, and the same bits as the untuned solve afterwards."""
    if name == "gbm":
        e = W.gbm(N=4096)
        s = ens.Solver(0, precision=32, dt=e.dt, seed=e.seed)
        args = (to_dev(e.params), to_dev(e.u0), to_dev(e.tspan), "em", 0.0, 0.0, e.theta)
    else:
        e = W.stiff(name, N=1024)
        s = ens.Solver(0, precision=32)
        if e.h0:
            s.set(h0=e.h0)
        args = (to_dev(e.params), to_dev(e.u0), to_dev(e.tspan), e.alg, e.abstol, e.reltol,
                e.theta)
    banner(f"autotune {name}")
    ref = to_host(s.solve(e.system, *args))
    ms, cfg = s.autotune(e.system, *args)
    print(f"autotune {name}:", ms, cfg)
    assert ms > 0
    if name in ("gbm", "pollu"):
        assert cfg["form"] == 0 and cfg["block"] in (64, 128, 256)
    if name == "pollu":
        assert cfg["tpl"] == 1
    out = to_host(s.solve(e.system, *args))
    assert np.array_equal(out.view(np.uint8), ref.view(np.uint8))
    s.close()


@pytest.mark.parametrize("name", ["lorenz_fp32", "robertson"])
def test_full_size_in_the_benchmarked_launch(ens, orc, name):
    """The benchmark's workloads at their full sizes in exactly the launch
    bench.py times: 2^24 Lorenz with 16 saves read off Tsit5's dense output
    (save mode 1) in the cost-sorted form with block 256, and 2^20 Robertson
    (Rodas4, landing saves) in the same form.  Every trajectory finishes with
    status 0, 4096 sampled trajectories match the FP64 oracle at tol 1e-12
    within the FP32 bar, and the plain and both persistent forms in the same
    save mode give the same bits on the sample."""
    import torch
    e = W.lorenz_fp32() if name == "lorenz_fp32" else W.robertson()
    mode = 1 if name == "lorenz_fp32" else 0
    banner(f"{name} full size N={e.n}, sorted form block 256, save mode {mode}")
    s = ens.Solver(0, precision=32, form=2, block=256, save_mode=mode)
    if e.h0:
        s.set(h0=e.h0)
    status = torch.empty(e.n, dtype=torch.uint8, device="cuda")
    P, U, T = to_dev(e.params), to_dev(e.u0), to_dev(e.tspan)
    idx = W.sample_indices(e.n, 4096)
    idx_d = torch.from_numpy(idx.astype(np.int64)).cuda()
    out = s.solve(e.system, P, U, T, e.alg, e.abstol, e.reltol, e.theta, status=status)
    st = to_host(status)
    assert (st == 0).all()
    got = np.ascontiguousarray(to_host(out.index_select(2, idx_d)))
    sub = W.Ensemble(e.name, e.system, e.alg, np.ascontiguousarray(e.params[:, idx]),
                     np.ascontiguousarray(e.u0[:, idx]), np.ascontiguousarray(e.tspan[:, idx]),
                     e.theta, e.abstol, e.reltol, e.h0)
    truth, *_ = oracle_solve(orc, sub, tol=1e-12)
    err = normwise(got, truth)
    print("%s full size, sampled: max normwise error %.3e" % (name, err.max()))
    assert err.max() <= FP32_BAR
    for form in (0, 1, 3):
        s.set(form=form, block=256)
        o = s.solve(e.system, P, U, T, e.alg, e.abstol, e.reltol, e.theta, out=out)
        g = np.ascontiguousarray(to_host(o.index_select(2, idx_d)))
        assert np.array_equal(g.view(np.uint8), got.view(np.uint8)), form
    s.close()


def test_dense_output_fp64_matches_oracle(ens, orc):
    """Save mode 1 (Tsit5 dense output) in FP64 against the oracle's dense
    mode with the same settings: rounding-order differences only; and the
    same attempt counts for almost every trajectory."""
    e = W.lorenz_fp32(N=3001, seed=23)
    e.params, e.u0 = e.params.astype(np.float64), e.u0.astype(np.float64)
    banner(f"lorenz fp64 tsit5 dense output N={e.n}")
    out, st, stats = run(ens, e, 64, save_mode=1)
    assert (st == 0).all()
    ref, _, na, nr = orc.solve(orc.LORENZ, orc.TSIT5, e.params, e.u0, e.tspan, e.abstol,
                               e.reltol, e.theta, save_mode=1)
    err = normwise(out, ref)
    print("fp64 dense vs oracle dense: max %.3e median %.3e" % (err.max(), np.median(err)))
    assert err.max() <= FP64_SAME_ALG_BAR
    assert np.median(err) <= 1e-12
    assert np.mean((stats[0] == na) & (stats[1] == nr)) > 0.95


@pytest.mark.parametrize("form", [0, 1, 2, 3])
def test_dense_output_fp32_accuracy_and_forms(ens, orc, form):
    """FP32 dense output against the FP64 truth (landing oracle at 1e-12):
    within the FP32 bar, fewer attempts than the landing mode, and the three
    work-assignment forms give the same bits."""
    e = W.lorenz_fp32(N=4099, seed=24)
    banner(f"lorenz fp32 dense output form {form}")
    out, st, stats = run(ens, e, 32, save_mode=1, form=form)
    assert (st == 0).all()
    truth, *_ = oracle_solve(orc, e, tol=1e-12)
    err = normwise(out, truth)
    _, _, land = run(ens, e, 32)
    print("fp32 dense vs truth: max %.3e; attempts dense %.1f landing %.1f"
          % (err.max(), stats.sum(0).mean(), land.sum(0).mean()))
    assert err.max() <= FP32_BAR
    assert stats.sum(0).mean() < 0.85 * land.sum(0).mean()
    if form != 0:
        base, _, s0 = run(ens, e, 32, save_mode=1)
        assert np.array_equal(out.view(np.uint8), base.view(np.uint8))
        assert np.array_equal(stats, s0)


def test_dense_output_is_tsit5_only(ens):
    import paper_2304_06835_amd as ensmod
    e = W.robertson(N=64)
    with pytest.raises(ensmod.EnsError):
        run(ens, e, 32, save_mode=1)
