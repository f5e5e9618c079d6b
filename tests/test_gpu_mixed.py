"""ens_solve_mixed: several groups, each an ensemble of its own system, in
one persistent launch whose work queue hands out single-system chunks.
Every trajectory must get exactly the bits, status and step counts that
ens_solve gives it alone (same lane code, only the scheduling differs), and
the groups must match the FP64 oracle as their single-system solves do."""
import numpy as np
import pytest

from paper_2304_06835_amd import workloads as W
from tests.gpu_util import banner, normwise, to_dev, to_host
from tests.test_gpu_ode import FP32_BAR, FP64_SAME_ALG_BAR

pytestmark = pytest.mark.gpu

ORC_SYS = {"lorenz": 1, "robertson": 2, "linear": 0, "orego": 4}
ORC_ALG = {"tsit5": 1, "rodas4": 2, "ros23": 3, "rodas5p": 6}


@pytest.fixture(scope="module")
def ens():
    import torch
    import paper_2304_06835_amd as e
    assert torch.cuda.is_available()
    return e


def linear_group(N, seed, dtype):
    rng = np.random.default_rng(seed)
    A = rng.normal(0, 1, (N, 3, 3)) - 1.5 * np.eye(3)
    params = np.ascontiguousarray(A.reshape(N, 9).T, dtype=dtype)
    u0 = np.ascontiguousarray(rng.normal(0, 1, (3, N)), dtype=dtype)
    tspan = np.stack([np.zeros(N), rng.uniform(0.5, 2.0, N)])
    return W.Ensemble("linear", "linear", "", params, u0, tspan, np.array([1.0]),
                      abstol=1e-6, reltol=1e-6)


def groups_for(alg, precision):
    dt = np.float32 if precision == 32 else np.float64
    if alg == "tsit5":
        lor = W.lorenz_fp32(N=2051, seed=41)
        if precision == 64:
            lor.params, lor.u0 = lor.params.astype(dt), lor.u0.astype(dt)
        return [lor, linear_group(300, 42, dt)]
    rob = W.robertson(N=3001, dtype=dt, alg=alg)
    oreg = W.stiff("orego", N=515, dtype=dt, alg=alg)
    lor = W.lorenz_fp64(N=700)
    lor.params, lor.u0 = lor.params.astype(dt), lor.u0.astype(dt)
    lor.tspan = np.array([0.0, 1.0])      # a broadcast span in one group
    return [rob, oreg, lor, linear_group(130, 43, dt)]


def single(ens, e, alg, precision, theta, save_mode, h0):
    import torch
    s = ens.Solver(0, precision=precision, save_mode=save_mode, h0=h0)
    st = torch.empty(e.n, dtype=torch.uint8, device="cuda")
    sts = torch.empty((2, e.n), dtype=torch.int32, device="cuda")
    out = s.solve(e.system, to_dev(e.params), to_dev(e.u0), to_dev(e.tspan), alg, 1e-6, 1e-6,
                  theta, status=st, stats=sts)
    res = to_host(out), to_host(st), to_host(sts)
    s.close()
    return res


@pytest.mark.parametrize("alg,precision", [("rodas4", 32), ("rodas4", 64), ("rodas5p", 32),
                                           ("ros23", 32), ("tsit5", 32), ("tsit5", 64)])
def test_mixed_equals_single_system_solves(ens, alg, precision):
    import torch
    gs = groups_for(alg, precision)
    theta = [0.25, 0.5, 1.0] if alg != "tsit5" else list((np.arange(16) + 1.0) / 16)
    save_mode = 1 if alg == "tsit5" else 0
    h0 = 1e-4 if alg != "tsit5" else 0.0   # Robertson's first step, for every group
    banner(f"mixed {alg} fp{precision}: " + ", ".join(f"{e.system} {e.n}" for e in gs))
    s = ens.Solver(0, precision=precision, save_mode=save_mode, h0=h0)
    groups = []
    for e in gs:
        groups.append({"system": e.system, "params": to_dev(e.params), "u0": to_dev(e.u0),
                       "tspan": to_dev(e.tspan),
                       "status": torch.empty(e.n, dtype=torch.uint8, device="cuda"),
                       "stats": torch.empty((2, e.n), dtype=torch.int32, device="cuda")})
    outs = s.solve_mixed(groups, alg, 1e-6, 1e-6, theta)
    s.set(form=3)   # the persistent queue instead of one block per chunk
    outs2 = s.solve_mixed([{k: v for k, v in G.items() if k not in ("status", "stats")}
                           for G in groups], alg, 1e-6, 1e-6, theta)
    for o, o2 in zip(outs, outs2):
        assert np.array_equal(to_host(o).view(np.uint8), to_host(o2).view(np.uint8))
    for e, G, o in zip(gs, groups, outs):
        ref, st, sts = single(ens, e, alg, precision, theta, save_mode, h0)
        got = to_host(o)
        assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), e.system
        assert np.array_equal(to_host(G["status"]), st) and np.array_equal(to_host(G["stats"]),
                                                                           sts), e.system
        assert (st == 0).all(), e.system
    s.close()


@pytest.mark.parametrize("precision", [32, 64])
def test_mixed_groups_match_the_oracle(ens, orc, precision):
    """Robertson and Lorenz under Rodas4 in one launch: FP64 against the
    oracle with the same method (rounding order only), FP32 against the
    truth (oracle at tol 1e-12) within the FP32 bar."""
    dt = np.float32 if precision == 32 else np.float64
    rob = W.robertson(N=1500, dtype=dt)
    lor = W.lorenz_fp64(N=1000)
    lor.params, lor.u0 = lor.params.astype(dt), lor.u0.astype(dt)
    theta = [1.0]
    banner(f"mixed rodas4 vs oracle fp{precision}")
    s = ens.Solver(0, precision=precision, h0=1e-4)
    outs = s.solve_mixed([{"system": e.system, "params": to_dev(e.params), "u0": to_dev(e.u0),
                           "tspan": to_dev(e.tspan)} for e in (rob, lor)], "rodas4", 1e-6, 1e-6,
                         theta)
    for e, o in zip((rob, lor), outs):
        got = to_host(o)
        tol = None if precision == 64 else 1e-12
        ref = orc.solve(ORC_SYS[e.system], ORC_ALG["rodas4"], e.params, e.u0, e.tspan,
                        tol or 1e-6, tol or 1e-6, theta, h0=1e-4)[0]
        err = normwise(got, ref)
        print("mixed %s fp%d vs oracle: max %.3e median %.3e" % (e.system, precision, err.max(),
                                                                  np.median(err)))
        if precision == 64:
            assert err.max() <= FP64_SAME_ALG_BAR and np.median(err) <= 1e-11
        else:
            assert err.max() <= FP32_BAR
    s.close()


def test_mixed_edge_cases(ens):
    import torch
    s = ens.Solver(0, precision=32)
    rob = W.robertson(N=100)
    empty = {"system": "lorenz", "params": torch.empty((3, 0), device="cuda"),
             "u0": torch.empty((3, 0), device="cuda"),
             "tspan": torch.tensor([0.0, 1.0], dtype=torch.float64, device="cuda")}
    g = {"system": "robertson", "params": to_dev(rob.params), "u0": to_dev(rob.u0),
         "tspan": to_dev(rob.tspan)}
    out = s.solve_mixed([empty, g, empty], "rodas4", 1e-8, 1e-6, [1.0])
    ref = s.solve("robertson", to_dev(rob.params), to_dev(rob.u0), to_dev(rob.tspan), "rodas4",
                  1e-8, 1e-6, [1.0])
    assert out[0].shape == (1, 3, 0)
    assert np.array_equal(to_host(out[1]).view(np.uint8), to_host(ref).view(np.uint8))
    hires = W.stiff("hires", N=10)
    with pytest.raises(ens.EnsError, match="mixed set"):
        s.solve_mixed([{"system": "hires", "params": to_dev(hires.params),
                        "u0": to_dev(hires.u0), "tspan": to_dev(hires.tspan)}], "rodas4")
    with pytest.raises(ens.EnsError, match="n_groups"):
        s.solve_mixed([g] * 9, "rodas4")
    with pytest.raises(ens.EnsError, match="adaptive"):
        s.solve_mixed([g], "em")
    bad = dict(g, tspan=to_dev(np.stack([rob.tspan[0], rob.tspan[0] - 1.0])))
    out = s.solve_mixed([bad], "rodas4", 1e-8, 1e-6, [1.0],)
    assert np.isnan(to_host(out[0])).all()   # inverted spans: status 3, NaN saves
    s.close()
