"""GPU parity of the Rosenbrock23 kernels (ENS_ALG_ROS23) against the FP64
oracle's Rosenbrock23, through the C ABI.

Bars as for the other adaptive kernels: FP32 within 1e-4 normwise of the
FP64 truth (oracle at tol 1e-12); FP64 against the oracle run with the same
method, controller and tolerance, rounding-order differences only.
"""
import numpy as np
import pytest

from paper_2304_06835_amd import workloads as W
from tests.gpu_util import banner, normwise, to_dev, to_host
from tests.test_gpu_ode import FP32_BAR, FP64_SAME_ALG_BAR, run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ens():
    import torch
    import paper_2304_06835_amd as e
    assert torch.cuda.is_available()
    return e


SYS = {"lorenz": 1, "robertson": 2, "linear": 0}


def oracle(orc, e, alg=None, tol=None):
    at = e.abstol if tol is None else tol
    rt = e.reltol if tol is None else tol
    return orc.solve(SYS[e.system], alg or orc.ROS23, e.params, e.u0, e.tspan, at, rt, e.theta,
                     h0=e.h0)


def test_robertson_fp32_ros23(ens, orc):
    e = W.robertson(N=2053, alg="ros23")
    banner(f"robertson fp32 ros23 N={e.n}")
    out, st, stats = run(ens, e, 32)
    assert (st == 0).all()
    truth, *_ = oracle(orc, e, alg=orc.RODAS4, tol=1e-12)
    same, _, na, nr = oracle(orc, e)
    err = normwise(out, truth)
    eo = normwise(same, truth)
    print("ros23 robertson fp32 vs truth: max %.3e (oracle at same tol %.3e); attempts mean "
          "%.1f (oracle %.1f)" % (err.max(), eo.max(), stats.sum(0).mean(), (na + nr).mean()))
    assert err.max() <= FP32_BAR
    assert np.abs(out.sum(axis=1) - 1.0).max() < 1e-5


def test_robertson_fp64_matches_oracle(ens, orc):
    e = W.robertson(N=1500, dtype=np.float64, alg="ros23")
    banner(f"robertson fp64 ros23 N={e.n}")
    out, st, stats = run(ens, e, 64)
    assert (st == 0).all()
    ref, rst, na, nr = oracle(orc, e)
    err = normwise(out, ref)
    print("ros23 robertson fp64 vs oracle: max %.3e median %.3e" % (err.max(), np.median(err)))
    assert err.max() <= FP64_SAME_ALG_BAR
    assert np.median(err) <= 1e-11
    assert np.abs(out.sum(axis=1) - 1.0).max() < 1e-12
    assert np.mean((stats[0] == na) & (stats[1] == nr)) > 0.95


def test_lorenz_fp64_starting_step_heuristic(ens, orc):
    """Non-stiff Lorenz with the starting-step heuristic (h0 = 0, order 2)
    and 16 save times, FP64 against the oracle."""
    e = W.lorenz_fp32(N=1100, seed=31)
    e.params, e.u0 = e.params.astype(np.float64), e.u0.astype(np.float64)
    e.alg, e.abstol, e.reltol = "ros23", 1e-7, 1e-7
    banner(f"lorenz fp64 ros23 N={e.n}")
    out, st, stats = run(ens, e, 64)
    assert (st == 0).all()
    ref, _, na, nr = oracle(orc, e)
    err = normwise(out, ref)
    print("ros23 lorenz fp64 vs oracle: max %.3e median %.3e" % (err.max(), np.median(err)))
    assert err.max() <= FP64_SAME_ALG_BAR
    assert np.median(err) <= 1e-11


@pytest.mark.parametrize("precision", [32, 64])
def test_ros23_forms_bitwise_equal(ens, precision):
    e = W.robertson(N=3001, dtype=np.float32 if precision == 32 else np.float64, alg="ros23")
    banner(f"ros23 forms fp{precision}")
    base, st0, s0 = run(ens, e, precision)
    for opts in ({"block": 64, "tpl": 3}, {"form": 1}, {"form": 1, "refill": 4, "block": 128},
                 {"form": 2}, {"form": 2, "block": 256, "tpl": 2}, {"form": 3},
                 {"form": 3, "block": 128}):
        out, st, s = run(ens, e, precision, **opts)
        assert np.array_equal(out.view(np.uint8), base.view(np.uint8)), opts
        assert np.array_equal(s, s0), opts


def test_linear_closed_form(ens, orc):
    """du = A u with a rotation-decay block, FP64: against the closed form
    within the order-2 method's global error at tol 1e-9 (oracle: 3.7e-7
    on t in [0, 3]), and against the oracle itself."""
    N = 130
    A = np.array([[-1.0, 2.0, 0.0], [-2.0, -1.0, 0.0], [0.0, 0.0, -0.5]])
    params = np.repeat(A.reshape(9, 1), N, axis=1)
    u0 = np.repeat(np.array([[1.0], [0.0], [2.0]]), N, axis=1)
    tf = np.linspace(0.5, 3.0, N)
    tspan = np.stack([np.zeros(N), tf])
    theta = np.array([0.25, 0.5, 1.0])
    e = W.Ensemble("lin", "linear", "ros23", params, u0, tspan, theta, abstol=1e-9, reltol=1e-9)
    out, st, _ = run(ens, e, 64)
    assert (st == 0).all()
    t = theta[:, None] * tf[None, :]
    ex = np.stack([np.exp(-t) * np.cos(2 * t), -np.exp(-t) * np.sin(2 * t), 2 * np.exp(-0.5 * t)],
                  axis=1)
    assert np.abs(out - ex).max() < 1e-6
    ref, *_ = oracle(orc, e)
    assert np.abs(out - ref).max() < 1e-12


def test_full_size_in_the_benchmarked_launch(ens, orc):
    """2^20 Robertson trajectories in the launch the benchmark times (sorted
    form, block 256): status 0 everywhere, 4096 sampled trajectories within
    the FP32 bar of the FP64 truth, and the persistent form gives the same
    bits on the sample."""
    import torch
    e = W.robertson(alg="ros23")
    banner(f"robertson ros23 full size N={e.n}, sorted form")
    s = ens.Solver(0, precision=32, form=2, block=256)
    s.set(h0=e.h0)
    status = torch.empty(e.n, dtype=torch.uint8, device="cuda")
    P, U, T = to_dev(e.params), to_dev(e.u0), to_dev(e.tspan)
    out = s.solve(e.system, P, U, T, e.alg, e.abstol, e.reltol, e.theta, status=status)
    assert (to_host(status) == 0).all()
    idx = W.sample_indices(e.n, 4096)
    got = np.ascontiguousarray(to_host(out)[:, :, idx])
    sub = W.Ensemble(e.name, e.system, e.alg, np.ascontiguousarray(e.params[:, idx]),
                     np.ascontiguousarray(e.u0[:, idx]), np.ascontiguousarray(e.tspan[:, idx]),
                     e.theta, e.abstol, e.reltol, e.h0)
    truth, *_ = oracle(orc, sub, alg=orc.RODAS4, tol=1e-12)
    err = normwise(got, truth)
    print("ros23 robertson full size, sampled: max normwise error %.3e" % err.max())
    assert err.max() <= FP32_BAR
    del out
    s.set(form=1, block=256)
    out1 = s.solve(e.system, P, U, T, e.alg, e.abstol, e.reltol, e.theta)
    got1 = np.ascontiguousarray(to_host(out1)[:, :, idx])
    assert np.array_equal(got1.view(np.uint8), got.view(np.uint8))
    s.close()


def test_dense_output_rejected(ens):
    import paper_2304_06835_amd as ensmod
    e = W.robertson(N=64, alg="ros23")
    with pytest.raises(ensmod.EnsError):
        run(ens, e, 32, save_mode=1)
