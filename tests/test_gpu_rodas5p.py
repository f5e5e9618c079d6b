"""GPU parity of the Rodas5P kernels (ENS_ALG_RODAS5P, GPURodas5P of section
5.2.1) against the FP64 oracle's Rodas5P, through the C ABI.

Bars as for the other Rosenbrock kernels: FP64 against the oracle run with
the same method, controller and tolerance -- rounding order only, so the
same steps (identical attempt counts for >= 95% of trajectories) and a
median difference at rounding level; FP32 state within 1e-4 normwise of the
FP64 truth (oracle at tol 1e-12) and Robertson's y1 + y2 + y3 = 1 within
FP32 rounding.  The appendix-B.1 problems run in tests/test_gpu_stiff.py.
"""
import numpy as np
import pytest

from paper_2304_06835_amd import workloads as W
from tests.gpu_util import banner, normwise, to_dev, to_host
from tests.test_gpu_ode import FP32_BAR, FP64_SAME_ALG_BAR, run

pytestmark = pytest.mark.gpu

SYS = {"lorenz": 1, "robertson": 2}


@pytest.fixture(scope="module")
def ens():
    import torch
    import paper_2304_06835_amd as e
    assert torch.cuda.is_available()
    return e


def oracle(orc, e, alg=None, tol=None):
    at = e.abstol if tol is None else tol
    rt = e.reltol if tol is None else tol
    return orc.solve(SYS[e.system], alg or orc.RODAS5P, e.params, e.u0, e.tspan, at, rt,
                     e.theta, h0=e.h0)


def test_robertson_fp32_rodas5p(ens, orc):
    e = W.robertson(N=2053, alg="rodas5p")
    banner(f"robertson fp32 rodas5p N={e.n}")
    out, st, stats = run(ens, e, 32)
    assert (st == 0).all()
    truth, *_ = oracle(orc, e, alg=orc.RODAS4, tol=1e-12)
    same, _, na, nr = oracle(orc, e)
    err = normwise(out, truth)
    eo = normwise(same, truth)
    print("rodas5p robertson fp32 vs truth: max %.3e (oracle at same tol %.3e); attempts "
          "mean %.1f (oracle %.1f)" % (err.max(), eo.max(), stats.sum(0).mean(),
                                       (na + nr).mean()))
    assert err.max() <= FP32_BAR
    assert np.abs(out.sum(axis=1) - 1.0).max() < 1e-5


@pytest.mark.parametrize("system", ["robertson", "lorenz"])
def test_fp64_matches_oracle(ens, orc, system):
    if system == "robertson":
        e = W.robertson(N=1500, dtype=np.float64, alg="rodas5p")
    else:
        e = W.lorenz_fp64(N=1001)
        e.alg = "rodas5p"
    banner(f"{system} fp64 rodas5p N={e.n}")
    out, st, stats = run(ens, e, 64)
    assert (st == 0).all()
    ref, rst, na, nr = oracle(orc, e)
    err = normwise(out, ref)
    same = np.mean((stats[0] == na) & (stats[1] == nr))
    print("rodas5p %s fp64 vs oracle: max %.3e median %.3e identical attempts %.3f"
          % (system, err.max(), np.median(err), same))
    assert err.max() <= FP64_SAME_ALG_BAR
    assert np.median(err) <= 1e-12
    assert same >= 0.95
    if system == "robertson":
        assert np.abs(out.sum(axis=1) - 1.0).max() < 1e-12


@pytest.mark.parametrize("precision", [32, 64])
def test_forms_bitwise_equal(ens, precision):
    e = W.robertson(N=3001, dtype=np.float32 if precision == 32 else np.float64, alg="rodas5p")
    banner(f"rodas5p forms fp{precision}")
    base, st0, s0 = run(ens, e, precision)
    for opts in ({"block": 64, "tpl": 3}, {"form": 1}, {"form": 2}, {"form": 2, "block": 256},
                 {"form": 2, "block": 512, "tpl": 2}, {"form": 3}):
        out, st, s = run(ens, e, precision, **opts)
        assert np.array_equal(out.view(np.uint8), base.view(np.uint8)), opts
        assert np.array_equal(s, s0), opts


def test_fewer_steps_than_rodas4_on_robertson(ens):
    """Order 5 against order 4 at the same tolerance: Rodas5P takes fewer
    attempted steps per trajectory on the Robertson ensemble."""
    e5 = W.robertson(N=4096, alg="rodas5p")
    e4 = W.robertson(N=4096, alg="rodas4")
    _, _, s5 = run(ens, e5, 32)
    _, _, s4 = run(ens, e4, 32)
    print("attempts per trajectory: rodas5p %.1f rodas4 %.1f" % (s5.sum(0).mean(),
                                                                   s4.sum(0).mean()))
    assert s5.sum(0).mean() < s4.sum(0).mean()


def test_full_size_sorted_form(ens, orc):
    """The 2^20 Robertson ensemble in the sorted form (block 512, two rounds):
    every status 0 and 4096 sampled trajectories within the FP32 bar."""
    import torch
    e = W.robertson(alg="rodas5p")
    banner(f"robertson rodas5p full size N={e.n}")
    s = ens.Solver(0, precision=32, form=2, block=512, tpl=2, h0=e.h0)
    status = torch.empty(e.n, dtype=torch.uint8, device="cuda")
    out = s.solve(e.system, to_dev(e.params), to_dev(e.u0), to_dev(e.tspan), e.alg, e.abstol,
                  e.reltol, e.theta, status=status)
    assert (to_host(status) == 0).all()
    idx = W.sample_indices(e.n, 4096)
    got = np.ascontiguousarray(to_host(out)[:, :, idx])
    sub = W.Ensemble(e.name, e.system, e.alg, np.ascontiguousarray(e.params[:, idx]),
                     np.ascontiguousarray(e.u0[:, idx]), np.ascontiguousarray(e.tspan[:, idx]),
                     e.theta, e.abstol, e.reltol, e.h0)
    truth, *_ = oracle(orc, sub, alg=orc.RODAS4, tol=1e-12)
    err = normwise(got, truth)
    print("rodas5p robertson full size, sampled: max normwise error %.3e" % err.max())
    assert err.max() <= FP32_BAR
    s.close()
