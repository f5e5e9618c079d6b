"""The library's launches under HIP stream capture (torch.cuda.CUDAGraph over
the binding's current stream): ens_solve in the plain, cost-sorted and
chunk-queue forms (the queue counter is cleared by a kernel, not a memset
node) and ens_surrogate_solve_static, the entry point that allocates nothing.
A captured graph replays with the arrays' current contents: each of several
replays, with new inputs written eagerly and the device synchronised in
between, must equal an eager call on the same inputs bit for bit."""
import numpy as np
import pytest

from paper_2304_06835_amd import workloads as W
from tests.gpu_util import banner, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ens():
    import torch
    import paper_2304_06835_amd as e
    assert torch.cuda.is_available()
    return e


def bits(a):
    return np.ascontiguousarray(a).view(np.uint8)


@pytest.mark.parametrize("form", [0, 2, 3])
def test_captured_solve_replays_match_eager(ens, form):
    import torch
    e = W.lorenz_fp32(N=20011, seed=91)  # ragged: 78 blocks of 256 + 43
    banner(f"graph replay of ens_solve, form {form}")
    opts = dict(precision=32, form=form, save_mode=1)
    if form:
        opts["block"] = 256
    s = ens.Solver(0, **opts)
    ref_solver = ens.Solver(0, **opts)
    P, U, T = to_dev(e.params), to_dev(e.u0), to_dev(e.tspan)
    out = torch.empty((len(e.theta), 3, e.n), dtype=torch.float32, device="cuda")
    status = torch.empty(e.n, dtype=torch.uint8, device="cuda")
    stats = torch.empty((2, e.n), dtype=torch.int32, device="cuda")

    def call():
        s.solve("lorenz", P, U, T, "tsit5", e.abstol, e.reltol, e.theta, out=out,
                status=status, stats=stats)

    call()  # eager first: loads the kernels' code
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="thread_local"):
        call()
    rng = np.random.default_rng(17)
    for rep in range(3):
        p = e.params.copy()
        p[1] = rng.uniform(0.0, 28.0, e.n).astype(np.float32)   # new rho for every replay
        P.copy_(to_dev(p))
        out.fill_(float("nan"))
        status.fill_(9)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = (to_host(out), to_host(status), to_host(stats))
        st_ref = torch.empty_like(status)
        sa_ref = torch.empty_like(stats)
        ref = ref_solver.solve("lorenz", to_dev(p), U, T, "tsit5", e.abstol, e.reltol, e.theta,
                               status=st_ref, stats=sa_ref)
        torch.cuda.synchronize()
        assert (got[1] == 0).all(), rep
        assert np.array_equal(bits(got[0]), bits(to_host(ref))), rep
        assert np.array_equal(got[1], to_host(st_ref)), rep
        assert np.array_equal(got[2], to_host(sa_ref)), rep
    del g
    s.close()
    ref_solver.close()


def test_captured_static_surrogate_solve_replays_match_eager(ens):
    import torch
    banner("graph replay of ens_surrogate_solve_static")
    s = ens.Solver(0, precision=32)
    m = ens.Surrogate(s, seed=3)
    tr = W.lorenz_fp32(N=8192, seed=92)
    y = np.random.default_rng(93).normal(0, 2, (48, tr.n)).astype(np.float32)
    m.fit_norm(to_dev(tr.params), to_dev(tr.u0), to_dev(y))
    q = W.lorenz_fp32(N=30011, seed=94)
    q.params[1, ::997] = 40.0   # outside the training box: always the solver
    P, U, T = to_dev(q.params), to_dev(q.u0), to_dev(q.tspan)
    out = torch.empty((16, 3, q.n), dtype=torch.float32, device="cuda")
    used = torch.empty(q.n, dtype=torch.uint8, device="cuda")
    rep_t = torch.zeros(4, dtype=torch.float32, device="cuda")
    for tol in (1e30, 1e-3):   # network answers most queries / the solver answers all
        def call():
            m.solve(P, U, T, q.abstol, q.reltol, q.theta, audit_frac=0.02, fallback_tol=tol,
                    audit_seed=5, out=out, used=used, report=rep_t, static=True)

        call()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, capture_error_mode="thread_local"):
            call()
        for rep in range(3):
            u = q.u0.copy()
            u[0] += np.float32(1e-3 * (rep + 1))
            U.copy_(to_dev(u))
            out.fill_(float("nan"))
            used.fill_(7)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got = (to_host(out), to_host(used), to_host(rep_t))
            o2 = torch.empty_like(out)
            u2 = torch.empty_like(used)
            r2 = torch.zeros_like(rep_t)
            m.solve(P, to_dev(u), T, q.abstol, q.reltol, q.theta, audit_frac=0.02,
                    fallback_tol=tol, audit_seed=5, out=o2, used=u2, report=r2, static=True)
            torch.cuda.synchronize()
            assert np.array_equal(bits(got[0]), bits(to_host(o2))), (tol, rep)
            assert np.array_equal(got[1], to_host(u2)), (tol, rep)
            assert np.array_equal(got[2], to_host(r2)), (tol, rep)
            assert set(np.unique(got[1])) <= {0, 1, 2}
        del g
    m.close()
    s.close()
