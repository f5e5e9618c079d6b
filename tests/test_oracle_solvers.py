"""Pins for the oracle's adaptive ODE integrators (CPU only).

Each pin ties the oracle to something other than itself: a closed form, a
special case with a textbook answer, a measured convergence order, a
conservation law, or an independent library integrator (SciPy).
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm


def lorenz_f(p):
    s, r, b = p
    return lambda t, y: [s * (y[1] - y[0]), r * y[0] - y[1] - y[0] * y[2],
                         y[0] * y[1] - b * y[2]]


def robertson_f(k):
    k1, k2, k3 = k
    return lambda t, y: [-k1 * y[0] + k3 * y[1] * y[2],
                         k1 * y[0] - k3 * y[1] * y[2] - k2 * y[1] ** 2,
                         k2 * y[1] ** 2]


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("alg", [1, 2])
def test_linear_rotation_decay_closed_form(orc, alg):
    """du = A u with A = [[-1, 2], [-2, -1]] (+ a decoupled decay): exact
    solution e^{-t}(cos 2t, -sin 2t) for u0 = (1, 0), and z0 e^{-t/2}."""
    A = np.array([[-1.0, 2.0, 0.0], [-2.0, -1.0, 0.0], [0.0, 0.0, -0.5]])
    theta = np.array([0.1, 0.25, 0.5, 0.75, 1.0])
    tf = 3.0
    out, st, na, nr = orc.solve(orc.LINEAR, alg, A.reshape(9, 1), [[1.0], [0.0], [2.0]],
                                [0.0, tf], 1e-11, 1e-11, theta)
    assert st[0] == 0
    t = theta * tf
    exact = np.stack([np.exp(-t) * np.cos(2 * t), -np.exp(-t) * np.sin(2 * t),
                      2.0 * np.exp(-0.5 * t)], axis=1)
    assert np.abs(out[:, :, 0] - exact).max() < 1e-9


@pytest.mark.parametrize("alg", [1, 2])
def test_linear_random_matrices_vs_expm(orc, alg):
    rng = np.random.default_rng(11)
    N = 32
    As = rng.normal(0.0, 1.0, (N, 3, 3)) - 1.5 * np.eye(3)
    u0 = rng.normal(0.0, 1.0, (3, N))
    theta = np.array([0.5, 1.0])
    out, st, *_ = orc.solve(orc.LINEAR, alg, As.reshape(N, 9).T.copy(), u0, [0.0, 1.0],
                            1e-12, 1e-12, theta)
    assert (st == 0).all()
    for i in range(N):
        for j, th in enumerate(theta):
            ex = expm(As[i] * th) @ u0[:, i]
            assert np.abs(out[j, :, i] - ex).max() <= 1e-9 * max(1.0, np.abs(ex).max())


def test_lorenz_special_cases_exact(orc):
    """rho = 0, u0 = (1,0,0): y and z stay 0 and x = e^{-sigma t}.
    u0 = (0,0,z0): x = y = 0 and z = z0 e^{-beta t}, for any rho."""
    N = 4
    params = np.array([[10.0] * N, [0.0, 0.0, 5.0, 28.0], [8 / 3] * N])
    u0 = np.array([[1.0, 1.0, 0.0, 0.0], [0.0] * N, [0.0, 0.0, 3.0, -2.0]])
    theta = np.array([0.2, 0.6, 1.0])
    for alg in (1, 2):
        out, st, *_ = orc.solve(orc.LORENZ, alg, params, u0, [0.0, 1.0], 1e-12, 1e-12, theta)
        assert (st == 0).all()
        t = theta
        ex0 = np.stack([np.exp(-10 * t), 0 * t, 0 * t], axis=1)
        assert np.abs(out[:, :, 0] - ex0).max() < 1e-10
        for i, z0 in ((2, 3.0), (3, -2.0)):
            ex = np.stack([0 * t, 0 * t, z0 * np.exp(-8 / 3 * t)], axis=1)
            assert np.abs(out[:, :, i] - ex).max() < 1e-10


# ------------------------------------------------------- convergence orders

def _fixed_err(orc, alg, ns_list, p=(10.0, 15.0, 8 / 3), T=0.5):
    ref = solve_ivp(lorenz_f(p), [0, T], [1.0, 0.0, 0.0], method="DOP853",
                    rtol=2.3e-14, atol=1e-14).y[:, -1]
    errs = []
    for ns in ns_list:
        u, _ = orc.fixed(orc.LORENZ, alg, p, [1.0, 0.0, 0.0], T / ns, ns)
        errs.append(np.abs(u - ref).max())
    return np.array(errs)


def test_tsit5_global_order_5(orc):
    e = _fixed_err(orc, 1, [50, 100, 200])
    slopes = np.log2(e[:-1] / e[1:])
    assert np.all(np.abs(slopes - 5.0) < 0.25), slopes


def test_rodas4_global_order_4(orc):
    e = _fixed_err(orc, 2, [100, 200, 400, 800])
    slopes = np.log2(e[:-1] / e[1:])
    assert np.all(np.abs(slopes - 4.0) < 0.15), slopes


@pytest.mark.parametrize("alg,p,phat", [(1, 5, 4), (2, 4, 3)])
def test_local_error_orders(orc, alg, p, phat):
    """One-step error ~ h^{p+1} for the solution and h^{phat+1} for the
    embedded solution that drives the error estimate."""
    prm = (10.0, 15.0, 8 / 3)
    hs = np.array([0.01, 0.005, 0.0025])
    le, leh = [], []
    for h in hs:
        r = solve_ivp(lorenz_f(prm), [0, h], [1.0, 0.0, 0.0], method="DOP853",
                      rtol=2.3e-14, atol=1e-16).y[:, -1]
        u, uh = orc.fixed(orc.LORENZ, alg, prm, [1.0, 0.0, 0.0], h, 1)
        le.append(np.abs(u - r).max())
        leh.append(np.abs(uh - r).max())
    s = np.log2(np.array(le[:-1]) / le[1:])
    sh = np.log2(np.array(leh[:-1]) / leh[1:])
    assert np.all(np.abs(s - (p + 1)) < 0.4), s
    assert np.all(np.abs(sh - (phat + 1)) < 0.2), sh


def test_tolerance_proportionality(orc):
    """Global error of the adaptive solve falls as the tolerance falls."""
    p = np.array([[10.0], [21.0], [8 / 3]])
    ref = solve_ivp(lorenz_f(p[:, 0]), [0, 1], [1.0, 0.0, 0.0], method="DOP853",
                    rtol=2.3e-14, atol=1e-14).y[:, -1]
    errs = []
    for tol in (1e-4, 1e-6, 1e-8, 1e-10):
        out, st, *_ = orc.solve(orc.LORENZ, 1, p, [[1.0], [0.0], [0.0]], [0.0, 1.0],
                                tol, tol, [1.0])
        errs.append(np.abs(out[0, :, 0] - ref).max() / np.abs(ref).max())
    errs = np.array(errs)
    assert np.all(errs[1:] < errs[:-1] / 10), errs
    assert errs[-1] < 1e-8


# --------------------------------------------------- independent integrators

def test_lorenz_vs_scipy_dop853(orc):
    rng = np.random.default_rng(5)
    N = 256
    rho = rng.uniform(0.0, 28.0, N)
    params = np.stack([np.full(N, 10.0), rho, np.full(N, 8 / 3)])
    u0 = np.array([[1.0], [0.0], [0.0]]) + rng.normal(0, 0.01, (3, N))
    theta = np.array([0.25, 0.5, 1.0])
    out, st, *_ = orc.solve(orc.LORENZ, 1, params, u0, [0.0, 1.0], 1e-12, 1e-12, theta)
    assert (st == 0).all()
    worst = 0.0
    for i in range(N):
        r = solve_ivp(lorenz_f(params[:, i]), [0, 1], u0[:, i], method="DOP853",
                      rtol=2.3e-14, atol=1e-14, t_eval=theta).y.T
        e = np.abs(out[:, :, i] - r).max(axis=1) / np.abs(r).max(axis=1)
        worst = max(worst, e.max())
    assert worst < 1e-9, worst


def test_robertson_vs_scipy_radau(orc):
    k = (0.04, 3e7, 1e4)
    tf = 1e5
    theta = np.array([1.0, 1e2, 1e5]) / tf
    out, st, *_ = orc.solve(orc.ROBERTSON, 2, np.array(k).reshape(3, 1), [[1.0], [0.0], [0.0]],
                            [0.0, tf], 1e-12, 1e-12, theta, h0=1e-4)
    assert st[0] == 0
    r = solve_ivp(robertson_f(k), [0, tf], [1.0, 0.0, 0.0], method="Radau", rtol=1e-12,
                  atol=1e-16, t_eval=theta * tf).y.T
    e = np.abs(out[:, :, 0] - r).max(axis=1) / np.abs(r).max(axis=1)
    assert e.max() < 1e-8, e


def test_robertson_mass_invariant_and_limit(orc):
    """e^T f = 0 makes y1+y2+y3 = 1 hold for every Rosenbrock step (exactly,
    up to rounding), and y -> (0, 0, 1) for large t."""
    rng = np.random.default_rng(3)
    N = 64
    k = np.array([[0.04], [3e7], [1e4]]) * np.exp(rng.uniform(np.log(0.5), np.log(2), (3, N)))
    theta = np.array([1e-6, 1e-3, 0.1, 1.0])
    out, st, na, _ = orc.solve(orc.ROBERTSON, 2, k, np.tile([[1.0], [0.0], [0.0]], N),
                               [0.0, 1e9], 1e-8, 1e-6, theta, h0=1e-4)
    assert (st == 0).all()
    assert np.abs(out.sum(axis=1) - 1.0).max() < 1e-13
    assert np.all(out[-1, 2] > 0.999) and np.all(out[-1, 0] < 1e-3)
    assert np.all(np.diff(out[:, 2, :], axis=0) > 0)  # y3 grows monotonically


def test_robertson_k2_k3_zero_closed_form(orc):
    """k2 = k3 = 0: y1 = e^{-k1 t}, y2 = 1 - e^{-k1 t}, y3 = 0."""
    theta = np.array([0.1, 0.5, 1.0])
    out, st, *_ = orc.solve(orc.ROBERTSON, 2, np.array([[0.04], [0.0], [0.0]]),
                            [[1.0], [0.0], [0.0]], [0.0, 50.0], 1e-12, 1e-12, theta, h0=1e-4)
    t = theta * 50.0
    ex = np.stack([np.exp(-0.04 * t), 1 - np.exp(-0.04 * t), 0 * t], axis=1)
    assert np.abs(out[:, :, 0] - ex).max() < 1e-10


@pytest.mark.parametrize("sys", [0, 1, 2])
def test_analytic_jacobian_vs_central_differences(orc, sys):
    rng = np.random.default_rng(sys)
    n, m = orc.DIMS[sys]
    for _ in range(5):
        if sys == 2:
            p = np.array([0.04, 3e7, 1e4]) * rng.uniform(0.5, 2, 3)
            u = np.abs(rng.normal(0, 1, n)) * np.array([1.0, 1e-5, 1.0])
        else:
            p = rng.normal(0, 3, m)
            u = rng.normal(0, 2, n)
        J = orc.jac(sys, p, u)
        Jfd = np.empty((n, n))
        for j in range(n):
            h = 1e-6 * max(1.0, abs(u[j])) if sys != 2 else 1e-6 * max(1e-5, abs(u[j]))
            e = np.zeros(n)
            e[j] = h
            Jfd[:, j] = (orc.rhs(sys, p, u + e) - orc.rhs(sys, p, u - e)) / (2 * h)
        assert np.abs(J - Jfd).max() <= 1e-6 * max(1.0, np.abs(J).max())


def test_rhs_matches_paper_models(orc):
    """Appendix models, evaluated at one point by hand."""
    u = np.array([1.5, -2.0, 3.0])
    assert np.allclose(orc.rhs(1, [10.0, 28.0, 8 / 3], u),
                       [10 * (-3.5), 28 * 1.5 + 2.0 - 4.5, -3.0 - 8.0])
    y = np.array([0.9, 2e-5, 0.1])
    assert np.allclose(orc.rhs(2, [0.04, 3e7, 1e4], y),
                       [-0.036 + 1e4 * 2e-6, 0.036 - 1e4 * 2e-6 - 3e7 * 4e-10, 3e7 * 4e-10],
                       rtol=1e-14, atol=0)


# --------------------------------------------------- saves and failure codes

def test_save_points_and_degenerate_spans(orc):
    p = np.array([[10.0, 10.0], [21.0, 21.0], [8 / 3, 8 / 3]])
    u0 = np.array([[1.0, 1.0], [0.0, 0.0], [0.0, 0.0]])
    tspan = np.array([[0.0, 2.0], [1.0, 2.0]])  # second trajectory: tf == t0
    theta = np.array([0.5, 1.0])
    out, st, na, _ = orc.solve(orc.LORENZ, 1, p, u0, tspan, 1e-8, 1e-8, theta)
    assert (st == 0).all()
    assert np.array_equal(out[:, :, 1], np.tile(u0[:, 1], (2, 1)))
    assert na[1] == 0
    # the save at theta=0.5 equals a solve whose span ends there
    out2, *_ = orc.solve(orc.LORENZ, 1, p[:, :1], u0[:, :1], [0.0, 0.5], 1e-8, 1e-8, [1.0])
    assert np.abs(out2[0, :, 0] - out[0, :, 0]).max() < 1e-6


def test_failure_status_codes(orc):
    p = np.array([[10.0, 10.0, 10.0], [21.0, np.nan, 21.0], [8 / 3, 8 / 3, 8 / 3]])
    u0 = np.tile([[1.0], [0.0], [0.0]], 3)
    out, st, *_ = orc.solve(orc.LORENZ, 1, p, u0, [0.0, 1.0], 1e-8, 1e-8, [1.0])
    assert st[0] == 0 and st[1] == 3
    assert np.isnan(out[0, :, 1]).all()
    out, st, na, nr = orc.solve(orc.LORENZ, 1, p[:, :1], u0[:, :1], [0.0, 1.0], 1e-8, 1e-8,
                                [1.0], maxiters=3)
    assert st[0] == 1 and na[0] + nr[0] == 3
