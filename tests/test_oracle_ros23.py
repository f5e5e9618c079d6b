"""Pins for the oracle's Rosenbrock23 (the 2(3) pair of GPURosenbrock23,
section 5.2.1) -- CPU only.

The paper names the method without printing it; the oracle writes the
Shampine-Reichelt modified Rosenbrock formulas (ode23s).  The pins: the
formulas read as a Rosenbrock method satisfy the order conditions (2 for the
solution, 3 for the companion) and fail them when d or e32 is changed; the
oracle's step reproduces the closed-form stability function
R(z) = (1 + (1 - 2d) z) / (1 - d z)^2 (L-stable); measured local and global
orders on Lorenz; Robertson against SciPy's Radau and its mass invariant.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from tests import ordercond as oc
from tests.test_oracle_solvers import lorenz_f, robertson_f

D = 1.0 / (2.0 + np.sqrt(2.0))
E32 = 6.0 + np.sqrt(2.0)


def transformed_tableau(d=D, e32=E32):
    """The ode23s formulas as a 3-stage Rosenbrock method (stage vectors
    scaled by h): alpha, strictly lower beta = alpha + Gamma, gamma = d."""
    alpha = np.array([[0.0, 0, 0], [0.5, 0, 0], [0.0, 1.0, 0]])
    G = np.array([[0.0, 0, 0], [-d, 0, 0], [e32 * d - 2 * d, -e32 * d, 0]])
    return alpha, alpha + G, d


def test_formulas_are_a_rosenbrock_pair_of_orders_2_and_3():
    alpha, beta, g = transformed_tableau()
    b = np.array([0.0, 1.0, 0.0])
    bhat = np.array([1 / 6, 2 / 3, 1 / 6])
    assert np.abs(oc.rosenbrock_residuals(alpha, beta, b, g, 2)).max() < 1e-14
    assert np.abs(oc.rosenbrock_residuals(alpha, beta, bhat, g, 3)).max() < 1e-14
    assert np.abs(oc.rosenbrock_residuals(alpha, beta, b, g, 3)).max() > 1e-3
    # a wrong d or e32 breaks the order-3 companion
    for d, e32 in ((1.0 / (2.0 - np.sqrt(2.0)), E32), (D, 6.0 - np.sqrt(2.0)), (D, 6.0)):
        al, be, gg = transformed_tableau(d, e32)
        assert np.abs(oc.rosenbrock_residuals(al, be, bhat, gg, 3)).max() > 1e-3


def _one_step(orc, A, u0, h):
    return orc.fixed(orc.LINEAR, orc.ROS23, np.asarray(A, float).reshape(-1), u0, h, 1)


def test_stability_function_closed_form_and_l_stability(orc):
    """du = diag(l) u: one step multiplies component i by R(h l_i)."""
    R = lambda z: (1 + (1 - 2 * D) * z) / (1 - D * z) ** 2
    for h in (0.1, 1.0, 1e3):
        lam = np.array([-0.5, -20.0, -1e6])
        u, _ = _one_step(orc, np.diag(lam), [1.0, 2.0, -1.0], h)
        ex = np.array([1.0, 2.0, -1.0]) * R(h * lam)
        assert np.abs(u - ex).max() <= 1e-14 * max(1.0, np.abs(ex).max()), (h, u, ex)
    # L-stability: R(z) -> 0 as z -> -inf
    u, _ = _one_step(orc, np.diag([-1e12, -1e9, -1e6]), [1.0, 1.0, 1.0], 1.0)
    assert np.abs(u).max() < 1e-5
    # A-stability on the imaginary axis: a rotation block (eigenvalues +-i w)
    # maps u1 + i u2 to R(-i w h)(u1 + i u2), with |R| <= 1
    for wh in (0.3, 3.0, 300.0):
        A = [[0.0, wh, 0.0], [-wh, 0.0, 0.0], [0.0, 0.0, 0.0]]
        u, _ = _one_step(orc, A, [1.0, 0.0, 1.0], 1.0)
        r = R(-1j * wh)
        assert abs(complex(u[0], u[1]) - r) < 1e-14
        assert abs(r) <= 1.0 and u[2] == 1.0


def test_local_error_orders(orc):
    """One-step error ~ h^3 for the propagated solution and h^4 for the
    companion that drives the error estimate (exact Jacobian)."""
    prm = (10.0, 15.0, 8 / 3)
    hs = np.array([0.004, 0.002, 0.001])
    le, leh = [], []
    for h in hs:
        r = solve_ivp(lorenz_f(prm), [0, h], [1.0, 0.0, 0.0], method="DOP853",
                      rtol=2.3e-14, atol=1e-16).y[:, -1]
        u, uh = orc.fixed(orc.LORENZ, orc.ROS23, prm, [1.0, 0.0, 0.0], h, 1)
        le.append(np.abs(u - r).max())
        leh.append(np.abs(uh - r).max())
    s = np.log2(np.array(le[:-1]) / le[1:])
    sh = np.log2(np.array(leh[:-1]) / leh[1:])
    assert np.all(np.abs(s - 3) < 0.2), s
    assert np.all(np.abs(sh - 4) < 0.3), sh


def test_global_order_2(orc):
    p, T = (10.0, 15.0, 8 / 3), 0.5
    ref = solve_ivp(lorenz_f(p), [0, T], [1.0, 0.0, 0.0], method="DOP853",
                    rtol=2.3e-14, atol=1e-14).y[:, -1]
    errs = []
    for ns in (200, 400, 800, 1600):
        u, _ = orc.fixed(orc.LORENZ, orc.ROS23, p, [1.0, 0.0, 0.0], T / ns, ns)
        errs.append(np.abs(u - ref).max())
    slopes = np.log2(np.array(errs[:-1]) / errs[1:])
    assert np.all(np.abs(slopes - 2.0) < 0.1), slopes


def test_linear_adaptive_vs_closed_form(orc):
    """Against the closed form; the global error of an order-2 method under
    per-step error control falls about as tol^(2/3) (100x per 1000x)."""
    A = np.array([[-1.0, 2.0, 0.0], [-2.0, -1.0, 0.0], [0.0, 0.0, -0.5]])
    theta = np.array([0.1, 0.5, 1.0])
    t = theta * 3.0
    exact = np.stack([np.exp(-t) * np.cos(2 * t), -np.exp(-t) * np.sin(2 * t),
                      2.0 * np.exp(-0.5 * t)], axis=1)
    errs = []
    for tol in (1e-6, 1e-9):
        out, st, na, nr = orc.solve(orc.LINEAR, orc.ROS23, A.reshape(9, 1),
                                    [[1.0], [0.0], [2.0]], [0.0, 3.0], tol, tol, theta)
        assert st[0] == 0
        errs.append(np.abs(out[:, :, 0] - exact).max())
    print("ros23 linear errors", errs)
    assert errs[1] < 1e-6 and errs[0] / errs[1] > 30


def test_robertson_vs_scipy_radau(orc):
    """The paper's stiff CPU-vs-GPU problem (section 5.3): k = (0.04, 3e7,
    1e4), u0 = (1, 0, 0), t in [0, 1e5], h0 = 1e-4."""
    k = (0.04, 3e7, 1e4)
    tf = 1e5
    theta = np.array([1.0, 1e2, 1e4, 1e5]) / tf
    out, st, na, nr = orc.solve(orc.ROBERTSON, orc.ROS23, np.array(k).reshape(3, 1),
                                [[1.0], [0.0], [0.0]], [0.0, tf], 1e-10, 1e-8, theta, h0=1e-4)
    assert st[0] == 0
    r = solve_ivp(robertson_f(k), [0, tf], [1.0, 0.0, 0.0], method="Radau", rtol=1e-12,
                  atol=1e-16, t_eval=theta * tf).y.T
    e = np.abs(out[:, :, 0] - r) / np.maximum(np.abs(r), 1e-10 / 1e-8)
    print("ros23 robertson rel err", e.max(), "steps", na[0] + nr[0])
    assert e.max() < 2e-6, e


def test_robertson_mass_invariant_and_limit(orc):
    """e^T f = 0 and e^T J = 0 give e^T W = e^T: every stage vector sums to
    zero and y1 + y2 + y3 = 1 holds to rounding; y -> (0, 0, 1)."""
    rng = np.random.default_rng(4)
    N = 32
    k = np.array([[0.04], [3e7], [1e4]]) * np.exp(rng.uniform(np.log(0.5), np.log(2), (3, N)))
    theta = np.array([1e-6, 1e-3, 0.1, 1.0])
    out, st, *_ = orc.solve(orc.ROBERTSON, orc.ROS23, k, np.tile([[1.0], [0.0], [0.0]], N),
                            [0.0, 1e9], 1e-8, 1e-5, theta, h0=1e-4)
    assert (st == 0).all()
    assert np.abs(out.sum(axis=1) - 1.0).max() < 1e-13
    assert np.all(out[-1, 2] > 0.999) and np.all(out[-1, 0] < 1e-3)


def test_error_estimate_is_the_companion_difference(orc):
    """uhat = unew - err is the order-3 companion: on du = l u with a small
    step, unew - e^{hl} ~ (d - d^2 - 1/6) (hl)^3 and the companion's error is
    O((hl)^4)."""
    lam = -1.0
    eh = []
    for h in (2e-2, 1e-2):
        u, uh = _one_step(orc, np.diag([lam, lam, lam]), [1.0, 1.0, 1.0], h)
        z = h * lam
        assert abs((u[0] - np.exp(z)) / z**3 - (D - D * D - 1 / 6)) < 2e-3
        eh.append(abs(uh[0] - np.exp(z)))
        assert eh[-1] < 1e-2 * z**4
    assert 13.0 < eh[0] / eh[1] < 19.0  # h^4


def test_rejects_bad_algorithm(orc):
    with pytest.raises(ValueError):
        orc.fixed(orc.LORENZ, 7, (10.0, 28.0, 8 / 3), [1.0, 0.0, 0.0], 0.01, 1)
