"""Pins for the oracle's Rodas5P (GPURodas5P of section 5.2.1; the 1.0x
reference method of section 6.4's stiff comparison).  The paper prints no
tableau; the coefficients are those of Steinebach's Rodas5P (2023).  They are
pinned here by the Rosenbrock order conditions -- all 17 through order 5 for
the propagated solution and all 8 through order 4 for the embedded one,
written generically over rooted trees and first checked against the
explicit order-4 list and the Runge-Kutta conditions --, by the method's
stability function (stiffly accurate: R(-inf) = 0; A-stable on the imaginary
axis), by measured global and local orders, and by independent integrators
(SciPy's Radau and the closed form of linear systems)."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm

from tests import ordercond as oc
from tests.test_oracle_solvers import robertson_f

TOL = 1e-12


def test_tree_helper_reproduces_the_explicit_order_4_list(orc):
    """On RODAS4 the generic tree conditions give exactly the residuals of
    the eight explicit order-4 conditions (same trees, same values)."""
    g, a, C, m, mh = orc.rodas4_tableau()
    alpha, beta, b = oc.rosenbrock_from_transformed(g, a, C, m)
    al2, G, b2 = oc.rosenbrock_transformed_full(g, a, C, m)
    assert np.allclose(al2, alpha) and np.allclose(b2, b)
    explicit = oc.rosenbrock_residuals(alpha, beta, b, g, 4)
    generic = oc.rosenbrock_tree_residuals(al2, G, b2, 4)
    # trees ordered by size; within order 3 and 4 match them by value
    for q, (lo, hi) in ((1, (0, 1)), (2, (1, 2)), (3, (2, 4)), (4, (4, 8))):
        assert np.allclose(sorted(explicit[lo:hi]), sorted(generic[lo:hi]), atol=1e-13), q
    # RODAS4 has order 4, not 5
    assert np.abs(oc.rosenbrock_tree_residuals(al2, G, b2, 5)[8:]).max() > 1e-4


def test_tree_helper_reduces_to_rk():
    """Gamma = 0: the Rosenbrock tree conditions are the Runge-Kutta ones."""
    A = np.array([[0, 0, 0, 0], [0.5, 0, 0, 0], [0, 0.5, 0, 0], [0, 0, 1.0, 0]])
    b = np.array([1, 2, 2, 1]) / 6.0
    r = oc.rosenbrock_tree_residuals(A, np.zeros((4, 4)), b, 5)
    rk = oc.rk_residuals(A, b, A.sum(axis=1), 5)
    assert np.allclose(r, rk, atol=1e-15)
    assert np.abs(r[:8]).max() < TOL and np.abs(r[8:]).max() > 1e-3


def test_rodas5p_order_conditions(orc):
    g, a, C, m, mh = orc.rodas5p_tableau()
    alpha, G, b = oc.rosenbrock_transformed_full(g, a, C, m)
    _, _, bh = oc.rosenbrock_transformed_full(g, a, C, mh)
    r = oc.rosenbrock_tree_residuals(alpha, G, b, 5)
    rh = oc.rosenbrock_tree_residuals(alpha, G, bh, 5)
    assert len(r) == 17
    assert np.abs(r).max() < TOL, r
    assert np.abs(rh[:8]).max() < TOL, rh
    assert np.abs(rh[8:]).max() > 1e-4          # the embedded method is order 4
    # stiffly accurate: stage points 7 and 8 are the previous point plus the
    # previous stage, the solution the 8th point plus U_8, the embedded one
    # the 8th point itself; stages 6..8 sit at c = 1
    assert np.array_equal(a[6, :6], np.append(a[5, :5], 1.0))
    assert np.array_equal(a[7, :7], np.append(a[6, :6], 1.0))
    assert np.array_equal(m[:7], a[7, :7]) and m[7] == 1.0 and mh[7] == 0.0
    assert np.abs(alpha.sum(axis=1)[5:] - 1.0).max() < 1e-13


@pytest.mark.parametrize("which", ["a", "C", "m", "gamma"])
def test_rodas5p_conditions_catch_a_perturbed_coefficient(orc, which):
    g, a, C, m, mh = orc.rodas5p_tableau()
    rng = np.random.default_rng(2)
    for _ in range(12):
        a2, C2, m2, g2 = a.copy(), C.copy(), m.copy(), g
        i = int(rng.integers(1, 6))
        j = int(rng.integers(0, i))
        if which == "a":
            a2[i, j] += 1e-8
        elif which == "C":
            C2[i, j] += 1e-8
        elif which == "m":
            m2[int(rng.integers(0, 6))] += 1e-8
        else:
            g2 += 1e-8
        alpha, G, b = oc.rosenbrock_transformed_full(g2, a2, C2, m2)
        assert np.abs(oc.rosenbrock_tree_residuals(alpha, G, b, 5)).max() > 1e-11


def test_rodas5p_stability_function(orc):
    """L-stable: R(z) -> 0 as z -> -inf, |R| <= 1 on the imaginary axis and
    on the negative real axis; R(z) matches e^z to order 5 near 0."""
    g, a, C, m, mh = orc.rodas5p_tableau()
    alpha, G, b = oc.rosenbrock_transformed_full(g, a, C, m)
    assert abs(oc.rosenbrock_stability(alpha, G, b, -1e9)) < 1e-6
    for y in np.concatenate([np.linspace(0, 50, 501), np.logspace(2, 8, 30)]):
        assert abs(oc.rosenbrock_stability(alpha, G, b, 1j * y)) <= 1 + 1e-12
    for x in -np.logspace(-3, 8, 60):
        assert abs(oc.rosenbrock_stability(alpha, G, b, x)) <= 1 + 1e-12
    for z in (0.01, -0.02, 0.01j):
        assert abs(oc.rosenbrock_stability(alpha, G, b, z) - np.exp(z)) < 1e-11


def test_rodas5p_linear_problems_see_order_6(orc):
    """On du = A u only the chain trees matter (b^T B^(k-1) 1 = 1/k!), and
    Rodas5P satisfies them through k = 6: fixed steps on a linear system
    converge at order 6 towards e^{At} u0."""
    g, a, C, m, mh = orc.rodas5p_tableau()
    alpha, G, b = oc.rosenbrock_transformed_full(g, a, C, m)
    B, v, fact = alpha + G, np.ones(8), 1.0
    for k in range(1, 8):
        fact *= k
        r = b @ v - 1.0 / fact
        assert (abs(r) < TOL) if k <= 6 else (abs(r) > 1e-6), (k, r)
        v = B @ v
    A = np.array([[-1.0, 2.0, 0.0], [-2.0, -1.0, 0.5], [0.0, -0.5, -0.3]])
    u0 = np.array([1.0, 0.0, 2.0])
    ex = expm(A * 2.0) @ u0
    errs = []
    for k in (10, 20, 40):
        u, _ = orc.fixed(orc.LINEAR, orc.RODAS5P, A.reshape(9), u0, 2.0 / k, k)
        errs.append(np.abs(u - ex).max())
    slopes = np.log2(np.array(errs[:-1]) / errs[1:])
    assert np.all(np.abs(slopes - 6.0) < 0.25), slopes


def test_rodas5p_global_order_5(orc):
    """Fixed steps on Lorenz (nonlinear: every tree counts): order 5."""
    from tests.test_oracle_solvers import _fixed_err
    e = _fixed_err(orc, orc.RODAS5P, [50, 100, 200])
    slopes = np.log2(e[:-1] / e[1:])
    assert np.all(np.abs(slopes - 5.0) < 0.2), slopes


def test_rodas5p_local_orders(orc):
    """One-step errors on Lorenz: h^6 for the solution, h^5 for the embedded
    solution that drives the step-size control."""
    from tests.test_oracle_solvers import lorenz_f
    prm = (10.0, 15.0, 8 / 3)
    hs = np.array([0.01, 0.005, 0.0025])
    le, leh = [], []
    for h in hs:
        r = solve_ivp(lorenz_f(prm), [0, h], [1.0, 0.0, 0.0], method="DOP853",
                      rtol=2.3e-14, atol=1e-16).y[:, -1]
        u, uh = orc.fixed(orc.LORENZ, orc.RODAS5P, prm, [1.0, 0.0, 0.0], h, 1)
        le.append(np.abs(u - r).max())
        leh.append(np.abs(uh - r).max())
    s = np.log2(np.array(le[:-1]) / le[1:])
    sh = np.log2(np.array(leh[:-1]) / leh[1:])
    assert np.all(np.abs(s - 6) < 0.4), s
    assert np.all(np.abs(sh - 5) < 0.3), sh


def test_rodas5p_robertson_vs_radau_and_invariant(orc):
    k = (0.04, 3e7, 1e4)
    tf = 1e5
    theta = np.array([1.0, 1e2, 1e5]) / tf
    out, st, na, nr = orc.solve(orc.ROBERTSON, orc.RODAS5P, np.array(k).reshape(3, 1),
                                [[1.0], [0.0], [0.0]], [0.0, tf], 1e-12, 1e-12, theta,
                                h0=1e-4)
    assert st[0] == 0
    r = solve_ivp(robertson_f(k), [0, tf], [1.0, 0.0, 0.0], method="Radau", rtol=1e-12,
                  atol=1e-16, t_eval=theta * tf).y.T
    e = np.abs(out[:, :, 0] - r).max(axis=1) / np.abs(r).max(axis=1)
    assert e.max() < 1e-8, e
    assert np.abs(out.sum(axis=1) - 1.0).max() < 1e-13
    # fewer steps than RODAS4 at the same tight tolerance (order 5 vs 4)
    _, _, na4, nr4 = orc.solve(orc.ROBERTSON, orc.RODAS4, np.array(k).reshape(3, 1),
                               [[1.0], [0.0], [0.0]], [0.0, tf], 1e-12, 1e-12, theta, h0=1e-4)
    assert (na + nr)[0] < (na4 + nr4)[0]
