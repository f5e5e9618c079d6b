"""Pins for the oracle's Tsit5 dense output (save_mode 1) -- CPU only.

The paper names a free 4th-order interpolation for Tsit5 (section 5.2.1)
without printing it.  The oracle's coefficients are pinned here by what
defines them: the order conditions through order 4 for every theta, the end
conditions b(1) = b, b'(0) = e_1, b'(1) = e_7, an independent re-derivation
of the defect-minimising member of the family, the measured convergence
order of the interpolated value, and adaptive solves against closed forms.
"""
import numpy as np
import pytest

from tests import ordercond as oc


@pytest.fixture(scope="module")
def tab(orc):
    c, A, b, _ = orc.tsit5_tableau()
    return A, b, c, orc.tsit5_dense_table()


def test_order_conditions_hold_for_every_theta(tab):
    A, b, c, B = tab
    assert oc.dense_residuals(A, c, B, np.linspace(0.0, 1.0, 41)) < 1e-12


def test_end_conditions(tab):
    A, b, c, B = tab
    m = np.arange(1, 5)
    assert np.abs(B.sum(axis=1) - b).max() < 1e-12          # b(1) = b
    assert np.abs(B[:, 0] - np.eye(7)[0]).max() < 1e-12      # b'(0) = e_1
    assert np.abs(B @ m - np.eye(7)[6]).max() < 1e-12        # b'(1) = e_7


def test_plausible_mistakes_break_the_pins(tab):
    """The order-condition pin rejects a dropped term, a sign flip or two
    swapped rows of the table."""
    A, b, c, B = tab
    thetas = np.linspace(0.0, 1.0, 11)
    d1 = B.copy()
    d1[3, 2] = 0.0
    d2 = B.copy()
    d2[4, 1] = -d2[4, 1]
    d3 = B.copy()
    d3[[2, 3]] = d3[[3, 2]]
    for bad in (d1, d2, d3):
        assert oc.dense_residuals(A, c, bad, thetas) > 1e-3


def test_table_is_the_defect_minimising_extension(tab):
    """Re-derive the extension from the tableau (KKT system of the
    constrained least-squares problem) and compare."""
    A, b, c, B = tab
    B2 = oc.continuous_extension(A, b, c)
    assert np.abs(B2 - B).max() < 1e-9


def test_interpolated_value_converges_at_order_five_in_h(orc):
    """du = Au: the dense output inside the last of n fixed steps, at the
    fixed time t = 1.5 (theta = 0.5), against e^{At} u0.  The interpolant's
    local error is O(h^5) for a 4th-order extension, like the global error of
    the 5th-order solution, so the error at a fixed time falls as h^5; a
    broken coefficient leaves an O(h^4) or worse local error (slope <= 4)."""
    from scipy.linalg import expm
    Amat = np.array([[-1.0, 2.0, 0.0], [-2.0, -1.0, 0.3], [0.1, 0.0, -0.5]])
    u0 = np.array([1.0, 0.2, -0.4])
    errs, hs = [], []
    for n in (16, 32, 64):
        h = 2.0 * 1.5 / (2 * n - 1)           # (n - 1 + 0.5) h = 1.5
        u = orc.fixed_dense(orc.LINEAR, Amat.reshape(-1), u0, h, n, 0.5)
        ref = expm(Amat * 1.5) @ u0
        errs.append(np.abs(u - ref).max())
        hs.append(h)
    slopes = np.diff(np.log(errs)) / np.diff(np.log(hs))
    print("dense-output error slopes:", slopes)
    assert slopes.min() > 4.6


def test_theta_one_is_the_step_end(orc):
    """At theta = 1 the dense output is the propagated solution."""
    Amat = np.array([[-1.0, 2.0, 0.0], [-2.0, -1.0, 0.0], [0.0, 0.0, -0.5]])
    u0 = np.array([1.0, 0.0, 2.0])
    u_dense = orc.fixed_dense(orc.LINEAR, Amat.reshape(-1), u0, 0.1, 5, 1.0)
    u_step, _ = orc.fixed(orc.LINEAR, orc.TSIT5, Amat.reshape(-1), u0, 0.1, 5)
    assert np.abs(u_dense - u_step).max() < 1e-14


def test_adaptive_dense_solve_matches_closed_form(orc):
    A = np.array([[-1.0, 2.0, 0.0], [-2.0, -1.0, 0.0], [0.0, 0.0, -0.5]])
    theta = (np.arange(16) + 1.0) / 16.0
    tf = 3.0
    out, st, na, nr = orc.solve(orc.LINEAR, orc.TSIT5, A.reshape(9, 1), [[1.0], [0.0], [2.0]],
                                [0.0, tf], 1e-10, 1e-10, theta, save_mode=1)
    assert st[0] == 0
    t = theta * tf
    exact = np.stack([np.exp(-t) * np.cos(2 * t), -np.exp(-t) * np.sin(2 * t),
                      2.0 * np.exp(-0.5 * t)], axis=1)
    assert np.abs(out[:, :, 0] - exact).max() < 1e-8


def test_dense_lorenz_agrees_with_landing_and_takes_fewer_steps(orc):
    """The headline ensemble's distribution: dense output at tol 1e-10 vs
    the landing mode at tol 1e-12 (truth); and at the headline tolerance the
    dense mode needs fewer attempts (no step is cut by a save time)."""
    from paper_2304_06835_amd import workloads as W
    e = W.lorenz_fp32(N=256, seed=17)
    P, U = e.params.astype(np.float64), e.u0.astype(np.float64)
    truth = orc.solve(orc.LORENZ, orc.TSIT5, P, U, e.tspan, 1e-12, 1e-12, e.theta)[0]
    dense = orc.solve(orc.LORENZ, orc.TSIT5, P, U, e.tspan, 1e-10, 1e-10, e.theta,
                      save_mode=1)[0]
    err = orc.normwise_rel_err(dense, truth).max()
    assert err < 1e-7, err
    _, _, na0, nr0 = orc.solve(orc.LORENZ, orc.TSIT5, P, U, e.tspan, 1e-6, 1e-6, e.theta)
    out1, _, na1, nr1 = orc.solve(orc.LORENZ, orc.TSIT5, P, U, e.tspan, 1e-6, 1e-6, e.theta,
                                  save_mode=1)
    print("attempts per trajectory: landing %.1f, dense %.1f"
          % ((na0 + nr0).mean(), (na1 + nr1).mean()))
    assert (na1 + nr1).mean() < 0.85 * (na0 + nr0).mean()
    assert orc.normwise_rel_err(out1, truth).max() < 1e-4


def test_save_mode_rejected_for_bad_values(orc):
    with pytest.raises(ValueError):
        orc.solve(orc.LORENZ, orc.TSIT5, [[10.0], [28.0], [8 / 3]], [[1.0], [0.0], [0.0]],
                  [0.0, 1.0], 1e-6, 1e-6, [1.0], save_mode=2)
