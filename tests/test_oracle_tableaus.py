"""Pins for the oracle's coefficient tables (CPU only).

The tables are not printed in the paper (it cites Tsitouras 2011 for Tsit5,
section 5.2.1, and Hairer & Wanner for Rodas4).  They are pinned here by the
order conditions they must satisfy; the conditions' helper is itself checked
on textbook tableaus first.
"""
import numpy as np
import pytest

from tests import ordercond as oc

TOL = 2e-14


def rk4():
    A = np.zeros((4, 4))
    A[1, 0] = 0.5
    A[2, 1] = 0.5
    A[3, 2] = 1.0
    return A, np.array([1 / 6, 1 / 3, 1 / 3, 1 / 6]), np.array([0, 0.5, 0.5, 1.0])


def dopri5():
    """Dormand & Prince (1980) 5(4), as tabulated in HNW I, Table II.5.2."""
    A = np.zeros((7, 7))
    A[1, :1] = [1 / 5]
    A[2, :2] = [3 / 40, 9 / 40]
    A[3, :3] = [44 / 45, -56 / 15, 32 / 9]
    A[4, :4] = [19372 / 6561, -25360 / 2187, 64448 / 6561, -212 / 729]
    A[5, :5] = [9017 / 3168, -355 / 33, 46732 / 5247, 49 / 176, -5103 / 18656]
    A[6, :6] = [35 / 384, 0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84]
    b = A[6].copy()
    bhat = np.array([5179 / 57600, 0, 7571 / 16695, 393 / 640, -92097 / 339200,
                     187 / 2100, 1 / 40])
    c = np.array([0, 1 / 5, 3 / 10, 4 / 5, 8 / 9, 1, 1])
    return A, b, bhat, c


def test_tree_counts():
    # number of rooted trees with 1..6 vertices (OEIS A000081)
    assert [len(oc.trees(q)) for q in range(1, 7)] == [1, 1, 2, 4, 9, 20]


def test_helper_on_rk4():
    A, b, c = rk4()
    assert np.abs(oc.rk_residuals(A, b, c, 4)).max() < TOL
    assert np.abs(oc.rk_residuals(A, b, c, 5)).max() > 1e-3  # RK4 is not 5th order


def test_helper_on_dopri5():
    A, b, bhat, c = dopri5()
    assert np.abs(oc.rk_residuals(A, b, c, 5)).max() < TOL
    assert np.abs(oc.rk_residuals(A, bhat, c, 4)).max() < TOL
    assert np.abs(oc.rk_residuals(A, bhat, c, 5)).max() > 1e-5


def test_tsit5_order_conditions(orc):
    c, A, b, bt = orc.tsit5_tableau()
    assert np.abs(A.sum(axis=1) - c).max() < TOL            # row-sum (c_i = sum_j a_ij)
    assert np.abs(A[6] - b).max() == 0.0                     # FSAL: last row is b
    assert b[6] == 0.0
    assert np.abs(oc.rk_residuals(A, b, c, 5)).max() < TOL   # 17 conditions, order 5
    bhat = b - bt
    assert np.abs(oc.rk_residuals(A, bhat, c, 4)).max() < TOL  # 8 conditions, order 4
    assert np.abs(oc.rk_residuals(A, bhat, c, 5)).max() > 1e-6  # and no more
    assert abs(bt.sum()) < TOL


@pytest.mark.parametrize("which", ["A", "b", "bt", "c"])
def test_tsit5_conditions_catch_a_perturbed_coefficient(orc, which):
    """A single mistyped digit anywhere in the table breaks some condition."""
    c, A, b, bt = orc.tsit5_tableau()
    rng = np.random.default_rng(0)
    for _ in range(10):
        c2, A2, b2, bt2 = c.copy(), A.copy(), b.copy(), bt.copy()
        if which == "A":
            i = rng.integers(1, 7)
            j = rng.integers(0, i)
            A2[i, j] += 1e-9
            if i == 6:
                b2[j] += 1e-9
        elif which == "b":
            j = rng.integers(0, 6)
            b2[j] += 1e-9
        elif which == "bt":
            j = rng.integers(0, 7)
            bt2[j] += 1e-9
        else:
            j = rng.integers(1, 6)
            c2[j] += 1e-9
        bad = max(np.abs(A2.sum(axis=1) - c2).max(),
                  np.abs(oc.rk_residuals(A2, b2, c2, 5)).max(),
                  np.abs(oc.rk_residuals(A2, b2 - bt2, c2, 4)).max())
        assert bad > 1e-11


def test_rosenbrock_helper_reduces_to_rk():
    """With Gamma = 0 the Rosenbrock conditions are the RK ones (beta = alpha)."""
    A, b, c = rk4()
    assert np.abs(oc.rosenbrock_residuals(A, A, b, 0.0, 4)).max() < TOL
    A5, b5, _, _ = dopri5()
    A5[6] = 0.0  # drop the FSAL row: the conditions do not need it
    assert np.abs(oc.rosenbrock_residuals(A5, A5, b5, 0.0, 4)).max() < TOL
    # a 3rd-order RK (Kutta's) passes through order 3 and fails at 4
    A3 = np.array([[0, 0, 0], [0.5, 0, 0], [-1.0, 2.0, 0]])
    b3 = np.array([1 / 6, 2 / 3, 1 / 6])
    assert np.abs(oc.rosenbrock_residuals(A3, A3, b3, 0.0, 3)).max() < TOL
    assert np.abs(oc.rosenbrock_residuals(A3, A3, b3, 0.0, 4)).max() > 1e-3


def test_rosenbrock_helper_one_stage():
    """Linearly implicit Euler / midpoint: 1 stage, order 2 iff gamma = 1/2."""
    one = np.zeros((1, 1))
    b = np.array([1.0])
    assert np.abs(oc.rosenbrock_residuals(one, one, b, 0.5, 2)).max() < TOL
    assert np.abs(oc.rosenbrock_residuals(one, one, b, 1.0, 2)).max() > 0.1
    assert np.abs(oc.rosenbrock_residuals(one, one, b, 0.5, 3)).max() > 0.1


def test_rodas4_order_conditions(orc):
    g, a, C, m, mh = orc.rodas4_tableau()
    assert g == 0.25
    alpha, beta, b = oc.rosenbrock_from_transformed(g, a, C, m)
    _, _, bhat = oc.rosenbrock_from_transformed(g, a, C, mh)
    # stage abscissae of RODAS4: (0, 0.386, 0.21, 0.63, 1, 1)
    assert np.abs(alpha.sum(axis=1) - [0, 0.386, 0.21, 0.63, 1, 1]).max() < 1e-13
    assert np.abs(oc.rosenbrock_residuals(alpha, beta, b, g, 4)).max() < 1e-13
    assert np.abs(oc.rosenbrock_residuals(alpha, beta, bhat, g, 3)).max() < 1e-13
    assert np.abs(oc.rosenbrock_residuals(alpha, beta, bhat, g, 4)).max() > 1e-4
    # stiffly accurate: the last stage point is the embedded solution
    assert np.array_equal(a[5, :5], mh[:5]) and mh[5] == 0.0 and m[5] == 1.0


@pytest.mark.parametrize("which", ["a", "C", "m"])
def test_rodas4_conditions_catch_a_perturbed_coefficient(orc, which):
    g, a, C, m, mh = orc.rodas4_tableau()
    rng = np.random.default_rng(1)
    for _ in range(10):
        a2, C2, m2 = a.copy(), C.copy(), m.copy()
        i = rng.integers(1, 6)
        j = rng.integers(0, i)
        if which == "a":
            a2[i, j] += 1e-8
        elif which == "C":
            C2[i, j] += 1e-8
        else:
            m2[rng.integers(0, 6)] += 1e-8
        alpha, beta, b = oc.rosenbrock_from_transformed(g, a2, C2, m2)
        res = oc.rosenbrock_residuals(alpha, beta, b, g, 4)
        # a perturbation of the stage-6 row of C only enters through the error
        # estimate; require that the embedded conditions catch it then
        _, _, bh = oc.rosenbrock_from_transformed(g, a2, C2, mh)
        res_h = oc.rosenbrock_residuals(alpha, beta, bh, g, 3)
        assert max(np.abs(res).max(), np.abs(res_h).max()) > 1e-11
