"""Pins for the oracle's stiff test problems of appendix B.1 (OREGO, HIRES,
POLLU) -- CPU only.

The oracle writes POLLU as a table of 25 reactions and HIRES / OREGO as
formulas.  Pinned here by: conservation laws that follow from the chemistry
of the species (nitrogen, carbon and sulfur atoms in POLLU; the y7 + y8 pair
of HIRES), which any dropped or misplaced term breaks; the analytic
Jacobians against central differences; the time-rescaling identity
y(t; c k) = y(c t; k) of the HIRES ensemble (every rate, the source
included, must carry its parameter); and SciPy's Radau on the equations
transcribed here term by term from the paper, independently of the
oracle's table.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from paper_2304_06835_amd import workloads as W


def orego_f(k):
    k1, k2, k3 = k
    return lambda t, y: [k1 * (y[1] + y[0] * (1 - k2 * y[0] - y[1])),
                         (y[2] - (1 + y[0]) * y[1]) / k1,
                         k3 * (y[0] - y[2])]


def hires_f(k):
    a, b, c, d, e, f_, g, h, i, j, l, m = k   # 1.71 .43 8.32 .0007 8.75 10.03 .035 1.12 1.745 280 .69 1.81

    def f(t, y):
        y1, y2, y3, y4, y5, y6, y7, y8 = y
        return [-a * y1 + b * y2 + c * y3 + d,
                a * y1 - e * y2,
                -f_ * y3 + b * y4 + g * y5,
                c * y2 + a * y3 - h * y4,
                -i * y5 + b * y6 + b * y7,
                -j * y6 * y8 + l * y4 + a * y5 - b * y6 + l * y7,
                j * y6 * y8 - m * y7,
                -j * y6 * y8 + m * y7]
    return f


def pollu_f(k):
    k = np.concatenate([[0.0], k])            # 1-based like the paper

    def f(t, y):
        y = np.concatenate([[0.0], y])
        d = np.zeros(21)
        d[1] = (-k[1] * y[1] - k[10] * y[11] * y[1] - k[14] * y[1] * y[6] - k[23] * y[1] * y[4]
                - k[24] * y[19] * y[1] + k[2] * y[2] * y[4] + k[3] * y[5] * y[2]
                + k[9] * y[11] * y[2] + k[11] * y[13] + k[12] * y[10] * y[2] + k[22] * y[19]
                + k[25] * y[20])
        d[2] = (-k[2] * y[2] * y[4] - k[3] * y[5] * y[2] - k[9] * y[11] * y[2]
                - k[12] * y[10] * y[2] + k[1] * y[1] + k[21] * y[19])
        d[3] = -k[15] * y[3] + k[1] * y[1] + k[17] * y[4] + k[19] * y[16] + k[22] * y[19]
        d[4] = -k[2] * y[2] * y[4] - k[16] * y[4] - k[17] * y[4] - k[23] * y[1] * y[4] + k[15] * y[3]
        d[5] = (-k[3] * y[5] * y[2] + 2 * k[4] * y[7] + k[6] * y[7] * y[6] + k[7] * y[9]
                + k[13] * y[14] + k[20] * y[17] * y[6])
        d[6] = (-k[6] * y[7] * y[6] - k[8] * y[9] * y[6] - k[14] * y[1] * y[6]
                - k[20] * y[17] * y[6] + k[3] * y[5] * y[2] + 2 * k[18] * y[16])
        d[7] = -k[4] * y[7] - k[5] * y[7] - k[6] * y[7] * y[6] + k[13] * y[14]
        d[8] = k[4] * y[7] + k[5] * y[7] + k[6] * y[7] * y[6] + k[7] * y[9]
        d[9] = -k[7] * y[9] - k[8] * y[9] * y[6]
        d[10] = -k[12] * y[10] * y[2] + k[7] * y[9] + k[9] * y[11] * y[2]
        d[11] = -k[9] * y[11] * y[2] - k[10] * y[11] * y[1] + k[8] * y[9] * y[6] + k[11] * y[13]
        d[12] = k[9] * y[11] * y[2]
        d[13] = -k[11] * y[13] + k[10] * y[11] * y[1]
        d[14] = -k[13] * y[14] + k[12] * y[10] * y[2]
        d[15] = k[14] * y[1] * y[6]
        d[16] = -k[18] * y[16] - k[19] * y[16] + k[16] * y[4]
        d[17] = -k[20] * y[17] * y[6]
        d[18] = k[20] * y[17] * y[6]
        d[19] = (-k[21] * y[19] - k[22] * y[19] - k[24] * y[19] * y[1] + k[23] * y[1] * y[4]
                 + k[25] * y[20])
        d[20] = -k[25] * y[20] + k[24] * y[19] * y[1]
        return d[1:]
    return f


# species of POLLU (Verwer 1994): y1 NO2, y2 NO, y3 O3P, y4 O3, y5 HO2, y6 OH,
# y7 HCHO, y8 CO, y9 ALD (CH3CHO), y10 MEO2, y11 C2O3, y12 CO2, y13 PAN,
# y14 CH3O, y15 HNO3, y16 O1D, y17 SO2, y18 SO4, y19 NO3, y20 N2O5
ATOMS = {
    "N": {1: 1, 2: 1, 13: 1, 15: 1, 19: 1, 20: 2},
    "C": {7: 1, 8: 1, 9: 2, 10: 1, 11: 2, 12: 1, 13: 2, 14: 1},
    "S": {17: 1, 18: 1},
}


def atom_vector(el):
    w = np.zeros(20)
    for sp, c in ATOMS[el].items():
        w[sp - 1] = c
    return w


def test_pollu_conserves_nitrogen_carbon_sulfur(orc):
    rng = np.random.default_rng(2)
    k = np.array(W.STIFF["pollu"][0])
    for _ in range(20):
        y = rng.uniform(0.0, 1.0, 20)
        kk = k * rng.uniform(0.5, 2.0, 25)
        f = orc.rhs(orc.POLLU, kk, y)
        scale = np.abs(f).max()
        for el in ATOMS:
            assert abs(atom_vector(el) @ f) <= 1e-12 * scale, el
    # and along an adaptive solve
    e = W.stiff("pollu", N=16)
    out, st, *_ = orc.solve(orc.POLLU, orc.RODAS4, e.params, e.u0, e.tspan, 1e-10, 1e-8, e.theta)
    assert (st == 0).all()
    for el in ATOMS:
        w = atom_vector(el)
        q0 = w @ e.u0.astype(np.float64)
        q = np.einsum("c,scn->sn", w, out)
        assert np.abs(q - q0).max() <= 1e-9 * np.abs(q0).max(), el


def test_plausible_mistakes_break_the_pollu_atom_balance():
    """A dropped term or a product written to the wrong species breaks one of
    the three balances (checked on the test-side transcription)."""
    k = np.array(W.STIFF["pollu"][0])
    y = np.random.default_rng(3).uniform(0.1, 1.0, 20)
    f = np.array(pollu_f(k)(0, y))
    assert all(abs(atom_vector(el) @ f) < 1e-9 * np.abs(f).max() for el in ATOMS)
    r14 = k[13] * y[0] * y[5]
    bad1 = f.copy(); bad1[14] -= r14          # drop k14 y1 y6 from dy15
    bad2 = f.copy(); bad2[11] -= k[8] * y[10] * y[1]; bad2[10] += k[8] * y[10] * y[1]  # r9 -> y11
    for bad in (bad1, bad2):
        assert max(abs(atom_vector(el) @ bad) for el in ATOMS) > 1e-6


def test_hires_pair_invariant_and_time_rescaling(orc):
    """d(y7 + y8)/dt = 0; and with every rate (the source too) scaled by c,
    y(T; c k) = y(c T; k)."""
    rng = np.random.default_rng(4)
    k = np.array(W.STIFF["hires"][0])
    for _ in range(10):
        y = rng.uniform(0.0, 1.0, 8)
        f = orc.rhs(orc.HIRES, k, y)
        assert abs(f[6] + f[7]) <= 1e-13 * np.abs(f).max()
    u0 = np.array(W.STIFF["hires"][1])
    T = 100.0
    for c in (0.5, 1.7):
        a = orc.solve(orc.HIRES, orc.RODAS4, (c * k)[:, None], u0[:, None], [0.0, T],
                      1e-12, 1e-12, [1.0])[0][0, :, 0]
        b = orc.solve(orc.HIRES, orc.RODAS4, k[:, None], u0[:, None], [0.0, c * T],
                      1e-12, 1e-12, [1.0])[0][0, :, 0]
        assert np.abs(a - b).max() <= 1e-8 * np.abs(b).max(), c
        assert abs(a[6] + a[7] - u0[7]) <= 1e-12


@pytest.mark.parametrize("name", ["orego", "hires", "pollu"])
def test_analytic_jacobian_vs_central_differences(orc, name):
    sid = {"orego": orc.OREGO, "hires": orc.HIRES, "pollu": orc.POLLU}[name]
    e = W.stiff(name, N=8)
    n, m = orc.DIMS[sid]
    rng = np.random.default_rng(5)
    for i in range(4):
        p = e.params[:, i].astype(np.float64)
        y = np.abs(e.u0[:, i].astype(np.float64)) + rng.uniform(0.01, 1.0, n)
        J = orc.jac(sid, p, y)
        Jfd = np.empty((n, n))
        for j in range(n):
            d = 1e-6 * max(1.0, abs(y[j]))
            yp, ym = y.copy(), y.copy()
            yp[j] += d
            ym[j] -= d
            Jfd[:, j] = (orc.rhs(sid, p, yp) - orc.rhs(sid, p, ym)) / (2 * d)
        assert np.abs(J - Jfd).max() <= 1e-6 * max(1.0, np.abs(J).max()), name


@pytest.mark.parametrize("name,alg", [("orego", 2), ("hires", 2), ("pollu", 2),
                                      ("orego", 3), ("hires", 3), ("pollu", 3)])
def test_vs_scipy_radau_on_an_independent_transcription(orc, name, alg):
    sid = {"orego": orc.OREGO, "hires": orc.HIRES, "pollu": orc.POLLU}[name]
    fmk = {"orego": orego_f, "hires": hires_f, "pollu": pollu_f}[name]
    e = W.stiff(name, N=4)
    tol = 1e-10 if alg == 2 else 1e-9
    out, st, na, nr = orc.solve(sid, alg, e.params, e.u0, e.tspan, tol * 1e-2, tol, e.theta)
    assert (st == 0).all()
    worst = 0.0
    for i in range(e.n):
        p = e.params[:, i].astype(np.float64)
        tf = e.tspan[1, i]
        r = solve_ivp(fmk(p), [0, tf], e.u0[:, i].astype(np.float64), method="Radau",
                      rtol=1e-12, atol=1e-16, t_eval=e.theta * tf).y.T
        err = np.abs(out[:, :, i] - r).max(axis=1) / np.abs(r).max(axis=1)
        worst = max(worst, err.max())
    print(name, alg, "max normwise vs Radau", worst, "attempts", (na + nr).mean())
    assert worst < (1e-6 if alg == 2 else 2e-5), worst


def test_orego_with_the_printed_sign_blows_up():
    """The reading of OREGO: with the leading minus printed on dy1 the
    solution from y = (1, 2, 3) does not exist on [0, 30] (SciPy's Radau
    fails); the textbook sign gives the bounded oscillation."""
    k1, k2, k3 = W.STIFF["orego"][0]
    printed = lambda t, y: [-k1 * (y[1] + y[0] * (1 - k2 * y[0] - y[1])),
                            (y[2] - (1 + y[0]) * y[1]) / k1, k3 * (y[0] - y[2])]
    s = solve_ivp(printed, [0, 30], [1.0, 2.0, 3.0], method="Radau", rtol=1e-8, atol=1e-10)
    assert s.status != 0 or not np.isfinite(s.y).all() or np.abs(s.y).max() > 1e8
    s2 = solve_ivp(orego_f((k1, k2, k3)), [0, 30], [1.0, 2.0, 3.0], method="Radau",
                   rtol=1e-8, atol=1e-10)
    assert s2.status == 0 and np.abs(s2.y).max() < 2e5
