"""Pins for the oracle's fixed-step SDE schemes beyond the GBM Euler-Maruyama
of test_oracle_em.py -- CPU only: the weak order-2 scheme standing in for
GPUSIEA, and the sigma-factor CRN SDE (non-diagonal noise, 8 Wiener
processes) under Euler-Maruyama.

The weak orders are measured without Monte Carlo noise: for the linear SDE
dX = mu X dt + sigma X dW one step of either scheme is a polynomial in the
Gaussian increment, so Gauss-Hermite quadrature over dW gives the step's
exact first and second moments, which must match e^{mu h} and
e^{(2 mu + sigma^2) h} to O(h^{p+1}) for weak order p.  The oracle's step is
used as a black box.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from paper_2304_06835_amd import workloads as W


def step_moments(orc, alg, mu, sigma, h, nodes=12):
    x, w = np.polynomial.hermite.hermgauss(nodes)
    z, w = x * np.sqrt(2.0), w / np.sqrt(np.pi)      # N(0, 1) nodes and weights
    m1 = m2 = 0.0
    for zi, wi in zip(z, w):
        dW = np.full(4, np.sqrt(h) * zi)
        y = orc.sde_step(orc.GBM4, alg, [mu, sigma], [1.0, 1.0, 1.0, 1.0], h, dW)[0]
        m1 += wi * y
        m2 += wi * y * y
    return m1, m2


@pytest.mark.parametrize("alg,order", [("EM", 1), ("SIEA", 2)])
def test_weak_order_by_quadrature(orc, alg, order):
    mu, sigma = 0.8, 0.6
    hs = np.array([0.2, 0.1, 0.05, 0.025])
    e1, e2 = [], []
    for h in hs:
        m1, m2 = step_moments(orc, getattr(orc, alg), mu, sigma, h)
        e1.append(abs(m1 - np.exp(mu * h)))
        e2.append(abs(m2 - np.exp((2 * mu + sigma ** 2) * h)))
    s1 = np.diff(np.log(e1)) / np.diff(np.log(hs))
    s2 = np.diff(np.log(e2)) / np.diff(np.log(hs))
    print(alg, "per-step moment error slopes", s1, s2)
    # local weak error O(h^{p+1}) <=> global weak order p
    assert np.all(np.abs(s1 - (order + 1)) < 0.25), s1
    assert np.all(np.abs(s2 - (order + 1)) < 0.25), s2


def test_siea_without_noise_is_heun(orc):
    """sigma = 0: the scheme reduces to Heun's method, global order 2 on
    dX = mu X (Euler-Maruyama: order 1)."""
    for alg, order in ((orc.SIEA, 2), (orc.EM, 1)):
        errs, hs = [], [0.1, 0.05, 0.025]
        for h in hs:
            x = np.ones(4)
            for _ in range(round(1.0 / h)):
                x = orc.sde_step(orc.GBM4, alg, [0.7, 0.0], x, h, np.zeros(4))
            errs.append(abs(x[0] - np.exp(0.7)))
        s = np.diff(np.log(errs)) / np.diff(np.log(hs))
        assert np.all(np.abs(s - order) < 0.1), (alg, s)


def test_siea_monte_carlo_mean_on_the_philox_stream(orc):
    """2^16 paths drawn from the Philox/Box-Muller stream: the sample mean of
    X(1) sits within 4 standard errors of the scheme's exact mean
    (E[M])^N, E[M] from quadrature -- the stream behaves like N(0, 1)
    increments as far as the scheme sees."""
    mu, sigma, h, N = 0.3, 0.4, 1.0 / 16, 1 << 16
    m1, m2 = step_moments(orc, orc.SIEA, mu, sigma, h)
    params = np.tile([[mu], [sigma]], N)
    out = orc.sde(orc.GBM4, orc.SIEA, params, np.ones((4, N)), h, 16, seed=12345)
    x = out.reshape(-1)
    se = x.std() / np.sqrt(x.size)
    assert abs(x.mean() - m1 ** 16) < 4 * se, (x.mean(), m1 ** 16, se)
    assert abs(np.mean(x * x) - m2 ** 16) < 4 * np.std(x * x) / np.sqrt(x.size)


def crn_drift(p):
    S, D, tau, nu0, n, eta = p

    def f(t, y):
        s, a1, a2, a3 = y
        hs, hd = (S * max(s, 0.0)) ** n, (D * max(a3, 0.0)) ** n
        H = hs / (hs + hd + 1.0)
        return [nu0 + H - s, (s - a1) / tau, (a1 - a2) / tau, (a2 - a3) / tau]
    return f


def test_crn_without_noise_is_euler_on_the_ode(orc):
    """eta = 0: Euler-Maruyama on the CRN is explicit Euler on the drift,
    first order against SciPy's solution of the paper's drift equations."""
    for p in ([1.0, 2.0, 5.0, 0.1, 3.0, 0.0], [30.0, 0.5, 0.7, 0.05, 2.0, 0.0]):
        T = 2.0   # inside the transient, where the Euler error is the leading term
        ref = solve_ivp(crn_drift(p), [0, T], [p[3]] * 4, method="LSODA", rtol=1e-12,
                        atol=1e-14).y[:, -1]
        errs, hs = [], [0.1, 0.05, 0.025]
        for h in hs:
            x = orc.sde(orc.CRN, orc.EM, np.array(p)[:, None], np.full((4, 1), p[3]), h,
                        round(T / h), seed=1)[:, 0]
            errs.append(np.abs(x - ref).max())
        s = np.diff(np.log(errs)) / np.diff(np.log(hs))
        assert np.all(np.abs(s - 1.0) < 0.15), (p, s, errs)


def test_crn_noise_matrix(orc):
    """The step is linear in dW; unit increments read off the 4 x 8 noise
    matrix: two entries per row, eta sqrt(production) and -eta sqrt(decay) of
    each species' Langevin term; a concentration pushed below zero enters
    the square roots as 0."""
    S, D, tau, nu0, n, eta = p = [2.0, 3.0, 4.0, 0.1, 2.5, 0.05]
    x = np.array([0.3, 0.2, 0.5, 0.4])
    base = orc.sde_step(orc.CRN, orc.EM, p, x, 0.1, np.zeros(8))
    B = np.empty((4, 8))
    for j in range(8):
        B[:, j] = orc.sde_step(orc.CRN, orc.EM, p, x, 0.1, np.eye(8)[j]) - base
    H = (S * x[0]) ** n / ((S * x[0]) ** n + (D * x[3]) ** n + 1)
    ex = np.zeros((4, 8))
    ex[0, 0], ex[0, 1] = eta * np.sqrt(nu0 + H), -eta * np.sqrt(x[0])
    for c in range(1, 4):
        ex[c, 2 * c] = eta * np.sqrt(x[c - 1] / tau)
        ex[c, 2 * c + 1] = -eta * np.sqrt(x[c] / tau)
    assert np.abs(B - ex).max() < 1e-14
    xneg = np.array([-0.01, 0.2, -0.3, 0.4])
    b0 = orc.sde_step(orc.CRN, orc.EM, p, xneg, 0.1, np.zeros(8))
    for j in (1, 2, 5):   # sqrt(s), sqrt(s / tau), sqrt(A2 / tau) with s, A2 < 0
        assert np.array_equal(orc.sde_step(orc.CRN, orc.EM, p, xneg, 0.1, np.eye(8)[j]), b0)


def crn_reactions():
    """The sigma-factor CRN of the paper's appendix as Gillespie's chemical
    Langevin equation (the construction the appendix cites): eight
    production / decay reactions read off the drift, each changing one
    species by +-1, with propensities a_r(x) >= 0 --
      s:  0 -> s at nu0 + H(s, A3),   s -> 0 at s,
      Ak: 0 -> Ak at A(k-1) / tau,    Ak -> 0 at Ak / tau   (A0 = s),
    H = (S s)^n / ((S s)^n + (D A3)^n + 1).  The CLE is then
      dX = sum_r nu_r a_r dt + eta sum_r nu_r sqrt(a_r) dW_r."""
    def hill(x, p):
        S, D, tau, nu0, n, eta = p
        hs, hd = (S * x[0]) ** n, (D * x[3]) ** n
        return hs / (hs + hd + 1.0)
    R = [(0, +1, lambda x, p: p[3] + hill(x, p)), (0, -1, lambda x, p: x[0])]
    for k in (1, 2, 3):
        R.append((k, +1, lambda x, p, k=k: x[k - 1] / p[2]))
        R.append((k, -1, lambda x, p, k=k: x[k] / p[2]))
    return R


def test_crn_is_the_chemical_langevin_equation(orc):
    """Pin of the CRN's drift and diffusion independent of how the oracle
    writes them: at random positive states and parameters, the oracle's
    Euler-Maruyama step has drift sum_r a_r nu_r and a noise matrix b (read
    off with unit increments) whose covariance b b^T is
    eta^2 sum_r a_r nu_r nu_r^T, the CLE's; and each column of b is
    eta sqrt(a_r) nu_r of one reaction r, every reaction once."""
    rng = np.random.default_rng(17)
    R = crn_reactions()
    h = 0.05
    for _ in range(50):
        p = [rng.uniform(0.1, 100), rng.uniform(0.1, 100), rng.uniform(0.1, 100),
             rng.uniform(0.01, 0.2), rng.uniform(2, 4), rng.uniform(0.001, 0.1)]
        x = rng.uniform(0.01, 2.0, 4)
        eta = p[5]
        base = orc.sde_step(orc.CRN, orc.EM, p, x, h, np.zeros(8))
        drift = (base - x) / h
        nu = np.zeros((len(R), 4))
        a = np.empty(len(R))
        for r, (c, sgn, prop) in enumerate(R):
            nu[r, c] = sgn
            a[r] = prop(x, p)
        assert np.all(a >= 0)
        f = nu.T @ a
        assert np.abs(drift - f).max() <= 1e-9 * max(1.0, np.abs(f).max()), (drift, f)
        B = np.empty((4, 8))
        for j in range(8):
            B[:, j] = orc.sde_step(orc.CRN, orc.EM, p, x, h, np.eye(8)[j]) - base
        cov = eta ** 2 * (nu.T * a) @ nu
        assert np.abs(B @ B.T - cov).max() <= 1e-12 * np.abs(cov).max()
        cols = [eta * np.sqrt(a[r]) * nu[r] for r in range(len(R))]
        used = set()
        for j in range(8):
            hit = [r for r in range(len(R)) if r not in used
                   and np.abs(B[:, j] - cols[r]).max() <= 1e-12 * np.abs(cols[r]).max()]
            assert hit, (j, B[:, j])
            used.add(hit[0])


def test_em_gbm_unchanged_by_the_general_path(orc):
    rng = np.random.default_rng(3)
    P = np.stack([rng.uniform(-.5, .5, 64), rng.uniform(.05, .5, 64)])
    U = np.ones((4, 64))
    assert np.array_equal(orc.em(P, U, 1 / 256, 256, 4), orc.sde(orc.GBM4, orc.EM, P, U,
                                                                   1 / 256, 256, 4))


def test_siea_rejects_non_diagonal_noise(orc):
    with pytest.raises(ValueError):
        orc.sde(orc.CRN, orc.SIEA, np.ones((6, 1)), np.ones((4, 1)), 0.1, 1, 1)
