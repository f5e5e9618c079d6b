"""Order conditions for Runge-Kutta and Rosenbrock tableaus (test helper).

Runge-Kutta: for every rooted tree t with |t| <= p, b^T Phi(t) = 1/gamma(t)
(Butcher's elementary weights and densities; Hairer, Norsett & Wanner I,
section II.2).  Trees are generated recursively, so the helper can be checked
on textbook tableaus before it is trusted on the ones under test.

Rosenbrock: the eight conditions through order 4 of Hairer & Wanner II,
section IV.7, written in the beta_ij = alpha_ij + gamma_ij notation (sums over
the strictly lower parts), with right-hand sides that are polynomials in the
diagonal gamma.  With gamma_ij = 0 they reduce to the RK conditions for the
four tall/bushy trees, which the tests use to cross-check the two helpers.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np


@lru_cache(maxsize=None)
def trees(order: int):
    """All rooted trees with `order` vertices as canonical nested tuples."""
    if order == 1:
        return ((),)
    out = set()

    def partitions(rem, max_part):
        # multisets of subtree sizes summing to rem, non-increasing
        if rem == 0:
            yield ()
            return
        for k in range(min(rem, max_part), 0, -1):
            for rest in partitions(rem - k, k):
                yield (k,) + rest

    for sizes in partitions(order - 1, order - 1):
        combos = [()]
        for k in sizes:
            combos = [c + (t,) for c in combos for t in trees(k)]
        for c in combos:
            out.add(tuple(sorted(c)))
    return tuple(sorted(out))


def density(t) -> int:
    """gamma(t) = |t| * prod gamma(children)."""
    g = size(t)
    for ch in t:
        g *= density(ch)
    return g


def size(t) -> int:
    return 1 + sum(size(ch) for ch in t)


def elementary_weight(t, A, c):
    """Phi(t) as a stage vector: prod over children of A Phi(child)."""
    s = A.shape[0]
    v = np.ones(s)
    for ch in t:
        v = v * (A @ elementary_weight(ch, A, c)) if ch else v * c
    return v


def rk_residuals(A, b, c, p):
    """Residuals b^T Phi(t) - 1/gamma(t) for all trees of order <= p."""
    res = []
    for q in range(1, p + 1):
        for t in trees(q):
            res.append(float(b @ elementary_weight(t, A, c) - 1.0 / density(t)))
    return np.array(res)


def rosenbrock_from_transformed(gamma, a, C, m):
    """(alpha, strictly-lower beta, b) from the transformed coefficients.

    Gamma^{-1} = I/gamma - C, alpha = a Gamma, b = m Gamma, beta = alpha +
    (Gamma without its diagonal) (Hairer & Wanner II, section IV.7).
    """
    s = a.shape[0]
    G = np.linalg.inv(np.eye(s) / gamma - C)
    alpha = a @ G
    b = m @ G
    beta = alpha + G - np.diag(np.diag(G))
    return alpha, beta, b


def rosenbrock_residuals(alpha, beta, b, gamma, p):
    """The conditions through order p (<= 4) for a Rosenbrock method."""
    al = alpha.sum(axis=1)
    bp = beta.sum(axis=1)
    g = gamma
    conds = [
        (1, b.sum() - 1.0),
        (2, b @ bp - (0.5 - g)),
        (3, b @ al**2 - 1.0 / 3.0),
        (3, b @ beta @ bp - (1.0 / 6.0 - g + g * g)),
        (4, b @ al**3 - 0.25),
        (4, b @ (al * (alpha @ bp)) - (1.0 / 8.0 - g / 3.0)),
        (4, b @ beta @ al**2 - (1.0 / 12.0 - g / 3.0)),
        (4, b @ beta @ beta @ bp - (1.0 / 24.0 - g / 2.0 + 1.5 * g * g - g**3)),
    ]
    return np.array([r for (q, r) in conds if q <= p])


def rosenbrock_weight(t, alpha, B):
    """Elementary weight vector of tree t for a Rosenbrock method: a vertex
    with exactly one child couples through B = alpha + Gamma (the Jacobian
    term enters only linearly), a vertex with several children through
    alpha, one factor per child (Hairer & Wanner II, section IV.7)."""
    s = alpha.shape[0]
    if len(t) == 0:
        return np.ones(s)
    if len(t) == 1:
        return B @ rosenbrock_weight(t[0], alpha, B)
    v = np.ones(s)
    for ch in t:
        v = v * (alpha @ rosenbrock_weight(ch, alpha, B))
    return v


def rosenbrock_tree_residuals(alpha, Gamma, b, p):
    """b^T Phi(t) - 1/gamma(t) for every rooted tree with |t| <= p, Phi the
    Rosenbrock elementary weight with B = alpha + Gamma (Gamma lower
    triangular with its diagonal): any order, unlike the explicit list of
    rosenbrock_residuals, which it reproduces through order 4."""
    B = alpha + Gamma
    res = []
    for q in range(1, p + 1):
        for t in trees(q):
            res.append(float(b @ rosenbrock_weight(t, alpha, B) - 1.0 / density(t)))
    return np.array(res)


def rosenbrock_transformed_full(gamma, a, C, m):
    """(alpha, Gamma with diagonal, b) from transformed coefficients."""
    s = a.shape[0]
    G = np.linalg.inv(np.eye(s) / gamma - C)
    return a @ G, G, m @ G


def rosenbrock_stability(alpha, Gamma, b, z):
    """R(z) = 1 + z b^T (I - z (alpha + Gamma))^-1 1 on y' = lambda y."""
    B = alpha + Gamma
    s = B.shape[0]
    return 1.0 + z * (b @ np.linalg.solve(np.eye(s) - z * B, np.ones(s)))


def continuous_extension(A, b, c, p=4):
    """Coefficients B [s][p] of a dense output u(t + theta h) = u + h sum_i
    b_i(theta) k_i with b_i(theta) = sum_m B[i][m-1] theta^m, chosen as:
    order conditions through order p for every theta (b(theta)^T Phi(t) =
    theta^|t| / gamma(t)), b(1) = b, b'(0) = e_1 and b'(1) = e_s (C1 across
    steps of a first-same-as-last pair), and among those the one minimising
    the integral over theta in [0, 1] of the squared order-(p+1) defects.
    Equality-constrained least squares solved exactly through its KKT
    system (the integrals of polynomial products are exact)."""
    s = A.shape[0]
    nv = s * p
    rows, rhs = [], []
    for q in range(1, p + 1):
        for t in trees(q):
            phi = elementary_weight(t, A, c)
            for m in range(1, p + 1):
                r = np.zeros(nv)
                r[np.arange(s) * p + (m - 1)] = phi
                rows.append(r)
                rhs.append(1.0 / density(t) if m == q else 0.0)
    for i in range(s):
        r = np.zeros(nv)
        r[i * p:(i + 1) * p] = 1.0
        rows.append(r)
        rhs.append(b[i])
        r = np.zeros(nv)
        r[i * p] = 1.0
        rows.append(r)
        rhs.append(1.0 if i == 0 else 0.0)
        r = np.zeros(nv)
        r[i * p:(i + 1) * p] = np.arange(1, p + 1)
        rows.append(r)
        rhs.append(1.0 if i == s - 1 else 0.0)
    C = np.array(rows)
    d = np.array(rhs)
    # objective: sum over order-(p+1) trees of int_0^1 (sum_m theta^m w_m . x - theta^(p+1)/g)^2
    H = np.zeros((nv, nv))
    f = np.zeros(nv)
    for t in trees(p + 1):
        phi = elementary_weight(t, A, c)
        g = 1.0 / density(t)
        V = np.zeros((p, nv))  # coefficient of theta^m (m = 1..p) as a row over unknowns
        for m in range(1, p + 1):
            V[m - 1, np.arange(s) * p + (m - 1)] = phi
        M = np.array([[1.0 / (a + bb + 1) for bb in range(1, p + 1)] for a in range(1, p + 1)])
        H += V.T @ M @ V
        f += g * (V.T @ np.array([1.0 / (m + p + 2) for m in range(1, p + 1)]))
    # KKT: [2H C^T; C 0] [x; lam] = [2f; d]; C has dependent rows, so lstsq
    K = np.block([[2 * H, C.T], [C, np.zeros((C.shape[0], C.shape[0]))]])
    sol = np.linalg.lstsq(K, np.concatenate([2 * f, d]), rcond=1e-13)[0]
    return sol[:nv].reshape(s, p)


def dense_residuals(A, c, B, thetas, p=4):
    """max over theta and trees of order <= p of |b(theta)^T Phi(t) - theta^|t|/gamma(t)|."""
    worst = 0.0
    for th in thetas:
        bt = B @ np.array([th ** m for m in range(1, B.shape[1] + 1)])
        for q in range(1, p + 1):
            for t in trees(q):
                worst = max(worst, abs(bt @ elementary_weight(t, A, c) - th ** q / density(t)))
    return worst
