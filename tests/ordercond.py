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
