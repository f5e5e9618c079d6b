"""Seeded synthetic ensembles (inputs only; no integration arithmetic here).

Both the GPU path and the CPU oracle are fed from these generators, so that
they see bit-identical inputs.  Every draw uses numpy's PCG64 with a fixed
seed.  Arrays follow the library's structure-of-arrays layout: a quantity
with r rows per trajectory is a C-contiguous [r][N] array (column j of the
paper's U / P matrices, section 5.1.1, is trajectory j).

Workloads (the paper's models, appendix, with per-trajectory draws):
  lorenz_fp64   Lorenz, sigma=10, beta=8/3, rho ~ U[0,21], u0=(1,0,0),
                t in [0,1], Tsit5 atol=rtol=1e-8, final state saved; N=8192.
  lorenz_fp32   Lorenz, rho ~ U[0,28], u0=(1,0,0)+N(0,0.01^2) per component,
                t in [0,1], Tsit5 atol=rtol=1e-6, 16 evenly spaced saves
                (theta_j = (j+1)/16); N=2^24.
  robertson     Robertson kinetics, (k1,k2,k3) = (0.04, 3e7, 1e4) each scaled
                by exp(U[ln 0.5, ln 2]), u0=(1,0,0), t0=0, tf = exp(U[0, ln 1e5]),
                Rodas4 rtol=1e-6 atol=1e-8, h0=1e-4, final state; N=2^20.
  gbm           4 independent GBM components, mu ~ U[-0.5,0.5],
                sigma ~ U[0.05,0.5], u0=1, Euler-Maruyama dt=1/256 on [0,1];
                N=2^22; Philox key 4.
  surrogate     (rho, u0) draws from lorenz_fp32's distribution: training set
                2^20 (seed 5), validation 2^16 (seed 6), queries 2^24 (seed 7),
                audit sample seed 8.
  orego, hires, pollu
                the stiff test problems of appendix B.1 at the paper's 8192
                trajectories: OREGO's and POLLU's rate constants each scaled
                by its own exp(U[ln 0.5, ln 2]) per trajectory; HIRES's by one
                common factor exp(U[ln 0.5, ln 2]) per trajectory (its printed
                constants are tied sums of one another -- 10.03 = 8.32 + 1.71
                and the like -- and scaling them apart makes the solution grow
                without bound; a common factor c is a change of time scale,
                y(t; c k) = y(c t; k)); the printed initial state and time
                span, saves at 1/4, 1/2, 3/4 and 1 of the span, rtol=1e-6
                atol=1e-8, starting-step heuristic; seeds 9, 10, 11.
  crn           the sigma-factor CRN SDE (appendix): 10 values of each of the six
                parameters drawn uniformly from the appendix table's ranges
                (S, D, tau in [0.1, 100], nu0 in [0.01, 0.2], n in [2, 4], eta
                in [0.001, 0.1] -- the table's garbled rows read as one
                parameter each) and their Cartesian product, 10^6 trajectories;
                u0 = (nu0, nu0, nu0, nu0), t in [0, 1000], Euler-Maruyama
                dt = 0.1 (10^4 steps), 10 evenly spaced saves; Philox key 13;
                seed 12.
  gbm(alg="siea") the gbm ensemble under the weak order-2 scheme.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEEDS = {"lorenz_fp64": 1, "lorenz_fp32": 2, "robertson": 3, "gbm": 4,
         "surr_train": 5, "surr_val": 6, "surr_query": 7, "surr_audit": 8,
         "orego": 9, "hires": 10, "pollu": 11, "crn": 12}

FULL_N = {"lorenz_fp64": 8192, "lorenz_fp32": 1 << 24, "robertson": 1 << 20,
          "gbm": 1 << 22, "orego": 8192, "hires": 8192, "pollu": 8192, "crn": 10 ** 6}

# Ranges of the CRN parameters (S, D, tau, nu0, n, eta), appendix table.
CRN_RANGES = [(0.1, 100.0), (0.1, 100.0), (0.1, 100.0), (0.01, 0.2), (2.0, 4.0), (0.001, 0.1)]

# The stiff test problems of appendix B.1: printed rate constants, initial
# state and final time.  HIRES lists its 12 distinct constants (each stands
# for every occurrence of its value in the equations); POLLU k1..k25.
STIFF = {
    "orego": ([77.27, 8.375e-6, 0.161], [1.0, 2.0, 3.0], 30.0),
    "hires": ([1.71, 0.43, 8.32, 0.0007, 8.75, 10.03, 0.035, 1.12, 1.745, 280.0, 0.69, 1.81],
              [1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0057], 321.8122),
    "pollu": ([0.35, 26.6, 12300.0, 0.00086, 0.00082, 15000.0, 0.00013, 24000.0, 16500.0,
               9000.0, 0.022, 12000.0, 1.88, 16300.0, 4.8e6, 0.00035, 0.0175, 1.0e8, 4.44e11,
               1240.0, 2.1, 5.78, 0.0474, 1780.0, 3.12],
              [0.0, 0.2, 0.0, 0.04, 0.0, 0.0, 0.1, 0.3, 0.017, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0,
               0.007, 0.0, 0.0, 0.0], 60.0),
}


@dataclass
class Ensemble:
    name: str
    system: str            # "lorenz" | "robertson" | "gbm4" | "linear" | "orego" | ...
    alg: str               # "tsit5" | "rodas4" | "ros23" | "em"
    params: np.ndarray     # [m][N]
    u0: np.ndarray         # [n][N]
    tspan: np.ndarray      # [2][N] float64 (t0 row, tf row)
    theta: np.ndarray      # [n_save] float64, save fractions in (0, 1]
    abstol: float = 0.0
    reltol: float = 0.0
    h0: float = 0.0        # 0: starting-step heuristic
    dt: float = 0.0        # fixed-step algorithms
    n_steps: int = 0
    seed: int = 0          # Philox key for SDEs
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.u0.shape[1]


def _rows(*rows, dtype):
    return np.ascontiguousarray(np.stack(rows), dtype=dtype)


def lorenz_fp64(N: int = FULL_N["lorenz_fp64"], seed: int = SEEDS["lorenz_fp64"]):
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = rng.uniform(0.0, 21.0, N)
    params = _rows(np.full(N, 10.0), rho, np.full(N, 8.0 / 3.0), dtype=np.float64)
    u0 = _rows(np.ones(N), np.zeros(N), np.zeros(N), dtype=np.float64)
    tspan = _rows(np.zeros(N), np.ones(N), dtype=np.float64)
    return Ensemble("lorenz_fp64", "lorenz", "tsit5", params, u0, tspan,
                    np.array([1.0]), abstol=1e-8, reltol=1e-8)


def lorenz_draws(N: int, seed: int, dtype=np.float32):
    """(params [3][N], u0 [3][N]) from the rho ~ U[0,28], u0 ~ (1,0,0)+N(0,0.01^2)
    distribution, rounded to `dtype`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = rng.uniform(0.0, 28.0, N)
    pert = rng.normal(0.0, 0.01, (3, N))
    params = _rows(np.full(N, 10.0), rho, np.full(N, 8.0 / 3.0), dtype=dtype)
    u0 = np.ascontiguousarray(np.array([[1.0], [0.0], [0.0]]) + pert, dtype=dtype)
    return params, u0


def lorenz_fp32(N: int = FULL_N["lorenz_fp32"], seed: int = SEEDS["lorenz_fp32"]):
    params, u0 = lorenz_draws(N, seed, np.float32)
    tspan = _rows(np.zeros(N), np.ones(N), dtype=np.float64)
    theta = (np.arange(16, dtype=np.float64) + 1.0) / 16.0
    return Ensemble("lorenz_fp32", "lorenz", "tsit5", params, u0, tspan, theta,
                    abstol=1e-6, reltol=1e-6)


def robertson(N: int = FULL_N["robertson"], seed: int = SEEDS["robertson"],
              dtype=np.float32, alg: str = "rodas4"):
    rng = np.random.Generator(np.random.PCG64(seed))
    scale = np.exp(rng.uniform(np.log(0.5), np.log(2.0), (3, N)))
    k = np.array([[0.04], [3e7], [1e4]]) * scale
    tf = np.exp(rng.uniform(0.0, np.log(1e5), N))
    params = np.ascontiguousarray(k, dtype=dtype)
    u0 = _rows(np.ones(N), np.zeros(N), np.zeros(N), dtype=dtype)
    tspan = _rows(np.zeros(N), tf, dtype=np.float64)
    return Ensemble("robertson", "robertson", alg, params, u0, tspan,
                    np.array([1.0]), abstol=1e-8, reltol=1e-6, h0=1e-4)


def gbm(N: int = FULL_N["gbm"], seed: int = SEEDS["gbm"], alg: str = "em"):
    rng = np.random.Generator(np.random.PCG64(seed))
    mu = rng.uniform(-0.5, 0.5, N)
    sigma = rng.uniform(0.05, 0.5, N)
    params = _rows(mu, sigma, dtype=np.float32)
    u0 = np.ones((4, N), dtype=np.float32)
    tspan = _rows(np.zeros(N), np.ones(N), dtype=np.float64)
    return Ensemble("gbm", "gbm4", alg, params, u0, tspan, np.array([1.0]),
                    dt=1.0 / 256.0, n_steps=256, seed=seed)


def stiff(name: str, N: int = 0, seed: int = 0, dtype=np.float32, alg: str = "rodas4"):
    """One of the appendix-B.1 stiff problems (orego, hires, pollu) as an
    ensemble: per-trajectory rate constants k * exp(U[ln 0.5, ln 2]), one
    factor per constant (OREGO, POLLU) or one per trajectory (HIRES)."""
    k, y0, tf = STIFF[name]
    N = N or FULL_N[name]
    rng = np.random.Generator(np.random.PCG64(seed or SEEDS[name]))
    scale = np.exp(rng.uniform(np.log(0.5), np.log(2.0), (1 if name == "hires" else len(k), N)))
    params = np.ascontiguousarray(np.array(k)[:, None] * scale, dtype=dtype)
    u0 = np.ascontiguousarray(np.repeat(np.array(y0)[:, None], N, axis=1), dtype=dtype)
    tspan = _rows(np.zeros(N), np.full(N, tf), dtype=np.float64)
    return Ensemble(name, name, alg, params, u0, tspan, np.array([0.25, 0.5, 0.75, 1.0]),
                    abstol=1e-8, reltol=1e-6)


def crn(values_per_param: int = 10, seed: int = SEEDS["crn"], t_end: float = 1000.0,
        dt: float = 0.1, n_save: int = 10):
    """The CRN parameter sweep: values_per_param uniform draws per parameter,
    all combinations (values_per_param^6 trajectories, parameter 0 varying
    slowest), u0 = nu0 in every species."""
    rng = np.random.Generator(np.random.PCG64(seed))
    axes = [np.sort(rng.uniform(lo, hi, values_per_param)) for lo, hi in CRN_RANGES]
    grid = np.meshgrid(*axes, indexing="ij")
    params = np.ascontiguousarray(np.stack([g.reshape(-1) for g in grid]), dtype=np.float32)
    N = params.shape[1]
    u0 = np.ascontiguousarray(np.repeat(params[3:4], 4, axis=0))
    tspan = _rows(np.zeros(N), np.full(N, t_end), dtype=np.float64)
    n_steps = int(round(t_end / dt))
    theta = (np.arange(n_save, dtype=np.float64) + 1.0) / n_save
    return Ensemble("crn", "crn", "em", params, u0, tspan, theta, dt=dt, n_steps=n_steps,
                    seed=13)


def sample_indices(N: int, k: int) -> np.ndarray:
    """Every (N/k)-th trajectory: the fixed oracle subsample of a large ensemble."""
    if k >= N:
        return np.arange(N)
    return (np.arange(k, dtype=np.int64) * (N // k)).astype(np.int64)
