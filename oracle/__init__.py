"""FP64 CPU oracle for the ensemble ODE/SDE hot path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and
this package imports nothing from it.

``liboracle.so`` is plain C (``oracle.c``) built with gcc; this module is a
thin numpy/ctypes face over it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

LINEAR, LORENZ, ROBERTSON, GBM4, OREGO, HIRES, POLLU, CRN = 0, 1, 2, 3, 4, 5, 6, 7
TSIT5, RODAS4, ROS23, EM, SIEA, RODAS5P = 1, 2, 3, 4, 5, 6
DIMS = {LINEAR: (3, 9), LORENZ: (3, 3), ROBERTSON: (3, 3), GBM4: (4, 2), OREGO: (3, 3),
        HIRES: (8, 12), POLLU: (20, 25), CRN: (4, 6)}
NOISES = {GBM4: 4, CRN: 8}


def build(verbose: bool = False) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wextra", "-Wno-unused-parameter",
           os.path.join(HERE, "oracle.c"), "-o", LIB_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        ip = ctypes.POINTER(ctypes.c_int)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.orc_solve.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, dp, dp, dp,
                                ctypes.c_double, ctypes.c_double, dp, ctypes.c_int, dp,
                                ip, i64p, i64p, ctypes.c_double, ctypes.c_int64,
                                ctypes.c_int]
        L.orc_solve_mode.argtypes = L.orc_solve.argtypes + [ctypes.c_int]
        L.orc_fixed.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_double,
                                ctypes.c_int, dp, dp]
        L.orc_fixed_dense.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_double, dp]
        L.orc_tsit5_dense_table.argtypes = [dp]
        L.orc_tsit5_dense_table.restype = None
        L.orc_rhs.argtypes = [ctypes.c_int, dp, dp, dp]
        L.orc_jac.argtypes = [ctypes.c_int, dp, dp, dp]
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox4x32_10.restype = None
        L.orc_uniform.argtypes = [ctypes.c_uint32]
        L.orc_uniform.restype = ctypes.c_double
        L.orc_box_muller.argtypes = [ctypes.c_uint32, ctypes.c_uint32, dp, dp]
        L.orc_box_muller.restype = None
        L.orc_em.argtypes = [ctypes.c_int, ctypes.c_int64, dp, dp, ctypes.c_double,
                             ctypes.c_int, ctypes.c_uint64, i64p, dp, ctypes.c_int]
        L.orc_sde.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, dp, dp,
                              ctypes.c_double, ctypes.c_int, ctypes.c_uint64, i64p, dp,
                              ctypes.c_int]
        L.orc_sde_step.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_double, dp, dp]
        L.orc_tsit5_tableau.argtypes = [dp, dp, dp, dp]
        L.orc_tsit5_tableau.restype = None
        L.orc_rodas4_tableau.argtypes = [dp, dp, dp, dp, dp]
        L.orc_rodas4_tableau.restype = None
        L.orc_rodas5p_tableau.argtypes = [dp, dp, dp, dp, dp]
        L.orc_rodas5p_tableau.restype = None
        _lib = L
    return _lib


def _p(a, ctype=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_threads() -> int:
    return len(os.sched_getaffinity(0))


def solve(system, alg, params, u0, tspan, atol, rtol, theta, h0=0.0,
          maxiters=10**6, nthreads=None, save_mode=0):
    """Adaptive ensemble solve.  params [m][N], u0 [n][N], tspan [2][N] or [2].
    save_mode 0: steps land on every save time; 1 (Tsit5): steps land on the
    last save time only and the others come from the dense output.

    Returns (out [n_save][n][N], status [N], naccept [N], nreject [N]).
    """
    params, u0 = _f64(params), _f64(u0)
    n, m = DIMS[system]
    N = u0.shape[1]
    assert params.shape == (m, N) and u0.shape == (n, N)
    tspan = _f64(tspan)
    if tspan.ndim == 1:
        tspan = np.repeat(tspan[:, None], N, axis=1).copy()
    theta = _f64(theta)
    out = np.empty((len(theta), n, N))
    st = np.empty(N, dtype=np.int32)
    na = np.empty(N, dtype=np.int64)
    nr = np.empty(N, dtype=np.int64)
    rc = lib().orc_solve_mode(system, alg, N, _p(params), _p(u0), _p(tspan), atol, rtol,
                              _p(theta), len(theta), _p(out), _p(st, ctypes.c_int),
                              _p(na, ctypes.c_int64), _p(nr, ctypes.c_int64), h0,
                              maxiters, nthreads or default_threads(), save_mode)
    if rc != 0:
        raise ValueError("orc_solve rejected its arguments")
    return out, st, na, nr


def fixed(system, alg, p, u0, h, n_steps):
    """n_steps fixed steps; returns (u, uhat) for one trajectory."""
    n, _ = DIMS[system]
    p, u0 = _f64(p), _f64(u0)
    u = np.empty(n)
    uh = np.empty(n)
    if lib().orc_fixed(system, alg, _p(p), _p(u0), h, n_steps, _p(u), _p(uh)) != 0:
        raise ValueError("orc_fixed rejected its arguments")
    return u, uh


def fixed_dense(system, p, u0, h, n_steps, theta):
    """n_steps fixed Tsit5 steps, the last read at its dense output:
    u(t0 + (n_steps - 1 + theta) h) for one trajectory."""
    n, _ = DIMS[system]
    p, u0 = _f64(p), _f64(u0)
    u = np.empty(n)
    if lib().orc_fixed_dense(system, _p(p), _p(u0), h, n_steps, theta, _p(u)) != 0:
        raise ValueError("orc_fixed_dense rejected its arguments")
    return u


def tsit5_dense_table():
    """B [7][4]: b_i(theta) = sum_m B[i][m] theta^(m+1)."""
    B = np.empty(28)
    lib().orc_tsit5_dense_table(_p(B))
    return B.reshape(7, 4)


def rhs(system, p, u):
    n, _ = DIMS[system]
    du = np.empty(n)
    lib().orc_rhs(system, _p(_f64(p)), _p(_f64(u)), _p(du))
    return du


def jac(system, p, u):
    n, _ = DIMS[system]
    J = np.empty((n, n))
    lib().orc_jac(system, _p(_f64(p)), _p(_f64(u)), _p(J))
    return J


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.empty(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32),
                            _p(o, ctypes.c_uint32))
    return o


def uniform(x: int) -> float:
    return lib().orc_uniform(x)


def box_muller(x0: int, x1: int):
    a = ctypes.c_double()
    b = ctypes.c_double()
    lib().orc_box_muller(x0, x1, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def em(params, u0, dt, n_steps, seed, ids=None, nthreads=None):
    """Euler-Maruyama ensemble for the 4-component GBM; returns [4][N].

    ids: trajectory ids (Philox counters) of the columns; default 0..N-1.
    """
    params, u0 = _f64(params), _f64(u0)
    N = u0.shape[1]
    assert params.shape == (2, N) and u0.shape == (4, N)
    out = np.empty((4, N))
    idp = None
    if ids is not None:
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        assert ids.shape == (N,)
        idp = _p(ids, ctypes.c_int64)
    rc = lib().orc_em(GBM4, N, _p(params), _p(u0), dt, n_steps, seed, idp, _p(out),
                      nthreads or default_threads())
    if rc != 0:
        raise ValueError("orc_em rejected its arguments")
    return out


def sde(system, alg, params, u0, dt, n_steps, seed, ids=None, nthreads=None):
    """Fixed-step SDE ensemble (EM for GBM4 and CRN, SIEA for GBM4); returns
    the final state [n][N].  ids: Philox trajectory ids of the columns."""
    params, u0 = _f64(params), _f64(u0)
    n, m = DIMS[system]
    N = u0.shape[1]
    assert params.shape == (m, N) and u0.shape == (n, N)
    out = np.empty((n, N))
    idp = None
    if ids is not None:
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        assert ids.shape == (N,)
        idp = _p(ids, ctypes.c_int64)
    rc = lib().orc_sde(system, alg, N, _p(params), _p(u0), dt, n_steps, seed, idp, _p(out),
                       nthreads or default_threads())
    if rc != 0:
        raise ValueError("orc_sde rejected its arguments")
    return out


def sde_step(system, alg, p, x, h, dW):
    """One SDE step of size h from x with Wiener increments dW."""
    n, _ = DIMS[system]
    p, x, dW = _f64(p), _f64(x), _f64(dW)
    assert dW.shape == (NOISES[system],)
    out = np.empty(n)
    if lib().orc_sde_step(system, alg, _p(p), _p(x), h, _p(dW), _p(out)) != 0:
        raise ValueError("orc_sde_step rejected its arguments")
    return out


def tsit5_tableau():
    c, a, b, bt = np.empty(7), np.empty(49), np.empty(7), np.empty(7)
    lib().orc_tsit5_tableau(_p(c), _p(a), _p(b), _p(bt))
    return c, a.reshape(7, 7), b, bt


def rodas4_tableau():
    g = ctypes.c_double()
    a, C, m, mh = np.empty(36), np.empty(36), np.empty(6), np.empty(6)
    lib().orc_rodas4_tableau(ctypes.byref(g), _p(a), _p(C), _p(m), _p(mh))
    return g.value, a.reshape(6, 6), C.reshape(6, 6), m, mh


def rodas5p_tableau():
    g = ctypes.c_double()
    a, C, m, mh = np.empty(64), np.empty(64), np.empty(8), np.empty(8)
    lib().orc_rodas5p_tableau(ctypes.byref(g), _p(a), _p(C), _p(m), _p(mh))
    return g.value, a.reshape(8, 8), C.reshape(8, 8), m, mh


def normwise_rel_err(x, ref):
    """Per (save, trajectory): ||x - ref||_inf / ||ref||_inf over components.

    x, ref: [n_save][n][N].  Returns [n_save][N].
    """
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    num = np.max(np.abs(x - ref), axis=1)
    den = np.max(np.abs(ref), axis=1)
    return num / den
