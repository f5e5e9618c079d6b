"""Ensemble ODE/SDE solving on AMD MI355X (gfx950).

Python face of libens.so (C ABI in include/ens.h): torch tensors in, torch
tensors out.  PyTorch only provides device memory and streams; every step of
the integration runs in the library's HIP kernels.  If libens.so is missing
the calls raise -- there is no CPU path.

    import torch, paper_2304_06835_amd as ens
    out = ens.solve("lorenz", params, u0, torch.tensor([0.0, 1.0], device="cuda"),
                    alg="tsit5", abstol=1e-6, reltol=1e-6, save_times=[0.5, 1.0])
"""
from __future__ import annotations

import ctypes
from typing import Iterable, Optional

from . import _native
from ._native import ALGS, OPTS, SYSTEMS, EnsError

__all__ = ["Solver", "Surrogate", "solve", "EnsError", "SYSTEMS", "ALGS", "system_dims"]


def system_dims(system: str):
    n, m = ctypes.c_int(), ctypes.c_int()
    rc = _native.lib().ens_system_dims(SYSTEMS[system], ctypes.byref(n), ctypes.byref(m))
    if rc != 0:
        raise EnsError(rc, f"unknown system {system}")
    return n.value, m.value


def _torch():
    import torch
    return torch


class Solver:
    """One ens_ctx on one HIP device.  Options persist across solve() calls."""

    def __init__(self, device: int = 0, **opts):
        self._L = _native.lib()
        self.device = device
        self._ctx = ctypes.c_void_p()
        rc = self._L.ens_create(ctypes.byref(self._ctx), device)
        if rc != 0:
            raise EnsError(rc, f"ens_create(device={device}) failed")
        if opts:
            self.set(**opts)

    def _check(self, rc: int):
        if rc != 0:
            raise EnsError(rc, self._L.ens_last_error(self._ctx).decode())

    def set(self, **opts) -> "Solver":
        for k, v in opts.items():
            self._check(self._L.ens_set_option(self._ctx, OPTS[k], float(v)))
        return self

    def get(self, key: str) -> float:
        v = ctypes.c_double()
        self._check(self._L.ens_get_option(self._ctx, OPTS[key], ctypes.byref(v)))
        return v.value

    def close(self):
        if self._ctx:
            self._L.ens_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- argument marshalling ------------------------------------------------
    def _prepare(self, system, params, u0, tspan, alg, save_times, out, status, stats,
                 stream):
        torch = _torch()
        sys_id, alg_id = SYSTEMS[system], ALGS[alg]
        n, m = system_dims(system)
        if u0.dim() != 2 or u0.shape[0] != n:
            raise ValueError(f"u0 must be [{n}][N], got {tuple(u0.shape)}")
        N = u0.shape[1]
        if params.shape != (m, N):
            raise ValueError(f"params must be [{m}][{N}], got {tuple(params.shape)}")
        for name, t in (("params", params), ("u0", u0), ("tspan", tspan)):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous device tensor")
        dtype = torch.float64 if int(self.get("precision")) == 64 else torch.float32
        if params.dtype != dtype or u0.dtype != dtype:
            raise ValueError(f"params and u0 must be {dtype} at this precision")
        if tspan.dtype != torch.float64:
            raise ValueError("tspan must be float64")
        if tspan.shape == (2,):
            self.set(tspan_broadcast=1)
        elif tspan.shape == (2, N):
            self.set(tspan_broadcast=0)
        else:
            raise ValueError(f"tspan must be [2] or [2][{N}]")
        theta = [float(x) for x in save_times]
        th = (ctypes.c_double * len(theta))(*theta)
        if out is None:
            out = torch.empty((len(theta), n, N), dtype=dtype, device=u0.device)
        elif out.shape != (len(theta), n, N) or out.dtype != dtype or not out.is_contiguous():
            raise ValueError("out has the wrong shape, dtype or layout")
        if status is not None and (status.dtype != torch.uint8 or status.numel() != N):
            raise ValueError("status must be uint8 [N]")
        if stats is not None and (stats.dtype != torch.int32 or stats.shape != (2, N)):
            raise ValueError("stats must be int32 [2][N]")
        self._check(self._L.ens_set_ptr(self._ctx, _native.PTRS["status"],
                                        status.data_ptr() if status is not None else None))
        self._check(self._L.ens_set_ptr(self._ctx, _native.PTRS["stats"],
                                        stats.data_ptr() if stats is not None else None))
        if stream is None:
            stream = torch.cuda.current_stream(u0.device).cuda_stream
        elif not isinstance(stream, int):
            stream = stream.cuda_stream
        return sys_id, alg_id, N, th, len(theta), out, stream

    def solve(self, system: str, params, u0, tspan, alg: str = "tsit5",
              abstol: float = 1e-6, reltol: float = 1e-6,
              save_times: Iterable[float] = (1.0,), out=None, status=None, stats=None,
              stream=None):
        """Enqueue ens_solve on `stream` (default: torch's current stream).

        params [m][N], u0 [n][N] in the precision's dtype; tspan float64 [2]
        or [2][N]; returns out [n_save][n][N] (allocated if not given).
        """
        sys_id, alg_id, N, th, ns, out, s = self._prepare(
            system, params, u0, tspan, alg, save_times, out, status, stats, stream)
        self._check(self._L.ens_solve(self._ctx, sys_id, N, params.data_ptr(), u0.data_ptr(),
                                      tspan.data_ptr(), alg_id, abstol, reltol, th, ns,
                                      out.data_ptr(), s))
        return out

    def solve_mixed(self, groups, alg: str = "rodas4", abstol: float = 1e-6,
                    reltol: float = 1e-6, save_times: Iterable[float] = (1.0,), stream=None):
        """ens_solve_mixed: one persistent launch over several groups, each a
        dict with system, params, u0, tspan and optionally out, status, stats
        (torch device tensors, laid out as for solve()).  Returns the list of
        output tensors, one per group."""
        torch = _torch()
        theta = [float(x) for x in save_times]
        th = (ctypes.c_double * len(theta))(*theta)
        dtype = torch.float64 if int(self.get("precision")) == 64 else torch.float32
        arr = (_native.Group * len(groups))()
        outs = []
        for g, G in enumerate(groups):
            system, params, u0, tspan = G["system"], G["params"], G["u0"], G["tspan"]
            n, m = system_dims(system)
            N = u0.shape[1]
            if u0.shape != (n, N) or params.shape != (m, N):
                raise ValueError(f"group {g}: params must be [{m}][N] and u0 [{n}][N]")
            for name, t in (("params", params), ("u0", u0), ("tspan", tspan)):
                if not t.is_cuda or not t.is_contiguous():
                    raise ValueError(f"group {g}: {name} must be a contiguous device tensor")
            if params.dtype != dtype or u0.dtype != dtype or tspan.dtype != torch.float64:
                raise ValueError(f"group {g}: params/u0 must be {dtype}, tspan float64")
            if tspan.shape not in ((2,), (2, N)):
                raise ValueError(f"group {g}: tspan must be [2] or [2][N]")
            out = G.get("out")
            if out is None:
                out = torch.empty((len(theta), n, N), dtype=dtype, device=u0.device)
            elif out.shape != (len(theta), n, N) or out.dtype != dtype or not out.is_contiguous():
                raise ValueError(f"group {g}: out has the wrong shape, dtype or layout")
            st, sts = G.get("status"), G.get("stats")
            if st is not None and (st.dtype != torch.uint8 or st.numel() != N):
                raise ValueError(f"group {g}: status must be uint8 [N]")
            if sts is not None and (sts.dtype != torch.int32 or sts.shape != (2, N)):
                raise ValueError(f"group {g}: stats must be int32 [2][N]")
            arr[g] = _native.Group(SYSTEMS[system], 1 if tspan.shape == (2,) else 0, N,
                                   params.data_ptr(), u0.data_ptr(), tspan.data_ptr(),
                                   out.data_ptr(), st.data_ptr() if st is not None else None,
                                   sts.data_ptr() if sts is not None else None)
            outs.append(out)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        elif not isinstance(stream, int):
            stream = stream.cuda_stream
        self._check(self._L.ens_solve_mixed(self._ctx, len(groups), arr, ALGS[alg], abstol,
                                            reltol, th, len(theta), stream))
        return outs

    def autotune(self, system: str, params, u0, tspan, alg: str = "tsit5",
                 abstol: float = 1e-6, reltol: float = 1e-6,
                 save_times: Iterable[float] = (1.0,), out=None, stream=None):
        """Run ens_autotune on a probe ensemble; returns (best_ms, config)."""
        sys_id, alg_id, N, th, ns, out, s = self._prepare(
            system, params, u0, tspan, alg, save_times, out, None, None, stream)
        best = ctypes.c_double()
        self._check(self._L.ens_autotune(self._ctx, sys_id, N, params.data_ptr(),
                                         u0.data_ptr(), tspan.data_ptr(), alg_id, abstol,
                                         reltol, th, ns, out.data_ptr(), s,
                                         ctypes.byref(best)))
        cfg = {k: int(self.get(k)) for k in ("form", "block", "tpl", "refill")}
        cfg["cached"] = bool(self.get("autotune_cached"))
        return best.value, cfg

    def set_autotune_file(self, path: Optional[str]):
        """Persist autotuner results to a JSON file (None: clear the cache)."""
        self._check(self._L.ens_set_autotune_file(
            self._ctx, None if path is None else str(path).encode()))


_default = {}


def solve(system: str, params, u0, tspan, alg: str = "tsit5", abstol: float = 1e-6,
          reltol: float = 1e-6, save_times: Iterable[float] = (1.0,), out=None,
          stream=None, status=None, stats=None, device: Optional[int] = None, **opts):
    """One-call face of ens_solve on a per-device default context.

    Options (precision, form, block, tpl, refill, grid, dt, seed, h0,
    maxiters) are applied to that context before the call.
    """
    dev = u0.device.index if device is None else device
    dev = 0 if dev is None else dev
    s = _default.get(dev)
    if s is None:
        s = _default[dev] = Solver(dev)
    if "precision" not in opts:
        opts["precision"] = 64 if u0.dtype == _torch().float64 else 32
    s.set(**opts)
    return s.solve(system, params, u0, tspan, alg, abstol, reltol, save_times, out,
                   status, stats, stream)


class Surrogate:
    """The learned surrogate of include/ens.h (ens_surrogate_*), bound to a Solver.

    Lorenz queries in the ens_solve layout at precision 32: params [3][N]
    (sigma, rho, beta), u0 [3][N]; outputs [16][3][N].
    """

    NPARAM = _native.SURR_NPARAM

    def __init__(self, solver: Solver, seed: int = 0):
        self.solver = solver
        self._L = solver._L
        self._s = ctypes.c_void_p()
        solver._check(self._L.ens_surrogate_create(solver._ctx, seed, ctypes.byref(self._s)))

    def close(self):
        if self._s:
            self._L.ens_surrogate_destroy(self._s)
            self._s = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _stream(stream):
        torch = _torch()
        if stream is None:
            return torch.cuda.current_stream().cuda_stream
        return stream if isinstance(stream, int) else stream.cuda_stream

    def _c(self, rc):
        self.solver._check(rc)

    def buffer(self, which: str, stream=None):
        """A device copy of one model buffer (master, weights_bf16, grad, adam_m,
        adam_v, norm)."""
        torch = _torch()
        n = 160 if which == "norm" else self.NPARAM
        dt = torch.int16 if which == "weights_bf16" else torch.float32
        t = torch.empty(n, dtype=dt, device=f"cuda:{self.solver.device}")
        self._c(self._L.ens_surrogate_copy(self.solver._ctx, self._s, _native.SURR_BUFFERS[which],
                                           t.data_ptr(), 0, self._stream(stream)))
        return t

    def load(self, which: str, t, stream=None):
        """Overwrite one model buffer from a device tensor of its size."""
        assert t.is_cuda and t.is_contiguous()
        self._c(self._L.ens_surrogate_copy(self.solver._ctx, self._s, _native.SURR_BUFFERS[which],
                                           t.data_ptr(), 1, self._stream(stream)))

    def save_file(self, path):
        """Write weights, Adam state and normalisation to `path` (ens_surrogate_save)."""
        self._c(self._L.ens_surrogate_save(self.solver._ctx, self._s, str(path).encode()))

    def load_file(self, path):
        """Read a model written by save_file (ens_surrogate_load)."""
        self._c(self._L.ens_surrogate_load(self.solver._ctx, self._s, str(path).encode()))

    @property
    def step(self) -> int:
        v = ctypes.c_int64()
        self._c(self._L.ens_surrogate_get_step(self._s, ctypes.byref(v)))
        return v.value

    @step.setter
    def step(self, k: int):
        self._c(self._L.ens_surrogate_set_step(self._s, int(k)))

    def fit_norm(self, params, u0, y, stream=None):
        self._c(self._L.ens_surrogate_fit_norm(self.solver._ctx, self._s, params.data_ptr(),
                                               u0.data_ptr(), y.data_ptr(), u0.shape[1],
                                               self._stream(stream)))

    def train_step(self, params, u0, y, first, batch, mult=1, add=0, lr=1e-3, loss=None,
                   stream=None):
        self._c(self._L.ens_surrogate_train_step(
            self.solver._ctx, self._s, params.data_ptr(), u0.data_ptr(), y.data_ptr(),
            u0.shape[1], first, batch, mult, add, lr,
            loss.data_ptr() if loss is not None else None, self._stream(stream)))

    def train(self, params, u0, y, epochs, batch=4096, lr_max=1e-3, lr_min=1e-5, seed=0,
              stream=None):
        """Returns the per-epoch loss (device tensor [epochs])."""
        torch = _torch()
        losses = torch.zeros(epochs, dtype=torch.float32, device=u0.device)
        self._c(self._L.ens_surrogate_train(
            self.solver._ctx, self._s, params.data_ptr(), u0.data_ptr(), y.data_ptr(),
            u0.shape[1], epochs, batch, lr_max, lr_min, seed, losses.data_ptr(),
            self._stream(stream)))
        return losses

    def predict(self, params, u0, out=None, stream=None):
        torch = _torch()
        N = u0.shape[1]
        if out is None:
            out = torch.empty((16, 3, N), dtype=torch.float32, device=u0.device)
        self._c(self._L.ens_surrogate_predict(self.solver._ctx, self._s, params.data_ptr(),
                                              u0.data_ptr(), N, out.data_ptr(),
                                              self._stream(stream)))
        return out

    def solve(self, params, u0, tspan, abstol, reltol, save_times, audit_frac=0.01,
              fallback_tol=1e-3, audit_seed=8, out=None, used=None, report=None, stream=None,
              static=False):
        """Audited surrogate solve; returns (out, used [N] uint8, report [4]).
        static=True: ens_surrogate_solve_static (no device allocation, at most
        2^20 queries)."""
        torch = _torch()
        N = u0.shape[1]
        dev = u0.device
        if out is None:
            out = torch.empty((16, 3, N), dtype=torch.float32, device=dev)
        if used is None:
            used = torch.empty(N, dtype=torch.uint8, device=dev)
        if report is None:
            report = torch.zeros(4, dtype=torch.float32, device=dev)
        if tspan.shape == (2,):
            self.solver.set(tspan_broadcast=1)
        else:
            self.solver.set(tspan_broadcast=0)
        theta = [float(x) for x in save_times]
        th = (ctypes.c_double * len(theta))(*theta)
        fn = self._L.ens_surrogate_solve_static if static else self._L.ens_surrogate_solve
        self._c(fn(
            self.solver._ctx, self._s, params.data_ptr(), u0.data_ptr(), tspan.data_ptr(),
            abstol, reltol, th, len(theta), N, audit_frac, fallback_tol, audit_seed,
            out.data_ptr(), used.data_ptr(), report.data_ptr(), self._stream(stream)))
        return out, used, report
