"""The C ABI library loads and exports every symbol include/ens.h declares.

CPU only: no compute call is made (those need a GPU and live in test_gpu_*).
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ens.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(ens_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2304_06835_amd import _native
    return _native.lib()


def test_header_parsed():
    names = declared_functions()
    assert "ens_solve" in names and "ens_create" in names and len(names) >= 9


def test_every_declared_symbol_is_exported(lib):
    from paper_2304_06835_amd import _native
    names = declared_functions()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_native.EXPORTS)


def test_dims_and_null_handling(lib):
    n, m = ctypes.c_int(), ctypes.c_int()
    # (state size, parameters per trajectory): Lorenz (sigma, rho, beta),
    # Robertson's three rates, the GBMs' (mu, sigma), OREGO's three, HIRES's
    # twelve and POLLU's 25 rate constants, the CRN's (S, D, tau, nu0, n, eta)
    expect = {0: (3, 9), 1: (3, 3), 2: (3, 3), 3: (4, 2), 4: (3, 3), 5: (8, 12), 6: (20, 25),
              7: (4, 6)}
    for sid, (nn, mm) in expect.items():
        assert lib.ens_system_dims(sid, ctypes.byref(n), ctypes.byref(m)) == 0
        assert (n.value, m.value) == (nn, mm)
    assert lib.ens_system_dims(99, ctypes.byref(n), ctypes.byref(m)) == -1
    assert lib.ens_last_error(None) == b"null context"
    assert lib.ens_destroy(None) == 0
    assert lib.ens_set_option(None, 1, 32.0) == -1
    assert lib.ens_solve(None, 1, 1, None, None, None, 1, 1e-6, 1e-6, None, 1, None, None) == -1


def test_create_without_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    ctx = ctypes.c_void_p()
    assert lib.ens_create(ctypes.byref(ctx), 0) < 0
    assert not ctx.value


def test_product_package_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2304_06835_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", src, flags=re.M), f
                assert "liboracle" not in src and "oracle.h" not in src, f


def header_constants(prefix):
    text = open(HEADER).read()
    return {m.group(1).lower(): int(m.group(2))
            for m in re.finditer(r"^#define " + prefix + r"(\w+)\s+\(?(-?\d+)\)?", text, flags=re.M)}


def test_binding_constants_match_header():
    """The Python binding's name tables are the header's #defines: every
    system, algorithm, option, pointer slot and error code, same values."""
    from paper_2304_06835_amd import _native
    assert header_constants("ENS_SYS_") == _native.SYSTEMS
    assert header_constants("ENS_ALG_") == _native.ALGS
    assert header_constants("ENS_OPT_") == _native.OPTS
    assert header_constants("ENS_PTR_") == _native.PTRS
    errs = {k: v for k, v in header_constants("ENS_").items()
            if k in ("ok", "einval", "enomem", "edevice", "eunsupported")}
    assert errs == {"ok": _native.ENS_OK, "einval": _native.ENS_EINVAL,
                    "enomem": _native.ENS_ENOMEM, "edevice": _native.ENS_EDEVICE,
                    "eunsupported": _native.ENS_EUNSUPPORTED}
    assert header_constants("ENS_MAX_")["traj"] == _native.MAX_TRAJ == 2**32 - 2**11
    surr = header_constants("ENS_SURR_")
    assert {k: surr[k] for k in _native.SURR_BUFFERS} == _native.SURR_BUFFERS
    assert surr["nparam"] == _native.SURR_NPARAM
    assert surr["max_batch"] == _native.SURR_MAX_BATCH == 2**28



def test_valu_probe_library_loads_and_rejects_bad_kinds():
    """The issue-rate probes the benchmark prices instruction streams with are
    a separate shared object; it loads, exports its two entry points and each
    rejects an unknown kind or a null result pointer before touching a
    device."""
    path = os.path.join(ROOT, "paper_2304_06835_amd", "libvaluprobe.so")
    if not os.path.exists(path):
        pytest.skip("libvaluprobe.so not built")
    L = ctypes.CDLL(path)
    f = L.valu_probe_rate
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    r = ctypes.c_double(0.0)
    assert f(0, 99, 16, ctypes.byref(r)) == -1
    assert f(0, -1, 16, ctypes.byref(r)) == -1
    assert f(0, 0, 0, ctypes.byref(r)) == -1
    assert f(0, 0, 16, None) == -1
    g = L.mfma_mix_rate
    g.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    assert g(0, 3, 16, ctypes.byref(r)) == -1
    assert g(0, -1, 16, ctypes.byref(r)) == -1
    assert g(0, 0, 0, ctypes.byref(r)) == -1
    assert g(0, 0, 16, None) == -1
