"""GPU parity of the Euler-Maruyama kernel and its Philox stream."""
import numpy as np
import pytest

from paper_2304_06835_amd import workloads as W
from tests.gpu_util import banner, to_dev, to_host
from tests.test_oracle_em import em_moment_z

pytestmark = pytest.mark.gpu

# FP32 path vs the FP64 oracle on the same Philox words: each of the 256
# steps multiplies X by (1 + mu h + sigma sqrt(h) Z) with Z carrying a few FP32
# ulps (log, sqrt, sin/cos) and the product one more, so the relative path
# error is bounded by about 256 * 8 * 2^-24 = 1.2e-4 and is typically ~1e-6.
PATH_BAR = 1.2e-4


@pytest.fixture(scope="module")
def ens():
    import torch
    import paper_2304_06835_amd as e
    assert torch.cuda.is_available()
    return e


def test_philox_words_bit_exact(ens, orc):
    import torch
    N = 1000
    seed = (0xDEADBEEF << 32) | 0x12345678
    banner("philox fill")
    s = ens.Solver(0)
    out = torch.empty((4, N), dtype=torch.int32, device="cuda")
    L = ens._native.lib()
    for step in (0, 1, 255, 2**31 + 7):
        rc = L.ens_philox_fill(s._ctx, seed, N, step, out.data_ptr(), None)
        assert rc == 0
        got = to_host(out).view(np.uint32)
        for i in (0, 1, 2, 511, 999):
            want = orc.philox4x32_10([step, i, 0, 0], [seed & 0xFFFFFFFF, seed >> 32])
            assert list(got[:, i]) == list(want)
    s.close()


def run_em(ens, e, **opts):
    import torch
    s = ens.Solver(0, precision=32, dt=e.dt, seed=e.seed, **opts)
    out = s.solve("gbm4", to_dev(e.params), to_dev(e.u0), to_dev(e.tspan), "em", 0.0, 0.0,
                  e.theta)
    torch.cuda.synchronize()
    r = to_host(out)
    s.close()
    return r


def test_em_paths_match_oracle(ens, orc):
    e = W.gbm(N=3001)
    banner(f"em gbm4 N={e.n}")
    out = run_em(ens, e)
    ref = orc.em(e.params, e.u0, e.dt, e.n_steps, e.seed)
    rel = np.abs(out[0] - ref) / np.abs(ref)
    print("em path rel err: max %.3e median %.3e" % (rel.max(), np.median(rel)))
    assert rel.max() <= PATH_BAR
    assert np.median(rel) <= 1e-5


def test_em_intermediate_saves(ens, orc):
    e = W.gbm(N=257)
    e.theta = np.array([0.25, 0.5, 1.0])
    out = run_em(ens, e)
    for j, th in enumerate(e.theta):
        ref = orc.em(e.params, e.u0, e.dt, int(th * 256), e.seed)
        assert np.abs(out[j] / ref - 1).max() <= PATH_BAR


def test_em_block_shapes_bitwise_equal(ens):
    e = W.gbm(N=5000)
    base = run_em(ens, e)
    for b in (64, 128):
        assert np.array_equal(run_em(ens, e, block=b).view(np.uint8), base.view(np.uint8))


def test_em_full_size_moments(ens):
    """The full 2^22-trajectory ensemble: standardised first and second
    moments of every component against the exact discrete EM moments."""
    e = W.gbm()
    banner(f"em full size N={e.n}")
    out = run_em(ens, e)[0]
    mu = e.params[0].astype(np.float64)
    sg = e.params[1].astype(np.float64)
    for c in range(4):
        z1, z2 = em_moment_z(out[c].astype(np.float64), mu, sg, e.dt, e.n_steps)
        print(f"component {c}: z1 {z1:+.2f} z2 {z2:+.2f}")
        assert abs(z1) < 5 and abs(z2) < 5
