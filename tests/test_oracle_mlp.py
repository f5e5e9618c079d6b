"""Pins for the MLP oracle (CPU): library routines and finite differences."""
import numpy as np
import pytest
import torch

from oracle import mlp

SMALL = (4, 16, 16, 16, 6)


def rand_theta(dims, seed=0, scale=0.5):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, mlp.layout(dims)[1])


def torch_net(theta, dims):
    layers = mlp.unpack(theta, dims)
    ps = []
    for W, b in layers:
        ps.append(torch.tensor(W, dtype=torch.float64, requires_grad=True))
        ps.append(torch.tensor(b, dtype=torch.float64, requires_grad=True))

    def f(X):
        A = X
        for k in range(len(layers)):
            A = torch.nn.functional.linear(A, ps[2 * k], ps[2 * k + 1])
            if k < len(layers) - 1:
                A = torch.nn.functional.silu(A)
        return A
    return f, ps


def test_layout_size():
    assert mlp.N_PARAMS == 4 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 48 + 48 == 145200


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e-20, 1000),
                        rng.normal(0, 1e20, 1000), [0.0, -0.0, 1.0, 1.00390625]])
    want = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), want)


def test_forward_matches_torch_without_rounding():
    th = rand_theta(SMALL)
    X = np.random.default_rng(2).normal(0, 1, (33, 4))
    Y, _ = mlp.forward(th, X, bf16=False, dims=SMALL)
    f, _ = torch_net(th, SMALL)
    assert np.abs(Y - f(torch.tensor(X)).detach().numpy()).max() < 1e-12


def test_gradient_matches_autograd_and_finite_differences():
    th = rand_theta(SMALL, 3)
    rng = np.random.default_rng(4)
    X = rng.normal(0, 1, (17, 4))
    T = rng.normal(0, 1, (17, SMALL[-1]))
    L, g, _ = mlp.loss_and_grad(th, X, T, bf16=False, dims=SMALL)
    f, ps = torch_net(th, SMALL)
    Lt = torch.mean((f(torch.tensor(X)) - torch.tensor(T)) ** 2)
    Lt.backward()
    gt = np.concatenate([p.grad.numpy().reshape(-1) for p in ps])
    assert abs(L - Lt.item()) < 1e-13
    assert np.abs(g - gt).max() < 1e-12
    # central differences on a random subset of parameters
    idx = rng.choice(len(th), 40, replace=False)
    for k in idx:
        e = np.zeros_like(th)
        e[k] = 1e-6
        Lp = mlp.loss_and_grad(th + e, X, T, bf16=False, dims=SMALL)[0]
        Lm = mlp.loss_and_grad(th - e, X, T, bf16=False, dims=SMALL)[0]
        assert abs((Lp - Lm) / 2e-6 - g[k]) <= 1e-6 * max(1.0, abs(g[k]))


def test_bf16_emulation_is_a_small_perturbation():
    th = rand_theta(mlp.DIMS, 5, scale=0.05)
    rng = np.random.default_rng(6)
    X = rng.normal(0, 1, (64, 4))
    T = rng.normal(0, 1, (64, 48))
    _, g0, Y0 = mlp.loss_and_grad(th, X, T, bf16=False)
    _, g1, Y1 = mlp.loss_and_grad(th, X, T, bf16=True)
    assert np.abs(Y1 - Y0).max() / np.abs(Y0).max() < 3e-2
    assert np.linalg.norm(g1 - g0) / np.linalg.norm(g0) < 3e-2
    assert not np.array_equal(Y0, Y1)


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(7)
    th = rng.normal(0, 1, 50)
    p = torch.tensor(th.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    for t in range(1, 8):
        g = rng.normal(0, 1, 50)
        opt.zero_grad()
        p.grad = torch.tensor(g)
        opt.step()
        th, m, v = mlp.adam(th, m, v, g, t, 1e-2)
    assert np.abs(th - p.detach().numpy()).max() < 1e-13


@pytest.mark.parametrize("seed", [0, 1])
def test_adam_first_step_is_lr_times_sign(seed):
    """With bias correction the first update is lr * g / (|g| + eps')."""
    g = np.random.default_rng(seed).normal(0, 1, 20)
    th, _, _ = mlp.adam(np.zeros(20), np.zeros(20), np.zeros(20), g, 1, 1e-3)
    assert np.allclose(th, -1e-3 * np.sign(g), rtol=1e-6)
