"""FP64 numpy oracle of the learned surrogate -- TEST INFRASTRUCTURE.

The surrogate is a plain multilayer perceptron, (rho, x0, y0, z0) -> 256 ->
256 -> 256 -> 48 (the Lorenz state at 16 save times), SiLU hidden
activations.  Nothing in the paper defines it; the definitions below are the
textbook ones, written so that each GPU kernel has a counterpart:

  forward   A0 = r(X);  Z_l = A_{l-1} r(W_l)^T + b_l;  A_l = r(silu(Z_l))
            for the hidden layers, Y = A_3 r(W_4)^T + b_4,
  loss      L = mean over batch and outputs of (Y - T)^2,
  backward  G_4 = 2 (Y - T) / (B * 48);  dW_l = r(G_l)^T A_{l-1};
            db_l = sum_batch G_l;  G_{l-1} = (r(G_l) r(W_l)) * silu'(Z_{l-1}),
  Adam      Kingma & Ba (2015), Algorithm 1, with bias correction,

where r() rounds to bfloat16 (round to nearest even) when `bf16` is set, the
precision the MFMA kernels see, and is the identity otherwise.  Arithmetic is
FP64 throughout (the GPU accumulates in FP32).

Parameter layout (one flat vector): for each layer l = 1..4, W_l as a
row-major [out][in] matrix followed by b_l [out].
"""
from __future__ import annotations

import numpy as np

DIMS = (4, 256, 256, 256, 48)


def layout(dims=DIMS):
    """[(w_offset, (out, in), b_offset, out)] for each layer, and the total."""
    off = 0
    lay = []
    for i in range(len(dims) - 1):
        nin, nout = dims[i], dims[i + 1]
        lay.append((off, (nout, nin), off + nout * nin, nout))
        off += nout * nin + nout
    return lay, off


N_PARAMS = layout()[1]


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), via float32, as floats."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((u >> 16) & 1)
    r = ((u + bias) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def _r(x, bf16):
    return bf16_round(x) if bf16 else np.asarray(x, dtype=np.float64)


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def unpack(theta, dims=DIMS):
    lay, n = layout(dims)
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (n,)
    return [(theta[w:w + o * i].reshape(o, i), theta[b:b + nb]) for (w, (o, i), b, nb) in lay]


def forward(theta, X, bf16=True, dims=DIMS):
    """X [B][in] -> (Y [B][out], cache)."""
    layers = unpack(theta, dims)
    A = _r(X, bf16)
    acts, pre = [A], []
    for l, (W, b) in enumerate(layers):
        Z = A @ _r(W, bf16).T + b
        pre.append(Z)
        if l < len(layers) - 1:
            A = _r(silu(Z), bf16)
            acts.append(A)
        else:
            A = Z
    return A, {"acts": acts, "pre": pre}


def backward(theta, cache, G, bf16=True, dims=DIMS):
    """Gradient of the loss w.r.t. the flat parameters, given G = dL/dY."""
    layers = unpack(theta, dims)
    lay, n = layout(dims)
    grad = np.zeros(n)
    acts, pre = cache["acts"], cache["pre"]
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        Gr = _r(G, bf16)
        w, (o, i), b, nb = lay[l]
        grad[w:w + o * i] = (Gr.T @ acts[l]).reshape(-1)
        grad[b:b + nb] = G.sum(axis=0)
        if l > 0:
            G = (Gr @ _r(W, bf16)) * silu_grad(pre[l - 1])
    return grad


def loss_and_grad(theta, X, T, bf16=True, dims=DIMS):
    Y, cache = forward(theta, X, bf16, dims)
    B, K = Y.shape
    L = np.mean((Y - T) ** 2)
    G = 2.0 * (Y - T) / (B * K)
    return L, backward(theta, cache, G, bf16, dims), Y


def adam(theta, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1); t counts from 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1**t)
    vhat = v / (1.0 - b2**t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
