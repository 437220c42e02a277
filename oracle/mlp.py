"""Learned start density: descriptors, MLP, loss, gradients and Adam (oracle, FP64).

The start density of an SCF run may come from a small per-grid-point network
instead of the superposition of atomic densities:

  descriptors  d_k(x) = sum_J sum_L exp(-|x - R_J - L|^2 / (2 w_k^2)),
               k = 1..K, widths w_k geometric between w_min and w_max;
  inputs       u = (d - mean) / std, per channel (training-set statistics);
  network      a_0 = u, a_l = SiLU(W_l a_{l-1} + b_l) for the hidden layers,
               z = W_out a_L + b_out, y = softplus(z)  (y models rho / rho_bar,
               rho_bar = N_e / volume);
  density      rho_0(x) = N_e y(x) / (h^3 sum_x y(x));
  loss         mean over a batch of (y - rho_target / rho_bar)^2;
  training     Adam (Kingma & Ba): m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
               theta <- theta - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

SiLU(z) = z sigmoid(z), SiLU'(z) = sigmoid(z) (1 + z (1 - sigmoid(z)));
softplus(z) = log(1 + e^z), softplus'(z) = sigmoid(z).

Parameters are one flat vector, layer by layer: W_l (n_out x n_in, row-major:
W[o, i] at o * n_in + i) then b_l (n_out), for l = 1..L+1.

Pins (tests): descriptors against a brute-force three-dimensional image sum;
gradients against central differences of the loss; the first Adam step in
closed form (-lr g / (|g| + eps)).
"""

from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np


def widths(k: int, w_min: float, w_max: float) -> np.ndarray:
    return w_min * (w_max / w_min) ** (np.arange(k) / (k - 1))


def _periodic_1d(x: np.ndarray, r0: float, a: float, w2: float) -> np.ndarray:
    d0 = x - r0
    d0 = d0 - a * np.round(d0 / a)
    m = int(math.ceil(math.sqrt(50.0 * w2) / a)) + 1
    out = np.zeros_like(x)
    for img in range(-m, m + 1):
        d = d0 - img * a
        out += np.exp(-d * d / w2)
    return out


def descriptors(n: int, a: float, pos: np.ndarray, w: np.ndarray) -> np.ndarray:
    """(N_grid, K): the Gaussian sum factorises over the axes (exactly)."""
    x = np.arange(n) * (a / n)
    out = np.zeros((n ** 3, len(w)))
    for k, wk in enumerate(w):
        w2 = 2.0 * wk * wk
        for p in pos:
            g = [_periodic_1d(x, p[ax], a, w2) for ax in range(3)]
            out[:, k] += (g[2][:, None, None] * g[1][None, :, None] * g[0][None, None, :]).reshape(-1)
    return out


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def layer_shapes(n_in: int, hidden: int, n_hidden_layers: int) -> List[Tuple[int, int]]:
    dims = [n_in] + [hidden] * n_hidden_layers + [1]
    return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]


def param_count(shapes) -> int:
    return sum(o * i + o for o, i in shapes)


def unpack(theta: np.ndarray, shapes):
    out, off = [], 0
    for o, i in shapes:
        W = theta[off:off + o * i].reshape(o, i)
        off += o * i
        b = theta[off:off + o]
        off += o
        out.append((W, b))
    return out


def init_params(shapes, seed: int) -> np.ndarray:
    """Uniform(-1/sqrt(n_in), 1/sqrt(n_in)) for weights and biases, seeded."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for o, i in shapes:
        bound = 1.0 / math.sqrt(i)
        parts.append(rng.uniform(-bound, bound, o * i))
        parts.append(rng.uniform(-bound, bound, o))
    return np.concatenate(parts)


def forward(theta, shapes, u: np.ndarray):
    """u: (P, n_in) -> y (P,), with the pre-activations kept for backprop."""
    layers = unpack(theta, shapes)
    acts, pre = [u], []
    a = u
    for li, (W, b) in enumerate(layers):
        z = a @ W.T + b
        pre.append(z)
        a = silu(z) if li < len(layers) - 1 else z
        acts.append(a)
    y = softplus(pre[-1][:, 0])
    return y, acts, pre


def loss_and_grad(theta, shapes, u: np.ndarray, target: np.ndarray):
    """loss = mean (y - target)^2 and its gradient with respect to theta."""
    layers = unpack(theta, shapes)
    y, acts, pre = forward(theta, shapes, u)
    P = len(y)
    r = y - target
    loss = float(np.mean(r * r))
    dz = (2.0 / P) * r * sigmoid(pre[-1][:, 0])  # d loss / d z_out
    delta = dz[:, None]
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        a_in = acts[li]
        grads.append((delta.T @ a_in, delta.sum(axis=0)))
        if li > 0:
            delta = (delta @ W) * silu_grad(pre[li - 1])
    grads.reverse()
    g = np.concatenate([np.concatenate([gW.reshape(-1), gb]) for gW, gb in grads])
    return loss, g


def adam_step(theta, m, v, g, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def density(theta, shapes, u: np.ndarray, n_e: float, h: float) -> np.ndarray:
    y, _, _ = forward(theta, shapes, u)
    return n_e * y / (h ** 3 * y.sum())
