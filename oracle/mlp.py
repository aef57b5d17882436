"""FP64 CPU oracle of the surrogate network (test infrastructure only).

The network is not part of the paper: it models the variational energy
E(theta) of the hardware-efficient ansatz.  Definition:
    z1 = W1 x + b1, h1 = gelu(z1), z2 = W2 h1 + b2, h2 = gelu(z2),
    y  = w3 . h2 + b3,  gelu(x) = x Phi(x) = x (1 + erf(x / sqrt 2)) / 2,
    L  = mean_b (y_b - e_b)^2 + lambda / (B n_in) sum_b |dy/dx(x_b) - g_b|^2.
Everything is evaluated with plain torch CPU float64 ops; dy/dx and the
parameter gradient (which needs second derivatives) come from torch's
autograd with create_graph=True, i.e. the definition differentiated by the
library primitive, with no hand-written backward.

``bf16`` rounds x and the weights to bfloat16 (round to nearest even) before
use, the way the device kernels round the inputs of every matrix product;
intermediate activations stay in float64, so the comparison tolerance has to
cover the rounding of activations on the device (see the tests).
"""
from __future__ import annotations

import math

import numpy as np
import torch

LAYOUT = ("W1", "b1", "W2", "b2", "w3", "b3")


def unpack(flat, n_in, h1, h2):
    shapes = {"W1": (h1, n_in), "b1": (h1,), "W2": (h2, h1), "b2": (h2,), "w3": (h2,), "b3": (1,)}
    out, o = {}, 0
    for k in LAYOUT:
        n = int(np.prod(shapes[k]))
        out[k] = flat[o:o + n].reshape(shapes[k])
        o += n
    return out


def gelu(z):
    return 0.5 * z * (1.0 + torch.special.erf(z / math.sqrt(2.0)))


def _round_bf16(t):
    return t.to(torch.bfloat16).to(torch.float64)


def forward(flat, x, dims, bf16=False):
    """y [B] for x [B, n_in] (numpy or torch), float64."""
    n_in, h1, h2 = dims
    p = unpack(torch.as_tensor(np.asarray(flat), dtype=torch.float64), n_in, h1, h2)
    x = torch.as_tensor(np.asarray(x), dtype=torch.float64)
    if bf16:
        x = _round_bf16(x)
        p = {k: (_round_bf16(v) if k in ("W1", "W2") else v) for k, v in p.items()}
    z1 = x @ p["W1"].T + p["b1"]
    z2 = gelu(z1) @ p["W2"].T + p["b2"]
    return gelu(z2) @ p["w3"] + p["b3"][0]


def loss_and_grads(flat, x, e, g, lam, dims):
    """(loss, dL/dparams flat, y, dy/dx) in float64 by autograd."""
    n_in, h1, h2 = dims
    P = torch.tensor(np.asarray(flat, np.float64), requires_grad=True)
    p = unpack(P, n_in, h1, h2)
    X = torch.tensor(np.asarray(x, np.float64), requires_grad=True)
    z1 = X @ p["W1"].T + p["b1"]
    z2 = gelu(z1) @ p["W2"].T + p["b2"]
    y = gelu(z2) @ p["w3"] + p["b3"][0]
    B = X.shape[0]
    E = torch.as_tensor(np.asarray(e, np.float64))
    loss = ((y - E) ** 2).mean()
    gx = None
    if g is not None and lam != 0.0:
        (gx,) = torch.autograd.grad(y.sum(), X, create_graph=True)
        G = torch.as_tensor(np.asarray(g, np.float64))
        loss = loss + lam / (B * n_in) * ((gx - G) ** 2).sum()
    (dP,) = torch.autograd.grad(loss, P, retain_graph=True)
    if gx is None:
        (gx,) = torch.autograd.grad(y.sum(), X)
    return float(loss.detach()), dP.numpy().copy(), y.detach().numpy().copy(), gx.detach().numpy().copy()
