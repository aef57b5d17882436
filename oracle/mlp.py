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

``bf16=True`` gives the variant whose rounding points are those of the
device kernels: every operand of a matrix product -- in the forward pass, in
the input gradient dy/dx and in both backward passes of the parameter
gradient -- is rounded to bfloat16 (round to nearest even) before the
product, which is then accumulated in float64.  The output layer's forward
dot product y = h2 . w3 + b3, its input-side gradient dy (x) w3 and every
elementwise step (bias, GELU and its derivatives, the loss terms) are not
rounded.  This is implemented with two autograd Functions whose forward and
backward formulas are the plain products with those roundings applied to
their operands (gradients pass straight through a rounding), so the
parameter gradient is still the definition differentiated by autograd, with
no hand-written backward.
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


class _BMatmul(torch.autograd.Function):
    """A @ B with both operands rounded to bfloat16, float64 accumulation.
    Backward: dA = dC @ B^T and dB = A^T @ dC, each again a rounded product
    (so a second differentiation rounds the same way)."""

    @staticmethod
    def forward(ctx, A, B):
        ctx.save_for_backward(A, B)
        return _round_bf16(A) @ _round_bf16(B)

    @staticmethod
    def backward(ctx, dC):
        A, B = ctx.saved_tensors
        dA = _BMatmul.apply(dC, B.transpose(0, 1)) if ctx.needs_input_grad[0] else None
        dB = _BMatmul.apply(A.transpose(0, 1), dC) if ctx.needs_input_grad[1] else None
        return dA, dB


class _OutDot(torch.autograd.Function):
    """y = H @ w (H [B, h], w [h]) in float64 without rounding; backward
    dH = dy (x) w (not rounded) and dw = H^T dy as a rounded product."""

    @staticmethod
    def forward(ctx, H, w):
        ctx.save_for_backward(H, w)
        return H @ w

    @staticmethod
    def backward(ctx, dy):
        H, w = ctx.saved_tensors
        dH = dy[:, None] * w[None, :] if ctx.needs_input_grad[0] else None
        dw = _BMatmul.apply(H.transpose(0, 1), dy[:, None])[:, 0] if ctx.needs_input_grad[1] else None
        return dH, dw


def _net(p, X, bf16):
    """y for the parameter dict p and inputs X (the network's definition)."""
    if bf16:
        z1 = _BMatmul.apply(X, p["W1"].transpose(0, 1)) + p["b1"]
        z2 = _BMatmul.apply(gelu(z1), p["W2"].transpose(0, 1)) + p["b2"]
        return _OutDot.apply(gelu(z2), p["w3"]) + p["b3"][0]
    z1 = X @ p["W1"].T + p["b1"]
    z2 = gelu(z1) @ p["W2"].T + p["b2"]
    return gelu(z2) @ p["w3"] + p["b3"][0]


def forward(flat, x, dims, bf16=False):
    """y [B] for x [B, n_in] (numpy or torch), float64."""
    n_in, h1, h2 = dims
    p = unpack(torch.as_tensor(np.asarray(flat), dtype=torch.float64), n_in, h1, h2)
    x = torch.as_tensor(np.asarray(x), dtype=torch.float64)
    with torch.no_grad():
        return _net(p, x, bf16)


def loss_and_grads(flat, x, e, g, lam, dims, bf16=False):
    """(loss, dL/dparams flat, y, dy/dx) in float64 by autograd; bf16 as in
    the module docstring."""
    n_in, h1, h2 = dims
    P = torch.tensor(np.asarray(flat, np.float64), requires_grad=True)
    p = unpack(P, n_in, h1, h2)
    X = torch.tensor(np.asarray(x, np.float64), requires_grad=True)
    y = _net(p, X, bf16)
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
