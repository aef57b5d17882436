"""Element-wise error bounds for the surrogate network's device results.

The device evaluates the network (and its input gradient and the parameter
gradient with the gradient-matching term) as a fixed sequence of steps:
matrix products whose FP32 operands are rounded to BF16 (nearest even) and
accumulated in FP32, and FP32 elementwise steps (bias, GELU and its first two
derivatives, scalings, column sums, the output dot product).  This module
walks the same sequence in float64 and carries, for every intermediate, its
value v (the BF16-rounding model of oracle/mlp.py) and a bound d >= 0 on the
distance of the device's FP32 value from v:

* a rounding to BF16 adds nothing where [v - d, v + d] holds no rounding
  boundary (every device value in it rounds to the same BF16 number as v);
  elsewhere it allows the full step between the neighbouring BF16 values;
* a K-term FP32 accumulation of exact BF16 x BF16 products adds
  K 2^-24 sum |a| |b|;
* an FP32 elementwise step adds a relative 2^-24 per rounding, and the
  library's erff/expf are allowed 2^-20 (16 ulp) of the result's scale;
  input deviations propagate through local derivative bounds of GELU (the
  derivative at the value plus the half-width of the interval times a global
  bound of the next derivative).

The resulting values must equal oracle.mlp's BF16 mode (which gets them from
autograd, with no hand-written backward), so the bound is tied to the
network's definition; the device must then lie within the bound element by
element.  Test infrastructure only."""
from __future__ import annotations

import math

import numpy as np
import torch

U = 2.0 ** -24    # FP32 unit roundoff
EPS_FN = 2.0 ** -20  # allowance for erff / expf and the ops around them
L_G2, L_G3, L_G4 = 0.80, 0.78, 1.60  # sup |gelu''|, |gelu'''|, |gelu''''| over the reals


def _t(a):
    return torch.as_tensor(np.asarray(a), dtype=torch.float64)


def bf(v):
    """FP32 value -> BF16 (nearest even) -> float64, as the device rounds."""
    return v.to(torch.float32).to(torch.bfloat16).to(torch.float64)


class V:
    """value + deviation bound"""

    __slots__ = ("v", "d")

    def __init__(self, v, d=None):
        self.v = v
        self.d = torch.zeros_like(v) if d is None else d

    @property
    def T(self):
        return V(self.v.transpose(0, 1), self.d.transpose(0, 1))


def rnd(x: V):
    """(BF16 value, bound on the device's BF16 value's distance from it)."""
    r = bf(x.v)
    w = x.d * (1 + 2.0 ** -20) + 1e-300
    lo, hi = bf(x.v - w), bf(x.v + w)
    delta = torch.maximum((lo - r).abs(), (hi - r).abs())
    return r, delta


def gemm(a: V, b: V, acc: V | None = None) -> V:
    """a @ b with both operands rounded to BF16, FP32 accumulation
    (optionally added to acc, the device's beta = 1)."""
    ra, da = rnd(a)
    rb, db = rnd(b)
    K = ra.shape[1]
    v = ra @ rb
    S = (ra.abs() + da) @ (rb.abs() + db)
    d = da @ rb.abs() + ra.abs() @ db + da @ db + (K + 1) * U * S
    if acc is not None:
        v = v + acc.v
        d = d + acc.d + U * (v.abs() + d)
    return V(v, d)


def add(a: V, b: V) -> V:
    v = a.v + b.v
    return V(v, a.d + b.d + U * (a.v.abs() + b.v.abs()))


def mul(a: V, b: V) -> V:
    v = a.v * b.v
    return V(v, a.v.abs() * b.d + b.v.abs() * a.d + a.d * b.d + U * (v.abs() + a.d * b.v.abs() + a.v.abs() * b.d))


def scale(s: float, a: V, s_rel=3 * U) -> V:
    """s * a with s itself an FP32 expression of relative error s_rel"""
    v = s * a.v
    return V(v, abs(s) * a.d + (s_rel + U) * (v.abs() + abs(s) * a.d))


def _phi(z):
    return torch.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


def _g1(z):
    return 0.5 * (1 + torch.special.erf(z / math.sqrt(2))) + z * _phi(z)


def _g2(z):
    return _phi(z) * (2 - z * z)


def _g3(z):
    return _phi(z) * (z ** 3 - 4 * z)


# Over [z - d, z + d], |f'| <= |f'(z)| + d sup|f''| (the derivative bounds
# are local, which keeps saturated units from inflating the bound).
def gelu(z: V) -> V:
    v = 0.5 * z.v * (1 + torch.special.erf(z.v / math.sqrt(2)))
    lip = _g1(z.v).abs() + L_G2 * z.d
    return V(v, lip * z.d + EPS_FN * (0.5 * z.v.abs() + v.abs() + 1e-30))


def gelu_d(z: V) -> V:
    v = _g1(z.v)
    lip = _g2(z.v).abs() + L_G3 * z.d
    return V(v, lip * z.d + EPS_FN * (1 + z.v.abs() * _phi(z.v)))


def gelu_dd(z: V) -> V:
    v = _g2(z.v)
    lip = _g3(z.v).abs() + L_G4 * z.d
    return V(v, lip * z.d + EPS_FN * _phi(z.v) * (2 + z.v * z.v))


def colsum(x: V) -> V:
    M = x.v.shape[0]
    v = x.v.sum(0)
    return V(v, x.d.sum(0) + (M + 1) * U * (x.v.abs().sum(0) + x.d.sum(0)))


def rowdot(h: V, w: V, b: V) -> V:
    """y[m] = h[m] . w + b (FP32, no rounding to BF16)"""
    N = h.v.shape[1]
    v = h.v @ w.v + b.v
    d = h.d @ w.v.abs() + (N + 10) * U * (h.v.abs() @ w.v.abs() + h.d @ w.v.abs()) + U * (v.abs() + b.v.abs())
    return V(v, d)


def bcast_row(w: V, M: int) -> V:
    return V(w.v[None, :].expand(M, -1), w.d[None, :].expand(M, -1))


def model(flat, x, e=None, g=None, lam=0.0, dims=None, backward=True, want_dx=True):
    """Walk the device's steps.  Returns a dict of V: y, gx (when computed)
    and, with backward, the parameter gradient blocks gW1, gb1, gW2, gb2,
    gw3, gb3.  flat: the FP32 parameters (W1[h1][n_in], b1, W2[h2][h1], b2,
    w3, b3); x, e, g: FP32 inputs."""
    n_in, h1, h2 = dims
    f = _t(flat)
    o = 0
    P = {}
    for k, shp in (("W1", (h1, n_in)), ("b1", (h1,)), ("W2", (h2, h1)), ("b2", (h2,)), ("w3", (h2,)), ("b3", (1,))):
        n = int(np.prod(shp))
        P[k] = V(f[o:o + n].reshape(shp))
        o += n
    X = V(_t(x))
    B = X.v.shape[0]
    sob = backward and g is not None and lam != 0.0
    out = {}
    # forward: Z1 = x W1^T + b1, H1 = gelu(Z1), Z2 = H1 W2^T + b2, H2 = gelu(Z2)
    Z1 = add(gemm(X, P["W1"].T), bcast_row(P["b1"], B))
    H1 = gelu(Z1)
    Z2 = add(gemm(H1, P["W2"].T), bcast_row(P["b2"], B))
    H2 = gelu(Z2)
    y = rowdot(H2, P["w3"], V(P["b3"].v.expand(B), P["b3"].d.expand(B)))
    out["y"] = y
    need_dx = want_dx or sob
    if need_dx:
        # A2 = gelu'(Z2) w3, U = A2 W2, A1 = gelu'(Z1) U, Gx = A1 W1
        gd2, gd1 = gelu_d(Z2), gelu_d(Z1)
        A2 = mul(gd2, bcast_row(P["w3"], B))
        Uu = gemm(A2, P["W2"])
        A1 = mul(gd1, Uu)
        Gx = gemm(A1, P["W1"])
        out["gx"] = Gx
    if not backward:
        return out
    E = V(_t(e))
    if sob:
        s = 2.0 * lam / (B * n_in)
        R = add(scale(s, Gx), scale(-s, V(_t(g))))
        gW1 = gemm(A1.T, R)
        dA1 = gemm(R, P["W1"].T)
        dU = mul(gd1, dA1)
        dZ1 = mul(mul(gelu_dd(Z1), Uu), dA1)
        gW2 = gemm(A2.T, dU)
        dA2 = gemm(dU, P["W2"].T)
        gw3 = colsum(mul(gd2, dA2))
        gw3 = V(gw3.v[None, :], gw3.d[None, :])
        dZ2 = mul(mul(gelu_dd(Z2), bcast_row(P["w3"], B)), dA2)
    dy = add(scale(2.0 / B, y), scale(-2.0 / B, E))
    dyc = V(dy.v[:, None], dy.d[:, None])
    gw3 = gemm(dyc.T, H2, gw3 if sob else None)
    gb3 = colsum(dyc)
    T = mul(dyc, V(P["w3"].v[None, :], P["w3"].d[None, :]))  # dy (x) w3
    gdZ2 = gelu_d(Z2)
    dZ2 = add(dZ2, mul(gdZ2, T)) if sob else mul(gdZ2, T)
    gb2 = colsum(dZ2)
    gW2 = gemm(dZ2.T, H1, gW2 if sob else None)
    dH1 = gemm(dZ2, P["W2"])
    gdZ1 = gelu_d(Z1)
    dZ1 = add(dZ1, mul(gdZ1, dH1)) if sob else mul(gdZ1, dH1)
    gb1 = colsum(dZ1)
    gW1 = gemm(dZ1.T, X, gW1 if sob else None)
    out.update(gW1=gW1, gb1=gb1, gW2=gW2, gb2=gb2, gw3=V(gw3.v[0], gw3.d[0]), gb3=gb3)
    return out


BLOCKS = ("gW1", "gb1", "gW2", "gb2", "gw3", "gb3")


def flat_grad(out):
    v = torch.cat([out[k].v.reshape(-1) for k in BLOCKS])
    d = torch.cat([out[k].d.reshape(-1) for k in BLOCKS])
    return V(v, d)


def excess(got, ref: V, safety=2.0):
    """max over elements of |got - v| / (safety d + tiny): <= 1 passes."""
    got = _t(got).reshape(ref.v.shape)
    return float(((got - ref.v).abs() / (safety * ref.d + 1e-30)).max())
