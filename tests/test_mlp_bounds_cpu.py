"""CPU checks of the surrogate network's BF16-rounding oracle and of the
element-wise bounds the GPU test applies to the device's results.

* The rounding variant of oracle/mlp.py, with its rounding switched off,
  equals the plain float64 definition (its product rules are the right
  derivatives), and with rounding on it equals the step-by-step value model
  of tests/mlp_bounds.py (the device's rounding points are the definition's).
* An FP32 evaluation of the device's steps (a stand-in for the device, on the
  CPU) lies within the bounds; the same evaluation with one plausible mistake
  planted -- a dropped second-derivative term, a rounding in the wrong place,
  a wrong factor in the gradient-matching term, 10 % errors in the entries
  of the bias gradients 50 times smaller than their block's largest --
  falls outside them."""
import numpy as np
import pytest
import torch

import oracle.mlp as omlp
from tests import mlp_bounds as MB

DIMS = (24, 40, 32)
B = 7


def _problem(seed, dims=DIMS, batch=B):
    n_in, h1, h2 = dims
    rng = np.random.default_rng(seed)
    flat = np.concatenate([rng.normal(size=h1 * n_in) / np.sqrt(n_in), 0.1 * rng.normal(size=h1),
                           rng.normal(size=h2 * h1) / np.sqrt(h1), 0.1 * rng.normal(size=h2),
                           rng.normal(size=h2) / np.sqrt(h2), [0.05]]).astype(np.float32)
    x = rng.uniform(0, 2 * np.pi, (batch, n_in)).astype(np.float32)
    e = rng.normal(size=batch).astype(np.float32)
    g = (0.1 * rng.normal(size=(batch, n_in))).astype(np.float32)
    return flat, x, e, g


def test_rounding_variant_without_rounding_is_the_definition(monkeypatch):
    flat, x, e, g = _problem(1)
    ref = omlp.loss_and_grads(flat.astype(np.float64), x, e, g, 1.0, DIMS)
    monkeypatch.setattr(omlp, "_round_bf16", lambda t: t)
    got = omlp.loss_and_grads(flat.astype(np.float64), x, e, g, 1.0, DIMS, bf16=True)
    assert abs(got[0] - ref[0]) <= 1e-12 * abs(ref[0])
    for a, b in zip(got[1:], ref[1:]):
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


@pytest.mark.parametrize("lam", [0.0, 1.0])
def test_value_model_equals_rounding_oracle(lam):
    flat, x, e, g = _problem(2)
    L, dP, y, gx = omlp.loss_and_grads(flat.astype(np.float64), x, e, g, lam, DIMS, bf16=True)
    m = MB.model(flat, x, e, g, lam, DIMS)
    for got, ref in ((y, m["y"]), (gx, m["gx"]), (dP, MB.flat_grad(m))):
        ref_v = ref.v.numpy().reshape(-1)
        diff = np.abs(np.asarray(got).reshape(-1) - ref_v)
        assert np.all(diff <= 1e-3 * ref.d.numpy().reshape(-1) + 1e-300), float(diff.max())


def _device_standin(flat, x, e, g, lam, dims, plant=None):
    """The device's steps evaluated in FP32 on the CPU (products of BF16-
    rounded operands); `plant` names one deliberate mistake."""
    n_in, h1, h2 = dims
    f = torch.tensor(flat)
    o, P = 0, {}
    for k, shp in (("W1", (h1, n_in)), ("b1", (h1,)), ("W2", (h2, h1)), ("b2", (h2,)), ("w3", (h2,)), ("b3", (1,))):
        n = int(np.prod(shp))
        P[k] = f[o:o + n].reshape(shp)
        o += n
    X, E, G = torch.tensor(x), torch.tensor(e), torch.tensor(g)
    bf = lambda t: t.to(torch.bfloat16).to(torch.float32)
    mm = lambda a, b: bf(a) @ bf(b)
    s2 = torch.tensor(0.5 ** 0.5, dtype=torch.float32)
    gelu = lambda z: 0.5 * z * (1 + torch.erf(z * s2))
    phi = lambda z: 0.3989422804014327 * torch.exp(-0.5 * z * z)
    gd = lambda z: 0.5 * (1 + torch.erf(z * s2)) + z * phi(z)
    gdd = lambda z: phi(z) * (2 - z * z)
    Bn = X.shape[0]
    Z1 = mm(X, P["W1"].T) + P["b1"]
    H1 = gelu(Z1)
    Z2 = mm(H1, P["W2"].T) + P["b2"]
    H2 = gelu(Z2)
    y = H2 @ P["w3"] + P["b3"]
    w3a = bf(P["w3"]) if plant == "round_w3" else P["w3"]
    A2 = gd(Z2) * w3a
    U = mm(A2, P["W2"])
    A1 = gd(Z1) * U
    Gx = mm(A1, P["W1"])
    s = 2.0 * lam / (Bn * n_in) * (0.5 if plant == "half_lambda" else 1.0)
    R = s * Gx - s * G
    gW1 = mm(A1.T, R)
    dA1 = mm(R, P["W1"].T)
    dU = gd(Z1) * dA1
    dZ1 = gdd(Z1) * U * dA1
    if plant == "drop_gdd1":
        dZ1 = torch.zeros_like(dZ1)
    gW2 = mm(A2.T, dU)
    dA2 = mm(dU, P["W2"].T)
    gw3 = (gd(Z2) * dA2).sum(0)
    dZ2 = gdd(Z2) * P["w3"] * dA2
    dy = 2.0 / Bn * y - 2.0 / Bn * E
    gw3 = gw3 + mm(dy[None, :], H2)[0]
    gb3 = dy.sum(0, keepdim=True)
    dZ2 = dZ2 + gd(Z2) * (dy[:, None] * P["w3"][None, :])
    gb2 = dZ2.sum(0)
    gW2 = gW2 + mm(dZ2.T, H1)
    dH1 = mm(dZ2, P["W2"])
    dZ1 = dZ1 + gd(Z1) * dH1
    gb1 = dZ1.sum(0)
    gW1 = gW1 + mm(dZ1.T, X)
    grads = torch.cat([gW1.reshape(-1), gb1, gW2.reshape(-1), gb2, gw3, gb3])
    if plant == "small_entries":
        # every entry of the bias gradients 50x below its block's largest, 10 % off
        o = h1 * n_in
        for lo, hi in ((o, o + h1), (o + h1 + h2 * h1, o + h1 + h2 * h1 + h2)):
            blk = grads[lo:hi]
            small = blk.abs() < blk.abs().max() / 50
            blk[small] = blk[small] * 1.1
    return y, Gx, grads


def _excess(dev, m):
    y, gx, grads = dev
    return max(MB.excess(y.double(), m["y"]), MB.excess(gx.double(), m["gx"]),
               MB.excess(grads.double(), MB.flat_grad(m)))


def test_fp32_standin_within_bounds():
    for seed in (3, 4):
        flat, x, e, g = _problem(seed)
        m = MB.model(flat, x, e, g, 1.0, DIMS)
        ex = _excess(_device_standin(flat, x, e, g, 1.0, DIMS), m)
        assert ex <= 1.0, ex


@pytest.mark.parametrize("plant", ["drop_gdd1", "round_w3", "half_lambda", "small_entries"])
def test_planted_mistake_exceeds_bounds(plant):
    flat, x, e, g = _problem(3)
    m = MB.model(flat, x, e, g, 1.0, DIMS)
    ex = _excess(_device_standin(flat, x, e, g, 1.0, DIMS, plant), m)
    assert ex > 1.0, (plant, ex)
