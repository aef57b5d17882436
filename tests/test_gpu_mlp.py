"""Surrogate-network kernels vs the FP64 oracle.

GEMM: inputs rounded to BF16 exactly as the kernel rounds them, products
exact in FP32, so |C - C_ref| <= (K-1) 2^-24 sum_k |a_k b_k| (FP32
accumulation bound) element by element.  Network: the output, the input
gradient and every parameter-gradient entry are compared element by element
with the bounds of tests/mlp_bounds.py -- the device's steps walked in
float64 with the BF16 roundings where the kernels round, FP32 accumulation
bounds and flips of a BF16 rounding allowed only where the bound straddles
a rounding boundary -- whose values equal oracle.mlp's BF16 mode (autograd
of the network's definition)."""
import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from paper_2406_19212_amd import workloads as W
from tests import mlp_bounds as MB
from paper_2406_19212_amd.mlp import MLP, gemm_bf16

pytestmark = pytest.mark.gpu


def bf(x):
    return torch.as_tensor(x).to(torch.bfloat16).to(torch.float64)


# shapes reach all three block tiles (32: small grids; 64: (768, 770, 96);
# 128: the two 2048-wide cases), aligned float4 and scalar loads, and K
# tails inside and beyond a 32-wide k step
@pytest.mark.parametrize("M,N,K", [(70, 130, 45), (64, 64, 16), (1, 512, 37), (513, 3, 320), (5, 7, 1),
                                   (768, 770, 96), (2050, 2048, 64), (2048, 2052, 36)])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_bf16_layouts(M, N, K, ta, tb):
    g = torch.Generator().manual_seed(M * 131 + N * 7 + K + 1000 * ta + 2000 * tb)
    A = torch.randn((K, M) if ta else (M, K), generator=g, dtype=torch.float32)
    Bm = torch.randn((N, K) if tb else (K, N), generator=g, dtype=torch.float32)
    Ad, Bd = bf(A), bf(Bm)
    opA = Ad.T if ta else Ad
    opB = Bd.T if tb else Bd
    ref = opA @ opB
    bound = (K - 1) * 2.0 ** -24 * (opA.abs() @ opB.abs()) + 1e-30
    C = gemm_bf16(A.cuda(), Bm.cuda(), bool(ta), bool(tb)).double().cpu()
    assert torch.all((C - ref).abs() <= bound), float(((C - ref).abs() / bound).max())
    # beta accumulation: C2 = 2 op(A)op(B) + 0.5 C0
    C0 = torch.randn(M, N, generator=g, dtype=torch.float32)
    C2 = gemm_bf16(A.cuda(), Bm.cuda(), bool(ta), bool(tb), C=C0.cuda().clone(), alpha=2.0, beta=0.5).double().cpu()
    ref2 = 2 * ref + 0.5 * C0.double()
    assert torch.all((C2 - ref2).abs() <= 2 * bound + 4 * 2.0 ** -24 * ref2.abs() + 1e-30)


def _init(dims, seed):
    n_in, h1, h2 = dims
    r = W.SplitMix64(seed)
    parts = [r.normal(h1 * n_in) / np.sqrt(n_in), np.zeros(h1), r.normal(h2 * h1) / np.sqrt(h1), np.zeros(h2),
             r.normal(h2) / np.sqrt(h2), np.zeros(1)]
    return np.concatenate(parts)


def _blocks(dims, v):
    n_in, h1, h2 = dims
    return omlp.unpack(np.asarray(v), n_in, h1, h2)


@pytest.mark.parametrize("lam", [0.0, 1.0])
def test_mlp_forward_and_gradients(lam):
    dims = (320, 512, 512)
    B = 37
    p = _init(dims, 7)
    net = MLP(*dims, max_batch=64)
    net.set_params(p)
    p32 = net.params.double().cpu().numpy()  # the FP32 parameters the device uses
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 2 * np.pi, (B, dims[0])).astype(np.float32)
    e = rng.normal(size=B).astype(np.float32)
    g = (0.1 * rng.normal(size=(B, dims[0]))).astype(np.float32)
    xt, et, gt = (torch.tensor(v, device="cuda") for v in (x, e, g))
    y, gx = net.forward(xt, want_grad=True)
    grads = net.backward(xt, et, gt if lam else None, lam).double().cpu().numpy()
    m = MB.model(p32, x, e, g, lam, dims)
    # the bound's values are the rounding oracle's (autograd of the definition)
    _, dP_bf, y_bf, gx_bf = omlp.loss_and_grads(p32, x, e, g, lam, dims, bf16=True)
    for want, ref in ((y_bf, m["y"]), (gx_bf, m["gx"]), (dP_bf, MB.flat_grad(m))):
        diff = np.abs(np.asarray(want).reshape(-1) - ref.v.numpy().reshape(-1))
        assert np.all(diff <= 1e-3 * ref.d.numpy().reshape(-1) + 1e-300), float(diff.max())
    # the device within the element-wise bounds (<= 1 passes)
    ex = {"y": MB.excess(y.double().cpu(), m["y"]), "gx": MB.excess(gx.double().cpu(), m["gx"])}
    got = _blocks(dims, grads)
    for pk, gk in zip(omlp.LAYOUT, MB.BLOCKS):
        ex[gk] = MB.excess(got[pk].reshape(-1), MB.V(m[gk].v.reshape(-1), m[gk].d.reshape(-1)))
    print("bound excess (<= 1 passes):", {k: round(v, 4) for k, v in ex.items()})
    assert max(ex.values()) <= 1.0, ex
    # and the BF16 network stays close to the float64 definition
    _, dP, y_ref, gx_ref = omlp.loss_and_grads(p32, x, e, g, lam, dims)
    assert np.max(np.abs(y.cpu().numpy() - y_ref)) <= 2e-2 * np.max(np.abs(y_ref))
    assert np.max(np.abs(gx.cpu().numpy() - gx_ref)) <= 2e-2 * np.max(np.abs(gx_ref))


def test_adam_step_and_input_descent():
    dims = (8, 16, 16)
    net = MLP(*dims, max_batch=8)
    p = _init(dims, 9)
    net.set_params(p)
    rng = np.random.default_rng(2)
    x = torch.tensor(rng.uniform(0, 6, (4, 8)).astype(np.float32), device="cuda")
    e = torch.tensor(rng.normal(size=4).astype(np.float32), device="cuda")
    g = net.backward(x, e).clone()
    p0 = net.params.clone()
    net.adam(lr=1e-2)
    # Adam's first step moves every parameter by lr * sign(g) (bias-corrected moments)
    gd, pd = g.double().cpu().numpy(), (net.params - p0).double().cpu().numpy()
    mask = np.abs(gd) > 1e-4  # where eps = 1e-8 changes the step by < 1e-4
    bad = np.where(~np.isclose(pd, -1e-2 * np.sign(gd), rtol=1e-3, atol=1e-7) & mask)[0]
    assert bad.size == 0, [(int(i), float(gd[i]), float(pd[i])) for i in bad[:10]] + [gd.size]
    # gradient descent on the inputs lowers the surrogate
    y0 = net.forward(x).clone()
    xs = x.clone()
    net.descend_inputs(xs, lr=0.05, steps=5)
    assert torch.all(net.forward(xs) < y0)
