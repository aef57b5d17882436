"""Handle over the surrogate network kernels (vqc_mlp_* in include/vqc.h).

n_in -> h1 -> h2 -> 1 with exact-erf GELU; FP32 parameters, BF16 matrix
products with FP32 accumulation.  Marshalling only: parameters live in the
library's device buffer, viewed here as a torch tensor.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import binding as B
from .api import stream_ptr
from .binding import check, lib


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def gemm_bf16(A, B_, ta=False, tb=False, C=None, alpha=1.0, beta=0.0):
    """C = alpha op(A) op(B) + beta C on the GPU (FP32 tensors)."""
    M = A.shape[1] if ta else A.shape[0]
    K = A.shape[0] if ta else A.shape[1]
    N = B_.shape[0] if tb else B_.shape[1]
    if C is None:
        C = torch.zeros(M, N, dtype=torch.float32, device=A.device)
    check(lib().vqc_gemm_bf16(M, N, K, _p(A), A.shape[1], int(ta), _p(B_), B_.shape[1], int(tb), _p(C), C.shape[1],
                              float(alpha), float(beta), ctypes.c_void_p(stream_ptr())), "vqc_gemm_bf16")
    return C


class MLP:
    def __init__(self, n_in, h1, h2, max_batch, device="cuda"):
        self.dims = (n_in, h1, h2)
        self.max_batch = max_batch
        h = ctypes.c_void_p()
        check(lib().vqc_mlp_create(ctypes.byref(h), n_in, h1, h2, max_batch, ctypes.c_void_p(stream_ptr())),
              "vqc_mlp_create")
        self.h = h
        p, g, n = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_size_t()
        check(lib().vqc_mlp_buffers(h, ctypes.byref(p), ctypes.byref(g), ctypes.byref(n)), "vqc_mlp_buffers")
        self.count = n.value
        self.params = _wrap(p.value, self.count, device)
        self.grads = _wrap(g.value, self.count, device)
        self.step = 0

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and B._lib is not None:
            B._lib.vqc_mlp_destroy(h)
            self.h = None

    def layout(self):
        n_in, h1, h2 = self.dims
        sizes = [("W1", (h1, n_in)), ("b1", (h1,)), ("W2", (h2, h1)), ("b2", (h2,)), ("w3", (h2,)), ("b3", (1,))]
        out, o = {}, 0
        for name, shp in sizes:
            k = int(np.prod(shp))
            out[name] = (o, shp)
            o += k
        return out

    def set_params(self, flat: np.ndarray):
        self.params.copy_(torch.as_tensor(np.asarray(flat, np.float32), device=self.params.device))

    def forward(self, x, want_grad=False):
        x = x.contiguous()
        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        g = torch.empty_like(x) if want_grad else None
        check(lib().vqc_mlp_forward(self.h, x.shape[0], _p(x), _p(y), _p(g)), "vqc_mlp_forward")
        return (y, g) if want_grad else y

    def backward(self, x, e, g=None, lam=0.0):
        check(lib().vqc_mlp_backward(self.h, x.shape[0], _p(x.contiguous()), _p(e.contiguous()),
                                     _p(g.contiguous() if g is not None else None), float(lam), None, None),
              "vqc_mlp_backward")
        return self.grads

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        check(lib().vqc_mlp_adam(self.h, float(lr), float(b1), float(b2), float(eps), self.step), "vqc_mlp_adam")

    def descend_inputs(self, x, lr, steps):
        check(lib().vqc_mlp_descend_inputs(self.h, x.shape[0], _p(x), float(lr), int(steps)),
              "vqc_mlp_descend_inputs")
        return x


def _wrap(ptr, count, device):
    """A torch view of a library-owned FP32 device buffer (kept alive by the MLP)."""
    # build through the CUDA array interface of a tiny holder object
    class _Holder:
        pass
    hold = _Holder()
    hold.__cuda_array_interface__ = {"shape": (count,), "typestr": "<f4", "data": (ptr, False), "version": 3,
                                     "strides": None}
    return torch.as_tensor(hold, device=device)
