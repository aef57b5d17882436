"""Thin Python handles over the C ABI (marshalling only).

``State``    StateVector / DensityMatrix (Sec. 2.1) in a torch complex128 tensor
``Circuit``  QCircuit (Sec. 2.3): fused forward, adjoint backward, autotune
``Batch``    many circuits / parameter sets run together (one launch per step)
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import binding as B
from .binding import check, lib


def stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def flatten_ops(ops) -> list:
    """QCircuit nesting (Sec. 2.3): an element may be an op, a Circuit or a
    list of elements; the result is the flat op sequence in order."""
    out = []
    for x in ops:
        if hasattr(x, "name"):
            out.append(x)
        elif isinstance(x, Circuit):
            out.extend(x.ops)
        else:
            out.extend(flatten_ops(x))
    return out


def ops_params(ops) -> int:
    m = -1
    for op in ops:
        for v in (getattr(op, "var", ()) or ()):
            m = max(m, int(v))
    return m + 1


def fuse_gates(n: int, ops, theta=None):
    """fuse_gates(circ): one-qubit gates absorbed into an adjacent two-qubit
    gate on their qubit; returns general matrix ops (workloads.Op "matrix",
    row-major numpy data) evaluated at theta (host values)."""
    from .workloads import Op
    arr = B.OpArray(ops)
    P = ops_params(ops)
    th = np.ascontiguousarray(np.zeros(max(1, P)) if theta is None else np.asarray(theta, np.float64).ravel())
    out = (B.vqc_op * max(1, len(ops)))()
    data = np.zeros(16 * max(1, len(ops)), np.complex128)
    cnt = ctypes.c_int()
    check(lib().vqc_fuse_gates(int(n), len(ops), arr.ptr(), P, th.ctypes.data, ctypes.cast(out, ctypes.c_void_p),
                               data.ctypes.data, ctypes.byref(cnt)), "vqc_fuse_gates")
    res = []
    for k in range(cnt.value):
        o = out[k]
        d = 1 << o.n_qubits
        M = data[16 * k:16 * k + d * d].reshape(d, d).T.copy()  # ABI column-major -> row-major
        res.append(Op("matrix", tuple(o.qubits[t] for t in range(o.n_qubits)), (), (), M))
    return res


class State:
    """An n-qubit pure state (2^n amplitudes) or vectorised density matrix
    (4^n entries, v[x + 2^n y] = rho[x][y]) in a torch complex128 tensor."""

    def __init__(self, n: int, mixed: bool = False, init=None, tensor=None, device="cuda", stream=None):
        self.n = int(n)
        self.mixed = bool(mixed)
        size = 1 << (2 * self.n if self.mixed else self.n)
        self.tensor = tensor if tensor is not None else torch.empty(size, dtype=torch.complex128, device=device)
        if self.tensor.numel() != size or self.tensor.dtype != torch.complex128 or not self.tensor.is_contiguous():
            raise ValueError("state tensor must be contiguous complex128 with %d entries" % size)
        self._stream = stream_ptr(stream)
        h = ctypes.c_void_p()
        host = None
        if init is not None:
            host = np.ascontiguousarray(np.asarray(init, np.complex128).ravel())
            if host.size != size:
                raise ValueError("init must hold %d amplitudes" % size)
        check(lib().vqc_state_init(ctypes.byref(h), B.VQC_MIXED if self.mixed else B.VQC_PURE, self.n,
                                   _dptr(self.tensor), None if host is None else host.ctypes.data,
                                   ctypes.c_void_p(self._stream)), "vqc_state_init")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and B._lib is not None:
            B._lib.vqc_state_destroy(h)
            self.h = None

    def reset(self):
        """|0..0> (or |0..0><0..0|) again, queued on the stream."""
        check(lib().vqc_state_reset(self.h), "vqc_state_reset")

    def apply_gate(self, qubits, matrix):
        """Eq. (3) / Eq. (twoqubitgate) with a row-major numpy matrix."""
        q = (ctypes.c_int * len(qubits))(*qubits)
        m = B.colmajor(matrix)
        check(lib().vqc_apply_gate(self.h, len(qubits), q, m.ctypes.data), "vqc_apply_gate")

    def apply_op(self, op):
        arr = B.OpArray([op])
        check(lib().vqc_apply_op(self.h, ctypes.byref(arr.arr[0])), "vqc_apply_op")

    def apply_channel(self, qubits, kraus):
        q = (ctypes.c_int * len(qubits))(*qubits)
        buf = np.ascontiguousarray(np.concatenate([B.colmajor(k) for k in kraus]))
        check(lib().vqc_apply_channel(self.h, len(qubits), q, len(kraus), buf.ctypes.data), "vqc_apply_channel")

    def expectation(self, terms) -> complex:
        ps = B.PauliSum(terms)
        out = B.vqc_c128()
        check(lib().vqc_expectation(self.h, ps.ref(), ctypes.byref(out)), "vqc_expectation")
        return complex(out.re, out.im)

    def expectation_noalloc(self, terms) -> complex:
        """expectation() through the allocation-free entry point (fixed library
        scratch; at most 1024 terms and 2^28 summed amplitudes)."""
        ps = B.PauliSum(terms)
        out = B.vqc_c128()
        check(lib().vqc_expectation_noalloc(self.h, ps.ref(), ctypes.byref(out)), "vqc_expectation_noalloc")
        return complex(out.re, out.im)

    def norm(self) -> float:
        out = ctypes.c_double()
        check(lib().vqc_norm(self.h, ctypes.byref(out)), "vqc_norm")
        return out.value

    def gather(self, idx) -> np.ndarray:
        idx = np.ascontiguousarray(np.asarray(idx, np.int64))
        out = np.zeros(idx.size, np.complex128)
        check(lib().vqc_gather(self.h, idx.size, idx.ctypes.data, out.ctypes.data), "vqc_gather")
        return out

    def measure(self, qubit: int, u: float):
        """measure!(state, qubit): collapse in place; returns (outcome, probability).
        u is the caller's uniform number in [0, 1)."""
        o = ctypes.c_int()
        p = ctypes.c_double()
        check(lib().vqc_measure(self.h, int(qubit), float(u), ctypes.byref(o), ctypes.byref(p)), "vqc_measure")
        return o.value, p.value

    def sample(self, u) -> np.ndarray:
        """Basis-state samples (int64) for the uniform numbers u in [0, 1)."""
        uu = np.ascontiguousarray(np.asarray(u, np.float64).ravel())
        out = np.zeros(max(1, uu.size), np.int64)
        check(lib().vqc_sample(self.h, uu.size, uu.ctypes.data, out.ctypes.data), "vqc_sample")
        return out[: uu.size]

    def numpy(self) -> np.ndarray:
        return self.tensor.cpu().numpy()


class Circuit:
    """QCircuit of ops (workloads.Op tuples) planned into fused passes."""

    def __init__(self, n: int, ops, n_params=None, mixed: bool = False, tune=None):
        self.n = int(n)
        self.mixed = bool(mixed)
        self.ops = flatten_ops(ops)
        self.n_params = ops_params(self.ops) if n_params is None else int(n_params)
        arr = B.OpArray(self.ops)
        t = None
        if tune is not None:
            t = B.vqc_tune(*[int(tune.get(k, 0)) for k in ("tile_bits", "low_bits", "reg_bits", "grid_blocks",
                                                           "remap", "jit")])
        h = ctypes.c_void_p()
        check(lib().vqc_circuit_create(ctypes.byref(h), self.n, B.VQC_MIXED if self.mixed else B.VQC_PURE,
                                       arr.n, arr.ptr(), self.n_params,
                                       ctypes.byref(t) if t is not None else None), "vqc_circuit_create")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and B._lib is not None:
            B._lib.vqc_circuit_destroy(h)
            self.h = None

    def stats(self) -> dict:
        s = B.vqc_circuit_stats()
        check(lib().vqc_circuit_stats_get(self.h, ctypes.byref(s)), "vqc_circuit_stats_get")
        return {"n_ops": s.n_ops, "n_elementary": s.n_elementary, "n_passes": s.n_passes,
                "n_stages": s.n_stages, "n_var": s.n_var, "n_params": s.n_params,
                "tile_bits": s.tune.tile_bits, "low_bits": s.tune.low_bits, "reg_bits": s.tune.reg_bits,
                "grid_blocks": s.tune.grid_blocks, "remap": s.tune.remap, "alg_bytes_per_amp": s.alg_bytes_per_amp,
                "n_adj_passes": s.n_adj_passes, "n_fwd_moves": s.n_fwd_moves, "n_adj_moves": s.n_adj_moves,
                "jit": s.tune.jit, "n_jit_passes": s.n_jit_passes, "jit_cached": bool(s.jit_cached),
                "jit_ms": s.jit_ms, "n_jit_adj_passes": s.n_jit_adj_passes}

    def _theta(self, theta):
        if self.n_params == 0:
            return None
        if not (isinstance(theta, torch.Tensor) and theta.is_cuda and theta.dtype == torch.float64
                and theta.is_contiguous() and theta.numel() >= self.n_params):
            raise ValueError("theta must be a contiguous float64 CUDA tensor with %d entries" % self.n_params)
        return theta

    def apply(self, state: State, theta=None):
        th = self._theta(theta)
        check(lib().vqc_apply_circuit(state.h, self.h, _dptr(th)), "vqc_apply_circuit")

    def apply_out(self, state: State, theta=None) -> State:
        """apply(circ, state): a new state holding the circuit applied to a copy
        of ``state`` (which is left unchanged)."""
        th = self._theta(theta)
        out = State(state.n, mixed=state.mixed, device=state.tensor.device)
        check(lib().vqc_apply_circuit_out(out.h, state.h, self.h, _dptr(th)), "vqc_apply_circuit_out")
        return out

    def __mul__(self, state: State) -> State:
        """circ * state (Sec. 2.4) for circuits without variational parameters."""
        return self.apply_out(state)

    def apply_timed(self, state: State, theta=None) -> np.ndarray:
        """Apply with HIP events between pass launches; returns ms per pass."""
        th = self._theta(theta)
        ms = np.zeros(max(1, self.stats()["n_passes"]), np.float32)
        check(lib().vqc_apply_circuit_timed(state.h, self.h, _dptr(th), ms.ctypes.data),
              "vqc_apply_circuit_timed")
        return ms

    def backward(self, theta, state: State, terms, grad=None, energy=True, init=None, budget=0):
        """Adjoint gradient of Re<psi|H|psi> (pure) or Tr(H rho) (mixed);
        ``state`` must hold the forward result.  Returns (grad, energy)."""
        th = self._theta(theta)
        if grad is None:
            grad = torch.zeros(max(1, self.n_params), dtype=torch.float64, device=state.tensor.device)
        ps = B.PauliSum(terms)
        e = ctypes.c_double()
        check(lib().vqc_backward(self.h, _dptr(th), state.h, ps.ref(), _dptr(grad),
                                 ctypes.byref(e) if energy else None, _dptr(init), int(budget)),
              "vqc_backward")
        return grad[: self.n_params], (e.value if energy else None)

    def backward_inverse(self, theta, state: State, terms, grad=None, energy=True, max_cond=0.0):
        """Adjoint gradient by Alg. 2 with channel inverses for Phi (two states,
        no checkpoints); ``state`` holds the forward result and is uncomputed in
        place.  Raises VQCError(VQC_ERR_ILL_CONDITIONED) when a channel's
        condition number exceeds ``max_cond`` (0: 1e8).  Returns (grad, energy)."""
        th = self._theta(theta)
        if grad is None:
            grad = torch.zeros(max(1, self.n_params), dtype=torch.float64, device=state.tensor.device)
        ps = B.PauliSum(terms)
        e = ctypes.c_double()
        check(lib().vqc_backward_inverse(self.h, _dptr(th), state.h, ps.ref(), _dptr(grad),
                                         ctypes.byref(e) if energy else None, float(max_cond)),
              "vqc_backward_inverse")
        return grad[: self.n_params], (e.value if energy else None)

    def autotune(self, state: State, theta=None, terms=None) -> dict:
        """Time candidate tunes on the scratch ``state`` and re-plan with the
        fastest: the forward pass, or with ``terms`` the forward pass plus the
        gradient of that observable.  Returns the chosen tune."""
        th = self._theta(theta)
        t = B.vqc_tune()
        ps = B.PauliSum(terms) if terms is not None else None
        check(lib().vqc_circuit_autotune_ex(self.h, state.h, _dptr(th), ps.ref() if ps else None,
                                            1 if terms is not None else 0, ctypes.byref(t)),
              "vqc_circuit_autotune_ex")
        return {"tile_bits": t.tile_bits, "low_bits": t.low_bits, "reg_bits": t.reg_bits,
                "grid_blocks": t.grid_blocks, "remap": t.remap, "jit": t.jit}


class Batch:
    """Items b = (circuit, state tensor, theta tensor) run together."""

    def __init__(self, circuits, states, thetas, stream=None):
        self.circuits = list(circuits)
        self.states = list(states)
        self.thetas = list(thetas)
        nB = len(self.circuits)
        ch = (ctypes.c_void_p * nB)(*[c.h.value for c in self.circuits])
        sp = (ctypes.c_void_p * nB)(*[s.data_ptr() for s in self.states])
        tp = (ctypes.c_void_p * nB)(*[(t.data_ptr() if t is not None else 0) for t in self.thetas])
        self._keep = (ch, sp, tp)
        h = ctypes.c_void_p()
        check(lib().vqc_batch_create(ctypes.byref(h), nB, ch, sp, tp, ctypes.c_void_p(stream_ptr(stream))),
              "vqc_batch_create")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and B._lib is not None:
            B._lib.vqc_batch_destroy(h)
            self.h = None

    def forward(self):
        check(lib().vqc_batch_forward(self.h), "vqc_batch_forward")

    def expectation(self, terms, out):
        ps = B.PauliSum(terms)
        check(lib().vqc_batch_expectation(self.h, ps.ref(), _dptr(out)), "vqc_batch_expectation")

    def _gptrs(self, grads):
        return (ctypes.c_void_p * len(grads))(*[g.data_ptr() for g in grads])

    def backward(self, terms, grads, energies=None, budget=0):
        ps = B.PauliSum(terms)
        gp = self._gptrs(grads)
        check(lib().vqc_batch_backward(self.h, ps.ref(), gp, _dptr(energies), int(budget)), "vqc_batch_backward")

    def backward_inverse(self, terms, grads, energies=None, max_cond=0.0):
        """Mixed items: Alg. 2 with channel inverses, all items per launch."""
        ps = B.PauliSum(terms)
        gp = self._gptrs(grads)
        check(lib().vqc_batch_backward_inverse(self.h, ps.ref(), gp, _dptr(energies), float(max_cond)),
              "vqc_batch_backward_inverse")

    def capture(self, terms, grads, energies=None, budget=0):
        ps = B.PauliSum(terms)
        gp = self._gptrs(grads)
        # the graph holds these device pointers: keep the tensors alive with it
        self._cap_keep = (ps, gp, list(grads), energies)
        check(lib().vqc_batch_capture(self.h, ps.ref(), gp, _dptr(energies), int(budget)), "vqc_batch_capture")

    def replay(self):
        check(lib().vqc_batch_replay(self.h), "vqc_batch_replay")
