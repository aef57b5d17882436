"""ctypes binding of libvqc.so (the C ABI in include/vqc.h).

Argument marshalling only: Python op lists and Pauli terms become the C
structs, numpy row-major matrices become the ABI's column-major layout, torch
tensors supply device pointers and the current HIP stream.  Every computation
runs in the HIP library; if the library is missing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libvqc.so")

c_double, c_int, c_void_p, c_uint64, c_int64, c_size_t = (
    ctypes.c_double, ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64, ctypes.c_size_t)

VQC_PURE, VQC_MIXED = 0, 1

TYPES = {
    "x": 1, "y": 2, "z": 3, "h": 4, "s": 5, "t": 6, "sx": 7, "sy": 8, "sw": 9,
    "rx": 10, "ry": 11, "rz": 12, "id": 13,
    "cz": 20, "cnot": 21, "swap": 22, "iswap": 23, "fsim": 24, "crx": 25, "cry": 26, "crz": 27,
    "control": 28, "matrix": 29, "toffoli": 30, "fredkin": 31, "ccontrol": 32,
    "amplitude_damping": 40, "phase_damping": 41, "depolarizing": 42, "depolarizing2": 43,
    "kraus": 44,
}
ARITY = {k: 1 for k in ("x", "y", "z", "h", "s", "t", "sx", "sy", "sw", "rx", "ry", "rz", "id",
                        "amplitude_damping", "phase_damping", "depolarizing")}
ARITY.update({k: 2 for k in ("cz", "cnot", "swap", "iswap", "fsim", "crx", "cry", "crz", "control",
                             "depolarizing2")})

STATUS = {0: "ok", -1: "invalid argument", -2: "qubit out of range or repeated",
          -3: "unsupported op or combination", -4: "pure/mixed mismatch",
          -5: "Kraus operators are not trace preserving", -6: "non-finite input",
          -7: "device out of memory", -8: "HIP runtime error",
          -9: "observable must have real coefficients", -10: "gate matrix is not unitary",
          -11: "channel inverse exceeds the condition-number bound",
          -12: "input exceeds the fixed scratch of the allocation-free call",
          -13: "circuit is bound to a live batch"}


class VQCError(RuntimeError):
    def __init__(self, status, where):
        super().__init__("%s: %s (%d)" % (where, STATUS.get(status, "?"), status))
        self.status = status


class vqc_c128(ctypes.Structure):
    _fields_ = [("re", c_double), ("im", c_double)]


class vqc_op(ctypes.Structure):
    _fields_ = [("type", c_int), ("n_qubits", c_int), ("qubits", c_int * 4),
                ("params", c_double * 5), ("param_index", c_int * 5),
                ("n_data", c_int), ("data", c_void_p)]


class vqc_pauli_sum(ctypes.Structure):
    _fields_ = [("n_terms", c_int), ("x_mask", c_void_p), ("z_mask", c_void_p),
                ("coeff_re", c_void_p), ("coeff_im", c_void_p)]


class vqc_tune(ctypes.Structure):
    _fields_ = [("tile_bits", c_int), ("low_bits", c_int), ("reg_bits", c_int), ("grid_blocks", c_int),
                ("remap", c_int), ("jit", c_int)]


class vqc_circuit_stats(ctypes.Structure):
    _fields_ = [("n_ops", c_int), ("n_elementary", c_int), ("n_passes", c_int), ("n_stages", c_int),
                ("n_var", c_int), ("n_params", c_int), ("tune", vqc_tune),
                ("alg_bytes_per_amp", c_double), ("n_adj_passes", c_int), ("n_fwd_moves", c_int),
                ("n_adj_moves", c_int), ("n_jit_passes", c_int), ("jit_cached", c_int), ("jit_ms", c_double),
                ("n_jit_adj_passes", c_int)]


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "vqc_status_string": (ctypes.c_char_p, [c_int]),
    "vqc_version": (c_int, []),
    "vqc_mat_from_external": (c_int, [c_int, c_void_p, c_void_p]),
    "vqc_state_init": (c_int, [ctypes.POINTER(c_void_p), c_int, c_int, c_void_p, c_void_p, c_void_p]),
    "vqc_state_reset": (c_int, [c_void_p]),
    "vqc_state_rebind": (c_int, [c_void_p, c_void_p, c_void_p]),
    "vqc_state_destroy": (c_int, [c_void_p]),
    "vqc_apply_gate": (c_int, [c_void_p, c_int, c_void_p, c_void_p]),
    "vqc_apply_op": (c_int, [c_void_p, ctypes.POINTER(vqc_op)]),
    "vqc_apply_channel": (c_int, [c_void_p, c_int, c_void_p, c_int, c_void_p]),
    "vqc_expectation": (c_int, [c_void_p, ctypes.POINTER(vqc_pauli_sum), ctypes.POINTER(vqc_c128)]),
    "vqc_expectation_noalloc": (c_int, [c_void_p, ctypes.POINTER(vqc_pauli_sum), ctypes.POINTER(vqc_c128)]),
    "vqc_norm": (c_int, [c_void_p, ctypes.POINTER(c_double)]),
    "vqc_gather": (c_int, [c_void_p, c_int, c_void_p, c_void_p]),
    "vqc_circuit_create": (c_int, [ctypes.POINTER(c_void_p), c_int, c_int, c_int, c_void_p, c_int,
                                   ctypes.POINTER(vqc_tune)]),
    "vqc_circuit_destroy": (c_int, [c_void_p]),
    "vqc_fuse_gates": (c_int, [c_int, c_int, c_void_p, c_int, c_void_p, c_void_p, c_void_p,
                               ctypes.POINTER(c_int)]),
    "vqc_measure": (c_int, [c_void_p, c_int, c_double, ctypes.POINTER(c_int), ctypes.POINTER(c_double)]),
    "vqc_sample": (c_int, [c_void_p, c_int, c_void_p, c_void_p]),
    "vqc_circuit_stats_get": (c_int, [c_void_p, ctypes.POINTER(vqc_circuit_stats)]),
    "vqc_apply_circuit": (c_int, [c_void_p, c_void_p, c_void_p]),
    "vqc_apply_circuit_out": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "vqc_apply_circuit_timed": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "vqc_backward": (c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(vqc_pauli_sum), c_void_p,
                             ctypes.POINTER(c_double), c_void_p, c_size_t]),
    "vqc_backward_inverse": (c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(vqc_pauli_sum), c_void_p,
                                     ctypes.POINTER(c_double), c_double]),
    "vqc_circuit_autotune": (c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(vqc_tune)]),
    "vqc_circuit_autotune_ex": (c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(vqc_pauli_sum), c_int,
                                        ctypes.POINTER(vqc_tune)]),
    "vqc_batch_create": (c_int, [ctypes.POINTER(c_void_p), c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "vqc_batch_destroy": (c_int, [c_void_p]),
    "vqc_batch_forward": (c_int, [c_void_p]),
    "vqc_batch_expectation": (c_int, [c_void_p, ctypes.POINTER(vqc_pauli_sum), c_void_p]),
    "vqc_batch_backward": (c_int, [c_void_p, ctypes.POINTER(vqc_pauli_sum), c_void_p, c_void_p, c_size_t]),
    "vqc_batch_backward_inverse": (c_int, [c_void_p, ctypes.POINTER(vqc_pauli_sum), c_void_p, c_void_p, c_double]),
    "vqc_batch_capture": (c_int, [c_void_p, ctypes.POINTER(vqc_pauli_sum), c_void_p, c_void_p, c_size_t]),
    "vqc_batch_replay": (c_int, [c_void_p]),
    "vqc_gemm_bf16": (c_int, [c_int, c_int, c_int, c_void_p, c_int, c_int, c_void_p, c_int, c_int, c_void_p, c_int,
                              ctypes.c_float, ctypes.c_float, c_void_p]),
    "vqc_mlp_create": (c_int, [ctypes.POINTER(c_void_p), c_int, c_int, c_int, c_int, c_void_p]),
    "vqc_mlp_destroy": (c_int, [c_void_p]),
    "vqc_mlp_buffers": (c_int, [c_void_p, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p),
                                ctypes.POINTER(c_size_t)]),
    "vqc_mlp_forward": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    "vqc_mlp_backward": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, ctypes.c_float, c_void_p,
                                 c_void_p]),
    "vqc_mlp_adam": (c_int, [c_void_p, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, c_int]),
    "vqc_mlp_descend_inputs": (c_int, [c_void_p, c_int, c_void_p, ctypes.c_float, c_int]),
}


def lib():
    """Load libvqc.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libvqc.so is not built (%s); run `python -m paper_2406_19212_amd.build`"
                               % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status, where):
    if status != 0:
        raise VQCError(status, where)


# ------------------------------------------------------------- marshalling

def colmajor(G) -> np.ndarray:
    """Row-major numpy matrix -> ABI column-major complex128 buffer."""
    G = np.asarray(G, np.complex128)
    return np.ascontiguousarray(G.T).ravel()


class OpArray:
    """vqc_op[] for a list of ops (workloads.Op or compatible); keeps the
    matrix buffers alive."""

    def __init__(self, ops):
        self.keep = []
        self.n = len(ops)
        self.arr = (vqc_op * max(1, self.n))()
        for i, op in enumerate(ops):
            name, qubits = op.name, tuple(op.qubits)
            params = tuple(getattr(op, "params", ()) or ())
            var = tuple(getattr(op, "var", ()) or ())
            data = getattr(op, "data", None)
            o = self.arr[i]
            o.type = TYPES[name]
            o.n_qubits = len(qubits)
            for k, q in enumerate(qubits):
                o.qubits[k] = int(q)
            for k in range(5):
                o.params[k] = float(params[k]) if k < len(params) else 0.0
                o.param_index[k] = int(var[k]) if k < len(var) else -1
            if data is not None:
                mats = data if isinstance(data, (list, tuple)) else [data]
                buf = np.ascontiguousarray(np.concatenate([colmajor(m) for m in mats]))
                self.keep.append(buf)
                o.n_data = buf.size
                o.data = buf.ctypes.data
            else:
                o.n_data = 0
                o.data = None

    def ptr(self):
        return ctypes.cast(self.arr, c_void_p)


class PauliSum:
    """vqc_pauli_sum for [(x_mask, z_mask, coeff), ...]."""

    def __init__(self, terms):
        self.xm = np.array([t[0] for t in terms], np.uint64)
        self.zm = np.array([t[1] for t in terms], np.uint64)
        c = np.array([complex(t[2]) for t in terms], np.complex128)
        self.cre = np.ascontiguousarray(c.real)
        self.cim = np.ascontiguousarray(c.imag)
        self.s = vqc_pauli_sum(len(terms), self.xm.ctypes.data if len(terms) else None,
                               self.zm.ctypes.data if len(terms) else None,
                               self.cre.ctypes.data if len(terms) else None,
                               self.cim.ctypes.data if len(terms) else None)

    def ref(self):
        return ctypes.byref(self.s)
