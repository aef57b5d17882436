"""CPU oracle for the variational-circuit hot path (test infrastructure only).

Plain FP64 definitions from arXiv:2406.19212 (JuliVQC), written in C
(``vqc_oracle.c``) and loaded here through ctypes.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package; the HIP path never does, and the two share no code.

What each function follows:
* ``gate_matrix`` / ``dgate_matrix`` / ``kraus``: the gate and channel
  definitions of Sec. 2.2 (with the readings listed in ``vqc_oracle.c``).
* ``apply_matrix`` / ``run``: Eq. (3), Eq. (twoqubitgate), Alg. 1 and
  Eq. (circuitevolve); on mixed states, Eq. (channel2) on vec(rho) (Sec. 3.4).
* ``expectation``: Sec. 2.5 (Pauli sums), Eq. (loss_pure) / Eq. (loss_mixed).
* ``grad_pure``: Sec. 3.3, Eqs. (diff_pure)-(diff_pure2) and Alg. 2.
* ``grad_mixed``: Sec. 3.5, Eqs. (diff_mixed)-(diff_mixed2), states before
  each op recomputed from stored ones.
* ``grad_mixed_inverse``: the same gradient by Alg. 2 with channel inverses
  for Phi (Sec. 3.3: the inverse form extends Alg. 2 to channels) and the
  adjoint superoperator for Psi; ``invert`` is its Gauss-Jordan step.
* ``measure`` / ``sample``: measure! of Sec. 2.4 (outcome, exact probability,
  collapse in place) and bitstring sampling by the inverse cumulative
  distribution over basis states.
* ``lanczos`` (in ``oracle.lanczos``) and ``mlp`` (in ``oracle.mlp``) cover
  the ground energy and the surrogate network, which the paper does not define.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")

CODES = {
    "x": 1, "y": 2, "z": 3, "h": 4, "s": 5, "t": 6, "sx": 7, "sy": 8, "sw": 9,
    "rx": 10, "ry": 11, "rz": 12, "id": 13,
    "cz": 20, "cnot": 21, "swap": 22, "iswap": 23, "fsim": 24, "crx": 25, "cry": 26,
    "crz": 27, "control": 28, "matrix": 29, "toffoli": 30, "fredkin": 31, "ccontrol": 32,
    "amplitude_damping": 40, "phase_damping": 41, "depolarizing": 42,
    "depolarizing2": 43, "kraus": 44,
}
CHANNELS = {"amplitude_damping", "phase_damping", "depolarizing", "depolarizing2", "kraus"}


class OrOp(ctypes.Structure):
    _fields_ = [
        ("code", ctypes.c_int), ("m", ctypes.c_int), ("q", ctypes.c_int * 4),
        ("prm", ctypes.c_double * 5), ("var", ctypes.c_int * 5),
        ("n_data", ctypes.c_int), ("data", ctypes.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        _lib.or_gate_matrix.argtypes = [P, P, P]
        _lib.or_gate_dmatrix.argtypes = [P, P, ctypes.c_int, P]
        _lib.or_channel_kraus.argtypes = [P, P]
        _lib.or_superop.argtypes = [ctypes.c_int, ctypes.c_int, P, P]
        _lib.or_apply.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P]
        _lib.or_apply_op.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P]
        _lib.or_run.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]
        _lib.or_expect.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, P]
        _lib.or_grad_pure.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int, P, P, P,
                                      ctypes.c_int, P, P, P]
        _lib.or_grad_mixed.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int, P, P,
                                       P, ctypes.c_int, P, P, ctypes.c_int]
        _lib.or_grad_mixed_inverse.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int, P, P,
                                               P, ctypes.c_int, P, P, P]
        _lib.or_invert.argtypes = [ctypes.c_int, P, P]
        _lib.or_measure.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, P, P]
        _lib.or_sample.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]
        _lib.or_set_threads.argtypes = [ctypes.c_int]
        _lib.or_get_threads.restype = ctypes.c_int
    return _lib


def set_threads(t: int) -> None:
    lib().or_set_threads(int(t))


def get_threads() -> int:
    return int(lib().or_get_threads())


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


class _OpTable:
    """ctypes op array; keeps the numpy buffers it points to alive."""

    def __init__(self, ops):
        self.keep = []
        self.arr = (OrOp * max(1, len(ops)))()
        for i, op in enumerate(ops):
            name = op.name if hasattr(op, "name") else op[0]
            qubits = tuple(op.qubits if hasattr(op, "qubits") else op[1])
            params = tuple(getattr(op, "params", ()) or ())
            var = tuple(getattr(op, "var", ()) or ())
            data = getattr(op, "data", None)
            o = self.arr[i]
            o.code = CODES[name]
            o.m = len(qubits)
            for k, q in enumerate(qubits):
                o.q[k] = int(q)
            for k in range(5):
                o.prm[k] = float(params[k]) if k < len(params) else 0.0
                o.var[k] = int(var[k]) if k < len(var) else -1
            if data is not None:
                if isinstance(data, (list, tuple)):
                    buf = np.ascontiguousarray(np.concatenate([np.asarray(d, np.complex128).ravel()
                                                               for d in data]))
                else:
                    buf = np.ascontiguousarray(np.asarray(data, np.complex128).ravel())
                self.keep.append(buf)
                o.n_data = buf.size
                o.data = buf.ctypes.data
            else:
                o.n_data = 0
                o.data = None

    def __len__(self):
        return len(self.arr)


def _one(name, qubits, params=(), var=(), data=None):
    from types import SimpleNamespace
    return SimpleNamespace(name=name, qubits=tuple(qubits), params=tuple(params), var=tuple(var),
                           data=data)


def gate_matrix(name, qubits=None, params=(), data=None, theta=None) -> np.ndarray:
    """Row-major G[out][in] of a gate (Sec. 2.2)."""
    m = len(qubits) if qubits is not None else (1 if name in ("x", "y", "z", "h", "s", "t", "sx",
                                                               "sy", "sw", "rx", "ry", "rz", "id")
                                                else 2)
    tab = _OpTable([_one(name, qubits or tuple(range(m)), params, (), data)])
    G = np.zeros(256, np.complex128)
    d = lib().or_gate_matrix(ctypes.byref(tab.arr[0]), None, _ptr(G))
    if d < 0:
        raise ValueError("not a gate: %s" % name)
    return G[: d * d].reshape(d, d).copy()


def dgate_matrix(name, params, k=0, m=None) -> np.ndarray:
    m = m or (1 if name in ("rx", "ry", "rz") else 2)
    tab = _OpTable([_one(name, tuple(range(m)), params)])
    G = np.zeros(256, np.complex128)
    d = lib().or_gate_dmatrix(ctypes.byref(tab.arr[0]), None, int(k), _ptr(G))
    if d < 0:
        raise ValueError("no derivative for %s param %d" % (name, k))
    return G[: d * d].reshape(d, d).copy()


def kraus(name, params=(), m=None, data=None):
    m = m or (2 if name == "depolarizing2" else 1)
    tab = _OpTable([_one(name, tuple(range(m)), params, (), data)])
    K = np.zeros(16 * 16 * 64, np.complex128)
    nk = lib().or_channel_kraus(ctypes.byref(tab.arr[0]), _ptr(K))
    if nk < 0:
        raise ValueError("not a channel: %s" % name)
    d = 1 << m
    return [K[s * d * d:(s + 1) * d * d].reshape(d, d).copy() for s in range(nk)]


def superop(kraus_list) -> np.ndarray:
    d = kraus_list[0].shape[0]
    m = d.bit_length() - 1
    K = np.ascontiguousarray(np.concatenate([k.ravel() for k in kraus_list]).astype(np.complex128))
    S = np.zeros((d * d) ** 2, np.complex128)
    lib().or_superop(m, len(kraus_list), _ptr(K), _ptr(S))
    return S.reshape(d * d, d * d)


def apply_matrix(v: np.ndarray, nbits: int, qubits, G: np.ndarray) -> None:
    """In place: Eq. (3) / Alg. 1 for an m-qubit matrix G (row-major)."""
    assert v.dtype == np.complex128 and v.flags.c_contiguous and v.size == 1 << nbits
    q = np.asarray(qubits, np.int32)
    Gc = np.ascontiguousarray(G, np.complex128)
    lib().or_apply(_ptr(v), int(nbits), len(q), _ptr(q), _ptr(Gc))


def apply_op_inplace(st: np.ndarray, n: int, op, theta=None, mixed: bool = False) -> None:
    """Apply one op to `st` in place (no copy of the state)."""
    assert st.dtype == np.complex128 and st.flags.c_contiguous
    tab = _OpTable([op])
    th = None if theta is None else np.ascontiguousarray(theta, np.float64)
    rc = lib().or_apply_op(_ptr(st), n, int(mixed), ctypes.byref(tab.arr[0]), None if th is None else _ptr(th))
    if rc:
        raise ValueError("oracle apply failed")


def initial_state(n: int, mixed: bool = False) -> np.ndarray:
    v = np.zeros(1 << (2 * n if mixed else n), np.complex128)
    v[0] = 1.0
    return v


def run(n: int, ops, theta=None, mixed: bool = False, init=None) -> np.ndarray:
    """Run a circuit from |0..0> (or `init`) and return the state (a copy)."""
    st = initial_state(n, mixed) if init is None else np.array(init, np.complex128).ravel().copy()
    tab = _OpTable(ops)
    th = None if theta is None else np.ascontiguousarray(theta, np.float64)
    rc = lib().or_run(_ptr(st), n, int(mixed), len(ops), tab.arr, None if th is None else _ptr(th))
    if rc:
        raise ValueError("oracle run failed at op %d" % (-1 - rc))
    return st


def _terms(terms):
    xm = np.array([t[0] for t in terms], np.uint64)
    zm = np.array([t[1] for t in terms], np.uint64)
    c = np.array([complex(t[2]) for t in terms], np.complex128)
    return xm, zm, c


def expectation(state: np.ndarray, n: int, terms, mixed: bool = False) -> complex:
    xm, zm, c = _terms(terms)
    st = np.ascontiguousarray(state, np.complex128).ravel()
    out = np.zeros(1, np.complex128)
    lib().or_expect(_ptr(st), n, int(mixed), len(terms), _ptr(xm), _ptr(zm), _ptr(c), _ptr(out))
    return complex(out[0])


def grad_pure(n: int, ops, theta, terms, init=None, n_params=None):
    """Alg. 2.  Returns (energy, grad, Phi after the sweep)."""
    xm, zm, c = _terms(terms)
    th = np.ascontiguousarray(theta, np.float64)
    P = int(n_params if n_params is not None else th.size)
    grad = np.zeros(max(P, 1), np.float64)
    e = np.zeros(1, np.float64)
    phi = np.zeros(1 << n, np.complex128)
    ini = None if init is None else np.ascontiguousarray(init, np.complex128)
    tab = _OpTable(ops)
    rc = lib().or_grad_pure(n, len(ops), tab.arr, _ptr(th), None if ini is None else _ptr(ini),
                            len(terms), _ptr(xm), _ptr(zm), _ptr(c), P, _ptr(grad), _ptr(e),
                            _ptr(phi))
    if rc:
        raise ValueError("oracle grad_pure failed (%d)" % rc)
    return float(e[0]), grad[:P], phi


def grad_mixed(n: int, ops, theta, terms, init=None, n_params=None, stride: int = 0):
    """Sec. 3.5 noisy gradient.  Returns (energy, grad)."""
    xm, zm, c = _terms(terms)
    th = np.ascontiguousarray(theta, np.float64)
    P = int(n_params if n_params is not None else th.size)
    grad = np.zeros(max(P, 1), np.float64)
    e = np.zeros(1, np.float64)
    ini = None if init is None else np.ascontiguousarray(init, np.complex128).ravel()
    tab = _OpTable(ops)
    rc = lib().or_grad_mixed(n, len(ops), tab.arr, _ptr(th), None if ini is None else _ptr(ini),
                             len(terms), _ptr(xm), _ptr(zm), _ptr(c), P, _ptr(grad), _ptr(e),
                             int(stride))
    if rc:
        raise ValueError("oracle grad_mixed failed (%d)" % rc)
    return float(e[0]), grad[:P]


def invert(A: np.ndarray) -> np.ndarray:
    """Inverse of a square matrix (D <= 64) by Gauss-Jordan with partial pivoting."""
    A = np.ascontiguousarray(A, np.complex128)
    D = A.shape[0]
    out = np.zeros((D, D), np.complex128)
    if lib().or_invert(D, _ptr(A), _ptr(out)):
        raise ValueError("singular matrix")
    return out


def grad_mixed_inverse(n: int, ops, theta, terms, init=None, n_params=None):
    """Noisy gradient by Alg. 2 with Phi <- M^{-1} Phi and Psi <- M^dagger Psi.
    Returns (energy, grad, Phi after the sweep)."""
    xm, zm, c = _terms(terms)
    th = np.ascontiguousarray(theta, np.float64)
    P = int(n_params if n_params is not None else th.size)
    grad = np.zeros(max(P, 1), np.float64)
    e = np.zeros(1, np.float64)
    phi = np.zeros(1 << (2 * n), np.complex128)
    ini = None if init is None else np.ascontiguousarray(init, np.complex128).ravel()
    tab = _OpTable(ops)
    rc = lib().or_grad_mixed_inverse(n, len(ops), tab.arr, _ptr(th), None if ini is None else _ptr(ini),
                                     len(terms), _ptr(xm), _ptr(zm), _ptr(c), P, _ptr(grad), _ptr(e),
                                     _ptr(phi))
    if rc:
        raise ValueError("oracle grad_mixed_inverse failed (%d)" % rc)
    return float(e[0]), grad[:P], phi


def measure(state: np.ndarray, n: int, q: int, u: float, mixed: bool = False):
    """In place: measure qubit q with the uniform number u; returns (outcome, prob)."""
    assert state.dtype == np.complex128 and state.flags.c_contiguous
    o = ctypes.c_int()
    p = ctypes.c_double()
    if lib().or_measure(_ptr(state), n, int(mixed), int(q), float(u), ctypes.byref(o), ctypes.byref(p)):
        raise ValueError("state of zero norm")
    return o.value, p.value


def sample(state: np.ndarray, n: int, u, mixed: bool = False) -> np.ndarray:
    """Basis-state samples for the uniform numbers u (inverse cumulative distribution)."""
    st = np.ascontiguousarray(state, np.complex128)
    uu = np.ascontiguousarray(u, np.float64)
    out = np.zeros(max(1, uu.size), np.int64)
    if lib().or_sample(_ptr(st), n, int(mixed), int(uu.size), _ptr(uu), _ptr(out)):
        raise ValueError("state of zero norm")
    return out[: uu.size]


def fuse_gates(ops, theta=None):
    """fuse_gates of Sec. 2.3 on an op list (noiseless), applied until no
    one-qubit gate sits next to a two-qubit gate on its qubit: a run of
    one-qubit gates on a qubit is absorbed into the two-qubit gate before it
    (U <- g U, in order), else into the one after it (U <- U g ... g');
    every result is a general matrix evaluated at theta.
    Returns [(qubits, row-major matrix)]."""
    def mat(op):
        params = list(getattr(op, "params", ()) or ())
        var = list(getattr(op, "var", ()) or ())
        params += [0.0] * (5 - len(params))
        for k, v in enumerate(var):
            if v is not None and v >= 0:
                params[k] = float(theta[v])
        return gate_matrix(op.name, tuple(op.qubits), tuple(params), getattr(op, "data", None))

    def on_bit(g, t):  # 4x4 of g on local bit t (local index b0 + 2 b1)
        return np.kron(np.eye(2), g) if t == 0 else np.kron(g, np.eye(2))

    ops = list(ops)
    nxt = [None] * len(ops)
    seen = {}
    for j in range(len(ops) - 1, -1, -1):  # seen[q]: next two-qubit op on q
        qs = tuple(ops[j].qubits)
        if len(qs) == 1:
            nxt[j] = seen.get(qs[0])
        else:
            for q in qs:
                seen[q] = j
    out, last, pending = [], {}, {}
    for j, op in enumerate(ops):
        qs = tuple(op.qubits)
        if op.name in CHANNELS:
            raise ValueError("fuse_gates: noiseless circuits only")
        G = mat(op)
        if len(qs) == 1:
            k = last.get(qs[0])
            if k is not None and len(out[k][0]) == 2:
                out[k][1] = on_bit(G, out[k][0].index(qs[0])) @ out[k][1]
            elif nxt[j] is not None:
                pending.setdefault(nxt[j], []).append(j)
            else:
                out.append([qs, G])
                last[qs[0]] = len(out) - 1
        else:
            U = G
            for pj in reversed(pending.get(j, [])):
                U = U @ on_bit(mat(ops[pj]), qs.index(ops[pj].qubits[0]))
            out.append([qs, U])
            for q in qs:
                last[q] = len(out) - 1
    return [(tuple(q), M) for q, M in out]
