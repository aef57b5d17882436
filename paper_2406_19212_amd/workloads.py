"""Seeded synthetic inputs shared by the HIP path, its tests and the CPU oracle.

This module describes circuits, parameters and observables as plain data: gate
*names*, qubit indices, angles, Pauli masks and coefficients, bitstrings.  It
holds none of the method's arithmetic (no gate matrix, no state update, no
expectation value); each consumer turns the names into numbers on its own.

Conventions
-----------
* qubits are 0-based; qubit k is bit k of the amplitude index (the paper's
  column-major storage with the first qubit fastest, Sec. 2.1).
* an op is ``Op(name, qubits, params, var, data)``: ``params`` are the
  parameter values, ``var[k]`` is the index of parameter ``k`` in the flat
  variational vector theta (or -1 when the parameter is fixed, the paper's
  ``isparas=false``, Sec. 2.2), ``data`` is a complex matrix or Kraus list for
  ``matrix``/``control``/``kraus`` ops (row-major ``G[out][in]``, local index
  ``sum_t b_{q_t} 2^t``, first listed qubit = least significant bit).
* a Pauli term is ``(x_mask, z_mask, coeff)``; a Y on qubit k sets bit k in
  both masks.

Random numbers come from one counter-based generator, SplitMix64 (Steele,
Lea, Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
value i of stream ``seed`` is ``mix64(seed + (i + 1) * 0x9E3779B97F4A7C15)``.
Uniform doubles take the top 53 bits; normals use Box-Muller.
"""
from __future__ import annotations

import math
from typing import NamedTuple, Sequence

import numpy as np

__all__ = [
    "Op", "SplitMix64", "uniform", "normal", "brickwall", "noisy_brickwall",
    "rqc_grid", "rqc_bitstrings", "hea", "theta_uniform", "tfim", "zz",
    "pauli_string", "heisenberg_1d", "random_state", "random_density",
    "random_unitary", "random_kraus", "count_params", "CONFIG_SEED",
]

# default seed per workload: 2406_19212 + config index
CONFIG_SEED = [240619212 + i for i in range(5)]

_GOLD = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
TWO_PI = 2.0 * math.pi


class Op(NamedTuple):
    name: str
    qubits: tuple
    params: tuple = ()
    var: tuple = ()
    data: object = None


def _mix64(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


class SplitMix64:
    """Counter-based SplitMix64 stream: draw i is mix64(seed + (i+1)*golden)."""

    def __init__(self, seed: int):
        self.seed = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
        self.counter = 0

    def u64(self, count: int) -> np.ndarray:
        i = np.arange(self.counter + 1, self.counter + 1 + count, dtype=np.uint64)
        self.counter += count
        with np.errstate(over="ignore"):
            return _mix64(self.seed + i * _GOLD)

    def uniform(self, count: int) -> np.ndarray:
        """Doubles in [0, 1) from the top 53 bits."""
        return (self.u64(count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)

    def normal(self, count: int) -> np.ndarray:
        """Standard normals by Box-Muller (one normal per pair of uniforms)."""
        u = self.uniform(2 * count).reshape(count, 2)
        r = np.sqrt(-2.0 * np.log1p(-u[:, 0]))
        return r * np.cos(TWO_PI * u[:, 1])

    def integers(self, count: int, high: int) -> np.ndarray:
        return (self.uniform(count) * high).astype(np.int64)


def uniform(seed: int, count: int, lo: float = 0.0, hi: float = TWO_PI) -> np.ndarray:
    return lo + (hi - lo) * SplitMix64(seed).uniform(count)


def normal(seed: int, count: int) -> np.ndarray:
    return SplitMix64(seed).normal(count)


def count_params(ops: Sequence[Op]) -> int:
    m = -1
    for op in ops:
        for v in op.var:
            m = max(m, v)
    return m + 1


# ---------------------------------------------------------------- circuits

def brickwall(n: int, layers: int, seed: int):
    """Layered rotations + brick-wall CZ (n=12, 20 layers is the noiseless
    benchmark circuit).  Layer l: for each qubit q, Rx, Ry, Rz (in that order)
    with theta index (l*n + q)*3 + g; then CZ(2k, 2k+1) for even l and
    CZ(2k+1, 2k+2) for odd l.  Returns (ops, theta)."""
    theta = uniform(seed, layers * n * 3)
    ops = []
    for l in range(layers):
        for q in range(n):
            for g, name in enumerate(("rx", "ry", "rz")):
                k = (l * n + q) * 3 + g
                ops.append(Op(name, (q,), (float(theta[k]),), (k,)))
        start = 0 if l % 2 == 0 else 1
        for a in range(start, n - 1, 2):
            ops.append(Op("cz", (a, a + 1)))
    return ops, theta


def noisy_brickwall(n: int, layers: int, seed: int, p1: float = 1e-3,
                    gamma: float = 1e-3, p2: float = 1e-2):
    """The brick-wall circuit with noise: after each Rx, Ry, Rz a single-qubit
    depolarizing channel (p1) then amplitude damping (gamma) on that qubit;
    after each CZ a two-qubit depolarizing channel (p2) on the same pair."""
    base, theta = brickwall(n, layers, seed)
    ops = []
    for op in base:
        ops.append(op)
        if op.name in ("rx", "ry", "rz"):
            ops.append(Op("depolarizing", op.qubits, (p1,)))
            ops.append(Op("amplitude_damping", op.qubits, (gamma,)))
        elif op.name == "cz":
            ops.append(Op("depolarizing2", op.qubits, (p2,)))
    return ops, theta


def noisy_batch(seed: int, count: int = 32, widths=(8, 10, 12), layers: int = 20):
    """Batch of noisy brick-wall circuits of uneven width: circuit i has
    n = widths[i % len(widths)] and its own angle seed."""
    out = []
    for i in range(count):
        n = widths[i % len(widths)]
        ops, theta = noisy_brickwall(n, layers, seed * 1000 + i)
        out.append((n, ops, theta))
    return out


_RQC_SEQ = "ABCDCDAB"


def rqc_couplers(rows: int, cols: int, pattern: str):
    """Grid couplers for one of the four patterns.  Qubit (r, c) = cols*r + c.
    A/B: horizontal pairs with c even / odd; C/D: vertical pairs with r even / odd."""
    out = []
    if pattern in "AB":
        par = 0 if pattern == "A" else 1
        for r in range(rows):
            for c in range(par, cols - 1, 2):
                out.append((cols * r + c, cols * r + c + 1))
    else:
        par = 0 if pattern == "C" else 1
        for r in range(par, rows - 1, 2):
            for c in range(cols):
                out.append((cols * r + c, cols * (r + 1) + c))
    return out


def rqc_grid(rows: int, cols: int, cycles: int, seed: int, cut_row: int | None = None):
    """Random circuit on a rows x cols grid (4x7 = 28 qubits, 20 cycles is the
    large-state benchmark).  Each cycle: one of sqrt(X), sqrt(Y), sqrt(W) on
    every qubit (uniform in cycle 0, afterwards uniform over the two gates that
    differ from the previous one on that qubit), then fSim(theta, phi) on the
    couplers of pattern ABCDCDAB[cycle % 8]; theta = pi/2 + N(0, 0.01) and
    phi = pi/6 + N(0, 0.01) drawn once per coupler.

    ``cut_row``: if given, couplers that join row cut_row-1 to row cut_row are
    dropped, which splits the circuit into two independent halves (qubits
    below cols*cut_row and the rest); used for sampled checks at full size."""
    rng = SplitMix64(seed)
    n = rows * cols
    all_couplers = sorted(set(sum((rqc_couplers(rows, cols, p) for p in "ABCD"), [])))
    z = rng.normal(2 * len(all_couplers)).reshape(-1, 2)
    ang = {cp: (math.pi / 2 + 0.01 * z[i, 0], math.pi / 6 + 0.01 * z[i, 1])
           for i, cp in enumerate(all_couplers)}
    names = ("sx", "sy", "sw")
    prev = [-1] * n
    ops = []
    for cyc in range(cycles):
        u = rng.uniform(n)
        for q in range(n):
            if prev[q] < 0:
                g = int(u[q] * 3)
            else:
                choices = [k for k in range(3) if k != prev[q]]
                g = choices[int(u[q] * 2)]
            prev[q] = g
            ops.append(Op(names[g], (q,)))
        for (a, b) in rqc_couplers(rows, cols, _RQC_SEQ[cyc % len(_RQC_SEQ)]):
            if cut_row is not None and a < cols * cut_row <= b:
                continue
            th, ph = ang[(a, b)]
            ops.append(Op("fsim", (a, b), (float(th), float(ph), 0.0, 0.0, 0.0), (-1,) * 5))
    return ops


def rqc_bitstrings(n: int, count: int, seed: int) -> np.ndarray:
    """``count`` distinct uniformly drawn n-bit output indices (int64)."""
    rng = SplitMix64(seed)
    seen, out = set(), []
    while len(out) < count:
        for v in (rng.u64(count) >> np.uint64(64 - n)).astype(np.int64):
            if int(v) not in seen:
                seen.add(int(v))
                out.append(int(v))
                if len(out) == count:
                    break
    return np.array(out, dtype=np.int64)


def hea(n: int, layers: int):
    """Hardware-efficient ansatz: per layer Ry on every qubit, Rz on every
    qubit, then CNOT(i, i+1) for i = 0..n-2.  theta index (2l + g)*n + q with
    g = 0 for Ry and 1 for Rz.  Parameter values in the ops are placeholders;
    the flat theta vector supplies them."""
    ops = []
    for l in range(layers):
        for g, name in enumerate(("ry", "rz")):
            for q in range(n):
                ops.append(Op(name, (q,), (0.0,), ((2 * l + g) * n + q,)))
        for i in range(n - 1):
            ops.append(Op("cnot", (i, i + 1)))
    return ops


def theta_uniform(seed: int, batch: int, count: int) -> np.ndarray:
    """[batch, count] angles uniform in [0, 2 pi)."""
    return uniform(seed, batch * count).reshape(batch, count)


# -------------------------------------------------------------- observables

_PAULI_BITS = {"x": (1, 0), "y": (1, 1), "z": (0, 1)}


def pauli_string(spec: dict, coeff: complex = 1.0):
    """{qubit: 'x'|'y'|'z'} -> (x_mask, z_mask, coeff)."""
    xm = zm = 0
    for q, p in spec.items():
        bx, bz = _PAULI_BITS[p.lower()]
        xm |= bx << q
        zm |= bz << q
    return (xm, zm, complex(coeff))


def tfim(n: int, h: float = 1.0):
    """Open transverse-field Ising chain: sum_i Z_i Z_{i+1} + h sum_i X_i."""
    terms = [pauli_string({i: "z", i + 1: "z"}, 1.0) for i in range(n - 1)]
    terms += [pauli_string({i: "x"}, h) for i in range(n)]
    return terms


def zz(i: int, j: int, coeff: float = 1.0):
    return [pauli_string({i: "z", j: "z"}, coeff)]


def heisenberg_1d(L: int, hz: float = 1.0, J: float = 1.0):
    """The Hamiltonian of the paper's Listing 5 (0-based sites): hz Z_i on
    every site, J (XX + YY + ZZ) on nearest neighbours."""
    terms = [pauli_string({i: "z"}, hz) for i in range(L)]
    for i in range(L - 1):
        for p in "xyz":
            terms.append(pauli_string({i: p, i + 1: p}, J))
    return terms


# ------------------------------------------------------ random test inputs

def _cgauss(rng: SplitMix64, shape) -> np.ndarray:
    cnt = int(np.prod(shape))
    z = rng.normal(2 * cnt)
    return (z[:cnt] + 1j * z[cnt:]).reshape(shape)


def random_state(n: int, seed: int) -> np.ndarray:
    v = _cgauss(SplitMix64(seed), (1 << n,))
    return v / np.linalg.norm(v)


def random_density(n: int, seed: int, rank: int | None = None) -> np.ndarray:
    """Random density matrix rho[x][y] (PSD, trace 1)."""
    d = 1 << n
    a = _cgauss(SplitMix64(seed), (d, rank or d))
    rho = a @ a.conj().T
    return rho / np.trace(rho).real


def random_unitary(d: int, seed: int) -> np.ndarray:
    """Haar-random d x d unitary (QR of a complex Gaussian with phase fix)."""
    z = _cgauss(SplitMix64(seed), (d, d))
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[None, :]


def random_kraus(d: int, count: int, seed: int):
    """``count`` Kraus operators of a random channel on a d-dim space: the
    blocks of a random (count*d) x d isometry."""
    z = _cgauss(SplitMix64(seed), (count * d, d))
    q, _ = np.linalg.qr(z)
    return [q[s * d:(s + 1) * d, :].copy() for s in range(count)]
