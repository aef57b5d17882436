"""Three-qubit gates (Toffoli, Fredkin, doubly controlled U, general 8x8
matrices): single ops on pure and mixed states, and circuits forward and
backward (the named gates run as exact one- and two-qubit sequences, a
general 8x8 matrix as one register op on three register bits in any order,
also in the circuit-specialised kernels), against the oracle's dense
definitions."""
import itertools

import numpy as np
import pytest
import torch

import oracle
from paper_2406_19212_amd import Circuit, State
from paper_2406_19212_amd import workloads as W
from paper_2406_19212_amd.workloads import Op

pytestmark = pytest.mark.gpu
AMP_TOL, GRAD_TOL = 1e-12, 1e-10


def maxdiff(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


def gate3_cases(n, seed):
    out = []
    for k, qs in enumerate(itertools.permutations(range(n), 3)):
        if k % 3:
            continue
        out.append(Op("toffoli", qs))
        out.append(Op("fredkin", qs))
        out.append(Op("ccontrol", qs, (), (), W.random_unitary(2, seed + k)))
        out.append(Op("matrix", qs, (), (), W.random_unitary(8, seed + 100 + k)))
    return out


@pytest.mark.parametrize("n,mixed", [(3, False), (6, False), (3, True), (4, True)])
def test_single_three_qubit_ops(n, mixed):
    if mixed:
        v = W.random_density(n, 70 + n).reshape(-1, order="F").copy()
    else:
        v = W.random_state(n, 70 + n)
    worst = 0.0
    for op in gate3_cases(n, 10 * n):
        st = State(n, mixed=mixed, init=v)
        st.apply_op(op)
        worst = max(worst, maxdiff(st.numpy(), oracle.run(n, [op], mixed=mixed, init=v)))
    print("n=%d mixed=%d: worst %.2e" % (n, mixed, worst))
    assert worst < AMP_TOL


def circuit_with_gate3(n, layers, seed, noisy=False):
    rng = np.random.default_rng(seed)
    ops, P = [], 0
    for layer in range(layers):
        for q in range(n):
            ops.append(Op("ry", (q,), (0.0,), (P,)))
            P += 1
            if noisy:
                ops.append(Op("depolarizing", (q,), (0.02,)))
        a, b, c = (int(v) for v in rng.choice(n, 3, replace=False))
        kind = ["toffoli", "fredkin", "ccontrol", "matrix"][layer % 4]
        data = {"ccontrol": W.random_unitary(2, seed + layer), "matrix": W.random_unitary(8, seed + 50 + layer)}
        ops.append(Op(kind, (a, b, c), (), (), data.get(kind)))
        if layer % 2:  # a second general matrix, qubits in another order
            ops.append(Op("matrix", (c, a, b), (), (), W.random_unitary(8, seed + 70 + layer)))
        for q in range(layer % 2, n - 1, 2):
            ops.append(Op("cz", (q, q + 1)))
            if noisy:
                ops.append(Op("amplitude_damping", (q + 1,), (0.03,)))
        ops.append(Op("rz", (int(rng.integers(n)),), (0.0,), (P,)))
        P += 1
    return ops, rng.uniform(-3, 3, P)


@pytest.mark.parametrize("n,tune", [(7, None), (9, {"tile_bits": 6, "low_bits": 2}),
                                    (13, {"tile_bits": 8, "low_bits": 3, "remap": 1}),
                                    (13, {"tile_bits": 9, "low_bits": 3, "reg_bits": 4, "jit": 1}),
                                    (14, {"tile_bits": 10, "low_bits": 4, "reg_bits": 3, "remap": 1, "jit": 1}),
                                    (3, None)])
def test_pure_circuit_with_three_qubit_gates(n, tune):
    ops, th = circuit_with_gate3(n, 8, 80 + n)
    c = Circuit(n, ops, tune=tune)
    if tune and tune.get("jit") == 1:
        assert c.stats()["n_jit_passes"] == c.stats()["n_passes"]
    st = State(n)
    tht = torch.tensor(th, device="cuda")
    c.apply(st, tht)
    assert maxdiff(st.numpy(), oracle.run(n, ops, th)) < AMP_TOL
    terms = W.tfim(n, 0.8)
    g, e = c.backward(tht, st, terms)
    e_ref, g_ref, _ = oracle.grad_pure(n, ops, th, terms)
    assert abs(e - e_ref) < AMP_TOL
    assert maxdiff(g.cpu().numpy(), g_ref) < GRAD_TOL


@pytest.mark.parametrize("n", [3, 5, 6])
def test_noisy_circuit_with_three_qubit_gates(n):
    ops, th = circuit_with_gate3(n, 8, 90 + n, noisy=True)
    c = Circuit(n, ops, mixed=True, n_params=len(th))
    tht = torch.tensor(th, device="cuda")
    st = State(n, mixed=True)
    c.apply(st, tht)
    assert maxdiff(st.numpy(), oracle.run(n, ops, th, mixed=True)) < AMP_TOL
    terms = W.zz(0, 1)
    g, e = c.backward(tht, st, terms)
    e_ref, g_ref = oracle.grad_mixed(n, ops, th, terms)
    assert abs(e - e_ref) < AMP_TOL and maxdiff(g.cpu().numpy(), g_ref) < GRAD_TOL
    g2, _ = c.backward_inverse(tht, st, terms)
    _, g2_ref, _ = oracle.grad_mixed_inverse(n, ops, th, terms)
    assert maxdiff(g2.cpu().numpy(), g2_ref) < GRAD_TOL
