"""Parity of the HIP path (through the C ABI) with the CPU oracle, element by
element on the same seeded inputs.  Bar: max-abs 1e-12 on amplitudes and
expectations, 1e-10 on gradients (FP64 throughout)."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2406_19212_amd import Circuit, State
from paper_2406_19212_amd import workloads as W

pytestmark = pytest.mark.gpu

AMP_TOL = 1e-12
GRAD_TOL = 1e-10
Op = W.Op

ONE_Q = ["x", "y", "z", "h", "s", "t", "sx", "sy", "sw"]
ONE_Q_P = ["rx", "ry", "rz"]
TWO_Q = ["cz", "cnot", "swap", "iswap"]
TWO_Q_P = ["crx", "cry", "crz"]


def gpu_state(n, psi, mixed=False):
    return State(n, mixed=mixed, init=psi)


def oracle_apply(n, psi, op, mixed=False):
    return oracle.run(n, [op], mixed=mixed, init=psi)


def maxdiff(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


@pytest.mark.parametrize("n", [1, 2, 5, 13])
def test_single_ops_every_position(n):
    psi = W.random_state(n, 1000 + n)
    rng = np.random.default_rng(n)
    cases = []
    for q in range(n):
        for g in ONE_Q:
            cases.append(Op(g, (q,)))
        for g in ONE_Q_P:
            cases.append(Op(g, (q,), (float(rng.uniform(-4, 4)),)))
        cases.append(Op("matrix", (q,), (), (), W.random_unitary(2, 7 * q + n)))
    for a in range(n):
        for b in range(n):
            if a == b or (n > 5 and (a + 2 * b) % 3):
                continue
            for g in TWO_Q:
                cases.append(Op(g, (a, b)))
            for g in TWO_Q_P:
                cases.append(Op(g, (a, b), (float(rng.uniform(-4, 4)),)))
            cases.append(Op("fsim", (a, b), tuple(float(v) for v in rng.uniform(-3, 3, 5))))
            cases.append(Op("control", (a, b), (), (), W.random_unitary(2, a * 31 + b)))
            cases.append(Op("matrix", (a, b), (), (), W.random_unitary(4, a * 37 + b)))
    worst = 0.0
    for op in cases:
        st = gpu_state(n, psi)
        st.apply_op(op)
        d = maxdiff(st.numpy(), oracle_apply(n, psi, op))
        worst = max(worst, d)
        assert d < AMP_TOL, (op.name, op.qubits, d)
    print("single ops n=%d cases=%d worst=%.2e" % (n, len(cases), worst))


def test_apply_gate_matrix_structures():
    n = 9
    psi = W.random_state(n, 77)
    mats = {
        "diag1": np.diag([np.exp(0.3j), np.exp(-1.1j)]),
        "phase1": np.diag([1, np.exp(0.7j)]),
        "dense1": W.random_unitary(2, 5),
        "diag2": np.diag(np.exp(1j * np.array([0.1, 0.2, 0.3, 0.4]))),
        "phase11": np.diag([1, 1, 1, -1]),
        "cx": oracle.gate_matrix("cnot", (0, 1)),
        "ctrl": oracle.gate_matrix("control", (0, 1), data=W.random_unitary(2, 9)),
        "fsim": oracle.gate_matrix("fsim", (0, 1), params=(0.4, 0.9, 0.1, 0.2, 0.3)),
        "dense2": W.random_unitary(4, 11),
    }
    for name, G in mats.items():
        m = 1 if G.shape[0] == 2 else 2
        for qs in ([0], [8], [4]) if m == 1 else ([0, 1], [8, 0], [3, 7], [6, 2]):
            st = gpu_state(n, psi)
            st.apply_gate(qs, G)
            ref = psi.copy()
            oracle.apply_matrix(ref, n, qs, G)
            assert maxdiff(st.numpy(), ref) < AMP_TOL, (name, qs)


@pytest.mark.parametrize("n,layers", [(6, 3), (12, 20), (15, 4)])
def test_brickwall_circuit(n, layers):
    ops, th = W.brickwall(n, layers, 5 + n)
    c = Circuit(n, ops)
    st = State(n)
    c.apply(st, torch.tensor(th, device="cuda"))
    ref = oracle.run(n, ops, th)
    d = maxdiff(st.numpy(), ref)
    print("brickwall n=%d layers=%d passes=%d maxdiff=%.2e" % (n, layers, c.stats()["n_passes"], d))
    assert d < AMP_TOL
    z0 = [W.pauli_string({0: "z"})]
    assert abs(st.expectation(z0) - oracle.expectation(ref, n, z0)) < AMP_TOL


@pytest.mark.parametrize("rows,cols,cycles", [(3, 3, 8), (3, 4, 20), (4, 5, 12)])
def test_random_grid_circuit(rows, cols, cycles):
    n = rows * cols
    ops = W.rqc_grid(rows, cols, cycles, 17 + n)
    c = Circuit(n, ops)
    st = State(n)
    c.apply(st)
    ref = oracle.run(n, ops)
    d = maxdiff(st.numpy(), ref)
    print("rqc %dx%d cycles=%d passes=%d maxdiff=%.2e" % (rows, cols, cycles, c.stats()["n_passes"], d))
    assert d < AMP_TOL
    assert abs(st.norm() - 1) < 1e-12


@pytest.mark.parametrize("tile,low,reg", [(5, 2, 4), (8, 3, 4), (10, 4, 4), (11, 5, 4), (13, 4, 4),
                                          (8, 3, 3), (11, 4, 3), (13, 5, 3)])
def test_tile_shapes_agree(tile, low, reg):
    n = 14
    ops = W.rqc_grid(2, 7, 10, 99)
    ref = oracle.run(n, ops)
    c = Circuit(n, ops, tune={"tile_bits": tile, "low_bits": low, "reg_bits": reg})
    st = State(n)
    c.apply(st)
    assert maxdiff(st.numpy(), ref) < AMP_TOL
    # the adjoint kernels of the same register width
    ops2 = W.hea(n, 2)
    th = W.theta_uniform(3, 1, W.count_params(ops2))[0]
    c2 = Circuit(n, ops2, tune={"tile_bits": tile, "low_bits": low, "reg_bits": reg})
    st2 = State(n)
    tht = torch.tensor(th, device="cuda")
    c2.apply(st2, tht)
    g, e = c2.backward(tht, st2, W.tfim(n))
    e_ref, g_ref, _ = oracle.grad_pure(n, ops2, th, W.tfim(n))
    assert maxdiff(g.cpu().numpy(), g_ref) < GRAD_TOL


def test_expectation_pure_and_mixed():
    n = 11
    psi = W.random_state(n, 3)
    terms = W.heisenberg_1d(n, 0.7, 1.3) + W.tfim(n, 0.4) + [
        W.pauli_string({0: "y", 5: "x", 10: "z"}, 0.3 - 0.2j), W.pauli_string({2: "y", 9: "y"}, -0.5)]
    st = gpu_state(n, psi)
    e = st.expectation(terms)
    assert abs(e - oracle.expectation(psi, n, terms)) < AMP_TOL
    assert abs(st.norm() - np.sum(np.abs(psi) ** 2)) < AMP_TOL
    m = 5
    rho = W.random_density(m, 4)
    v = rho.reshape(-1, order="F")
    sm = gpu_state(m, v, mixed=True)
    terms = W.heisenberg_1d(m) + [W.pauli_string({1: "y", 3: "x"}, 0.25j)]
    assert abs(sm.expectation(terms) - oracle.expectation(v, m, terms, mixed=True)) < AMP_TOL
    assert abs(sm.norm() - 1) < AMP_TOL


def test_channels_single_op():
    n = 4
    rho = W.random_density(n, 8)
    v = rho.reshape(-1, order="F").copy()
    cases = [Op("amplitude_damping", (2,), (0.3,)), Op("phase_damping", (0,), (0.2,)),
             Op("depolarizing", (3,), (0.15,)), Op("depolarizing2", (1, 3), (0.1,)),
             Op("depolarizing2", (2, 0), (0.05,)),
             Op("kraus", (1,), (), (), W.random_kraus(2, 3, 5)),
             Op("kraus", (3, 0), (), (), W.random_kraus(4, 2, 6)),
             Op("ry", (1,), (0.7,)), Op("cz", (0, 2)), Op("fsim", (3, 1), (0.4, 0.2, 0, 0, 0))]
    for op in cases:
        st = gpu_state(n, v, mixed=True)
        st.apply_op(op)
        ref = oracle_apply(n, v, op, mixed=True)
        assert maxdiff(st.numpy(), ref) < AMP_TOL, op.name
    st = gpu_state(n, v, mixed=True)
    K = W.random_kraus(4, 3, 9)
    st.apply_channel([2, 1], K)
    assert maxdiff(st.numpy(), oracle_apply(n, v, Op("kraus", (2, 1), (), (), K), mixed=True)) < AMP_TOL


@pytest.mark.parametrize("n,layers", [(4, 3), (6, 2)])
def test_noisy_circuit_forward(n, layers):
    ops, th = W.noisy_brickwall(n, layers, 31 + n, p1=0.02, gamma=0.03, p2=0.05)
    c = Circuit(n, ops, mixed=True)
    st = State(n, mixed=True)
    c.apply(st, torch.tensor(th, device="cuda"))
    ref = oracle.run(n, ops, th, mixed=True)
    assert maxdiff(st.numpy(), ref) < AMP_TOL
    assert abs(st.norm() - 1) < 1e-12


@pytest.mark.parametrize("kind,n,layers", [("hea", 10, 4), ("brick", 12, 3), ("hea", 5, 2)])
def test_pure_gradient(kind, n, layers):
    if kind == "hea":
        ops = W.hea(n, layers)
        th = W.theta_uniform(5, 1, W.count_params(ops))[0]
        terms = W.tfim(n, 1.0)
    else:
        ops, th = W.brickwall(n, layers, 8)
        terms = W.heisenberg_1d(n)
    c = Circuit(n, ops)
    st = State(n)
    tht = torch.tensor(th, device="cuda")
    c.apply(st, tht)
    g, e = c.backward(tht, st, terms)
    e_ref, g_ref, _ = oracle.grad_pure(n, ops, th, terms)
    gd = maxdiff(g.cpu().numpy(), g_ref)
    print("grad %s n=%d: |dE|=%.2e |dg|=%.2e" % (kind, n, abs(e - e_ref), gd))
    assert abs(e - e_ref) < AMP_TOL
    assert gd < GRAD_TOL
    # Alg. 2 leaves Phi at the initial state
    phi = st.numpy()
    assert abs(phi[0] - 1) < 1e-11 and np.max(np.abs(phi[1:])) < 1e-11


def test_pure_gradient_fsim_shared_and_controlled():
    n = 6
    ops = [Op("h", (q,)) for q in range(n)]
    ops += [Op("fsim", (0, 4), (0, 0, 0, 0, 0), (0, 1, 2, 3, 4)), Op("crx", (5, 1), (0,), (5,)),
            Op("cry", (1, 2), (0,), (6,)), Op("crz", (2, 0), (0,), (7,)), Op("ry", (3,), (0,), (0,)),
            Op("rz", (5,), (0,), (7,))]
    th = np.array([0.4, 0.9, -0.3, 0.2, 0.6, 1.3, -0.8, 2.1])
    terms = W.heisenberg_1d(n)
    c = Circuit(n, ops)
    st = State(n)
    tht = torch.tensor(th, device="cuda")
    c.apply(st, tht)
    g, e = c.backward(tht, st, terms)
    e_ref, g_ref, _ = oracle.grad_pure(n, ops, th, terms)
    assert maxdiff(g.cpu().numpy(), g_ref) < GRAD_TOL


@pytest.mark.parametrize("n,layers", [(3, 2), (4, 3)])
def test_noisy_gradient(n, layers):
    ops, th = W.noisy_brickwall(n, layers, 50 + n, p1=0.02, gamma=0.03, p2=0.05)
    terms = W.zz(0, 1)
    c = Circuit(n, ops, mixed=True)
    st = State(n, mixed=True)
    tht = torch.tensor(th, device="cuda")
    c.apply(st, tht)
    g, e = c.backward(tht, st, terms)
    e_ref, g_ref = oracle.grad_mixed(n, ops, th, terms)
    gd = maxdiff(g.cpu().numpy(), g_ref)
    print("noisy grad n=%d: |dE|=%.2e |dg|=%.2e" % (n, abs(e - e_ref), gd))
    assert abs(e - e_ref) < AMP_TOL
    assert gd < GRAD_TOL
    # a small checkpoint budget (more recomputation) gives the same gradient
    g2, _ = c.backward(tht, st, terms, budget=12 * 16 * (4 ** n))
    assert maxdiff(g2.cpu().numpy(), g_ref) < GRAD_TOL


def _mixed_gate_circuit(n, seed, n_sqrt):
    """Every gate type at seeded positions; `n_sqrt` phase-factored sqrt gates
    (a count that is not a multiple of 8 exercises the global-phase op)."""
    rng = np.random.default_rng(seed)
    ops, k = [], 0
    names1 = ["x", "y", "z", "h", "s", "t"]
    for i in range(6 * n):
        q = int(rng.integers(n))
        r = i % 9
        if r < 3:
            ops.append(Op(["rx", "ry", "rz"][r], (q,), (0.0,), (k,)))
            k += 1
        elif r < 5:
            ops.append(Op(names1[int(rng.integers(6))], (q,)))
        else:
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            two = ["cz", "cnot", "swap", "iswap", "crx", "fsim", "fsimd", "control"][int(rng.integers(8))]
            if two == "crx":
                ops.append(Op("crx", (a, b), (0.0,), (k,)))
                k += 1
            elif two == "fsim":
                ops.append(Op("fsim", (a, b), (0.0, 0.3, 0, 0, 0), (k, -1, -1, -1, -1)))
                k += 1
            elif two == "fsimd":
                ops.append(Op("fsim", (a, b), (0.7, 0.3, 0.1, -0.2, 0.05)))
            elif two == "control":
                ops.append(Op("control", (a, b), (), (), W.random_unitary(2, i)))
            else:
                ops.append(Op(two, (a, b)))
    for i in range(n_sqrt):
        ops.insert(int(rng.integers(len(ops))), Op(["sx", "sy", "sw"][i % 3], (int(rng.integers(n)),)))
    th = rng.uniform(-3, 3, k)
    return ops, th


@pytest.mark.parametrize("n,n_sqrt,tile,reg", [(12, 13, 11, 3), (13, 8, 10, 4), (9, 3, 8, 4)])
def test_every_kind_fused_forward_and_adjoint(n, n_sqrt, tile, reg):
    ops, th = _mixed_gate_circuit(n, 100 + n, n_sqrt)
    c = Circuit(n, ops, tune={"tile_bits": tile, "low_bits": 3, "reg_bits": reg})
    st = State(n)
    tht = torch.tensor(th, device="cuda")
    c.apply(st, tht)
    ref = oracle.run(n, ops, th)
    assert maxdiff(st.numpy(), ref) < AMP_TOL
    terms = W.heisenberg_1d(n, 0.3, 1.0)
    g, e = c.backward(tht, st, terms)
    e_ref, g_ref, _ = oracle.grad_pure(n, ops, th, terms)
    assert abs(e - e_ref) < AMP_TOL
    assert maxdiff(g.cpu().numpy(), g_ref) < GRAD_TOL
    phi = st.numpy()
    assert abs(phi[0] - 1) < 1e-11 and np.max(np.abs(phi[1:])) < 1e-11


EDGE_ANGLES = [0.0, math.pi / 2, math.pi, 1.5 * math.pi, 2 * math.pi, -math.pi, -math.pi / 2, 1e-9,
               math.pi - 1e-9, math.pi + 1e-9, 4 * math.pi - 1e-3, 3 * math.pi]


def _edge_circuit(n, seed):
    """Rotation-type ops (the kinds applied as in-place plane rotations) at
    angles where the cosine is 0, +-1 or changes sign, mixed with random ones."""
    rng = np.random.default_rng(seed)
    ops, th = [], []
    for i in range(5 * n):
        q = int(rng.integers(n))
        r = i % 5
        if r < 3:
            ops.append(Op(["rx", "ry", "rz"][r], (q,), (0.0,), (len(th),)))
            th.append(EDGE_ANGLES[i % len(EDGE_ANGLES)] if i % 2 == 0 else float(rng.uniform(0, 2 * math.pi)))
        elif r == 3:
            ops.append(Op(["s", "t", "z", "sx", "sy", "sw"][int(rng.integers(6))], (q,)))
        else:
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            ops.append(Op("fsim", (a, b), (0.0, 0.0, 0, 0, 0), (len(th), len(th) + 1, -1, -1, -1)))
            th.append(EDGE_ANGLES[i % len(EDGE_ANGLES)])
            th.append(EDGE_ANGLES[(3 * i + 1) % len(EDGE_ANGLES)])
    return ops, np.array(th)


@pytest.mark.parametrize("n,tile,reg", [(9, 8, 4), (10, 9, 3)])
def test_rotation_kinds_at_edge_angles(n, tile, reg):
    ops, th = _edge_circuit(n, 7 + n)
    c = Circuit(n, ops, n_params=len(th), tune={"tile_bits": tile, "low_bits": 3, "reg_bits": reg})
    psi0 = W.random_state(n, 11 + n)
    st = State(n, init=psi0)
    tht = torch.tensor(th, device="cuda")
    c.apply(st, tht)
    assert maxdiff(st.numpy(), oracle.run(n, ops, th, init=psi0)) < AMP_TOL
    st = State(n)
    c.apply(st, tht)
    terms = W.tfim(n, 0.7)
    g, e = c.backward(tht, st, terms)
    e_ref, g_ref, _ = oracle.grad_pure(n, ops, th, terms)
    assert abs(e - e_ref) < AMP_TOL
    assert maxdiff(g.cpu().numpy(), g_ref) < GRAD_TOL


def test_rotation_kinds_at_edge_angles_mixed():
    n = 4
    rng = np.random.default_rng(5)
    ops = []
    for i, a in enumerate(EDGE_ANGLES):
        q = int(rng.integers(n))
        ops.append(Op(["rx", "ry", "rz"][i % 3], (q,), (a,)))
        ops.append(Op(["s", "t", "z"][i % 3], (int(rng.integers(n)),)))
        p, r = (int(v) for v in rng.choice(n, 2, replace=False))
        ops.append(Op("fsim", (p, r), (a, EDGE_ANGLES[-1 - i], 0, 0, 0)))
    v = W.random_density(n, 3).reshape(-1, order="F")
    st = State(n, mixed=True, init=v)
    Circuit(n, ops, mixed=True).apply(st)
    assert maxdiff(st.numpy(), oracle.run(n, ops, mixed=True, init=v)) < AMP_TOL


@pytest.mark.parametrize("rows,cols,cycles,tile,low", [(3, 4, 14, 7, 3), (4, 4, 10, 8, 4), (3, 5, 12, 9, 2)])
def test_forward_with_qubit_moves(rows, cols, cycles, tile, low):
    """Forward plans that move qubits into the contiguous low block between
    passes (ping-pong through the circuit's second buffer) agree with the
    oracle and end in the standard layout."""
    n = rows * cols
    ops = W.rqc_grid(rows, cols, cycles, 41 + n)
    ref = oracle.run(n, ops)
    c = Circuit(n, ops, tune={"tile_bits": tile, "low_bits": low, "remap": 1})
    assert c.stats()["remap"] == 1
    c0 = Circuit(n, ops, tune={"tile_bits": tile, "low_bits": low, "remap": -1})
    print("passes with moves %d, without %d" % (c.stats()["n_passes"], c0.stats()["n_passes"]))
    psi0 = W.random_state(n, 5 + n)
    st = State(n, init=psi0)
    c.apply(st)
    assert maxdiff(st.numpy(), oracle.run(n, ops, init=psi0)) < AMP_TOL
    st = State(n)
    ms = c.apply_timed(st)
    assert len(ms) == c.stats()["n_passes"]
    assert maxdiff(st.numpy(), ref) < AMP_TOL
    # parametrised circuit with moves: forward and the adjoint gradient
    ops2 = W.hea(n, 5)
    th = W.theta_uniform(9, 1, W.count_params(ops2))[0]
    c2 = Circuit(n, ops2, tune={"tile_bits": tile, "low_bits": low, "remap": 1})
    s2 = c2.stats()
    print("hea: adjoint passes %d, moving %d" % (s2["n_adj_passes"], s2["n_adj_moves"]))
    assert s2["n_adj_moves"] > 0
    st2 = State(n)
    tht = torch.tensor(th, device="cuda")
    c2.apply(st2, tht)
    assert maxdiff(st2.numpy(), oracle.run(n, ops2, th)) < AMP_TOL
    g, e = c2.backward(tht, st2, W.tfim(n))
    e_ref, g_ref, _ = oracle.grad_pure(n, ops2, th, W.tfim(n))
    assert maxdiff(g.cpu().numpy(), g_ref) < GRAD_TOL
