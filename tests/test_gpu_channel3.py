"""Three-qubit Kraus channels (QuantumMap with m = 3) on density matrices:
as single ops the library applies sum_s K_s rho K_s^dagger term by term on
each 8 x 8 block, and inside circuits the same block kernel runs as a pass of
its own (adjoint Kraus sets for Psi, the inverse superoperator for Phi in the
inverse form); the oracle applies the 64 x 64 superoperator of Eq.
(channel2).  Amplitudes to 1e-12, gradients to 1e-10."""
import itertools

import numpy as np
import pytest
import torch

import oracle
from paper_2406_19212_amd import Circuit, State
from paper_2406_19212_amd import workloads as W
from paper_2406_19212_amd.binding import VQCError
from paper_2406_19212_amd.workloads import Op

pytestmark = pytest.mark.gpu
AMP_TOL = 1e-12
GRAD_TOL = 1e-10


def maxdiff(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


@pytest.mark.parametrize("n", [3, 4, 6, 9])
def test_three_qubit_kraus_matches_oracle(n):
    v = W.random_density(n, 90 + n).reshape(-1, order="F").copy()
    perms = list(itertools.permutations(range(n), 3))
    cases = [perms[0], perms[-1], perms[len(perms) // 2], (n - 1, 0, n // 2)]
    worst = 0.0
    for k, (qs, cnt) in enumerate(itertools.product(cases, (1, 3, 64))):
        K = W.random_kraus(8, cnt, 300 + 7 * n + k)
        st = State(n, mixed=True, init=v)
        st.apply_channel(list(qs), K)
        got = st.numpy()
        ref = oracle.run(n, [Op("kraus", qs, (), (), K)], mixed=True, init=v)
        worst = max(worst, maxdiff(got, ref))
        # the result is a density matrix: unit trace, Hermitian
        rho = got.reshape(1 << n, 1 << n, order="F")
        assert abs(np.trace(rho) - 1) < 1e-12
        assert maxdiff(rho, rho.conj().T) < 1e-12
    print("n=%d: worst %.2e" % (n, worst))
    assert worst < AMP_TOL


def test_unitary_kraus_equals_three_qubit_gate_and_apply_op():
    n = 5
    v = W.random_density(n, 123).reshape(-1, order="F").copy()
    U = W.random_unitary(8, 124)
    a = State(n, mixed=True, init=v)
    a.apply_channel([4, 1, 2], [U])
    b = State(n, mixed=True, init=v)
    b.apply_gate([4, 1, 2], U)
    assert maxdiff(a.numpy(), b.numpy()) < AMP_TOL
    K = W.random_kraus(8, 5, 125)
    c = State(n, mixed=True, init=v)
    c.apply_op(Op("kraus", (0, 3, 4), (), (), K))
    d = State(n, mixed=True, init=v)
    d.apply_channel([0, 3, 4], K)
    assert maxdiff(c.numpy(), d.numpy()) == 0.0


def _circuit_with_channels(n, layers, seed):
    """Ry layers, three-qubit channels close to unitaries on varying qubit
    orders, three-qubit gates, one-qubit noise and CZ."""
    from tests.test_oracle_pins import weak_kraus3
    rng = np.random.default_rng(seed)
    ops, P = [], 0
    for layer in range(layers):
        for q in range(n):
            ops.append(Op("ry", (q,), (0.0,), (P,)))
            P += 1
        a, b, c = (int(v) for v in rng.choice(n, 3, replace=False))
        ops.append(Op("kraus", (a, b, c), (), (), weak_kraus3(0.05, seed + layer)))
        if layer % 2:
            ops.append(Op("matrix", (c, b, a), (), (), W.random_unitary(8, seed + 40 + layer)))
        ops.append(Op("depolarizing", (int(rng.integers(n)),), (0.02,)))
        for q in range(layer % 2, n - 1, 2):
            ops.append(Op("cz", (q, q + 1)))
    return ops, rng.uniform(-3, 3, P)


@pytest.mark.parametrize("n,tune", [(3, None), (4, None), (6, None), (6, {"remap": -1, "low_bits": 3}), (7, None)])
def test_noisy_circuit_with_three_qubit_channels(n, tune):
    """Three-qubit channels inside circuits (passes of their own) against the
    oracle: state, energy, the checkpointed gradient and the inverse form."""
    ops, th = _circuit_with_channels(n, 4, 300 + n)
    c = Circuit(n, ops, mixed=True, n_params=len(th), tune=tune)
    tht = torch.tensor(th, device="cuda")
    st = State(n, mixed=True)
    c.apply(st, tht)
    assert maxdiff(st.numpy(), oracle.run(n, ops, th, mixed=True)) < AMP_TOL
    terms = W.zz(0, 1) + [W.pauli_string({n - 1: "x"}, 0.4)]
    g, e = c.backward(tht, st, terms)
    e_ref, g_ref = oracle.grad_mixed(n, ops, th, terms)
    print("n=%d: passes %d, |dE| %.1e, max|d grad| %.1e" % (n, c.stats()["n_passes"], abs(e - e_ref),
                                                          maxdiff(g.cpu().numpy(), g_ref)))
    assert abs(e - e_ref) < AMP_TOL
    assert maxdiff(g.cpu().numpy(), g_ref) < GRAD_TOL
    g2, e2 = c.backward_inverse(tht, st, terms)
    _, g2_ref, _ = oracle.grad_mixed_inverse(n, ops, th, terms)
    assert abs(e2 - e_ref) < AMP_TOL
    assert maxdiff(g2.cpu().numpy(), g2_ref) < GRAD_TOL
    # Phi was uncomputed back to |0..0><0..0| (up to the channels' conditioning)
    v0 = np.zeros(4 ** n, complex)
    v0[0] = 1
    assert maxdiff(st.numpy(), v0) < 1e-10


def test_three_qubit_channels_refused_where_unsupported():
    from paper_2406_19212_amd import Batch
    K = W.random_kraus(8, 2, 7)
    st = State(3, mixed=True)
    with pytest.raises(VQCError) as e:
        st.apply_channel([0, 1, 2], [k * 1.01 for k in K])  # not trace preserving
    assert e.value.status == -5
    with pytest.raises(VQCError) as e:
        State(3).apply_channel([0, 1, 2], K)  # pure state
    assert e.value.status == -4
    # batches do not take circuits with three-qubit channels
    c = Circuit(3, [Op("kraus", (0, 1, 2), (), (), K)], mixed=True)
    with pytest.raises(VQCError) as e:
        Batch([c], [torch.empty(64, dtype=torch.complex128, device="cuda")], [None])
    assert e.value.status == -3
    # complete dephasing of qubit 0 has a singular superoperator: the inverse
    # form refuses it, the checkpointed form does not need an inverse
    P0, P1 = np.diag([1, 0]), np.diag([0, 1])
    deph = [np.kron(np.eye(4), P0), np.kron(np.eye(4), P1)]  # qubit 0 = the least significant bit
    ops = [Op("ry", (0,), (0.0,), (0,)), Op("kraus", (0, 1, 2), (), (), deph), Op("rx", (1,), (0.0,), (1,))]
    cd = Circuit(3, ops, mixed=True, n_params=2)
    th = np.array([0.4, 1.1])
    tht = torch.tensor(th, device="cuda")
    s2 = State(3, mixed=True)
    cd.apply(s2, tht)
    g, _ = cd.backward(tht, s2, W.zz(0, 1))
    assert maxdiff(g.cpu().numpy(), oracle.grad_mixed(3, ops, th, W.zz(0, 1))[1]) < GRAD_TOL
    with pytest.raises(VQCError) as e:
        cd.backward_inverse(tht, s2, W.zz(0, 1))
    assert e.value.status == -11
