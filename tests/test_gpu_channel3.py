"""Three-qubit Kraus channels (QuantumMap with m = 3) as single ops on
density matrices: the library applies sum_s K_s rho K_s^dagger term by term on
each 8 x 8 block; the oracle applies the 64 x 64 superoperator of Eq.
(channel2).  Amplitudes to 1e-12."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2406_19212_amd import Circuit, State
from paper_2406_19212_amd import workloads as W
from paper_2406_19212_amd.binding import VQCError
from paper_2406_19212_amd.workloads import Op

pytestmark = pytest.mark.gpu
AMP_TOL = 1e-12


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


def test_three_qubit_channels_refused_where_unsupported():
    K = W.random_kraus(8, 2, 7)
    with pytest.raises(VQCError) as e:
        Circuit(3, [Op("kraus", (0, 1, 2), (), (), K)], mixed=True)
    assert e.value.status == -3
    st = State(3, mixed=True)
    with pytest.raises(VQCError) as e:
        st.apply_channel([0, 1, 2], [k * 1.01 for k in K])  # not trace preserving
    assert e.value.status == -5
    with pytest.raises(VQCError) as e:
        State(3).apply_channel([0, 1, 2], K)  # pure state
    assert e.value.status == -4
