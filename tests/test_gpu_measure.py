"""measure! (outcome, exact probability, collapse) and bitstring sampling on
the device against the oracle."""
import json
import os

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
GOLD = os.path.join(os.path.dirname(__file__), "golden", "listings.json")


def maxdiff(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


def weights(v, n, mixed):
    D = 1 << n
    if mixed:
        return np.real(v.reshape(D, D, order="F").diagonal()).copy()
    return np.abs(v) ** 2


@pytest.mark.parametrize("n,mixed", [(1, False), (5, False), (13, False), (1, True), (4, True), (6, True)])
def test_measure_chain_matches_oracle(n, mixed):
    if mixed:
        v = W.random_density(n, 40 + n).reshape(-1, order="F").copy()
    else:
        v = W.random_state(n, 40 + n) * 1.3  # not normalised: probabilities are relative
    st = State(n, mixed=mixed, init=v)
    ref = v.copy()
    rng = np.random.default_rng(n)
    for step, q in enumerate(rng.permutation(n)):
        w = weights(ref, n, mixed)
        idx = np.arange(1 << n)
        p0 = w[((idx >> q) & 1) == 0].sum() / w.sum()
        u = float(rng.uniform())
        if abs(u - p0) < 1e-9:
            u = (u + 0.5) % 1.0
        o, p = st.measure(int(q), u)
        o_ref, p_ref = oracle.measure(ref, n, int(q), u, mixed=mixed)
        assert o == o_ref and abs(p - p_ref) < AMP_TOL
        assert maxdiff(st.numpy(), ref) < AMP_TOL
    # every qubit measured: a basis state (pure) / diagonal projector (mixed)
    assert abs(st.norm() - 1) < AMP_TOL


def test_measure_listing4_and_errors():
    L4 = json.load(open(GOLD))["listing4_probability"]
    ops = [Op(a, tuple(b), tuple(c)) for a, b, c in L4["circuit"]]
    c = Circuit(2, ops)
    for u, want in ((0.9, 1), (0.1, 0)):
        st = State(2)
        c.apply(st)
        o, p = st.measure(L4["measured_qubit"], u)
        assert o == want
        assert abs(p - (L4["p_outcome_1"] if o else 1 - L4["p_outcome_1"])) < AMP_TOL
        amp = st.numpy()
        assert abs(abs(amp[3 if o else 0]) - 1) < AMP_TOL
    st = State(2)
    for bad in (-0.1, 1.0):
        with pytest.raises(VQCError):
            st.measure(0, bad)
    with pytest.raises(VQCError):
        st.measure(2, 0.5)
    z = State(3, init=np.zeros(8, complex))
    with pytest.raises(VQCError):
        z.measure(0, 0.5)
    with pytest.raises(VQCError):
        z.sample([0.5])


def check_samples(x, x_ref, v, n, mixed, u):
    """Equal to the oracle's left-to-right inverse CDF except where u*C lies
    within rounding of a boundary; there the sample must still be valid."""
    w = weights(v, n, mixed)
    C = np.cumsum(w)
    t = np.asarray(u) * C[-1]
    tol = 1e-12 * C[-1]
    diff = np.nonzero(x != x_ref)[0]
    for k in diff:
        xk = int(x[k])
        lo = C[xk - 1] if xk > 0 else 0.0
        assert w[xk] > 0 and lo <= t[k] + tol and C[xk] >= t[k] - tol, (k, xk, x_ref[k])
    return diff.size


@pytest.mark.parametrize("n,mixed,count", [(3, False, 500), (12, False, 20000), (14, False, 20000),
                                           (22, False, 50000), (5, True, 3000), (7, True, 20000)])
def test_sample_matches_oracle(n, mixed, count):
    if mixed:
        v = W.random_density(n, 50 + n).reshape(-1, order="F").copy()
    else:
        v = W.random_state(n, 50 + n)
        v[np.arange(v.size) % 7 == 3] = 0  # zero-weight basis states are never sampled
    st = State(n, mixed=mixed, init=v)
    rng = np.random.default_rng(60 + n)
    u = rng.uniform(size=count)
    u[:64] = (np.arange(64) + 0.5) / 64  # stratified head
    u[64] = 0.0
    x = st.sample(u)
    x_ref = oracle.sample(v, n, u, mixed=mixed)
    nd = check_samples(x, x_ref, v, n, mixed, u)
    print("n=%d mixed=%d: %d of %d samples differ from the oracle (all valid)" % (n, mixed, nd, count))
    assert nd <= count // 1000
    assert maxdiff(st.numpy(), v) == 0.0  # sampling leaves the state alone
    assert st.sample([]).size == 0


def test_sample_after_circuit_is_born_distribution():
    # a product of Ry rotations: the exact distribution is a product of cos^2 / sin^2
    n = 10
    ang = np.linspace(0.2, 2.9, n)
    c = Circuit(n, [Op("ry", (q,), (float(a),)) for q, a in enumerate(ang)])
    st = State(n)
    c.apply(st)
    K = 1 << 16
    x = st.sample((np.arange(K) + 0.5) / K)
    p = np.ones(1 << n)
    idx = np.arange(1 << n)
    for q, a in enumerate(ang):
        bit = (idx >> q) & 1
        p *= np.where(bit == 1, np.sin(a / 2) ** 2, np.cos(a / 2) ** 2)
    cnt = np.bincount(x, minlength=1 << n)
    # a sample at a rounding boundary may move to its neighbour
    assert np.all(np.abs(cnt - K * p) <= 2.0)
