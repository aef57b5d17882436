"""Density matrices of 6+ qubits run their forward and inverse-form adjoint on
11-bit LDS tiles with 16x16 superoperators; the checkpointed adjoint keeps
register-only passes.  Every path against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2406_19212_amd import Batch, Circuit, State
from paper_2406_19212_amd import workloads as W
from paper_2406_19212_amd.workloads import Op

pytestmark = pytest.mark.gpu
AMP_TOL, GRAD_TOL = 1e-12, 1e-10


def maxdiff(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


def every_kind(n, seed):
    rng = np.random.default_rng(seed)
    ops, P = [], 0
    for layer in range(3):
        for q in range(n):
            ops.append(Op(["rx", "ry", "rz"][(q + layer) % 3], (q,), (0.0,), (P,)))
            P += 1
            if (q + layer) % 2 == 0:
                ops.append(Op("depolarizing", (q,), (0.03,)))
            if q % 3 == 0:
                ops.append(Op("amplitude_damping", (q,), (0.05,)))
            ops.append(Op(["sx", "h", "t"][q % 3], (q,)))
        for q in range(layer % 2, n - 1, 2):
            ops.append(Op("cz", (q, q + 1)))
            ops.append(Op("depolarizing2", (q, q + 1), (0.02,)))
        a, b = (int(v) for v in rng.choice(n, 2, replace=False))
        ops.append(Op("crz", (a, b), (0.0,), (P,)))
        P += 1
        ops.append(Op("fsim", (b, a), (0.4, 0.9, 0, 0, 0)))
        ops.append(Op("kraus", (a, (a + 2) % n), (), (), W.random_kraus(4, 2, seed + layer)))
        ops.append(Op("kraus", (b,), (), (), W.random_kraus(2, 3, seed + 10 + layer)))
        ops.append(Op("toffoli", (0, 1, n - 1)))
    return ops, rng.uniform(-3, 3, P)


@pytest.mark.parametrize("n,remap", [(6, 0), (7, -1), (8, 1)])
def test_mixed_lds_forward_and_both_gradients(n, remap):
    ops, th = every_kind(n, 100 + n)
    c = Circuit(n, ops, mixed=True, n_params=len(th), tune={"remap": remap})
    s = c.stats()
    print("n=%d: LDS passes %d (moving %d), register passes %d, adjoint LDS passes" % (
        n, s["n_passes"], s["n_fwd_moves"], s["n_adj_passes"]))
    assert s["tile_bits"] == 11
    tht = torch.tensor(th, device="cuda")
    st = State(n, mixed=True)
    c.apply(st, tht)
    ref = oracle.run(n, ops, th, mixed=True)
    assert maxdiff(st.numpy(), ref) < AMP_TOL
    terms = W.tfim(n, 0.7)
    g, e = c.backward(tht, st, terms)
    e_ref, g_ref = oracle.grad_mixed(n, ops, th, terms)
    assert abs(e - e_ref) < AMP_TOL and maxdiff(g.cpu().numpy(), g_ref) < GRAD_TOL
    assert maxdiff(st.numpy(), ref) < AMP_TOL  # the checkpointed form leaves the state alone
    g2, e2 = c.backward_inverse(tht, st, terms, max_cond=1e6)
    e2_ref, g2_ref, phi = oracle.grad_mixed_inverse(n, ops, th, terms)
    assert abs(e2 - e2_ref) < AMP_TOL and maxdiff(g2.cpu().numpy(), g2_ref) < GRAD_TOL
    assert maxdiff(st.numpy(), phi) < 1e-11


def test_mixed_lds_batches():
    items = W.noisy_batch(88, 6, (6, 7, 8), 4)
    circs = [Circuit(n, ops, mixed=True, n_params=len(th)) for n, ops, th in items]
    states = [torch.empty(1 << (2 * n), dtype=torch.complex128, device="cuda") for n, *_ in items]
    thetas = [torch.tensor(th, device="cuda") for *_, th in items]
    grads = [torch.zeros(t.numel(), dtype=torch.float64, device="cuda") for t in thetas]
    en = torch.zeros(len(items), dtype=torch.float64, device="cuda")
    terms = W.zz(0, 1)
    bt = Batch(circs, states, thetas)
    bt.forward()
    for (n, ops, th), s in zip(items, states):
        assert maxdiff(s.cpu().numpy(), oracle.run(n, ops, th, mixed=True)) < AMP_TOL
    bt.backward(terms, grads, en)
    for (n, ops, th), g, e in zip(items, grads, en.cpu().numpy()):
        e_ref, g_ref = oracle.grad_mixed(n, ops, th, terms)
        assert abs(e - e_ref) < AMP_TOL and maxdiff(g.cpu().numpy(), g_ref) < GRAD_TOL
    for rep in range(2):
        bt.forward()
        bt.backward_inverse(terms, grads, en)
        for (n, ops, th), s, g, e in zip(items, states, grads, en.cpu().numpy()):
            e_ref, g_ref, phi = oracle.grad_mixed_inverse(n, ops, th, terms)
            assert abs(e - e_ref) < AMP_TOL and maxdiff(g.cpu().numpy(), g_ref) < GRAD_TOL
            assert maxdiff(s.cpu().numpy(), phi) < AMP_TOL


def test_batched_inverse_matches_checkpointed_form_at_n10():
    """Two items of the 20-layer noisy circuit at n = 10 in one batch: the
    inverse form agrees with the checkpointed form and with the single-item
    path (a missing barrier after direct last-stage stores once let the
    waves of one tile sum each other's reductions before they were written)."""
    items = [it for it in W.noisy_batch(W.CONFIG_SEED[3], 6, (8, 10, 12), 20) if it[0] == 10]
    items = [items[0], items[1], items[0]]
    circs = [Circuit(n, ops, mixed=True, n_params=len(th)) for n, ops, th in items]
    states = [torch.empty(1 << (2 * n), dtype=torch.complex128, device="cuda") for n, *_ in items]
    thetas = [torch.tensor(th, device="cuda") for *_, th in items]
    g_ck = [torch.zeros(t.numel(), dtype=torch.float64, device="cuda") for t in thetas]
    g_inv = [torch.zeros(t.numel(), dtype=torch.float64, device="cuda") for t in thetas]
    en = torch.zeros(len(items), dtype=torch.float64, device="cuda")
    terms = W.zz(0, 1)
    bt = Batch(circs, states, thetas)
    bt.forward()
    bt.backward(terms, g_ck, en)
    for rep in range(3):
        bt.forward()
        bt.backward_inverse(terms, g_inv, en)
        for a, b in zip(g_ck, g_inv):
            assert maxdiff(a.cpu().numpy(), b.cpu().numpy()) < GRAD_TOL
