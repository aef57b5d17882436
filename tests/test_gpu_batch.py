"""Batched launches and hipGraph replay agree with the per-item path and the
oracle; the autograd wrapper returns the oracle gradient."""
import numpy as np
import pytest
import torch

import oracle
from paper_2406_19212_amd import Batch, Circuit, State
from paper_2406_19212_amd import workloads as W
from paper_2406_19212_amd.autograd import energy

pytestmark = pytest.mark.gpu
AMP_TOL, GRAD_TOL = 1e-12, 1e-10


def test_batch_forward_backward_matches_oracle():
    n, L, B = 10, 3, 6
    ops = W.hea(n, L)
    P = W.count_params(ops)
    th = W.theta_uniform(11, B, P)
    terms = W.tfim(n, 1.0)
    circ = Circuit(n, ops, n_params=P)
    theta = torch.tensor(th, device="cuda")
    states = [torch.empty(1 << n, dtype=torch.complex128, device="cuda") for _ in range(B)]
    bt = Batch([circ] * B, states, [theta[b] for b in range(B)])
    bt.forward()
    for b in range(B):
        ref = oracle.run(n, ops, th[b])
        assert np.max(np.abs(states[b].cpu().numpy() - ref)) < AMP_TOL
    en = torch.zeros(B, dtype=torch.float64, device="cuda")
    bt.expectation(terms, en)
    grads = [torch.zeros(P, dtype=torch.float64, device="cuda") for _ in range(B)]
    en2 = torch.zeros(B, dtype=torch.float64, device="cuda")
    bt.backward(terms, grads, en2)
    for b in range(B):
        e_ref, g_ref, _ = oracle.grad_pure(n, ops, th[b], terms)
        assert abs(en[b].item() - e_ref) < AMP_TOL and abs(en2[b].item() - e_ref) < AMP_TOL
        assert np.max(np.abs(grads[b].cpu().numpy() - g_ref)) < GRAD_TOL


def test_batch_uneven_widths_pure():
    tune = {"tile_bits": 8, "low_bits": 3}
    items = []
    for i, n in enumerate([8, 11, 13, 9]):
        ops, th = W.brickwall(n, 3, 70 + i)
        items.append((n, ops, th, Circuit(n, ops, tune=tune)))
    states = [torch.empty(1 << n, dtype=torch.complex128, device="cuda") for n, *_ in items]
    thetas = [torch.tensor(th, device="cuda") for _, _, th, _ in items]
    bt = Batch([c for *_, c in items], states, thetas)
    bt.forward()
    terms = W.zz(0, 1) + [W.pauli_string({2: "x"}, 0.5)]
    grads = [torch.zeros(t.numel(), dtype=torch.float64, device="cuda") for t in thetas]
    bt.backward(terms, grads)
    for (n, ops, th, _), s, g in zip(items, states, grads):
        bt_ref = oracle.run(n, ops, th)
        e_ref, g_ref, _ = oracle.grad_pure(n, ops, th, terms)
        assert np.max(np.abs(g.cpu().numpy() - g_ref)) < GRAD_TOL


def test_batch_uneven_widths_noisy():
    items = []
    for i, n in enumerate([3, 4, 2]):
        ops, th = W.noisy_brickwall(n, 2, 80 + i, p1=0.02, gamma=0.03, p2=0.05)
        items.append((n, ops, th, Circuit(n, ops, mixed=True)))
    states = [torch.empty(1 << (2 * n), dtype=torch.complex128, device="cuda") for n, *_ in items]
    thetas = [torch.tensor(th, device="cuda") for _, _, th, _ in items]
    bt = Batch([c for *_, c in items], states, thetas)
    bt.forward()
    for (n, ops, th, _), s in zip(items, states):
        assert np.max(np.abs(s.cpu().numpy() - oracle.run(n, ops, th, mixed=True))) < AMP_TOL
    terms = W.zz(0, 1)
    grads = [torch.zeros(t.numel(), dtype=torch.float64, device="cuda") for t in thetas]
    en = torch.zeros(len(items), dtype=torch.float64, device="cuda")
    bt.backward(terms, grads, en)
    for k, ((n, ops, th, _), g) in enumerate(zip(items, grads)):
        e_ref, g_ref = oracle.grad_mixed(n, ops, th, terms)
        assert abs(en[k].item() - e_ref) < AMP_TOL
        assert np.max(np.abs(g.cpu().numpy() - g_ref)) < GRAD_TOL


def test_graph_replays_are_identical():
    n, L, B = 12, 4, 8
    ops = W.hea(n, L)
    P = W.count_params(ops)
    th = W.theta_uniform(12, B, P)
    terms = W.tfim(n, 1.0)
    circ = Circuit(n, ops, n_params=P)
    theta = torch.tensor(th, device="cuda")
    states = [torch.empty(1 << n, dtype=torch.complex128, device="cuda") for _ in range(B)]
    bt = Batch([circ] * B, states, [theta[b] for b in range(B)])
    grads = [torch.zeros(P, dtype=torch.float64, device="cuda") for _ in range(B)]
    en = torch.zeros(B, dtype=torch.float64, device="cuda")
    bt.capture(terms, grads, en)
    ref = None
    for rep in range(3):
        for g in grads:
            g.fill_(7.0)  # eager work between replays
        bt.replay()
        torch.cuda.synchronize()
        cur = torch.stack(grads).cpu().numpy().copy()
        if ref is None:
            ref = cur
            for b in range(B):
                e_ref, g_ref, _ = oracle.grad_pure(n, ops, th[b], terms)
                assert np.max(np.abs(cur[b] - g_ref)) < GRAD_TOL
                assert abs(en[b].item() - e_ref) < AMP_TOL
        else:
            assert np.array_equal(cur, ref)


@pytest.mark.parametrize("tile,low", [(8, 3), (9, 4)])
def test_batch_with_qubit_moves(tile, low):
    """Batched passes that move qubits run out of place through per-item
    second buffers (one for the forward, two for the adjoint); forward
    states, energies and gradients match the oracle, also on graph replays,
    and a mixed batch of moving and non-moving plans works."""
    n, L = 12, 5
    ops = W.hea(n, L)
    P = W.count_params(ops)
    B = 4
    th = W.theta_uniform(31 + tile, B, P)
    terms = W.tfim(n, 0.9)
    cm = Circuit(n, ops, n_params=P, tune={"tile_bits": tile, "low_bits": low, "remap": 1})
    cp = Circuit(n, ops, n_params=P, tune={"tile_bits": tile, "low_bits": low, "remap": -1})
    sm = cm.stats()
    print("fwd passes %d (moving %d), adjoint %d (moving %d); without moves %d / %d" % (
        sm["n_passes"], sm["n_fwd_moves"], sm["n_adj_passes"], sm["n_adj_moves"],
        cp.stats()["n_passes"], cp.stats()["n_adj_passes"]))
    assert sm["n_fwd_moves"] > 0 and sm["n_adj_moves"] > 0
    circs = [cm, cp, cm, cm]
    theta = torch.tensor(th, device="cuda")
    states = [torch.empty(1 << n, dtype=torch.complex128, device="cuda") for _ in range(B)]
    bt = Batch(circs, states, [theta[b] for b in range(B)])
    bt.forward()
    for b in range(B):
        assert np.max(np.abs(states[b].cpu().numpy() - oracle.run(n, ops, th[b]))) < AMP_TOL
    grads = [torch.zeros(P, dtype=torch.float64, device="cuda") for _ in range(B)]
    en = torch.zeros(B, dtype=torch.float64, device="cuda")
    bt.backward(terms, grads, en)
    refs = [oracle.grad_pure(n, ops, th[b], terms) for b in range(B)]
    for b in range(B):
        assert abs(en[b].item() - refs[b][0]) < AMP_TOL
        assert np.max(np.abs(grads[b].cpu().numpy() - refs[b][1])) < GRAD_TOL
    bt2 = Batch(circs, states, [theta[b] for b in range(B)])
    bt2.capture(terms, grads, en)
    for rep in range(2):
        for g in grads:
            g.fill_(7.0)
        bt2.replay()
        torch.cuda.synchronize()
        for b in range(B):
            assert np.max(np.abs(grads[b].cpu().numpy() - refs[b][1])) < GRAD_TOL


def test_autograd_energy():
    n = 8
    ops = W.hea(n, 3)
    P = W.count_params(ops)
    th = W.theta_uniform(21, 1, P)[0]
    terms = W.tfim(n, 0.7)
    circ = Circuit(n, ops, n_params=P)
    theta = torch.tensor(th, device="cuda", requires_grad=True)
    e = energy(circ, theta, terms)
    (3.0 * e).backward()
    e_ref, g_ref, _ = oracle.grad_pure(n, ops, th, terms)
    assert abs(e.item() - e_ref) < AMP_TOL
    assert np.max(np.abs(theta.grad.cpu().numpy() - 3.0 * g_ref)) < GRAD_TOL
