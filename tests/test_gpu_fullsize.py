"""Full-size workloads in the launch configurations the benchmark times.

* The 28-qubit random grid circuit (default tile 11, 4 low qubits, 4 register
  bits, qubit moves): its first 8 cycles against the oracle amplitude by
  amplitude (the whole 4 GiB state, compared in chunks); the full 20-cycle
  circuit through properties that hold at any size -- unit norm, and the
  circuit followed by its inverse (each gate's conjugate transpose as a dense
  matrix op, from the oracle's gate matrices) returning |0...0>.
* The 20-qubit VQE batch of 64 (graph capture and replay): sampled items
  against the oracle's gradient.
* The batch of 32 noisy circuits of uneven width, both gradient forms:
  sampled items against the oracle, all items form against form."""
import time

import numpy as np
import pytest
import torch

import oracle
from paper_2406_19212_amd import Circuit, State
from paper_2406_19212_amd import workloads as W
from paper_2406_19212_amd.workloads import Op

pytestmark = pytest.mark.gpu
AMP_TOL = 1e-12
N, ROWS, COLS = 28, 4, 7
SEED = W.CONFIG_SEED[1]


def chunked_maxdiff(a, b, chunk=1 << 24):
    worst = 0.0
    for s in range(0, a.size, chunk):
        worst = max(worst, float(np.max(np.abs(a[s:s + chunk] - b[s:s + chunk]))))
    return worst


def test_rqc28_prefix_matches_oracle():
    ops = W.rqc_grid(ROWS, COLS, 8, SEED)
    c = Circuit(N, ops)
    stats = c.stats()
    assert (stats["tile_bits"], stats["low_bits"]) == (11, 4)
    st = State(N)
    c.apply(st)
    got = st.numpy()
    del st
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    ref = oracle.run(N, ops)
    t_or = time.perf_counter() - t0
    d = chunked_maxdiff(got, ref)
    amax = max(float(np.max(np.abs(ref[s:s + (1 << 24)]))) for s in range(0, ref.size, 1 << 24))
    print("rqc28 8 cycles: %d gates, %d passes, oracle %.1f s, maxdiff %.2e (largest amplitude %.2e)"
          % (len(ops), stats["n_passes"], t_or, d, amax), flush=True)
    assert d < AMP_TOL
    # amplitudes here are ~2^-14: hold the error to 1e-12 of the largest one as well
    assert d < 1e-12 * amax


def test_rqc28_full_circuit_and_its_inverse():
    ops = W.rqc_grid(ROWS, COLS, 20, SEED)
    inv = []
    for op in reversed(ops):
        G = oracle.gate_matrix(op.name, tuple(range(len(op.qubits))), tuple(op.params))
        inv.append(Op("matrix", tuple(op.qubits), (), (), G.conj().T.copy()))
    c, ci = Circuit(N, ops), Circuit(N, inv)
    st = State(N)
    c.apply(st)
    assert abs(st.norm() - 1) < 1e-12
    ci.apply(st)
    amp0 = st.gather([0])[0]
    print("rqc28 20 cycles + inverse: passes %d + %d, |<0|psi> - 1| = %.2e"
          % (c.stats()["n_passes"], ci.stats()["n_passes"], abs(amp0 - 1)), flush=True)
    assert abs(amp0 - 1) < AMP_TOL
    assert abs(st.norm() - 1) < 1e-12


def test_vqe20_batch64_sampled_items():
    """The 20-qubit VQE workload as the benchmark launches it (64 parameter
    sets of the 40-layer ansatz, 1600 parameters, TFIM energy; captured and
    replayed as one graph): items 0 and 63 against the oracle's Alg. 2."""
    from paper_2406_19212_amd import Batch
    n, L, Bn = 20, 40, 64
    ops = W.hea(n, L)
    P = W.count_params(ops)
    th = W.theta_uniform(W.CONFIG_SEED[2], Bn, P)
    terms = W.tfim(n, 1.0)
    circ = Circuit(n, ops, n_params=P)
    theta = torch.tensor(th, device="cuda")
    states = [torch.empty(1 << n, dtype=torch.complex128, device="cuda") for _ in range(Bn)]
    bt = Batch([circ] * Bn, states, [theta[b] for b in range(Bn)])
    en = torch.zeros(Bn, dtype=torch.float64, device="cuda")
    grads = [torch.zeros(P, dtype=torch.float64, device="cuda") for _ in range(Bn)]
    bt.capture(terms, grads, en)
    bt.replay()
    torch.cuda.synchronize()
    for b in (0, Bn - 1):
        t0 = time.perf_counter()
        e_ref, g_ref, _ = oracle.grad_pure(n, ops, th[b], terms)
        d = float(np.max(np.abs(grads[b].cpu().numpy() - g_ref)))
        print("vqe20 item %d: |dE| %.2e, max|d grad| %.2e (oracle %.1f s)"
              % (b, abs(en[b].item() - e_ref), d, time.perf_counter() - t0), flush=True)
        assert abs(en[b].item() - e_ref) < AMP_TOL
        assert d < 1e-10


def test_noisy_batch32_sampled_items():
    """The batch of 32 noisy brick-wall circuits (n in {8, 10, 12}, 20 layers,
    <Z0 Z1>) as the benchmark launches it, both gradient forms: the first
    n = 8 and n = 10 items against the oracle's checkpointed noisy gradient;
    every item's two forms against each other (the n = 12 items are beyond
    the oracle's seconds)."""
    from paper_2406_19212_amd import Batch
    items = W.noisy_batch(W.CONFIG_SEED[3], 32, (8, 10, 12), 20)
    terms = W.zz(0, 1)
    circs = [Circuit(n, ops, mixed=True, n_params=len(th)) for n, ops, th in items]
    states = [torch.empty(1 << (2 * n), dtype=torch.complex128, device="cuda") for n, *_ in items]
    thetas = [torch.tensor(th, device="cuda") for *_, th in items]
    bt = Batch(circs, states, thetas)
    res = {}
    for form in ("checkpoint", "inverse"):
        grads = [torch.zeros(t.numel(), dtype=torch.float64, device="cuda") for t in thetas]
        en = torch.zeros(len(items), dtype=torch.float64, device="cuda")
        bt.forward()
        if form == "checkpoint":
            bt.backward(terms, grads, en)
        else:
            bt.backward_inverse(terms, grads, en)
        res[form] = ([g.cpu().numpy() for g in grads], en.cpu().numpy())
    gc, ec = res["checkpoint"]
    gi, ei = res["inverse"]
    worst = max(float(np.max(np.abs(a - b))) for a, b in zip(gc, gi))
    print("noisy batch32: checkpoint vs inverse max|d grad| %.2e" % worst, flush=True)
    assert worst < 1e-10
    assert float(np.max(np.abs(ec - ei))) < AMP_TOL
    for k in (0, 1):  # n = 8, n = 10
        n, ops, th = items[k]
        t0 = time.perf_counter()
        e_ref, g_ref = oracle.grad_mixed(n, ops, th, terms)
        d = float(np.max(np.abs(gc[k] - g_ref)))
        print("noisy item %d (n=%d): |dE| %.2e, max|d grad| %.2e (oracle %.1f s)"
              % (k, n, abs(ec[k] - e_ref), d, time.perf_counter() - t0), flush=True)
        assert abs(ec[k] - e_ref) < AMP_TOL
        assert d < 1e-10
