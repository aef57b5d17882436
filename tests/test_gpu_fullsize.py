"""Full-size workloads in the launch configurations the benchmark times.

* The 28-qubit random grid circuit (default tile 11, 4 low qubits, 4 register
  bits, qubit moves, 22 passes), all 20 cycles: its output -- the 1000 seeded
  bitstring amplitudes and the norm the benchmark reads -- and every other
  amplitude of the 4 GiB state against the oracle's run of the same circuit
  (Eq. (circuitevolve)); and the circuit followed by its inverse (each gate's
  conjugate transpose as a dense matrix op) returning |0...0>.
* The single unfused ops the benchmark times on the 28-qubit state (dense
  one-, two- and three-qubit matrices on qubit 27, CZ) against the oracle's
  Eq. (3) / Alg. 1 loops, from a seeded 28-qubit input state.
* The 20-qubit VQE batch of 64 (graph capture and replay): sampled items
  against the oracle's gradient.
* The batch of 32 noisy circuits of uneven width, both gradient forms:
  sampled items against the oracle, all items form against form; and a
  12-qubit noisy item (vec(rho) of 2^24 entries on the benchmark's 11-bit LDS
  tiles, two layers so that the oracle runs in seconds) alone and inside a
  batch of widths 8, 10, 12: state, energy and both gradient forms against
  the oracle (Sec. 3.5, Eq. (diff_mixed))."""
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


def test_rqc28_output_matches_oracle():
    ops = W.rqc_grid(ROWS, COLS, 20, SEED)
    idx = W.rqc_bitstrings(N, 1000, SEED + 1)  # the benchmark's output bitstrings
    c = Circuit(N, ops)
    stats = c.stats()
    assert (stats["tile_bits"], stats["low_bits"], stats["n_passes"]) == (11, 4, 22)
    st = State(N)
    c.apply(st)
    amps = st.gather(idx)
    nrm = st.norm()
    got = st.numpy()
    del st
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    ref = oracle.run(N, ops)
    t_or = time.perf_counter() - t0
    amax = max(float(np.max(np.abs(ref[s:s + (1 << 24)]))) for s in range(0, ref.size, 1 << 24))
    d_out = float(np.max(np.abs(amps - ref[idx])))
    nrm_ref = sum(float(np.sum(np.abs(ref[s:s + (1 << 24)]) ** 2)) for s in range(0, ref.size, 1 << 24))
    d_all = chunked_maxdiff(got, ref)
    print("rqc28 20 cycles: %d gates, %d passes, oracle %.1f s (%d threads); 1000 amplitudes max|d| %.2e "
          "(x 2^14 = %.2e), |d norm| %.2e, all amplitudes max|d| %.2e (largest %.2e)"
          % (len(ops), stats["n_passes"], t_or, oracle.get_threads(), d_out, d_out * 2 ** 14,
             abs(nrm - nrm_ref), d_all, amax), flush=True)
    assert d_out < AMP_TOL and d_out < 1e-12 * amax
    assert abs(nrm - nrm_ref) < AMP_TOL
    assert d_all < AMP_TOL and d_all < 1e-12 * amax


def test_single_ops_q27_match_oracle():
    """dense 1q on qubit 27, dense 2q on (3, 27), dense 3q on (0, 13, 27) and
    CZ on (5, 26), one after another on a 28-qubit state, each checked over
    every amplitude."""
    # seeded input with no product structure across any qubit: the sum of two
    # Kronecker products of random 14-qubit states, normalised
    a, b, c2, d = (W.random_state(14, 500 + k) for k in range(4))
    psi = np.multiply.outer(a, b).ravel()  # index = x_b + 2^14 x_a: a holds qubits 14..27
    psi += np.multiply.outer(c2, d).ravel()
    psi /= np.sqrt(sum(float(np.sum(np.abs(psi[s:s + (1 << 24)]) ** 2)) for s in range(0, psi.size, 1 << 24)))
    st = State(N, init=psi)
    cases = [Op("matrix", (27,), (), (), W.random_unitary(2, 1)),
             Op("matrix", (3, 27), (), (), W.random_unitary(4, 2)),
             Op("matrix", (0, 13, 27), (), (), W.random_unitary(8, 3)),
             Op("cz", (5, 26))]
    for op in cases:
        st.apply_op(op)
        oracle.apply_op_inplace(psi, N, op)
        d = chunked_maxdiff(st.numpy(), psi)
        print("28q single op %s %s: max|d| %.2e" % (op.name, op.qubits, d), flush=True)
        assert d < AMP_TOL


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


def _noisy_item_checks(tag, n, st_vec, e_ck, g_ck, e_inv, g_inv, ops, th, terms):
    t0 = time.perf_counter()
    rho_ref = oracle.run(n, ops, th, mixed=True)
    e_ref, g_ref, _ = oracle.grad_mixed_inverse(n, ops, th, terms)
    d_rho = float(np.max(np.abs(st_vec - rho_ref))) if st_vec is not None else 0.0
    print("%s n=%d: max|d rho| %.2e, |dE| %.2e / %.2e, max|d grad| checkpoint %.2e inverse %.2e (oracle %.1f s)"
          % (tag, n, d_rho, abs(e_ck - e_ref), abs(e_inv - e_ref), float(np.max(np.abs(g_ck - g_ref))),
             float(np.max(np.abs(g_inv - g_ref))), time.perf_counter() - t0), flush=True)
    assert d_rho < AMP_TOL
    assert abs(e_ck - e_ref) < AMP_TOL and abs(e_inv - e_ref) < AMP_TOL
    assert float(np.max(np.abs(g_ck - g_ref))) < 1e-10
    assert float(np.max(np.abs(g_inv - g_ref))) < 1e-10


def test_noisy_n12_item_matches_oracle():
    """A 12-qubit noisy brick-wall item (two layers, 238 ops, 72 angles) on
    the benchmark's tiles, single-item calls and inside a batch with an
    8- and a 10-qubit item (both gradient forms)."""
    from paper_2406_19212_amd import Batch
    terms = W.zz(0, 1)
    items = [(n,) + tuple(W.noisy_brickwall(n, 2, W.CONFIG_SEED[3] + 100 + n)) for n in (8, 10, 12)]
    n, ops, th = items[2]
    c = Circuit(n, ops, mixed=True, n_params=len(th))
    tht = torch.tensor(th, device="cuda")
    st = State(n, mixed=True)
    c.apply(st, tht)
    rho = st.numpy().copy()
    g_ck, e_ck = c.backward(tht, st, terms)
    st.reset()
    c.apply(st, tht)
    g_inv, e_inv = c.backward_inverse(tht, st, terms)
    _noisy_item_checks("single", n, rho, e_ck, g_ck.cpu().numpy(), e_inv, g_inv.cpu().numpy(), ops, th, terms)
    del st
    circs = [Circuit(m, o, mixed=True, n_params=len(t)) for m, o, t in items]
    states = [torch.empty(1 << (2 * m), dtype=torch.complex128, device="cuda") for m, *_ in items]
    thetas = [torch.tensor(t, device="cuda") for *_, t in items]
    bt = Batch(circs, states, thetas)
    res = {}
    for form in ("checkpoint", "inverse"):
        grads = [torch.zeros(t.numel(), dtype=torch.float64, device="cuda") for t in thetas]
        en = torch.zeros(len(items), dtype=torch.float64, device="cuda")
        bt.forward()
        if form == "checkpoint":
            rho_b = states[2].cpu().numpy().copy()
            bt.backward(terms, grads, en)
        else:
            bt.backward_inverse(terms, grads, en)
        res[form] = (grads[2].cpu().numpy(), float(en[2].item()))
    assert float(np.max(np.abs(rho_b - rho))) < AMP_TOL
    _noisy_item_checks("batch", n, None, res["checkpoint"][1], res["checkpoint"][0], res["inverse"][1],
                       res["inverse"][0], ops, th, terms)
