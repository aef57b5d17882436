"""Circuit-specialised forward and adjoint passes (compiled at run time for
the circuit's op sequence) against the oracle: every gate kind fused in one circuit, the
rotation kinds at edge angles, qubit moves between passes, both register
widths, a persistent grid, batched items of one circuit, and the on-disk code
cache.  Every case asks for the specialised kernels (vqc_tune.jit = 1), so a
failed compile fails the test instead of falling back to the interpreting
kernel."""
import math
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2406_19212_amd import Batch, Circuit, State
from paper_2406_19212_amd import workloads as W
from tests.test_gpu_parity import _edge_circuit, _mixed_gate_circuit

pytestmark = pytest.mark.gpu
AMP_TOL = 1e-12
GRAD_TOL = 1e-10


def maxdiff(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


def _jit_circuit(n, ops, **tune):
    tune.setdefault("jit", 1)
    c = Circuit(n, ops, n_params=W.count_params(ops), tune=tune)
    s = c.stats()
    assert s["n_jit_passes"] == s["n_passes"] > 0, s
    assert s["n_jit_adj_passes"] == s["n_adj_passes"] > 0, s
    return c


@pytest.mark.parametrize("n,n_sqrt,tile,reg,remap", [(12, 13, 11, 3, 1), (13, 8, 10, 4, -1), (14, 5, 11, 4, 1),
                                                     (9, 3, 8, 3, -1)])
def test_every_kind_specialised(n, n_sqrt, tile, reg, remap):
    ops, th = _mixed_gate_circuit(n, 300 + n, n_sqrt)
    c = _jit_circuit(n, ops, tile_bits=tile, low_bits=3, reg_bits=reg, remap=remap)
    tht = torch.tensor(th, device="cuda")
    psi0 = W.random_state(n, 31 + n)
    st = State(n, init=psi0)
    c.apply(st, tht)
    assert maxdiff(st.numpy(), oracle.run(n, ops, th, init=psi0)) < AMP_TOL
    # the interpreting kernel on the same plan gives the same state
    ci = Circuit(n, ops, n_params=len(th), tune={"tile_bits": tile, "low_bits": 3, "reg_bits": reg, "remap": remap,
                                                  "jit": -1})
    assert ci.stats()["n_jit_passes"] == 0
    si = State(n, init=psi0)
    ci.apply(si, tht)
    assert maxdiff(st.numpy(), si.numpy()) < AMP_TOL
    # the gradient (specialised adjoint passes, Alg. 2)
    st = State(n)
    c.apply(st, tht)
    terms = W.heisenberg_1d(n, 0.3, 1.0)
    g, e = c.backward(tht, st, terms)
    e_ref, g_ref, _ = oracle.grad_pure(n, ops, th, terms)
    assert abs(e - e_ref) < AMP_TOL
    assert maxdiff(g.cpu().numpy(), g_ref) < GRAD_TOL


@pytest.mark.parametrize("n,tile,reg", [(10, 9, 3), (11, 8, 4)])
def test_rotation_kinds_at_edge_angles_specialised(n, tile, reg):
    ops, th = _edge_circuit(n, 17 + n)
    c = _jit_circuit(n, ops, tile_bits=tile, low_bits=3, reg_bits=reg)
    psi0 = W.random_state(n, 21 + n)
    st = State(n, init=psi0)
    c.apply(st, torch.tensor(th, device="cuda"))
    assert maxdiff(st.numpy(), oracle.run(n, ops, th, init=psi0)) < AMP_TOL


@pytest.mark.parametrize("rows,cols,cycles,tile,low,grid", [(3, 5, 12, 9, 2, 0), (4, 4, 10, 8, 4, 0),
                                                            (4, 5, 8, 11, 4, 0), (4, 5, 8, 11, 4, 96)])
def test_grid_circuits_with_moves_specialised(rows, cols, cycles, tile, low, grid):
    """Random grid circuits whose plans move qubits between passes (including
    passes that only move qubits), and a persistent grid smaller than the
    tile count."""
    n = rows * cols
    ops = W.rqc_grid(rows, cols, cycles, 51 + n)
    c = _jit_circuit(n, ops, tile_bits=tile, low_bits=low, remap=1, grid_blocks=grid)
    assert c.stats()["n_fwd_moves"] > 0
    psi0 = W.random_state(n, 6 + n)
    st = State(n, init=psi0)
    c.apply(st)
    assert maxdiff(st.numpy(), oracle.run(n, ops, init=psi0)) < AMP_TOL
    st = State(n)
    ms = c.apply_timed(st)
    assert len(ms) == c.stats()["n_passes"]
    assert maxdiff(st.numpy(), oracle.run(n, ops)) < AMP_TOL


def test_batch_of_one_circuit_specialised():
    """A batch whose items share one circuit runs its forward steps on the
    specialised kernels (items with their own theta and qubit-move buffers)."""
    n, L, Bn = 13, 4, 5
    ops = W.hea(n, L)
    P = W.count_params(ops)
    th = W.theta_uniform(77, Bn, P)
    c = _jit_circuit(n, ops, remap=1)
    theta = torch.tensor(th, device="cuda")
    states = [torch.empty(1 << n, dtype=torch.complex128, device="cuda") for _ in range(Bn)]
    bt = Batch([c] * Bn, states, [theta[b] for b in range(Bn)])
    terms = W.tfim(n, 1.0)
    grads = [torch.zeros(P, dtype=torch.float64, device="cuda") for _ in range(Bn)]
    en = torch.zeros(Bn, dtype=torch.float64, device="cuda")
    bt.forward()
    for b in (0, Bn - 1):
        assert maxdiff(states[b].cpu().numpy(), oracle.run(n, ops, th[b])) < AMP_TOL
    bt.backward(terms, grads, en)
    for b in (0, 2, Bn - 1):
        e_ref, g_ref, _ = oracle.grad_pure(n, ops, th[b], terms)
        assert abs(en[b].item() - e_ref) < AMP_TOL
        assert maxdiff(grads[b].cpu().numpy(), g_ref) < GRAD_TOL


def test_code_cache_reused(tmp_path):
    """The second circuit of the same structure loads its code object from the
    cache (different angles: the parameters are read at run time)."""
    old = os.environ.get("VQC_JIT_CACHE")
    os.environ["VQC_JIT_CACHE"] = str(tmp_path)
    try:
        n = 11
        ops = W.hea(n, 3)
        P = W.count_params(ops)
        c1 = _jit_circuit(n, ops)
        assert not c1.stats()["jit_cached"]
        assert len(list(tmp_path.iterdir())) == 1
        c2 = _jit_circuit(n, ops)
        assert c2.stats()["jit_cached"]
        th = W.theta_uniform(5, 1, P)[0]
        st = State(n)
        c2.apply(st, torch.tensor(th, device="cuda"))
        assert maxdiff(st.numpy(), oracle.run(n, ops, th)) < AMP_TOL
    finally:
        if old is None:
            del os.environ["VQC_JIT_CACHE"]
        else:
            os.environ["VQC_JIT_CACHE"] = old


@pytest.mark.parametrize("env", [{"VQC_JIT_FWD_SPLIT": "0"}, {"VQC_JIT_HSQRT": "0"}, {"VQC_JIT_RECFREE": "0"},
                                 {"VQC_JIT_ADJ_SPLIT": "2"}, {"VQC_JIT_ADJ_SPLIT": "0"},
                                 {"VQC_JIT_ADJ_SPLIT": "0", "VQC_JIT_ADJ_SWZ": "1"},
                                 {"VQC_JIT_FWD_SPLIT": "0", "VQC_JIT_HSQRT": "0", "VQC_JIT_RECFREE": "0"}])
def test_specialised_pass_variants(env, monkeypatch):
    """The specialised passes' alternative forms (whole-amplitude LDS tile,
    rotation forms of the sqrt gates, a program entry read by every op, the
    adjoint on whole amplitudes or on its older driver with the fixed fold or a
    searched swizzle) give the oracle's state and
    gradient: a random grid circuit with qubit moves (sqrt gates, fSim) and
    the mixed-kind circuit."""
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    n = 20
    ops = W.rqc_grid(4, 5, 8, 71)
    c = _jit_circuit(n, ops, tile_bits=11, low_bits=4, remap=1)
    psi0 = W.random_state(n, 9)
    st = State(n, init=psi0)
    c.apply(st)
    assert maxdiff(st.numpy(), oracle.run(n, ops, init=psi0)) < AMP_TOL
    n = 12
    ops, th = _mixed_gate_circuit(n, 812, 9)
    c = _jit_circuit(n, ops, tile_bits=11, low_bits=3, reg_bits=3, remap=1)
    tht = torch.tensor(th, device="cuda")
    st = State(n)
    c.apply(st, tht)
    terms = W.heisenberg_1d(n, 0.3, 1.0)
    g, e = c.backward(tht, st, terms)
    e_ref, g_ref, _ = oracle.grad_pure(n, ops, th, terms)
    assert abs(e - e_ref) < AMP_TOL
    assert maxdiff(g.cpu().numpy(), g_ref) < GRAD_TOL
