"""The 28-qubit random grid circuit at its full size, in the launch
configuration the benchmark times (default tile 11, 4 low qubits, 4 register
bits, qubit moves): the first 8 cycles against the oracle amplitude by
amplitude (the whole 4 GiB state, compared in chunks), and the full 20-cycle
circuit through properties that hold at any size -- unit norm, and the
circuit followed by its inverse (each gate's conjugate transpose as a dense
matrix op, taken from the oracle's gate matrices) returning |0...0>."""
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
