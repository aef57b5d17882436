"""User-facing forms of Sec. 2.3-2.4: nested QCircuits, apply(circ, state) /
circ * state out of place, against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2406_19212_amd import Circuit, State
from paper_2406_19212_amd import workloads as W
from paper_2406_19212_amd.workloads import Op

pytestmark = pytest.mark.gpu


def test_nested_circuit_and_out_of_place_apply():
    n = 9
    ops, th = W.brickwall(n, 4, 121)
    inner = Circuit(n, ops[:40], n_params=len(th))
    nested = Circuit(n, [inner, [ops[40:70], [ops[70:]]]], n_params=len(th))
    assert len(nested.ops) == len(ops)
    tht = torch.tensor(th, device="cuda")
    src = State(n, init=W.random_state(n, 122))
    before = src.numpy().copy()
    out = nested.apply_out(src, tht)
    assert np.array_equal(src.numpy(), before)
    want = oracle.run(n, ops, th, init=before)
    assert np.max(np.abs(out.numpy() - want)) < 1e-12
    # circ * state for a circuit without variational parameters, pure and mixed
    fixed = [Op("h", (0,)), Op("cnot", (0, 1)), Op("toffoli", (0, 1, 2)), Op("sw", (3,))]
    c = Circuit(4, fixed)
    s0 = State(4)
    s1 = c * s0
    assert np.max(np.abs(s1.numpy() - oracle.run(4, fixed))) < 1e-12
    assert abs(s0.numpy()[0] - 1) == 0
    cm = Circuit(3, fixed[:3] + [Op("depolarizing", (2,), (0.1,))], mixed=True)
    r1 = cm * State(3, mixed=True)
    assert np.max(np.abs(r1.numpy() - oracle.run(3, cm.ops, mixed=True))) < 1e-12
