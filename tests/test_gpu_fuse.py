"""fuse_gates through the C ABI against the oracle's fuse_gates, and the fused
circuit's state on the device against the original circuit's."""
import numpy as np
import pytest
import torch

import oracle
from paper_2406_19212_amd import Circuit, State, fuse_gates
from paper_2406_19212_amd import workloads as W
from paper_2406_19212_amd.binding import VQCError
from paper_2406_19212_amd.workloads import Op

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["brick", "hea", "rqc"])
def test_fuse_gates_matches_oracle(kind):
    if kind == "brick":
        n = 10
        ops, th = W.brickwall(n, 5, 81)
    elif kind == "hea":
        n = 8
        ops = W.hea(n, 4)
        th = W.theta_uniform(82, 1, W.count_params(ops))[0]
    else:
        n = 12
        ops, th = W.rqc_grid(3, 4, 8, 83), None
    fused = fuse_gates(n, ops, th)
    ref = oracle.fuse_gates(ops, th if th is not None else np.zeros(1))
    assert [tuple(o.qubits) for o in fused] == [q for q, _ in ref]
    assert max(float(np.max(np.abs(o.data - M))) for o, (_, M) in zip(fused, ref)) < 1e-14
    # the fused circuit on the device gives the original circuit's state
    c = Circuit(n, fused)
    st = State(n)
    c.apply(st)
    want = oracle.run(n, ops, th)
    assert float(np.max(np.abs(st.numpy() - want))) < 1e-12
    print("%s: %d ops -> %d" % (kind, len(ops), len(fused)))


def test_fuse_gates_errors():
    with pytest.raises(VQCError) as ei:
        fuse_gates(3, [Op("h", (0,)), Op("depolarizing", (1,), (0.1,))])
    assert ei.value.status == -4
    assert fuse_gates(3, []) == []
