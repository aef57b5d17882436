"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments on the host before any launch."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2406_19212_amd import binding as B
from paper_2406_19212_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vqc.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vqc_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libvqc.so not built")
    return B.lib()


def test_header_declares_the_boundary():
    names = declared()
    for n in ("vqc_state_init", "vqc_apply_gate", "vqc_apply_channel", "vqc_expectation", "vqc_backward"):
        assert n in names


def test_library_exports_every_declared_symbol(L):
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(declared()) <= set(B._SIGS)


def test_status_strings(L):
    assert L.vqc_status_string(0) == b"ok"
    assert b"qubit" in L.vqc_status_string(-2)
    assert L.vqc_version() >= 100


def test_mat_from_external_cnot(L):
    # textbook CNOT with the control as the most significant bit
    tb = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], np.complex128)
    out = np.zeros(16, np.complex128)
    B.check(L.vqc_mat_from_external(2, np.ascontiguousarray(tb).ctypes.data, out.ctypes.data), "x")
    G = out.reshape(4, 4).T  # column-major -> row-major G[out][in]
    # native layout: control = local bit 0, target = local bit 1: |c=1,t=0> (1) -> |c=1,t=1> (3)
    ref = np.zeros((4, 4))
    ref[0, 0] = ref[2, 2] = ref[3, 1] = ref[1, 3] = 1
    assert np.array_equal(G, ref)


def test_mat_from_external_is_bit_reversal(L):
    U = W.random_unitary(8, 3)
    out = np.zeros(64, np.complex128)
    B.check(L.vqc_mat_from_external(3, np.ascontiguousarray(U).ctypes.data, out.ctypes.data), "x")
    G = out.reshape(8, 8).T
    rev = [int(format(i, "03b")[::-1], 2) for i in range(8)]
    assert np.array_equal(G, U[np.ix_(rev, rev)])
    assert L.vqc_mat_from_external(5, None, None) == -1


def _create(L, n, ops, mixed=False, n_params=None):
    arr = B.OpArray(ops)
    h = ctypes.c_void_p()
    np_ = W.count_params(ops) if n_params is None else n_params
    return L.vqc_circuit_create(ctypes.byref(h), n, 1 if mixed else 0, arr.n, arr.ptr(), np_, None)


def test_circuit_create_rejects_bad_ops_on_host(L):
    Op = W.Op
    assert _create(L, 3, [Op("h", (3,))]) == -2                      # out of range
    assert _create(L, 3, [Op("cz", (1, 1))]) == -2                   # repeated qubit
    assert _create(L, 3, [Op("cz", (0,))]) == -1                     # arity mismatch
    assert _create(L, 3, [Op("depolarizing", (0,), (0.1,))]) == -4   # channel on a pure circuit
    assert _create(L, 3, [Op("rx", (0,), (float("nan"),))]) == -6    # non-finite
    assert _create(L, 3, [Op("rx", (0,), (0.1,), (5,))], n_params=2) == -1  # theta index out of range
    bad = [np.eye(2) * 0.9, np.eye(2) * 0.1]
    assert _create(L, 2, [Op("kraus", (0,), (), (), bad)], mixed=True) == -5  # not trace preserving
    assert _create(L, 2, [Op("matrix", (0, 1, 2), (), (), np.eye(8))]) == -2  # qubit 2 of 2
    assert _create(L, 3, [Op("kraus", (0, 1, 2), (), (), [np.eye(8)])]) == -4  # a channel on a pure circuit
    assert _create(L, 3, [Op("matrix", (0, 1, 2), (), (), np.eye(4))]) == -1  # 8 x 8 data needed
    assert _create(L, 4, [Op("matrix", (0, 1, 2, 3), (), (), np.eye(16))]) == -3  # m = 4
    assert _create(L, 3, [Op("toffoli", (0, 1))]) == -1                         # arity
    assert _create(L, 3, [Op("ccontrol", (0, 1, 2), (), (), np.eye(2) * 2)]) == -10  # V needs a unitary U
    K3 = [np.eye(8)]
    K3bad = [1.01 * k for k in K3]
    assert _create(L, 3, [Op("kraus", (0, 1, 2), (), (), K3bad)], mixed=True) == -5  # 3q channel, not CPTP


def test_state_init_rejects_bad_sizes_on_host(L):
    h = ctypes.c_void_p()
    assert L.vqc_state_init(ctypes.byref(h), 0, 0, ctypes.c_void_p(1), None, None) == -1
    assert L.vqc_state_init(ctypes.byref(h), 0, 40, ctypes.c_void_p(1), None, None) == -1
    assert L.vqc_state_init(ctypes.byref(h), 1, 17, ctypes.c_void_p(1), None, None) == -1
    assert L.vqc_state_init(ctypes.byref(h), 0, 4, None, None, None) == -1


def test_new_entry_points_reject_bad_arguments_on_host(L):
    P = ctypes.c_void_p
    o, p = ctypes.c_int(), ctypes.c_double()
    assert L.vqc_measure(None, 0, 0.5, ctypes.byref(o), ctypes.byref(p)) == -1
    assert L.vqc_sample(None, 4, None, None) == -1
    assert L.vqc_backward_inverse(None, None, None, None, None, None, 0.0) == -1
    assert L.vqc_batch_backward_inverse(None, None, None, None, 0.0) == -1
    assert L.vqc_apply_circuit_out(None, None, None, None) == -1
    n_out = ctypes.c_int()
    assert L.vqc_fuse_gates(3, 1, None, 0, None, None, None, ctypes.byref(n_out)) == -1  # no ops array
    assert L.vqc_fuse_gates(0, 0, None, 0, None, None, None, ctypes.byref(n_out)) == -1  # n out of range
    # validation before any device work: a channel (noiseless only), a wide op, a bad theta index
    for ops, code in (([W.Op("depolarizing", (0,), (0.1,))], -4),
                      ([W.Op("toffoli", (0, 1, 2))], -3),
                      ([W.Op("rx", (0,), (0.1,), (3,))], -1)):
        arr = B.OpArray(ops)
        out = (B.vqc_op * 4)()
        data = np.zeros(64, np.complex128)
        th = np.zeros(2)
        assert L.vqc_fuse_gates(3, arr.n, arr.ptr(), 2, th.ctypes.data, ctypes.cast(out, P), data.ctypes.data,
                                ctypes.byref(n_out)) == code


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU only: --gpus above 1 exits with status 2
    and a message, before any GPU work."""
    import subprocess
    import sys
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(here, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_bench_traffic_only_for_the_recorded_sources(tmp_path, monkeypatch):
    """The bench line's measured HBM traffic comes from the committed counter
    summary only while the kernel sources have the digest recorded there;
    another digest, a missing file or a malformed figure gives null."""
    import sys
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, here)
    import bench
    f = tmp_path / "traffic.txt"
    f.write_text("# comment: with a colon\nsource_digest: %s\nbytes_per_pass: 8591374339\n" % bench.kernel_digest())
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic() == 8591374339.0
    f.write_text("source_digest: 0000000000000000\nbytes_per_pass: 8591374339\n")
    assert bench.measured_traffic() is None
    f.write_text("source_digest: %s\nbytes_per_pass: n/a\n" % bench.kernel_digest())
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic() is None
