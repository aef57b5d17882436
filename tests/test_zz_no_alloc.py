"""The allocation-free expectation entry point (vqc_expectation_noalloc):
its fixed per-GPU scratch gives the same value as vqc_expectation on
consecutive calls of shrinking size, pure and mixed, and inputs beyond the
scratch are refused before any work is queued."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2406_19212_amd import State, binding as B
from paper_2406_19212_amd import workloads as W

pytestmark = pytest.mark.gpu

AMP_TOL = 1e-12


def _terms(n, seed, count):
    """Random Pauli strings with complex coefficients (X, Y and Z letters)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        letters = rng.integers(0, 4, n)
        xm = zm = 0
        for q, l in enumerate(letters):
            if l in (1, 2):
                xm |= 1 << q
            if l in (2, 3):
                zm |= 1 << q
        out.append((xm, zm, complex(rng.normal(), rng.normal())))
    return out


def _both(st, terms):
    ps = B.PauliSum(terms)
    a, b = B.vqc_c128(), B.vqc_c128()
    B.check(B.lib().vqc_expectation(st.h, ps.ref(), ctypes.byref(a)), "vqc_expectation")
    B.check(B.lib().vqc_expectation_noalloc(st.h, ps.ref(), ctypes.byref(b)), "vqc_expectation_noalloc")
    return complex(a.re, a.im), complex(b.re, b.im)


def test_noalloc_matches_expectation_twice_shrinking():
    # first call: 22 qubits (1024 first-stage partials) and 60 terms;
    # second: 10 qubits and 7 terms, so stale partials of the first call lie
    # beyond the second call's range
    for n, count, seed in ((22, 60, 5), (10, 7, 6)):
        psi = W.random_state(n, seed)
        st = State(n, init=psi)
        terms = _terms(n, seed + 100, count)
        ref, got = _both(st, terms)
        assert abs(got - ref) <= AMP_TOL, (n, got, ref)
        assert got == ref  # same kernels, same fixed summation order
        if n <= 10:
            want = oracle.expectation(psi, n, terms)
            assert abs(got - want) <= AMP_TOL, (got, want)


def test_noalloc_mixed_and_tfim():
    n = 7
    rho = W.random_density(n, 31).reshape(-1, order="F").copy()  # v[x + 2^n y] = rho[x][y]
    st = State(n, mixed=True, init=rho)
    terms = W.tfim(n, 1.0) + _terms(n, 32, 5)
    ref, got = _both(st, terms)
    assert got == ref
    want = oracle.expectation(rho, n, terms, mixed=True)
    assert abs(got - want) <= AMP_TOL, (got, want)
    # then a smaller mixed state
    st2 = State(3, mixed=True, init=W.random_density(3, 33).reshape(-1, order="F").copy())
    ref2, got2 = _both(st2, W.tfim(3, 0.5))
    assert got2 == ref2


def test_noalloc_limits_refused():
    st = State(6, init=W.random_state(6, 41))
    ps = B.PauliSum([(0, 1, 1.0)] * 1025)
    out = B.vqc_c128()
    assert B.lib().vqc_expectation_noalloc(st.h, ps.ref(), ctypes.byref(out)) == -12
    # 2^29 amplitudes need more first-stage partials than the scratch holds
    big = State(29)
    ps1 = B.PauliSum([(0, 1, 1.0)])
    assert B.lib().vqc_expectation_noalloc(big.h, ps1.ref(), ctypes.byref(out)) == -12
    del big
    torch.cuda.empty_cache()
    # the largest size it takes: 28 qubits, |0..0> gives <Z_0> = 1
    top = State(28)
    assert top.expectation_noalloc([(0, 1, 1.0), (0, 0, 0.5)]) == complex(1.5, 0.0)
