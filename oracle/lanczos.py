"""Ground energy of a Pauli-sum Hamiltonian by Lanczos (test infrastructure).

The surrogate-assisted optimisation aims at the exact ground energy of the
transverse-field Ising chain; the paper gives no method for it.  Lanczos
(C. Lanczos 1950) with full reorthogonalisation in float64 on the sparse
matrix built term by term from the Pauli definition P|x> = i^{|Y|}
(-1)^{popcount(x & z)} |x ^ x_mask>; stops when the Ritz residual
|beta_k s_k| of the lowest Ritz pair falls below tol.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def sparse_hamiltonian(n: int, terms):
    N = 1 << n
    x = np.arange(N, dtype=np.int64)
    H = sp.csr_matrix((N, N), dtype=np.complex128)
    for xm, zm, c in terms:
        ny = bin(xm & zm).count("1") & 3
        ph = (1, 1j, -1, -1j)[ny]
        par = np.array([bin(v).count("1") & 1 for v in (x & zm)], dtype=np.int64) if n <= 12 else \
            _parity(x & zm)
        vals = complex(c) * ph * (1 - 2 * par)
        H = H + sp.csr_matrix((vals, (x ^ xm, x)), shape=(N, N))
    return H


def _parity(v):
    v = v.copy()
    p = np.zeros_like(v)
    while np.any(v):
        p ^= v & 1
        v >>= 1
    return p


def ground_energy(n: int, terms, tol: float = 1e-10, max_iter: int = 400, seed: int = 1):
    H = sparse_hamiltonian(n, terms)
    N = H.shape[0]
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(N) + 0j
    v /= np.linalg.norm(v)
    V = [v]
    alpha, beta = [], []
    w = H @ v
    for k in range(max_iter):
        a = np.vdot(V[-1], w).real
        alpha.append(a)
        w = w - a * V[-1] - (beta[-1] * V[-2] if beta else 0)
        for u in V:  # full reorthogonalisation
            w = w - np.vdot(u, w) * u
        b = np.linalg.norm(w)
        T = np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1)
        ev, evec = np.linalg.eigh(T)
        if b * abs(evec[-1, 0]) < tol or b < 1e-14:
            return float(ev[0])
        beta.append(b)
        V.append(w / b)
        w = H @ V[-1]
    raise RuntimeError("Lanczos did not converge")


def tfim_free_fermion(n: int, h: float = 1.0, J: float = 1.0) -> float:
    """Closed form for the open chain J sum Z_i Z_{i+1} + h sum X_i (Pfeuty
    1970): E0 = -sum of the singular values of the n x n upper-bidiagonal
    matrix with diagonal h and superdiagonal J."""
    M = np.diag(np.full(n, float(h))) + np.diag(np.full(n - 1, float(J)), 1)
    return float(-np.linalg.svd(M, compute_uv=False).sum())
