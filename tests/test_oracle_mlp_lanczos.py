"""Pins for the surrogate-network oracle (finite differences, the normal CDF)
and for the Lanczos ground energy (dense diagonalisation, free fermions)."""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla
from scipy.stats import norm

from oracle import lanczos
from oracle import mlp as omlp
from paper_2406_19212_amd import workloads as W

DIMS = (5, 4, 3)


def _params(seed, dims=DIMS):
    n_in, h1, h2 = dims
    count = h1 * n_in + h1 + h2 * h1 + h2 + h2 + 1
    return W.SplitMix64(seed).normal(count) * 0.7


def test_gelu_is_x_times_normal_cdf():
    import torch
    x = np.linspace(-6, 6, 41)
    assert np.max(np.abs(omlp.gelu(torch.tensor(x)).numpy() - x * norm.cdf(x))) < 1e-15


@pytest.mark.parametrize("lam", [0.0, 0.8])
def test_mlp_gradient_matches_finite_differences(lam):
    p = _params(3)
    rng = np.random.default_rng(4)
    x = rng.normal(size=(3, DIMS[0]))
    e = rng.normal(size=3)
    g = rng.normal(size=(3, DIMS[0]))
    L, dP, y, gx = omlp.loss_and_grads(p, x, e, g, lam, DIMS)
    h = 1e-6
    for k in range(p.size):
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (omlp.loss_and_grads(pp, x, e, g, lam, DIMS)[0] - omlp.loss_and_grads(pm, x, e, g, lam, DIMS)[0]) / (2 * h)
        assert abs(fd - dP[k]) < 1e-7 * max(1.0, abs(fd))
    # dy/dx against finite differences of the forward
    for b in range(3):
        for i in range(DIMS[0]):
            xp, xm = x.copy(), x.copy()
            xp[b, i] += h
            xm[b, i] -= h
            fd = (omlp.forward(p, xp, DIMS)[b] - omlp.forward(p, xm, DIMS)[b]).item() / (2 * h)
            assert abs(fd - gx[b, i]) < 1e-7


def test_mlp_loss_definition_by_hand():
    # one sample, explicit formula with numpy
    p = _params(5)
    x = np.array([[0.3, -0.2, 0.5, 0.1, -0.7]])
    prm = {k: v.numpy() if hasattr(v, "numpy") else v for k, v in omlp.unpack(p, *DIMS).items()}
    z1 = prm["W1"] @ x[0] + prm["b1"]
    h1 = z1 * norm.cdf(z1)
    z2 = prm["W2"] @ h1 + prm["b2"]
    y = prm["w3"] @ (z2 * norm.cdf(z2)) + prm["b3"][0]
    assert abs(omlp.forward(p, x, DIMS)[0].item() - y) < 1e-14


@pytest.mark.parametrize("n", [2, 3, 6, 9])
def test_free_fermion_matches_dense(n):
    H = lanczos.sparse_hamiltonian(n, W.tfim(n, 0.7)).toarray()
    assert np.allclose(H, H.conj().T)
    e0 = np.linalg.eigvalsh(H)[0]
    assert abs(lanczos.tfim_free_fermion(n, 0.7) - e0) < 1e-11


def test_lanczos_matches_dense_and_closed_form():
    n = 8
    terms = W.tfim(n, 1.0)
    e_l = lanczos.ground_energy(n, terms)
    H = lanczos.sparse_hamiltonian(n, terms)
    e_d = np.linalg.eigvalsh(H.toarray())[0]
    assert abs(e_l - e_d) < 1e-10
    assert abs(e_l - lanczos.tfim_free_fermion(n, 1.0)) < 1e-10
    # a Hamiltonian with Y terms (Listing 5's Heisenberg chain)
    hz = W.heisenberg_1d(6, 0.4, 1.0)
    H = lanczos.sparse_hamiltonian(6, hz).toarray()
    assert abs(lanczos.ground_energy(6, hz) - np.linalg.eigvalsh(H)[0]) < 1e-10


@pytest.mark.slow
def test_lanczos_tfim_12():
    n = 12
    e = lanczos.ground_energy(n, W.tfim(n, 1.0))
    assert abs(e - lanczos.tfim_free_fermion(n, 1.0)) < 1e-10


def test_surrogate_target_ground_energy():
    """The surrogate experiment's stated ground energy (16-qubit open chain,
    J = h = 1) is the free-fermion value, itself pinned to dense
    diagonalisation and Lanczos above."""
    from paper_2406_19212_amd.surrogate import GROUND_E_TFIM16
    assert abs(lanczos.tfim_free_fermion(16, 1.0) - GROUND_E_TFIM16) < 1e-12
