"""Surrogate-assisted optimisation: the loop's invariants and the network's
ability to learn an informative landscape from simulator labels."""
import numpy as np
import pytest
import torch

from paper_2406_19212_amd import surrogate
from paper_2406_19212_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_labels_match_single_item_simulator():
    sim = surrogate.Simulator(8, 2, batch=16)
    theta = torch.tensor(W.theta_uniform(5, 20, sim.P), device="cuda")
    E, G = sim.batch_energy_grad(theta)
    for i in (0, 7, 19):
        e, g = sim.energy_grad(theta[i].contiguous())
        assert abs(E[i].item() - e) < 1e-12
        assert torch.max(torch.abs(G[i] - g)).item() < 1e-10


def test_network_learns_local_landscape():
    """Trained on labels around one point, the network predicts held-out
    energies far better than the label spread and its input gradient points
    along the exact gradient."""
    sim = surrogate.Simulator(10, 3, batch=256)
    rng = W.SplitMix64(11)
    theta0 = torch.tensor(W.theta_uniform(3, 1, sim.P)[0], device="cuda")
    noise = torch.tensor(rng.normal(3000 * sim.P).reshape(3000, sim.P) * 0.15, device="cuda")
    theta = theta0 + noise
    E, G = sim.batch_energy_grad(theta)
    scale = (float(E.mean()), float(E.std()))
    net = surrogate.MLP(sim.P, 256, 256, max_batch=512)
    surrogate.init_params(net, 4)
    e_hat0, _ = surrogate.predict(net, theta[2500:], scale)
    surrogate.train(net, theta[:2500], E[:2500], G[:2500], epochs=40, scale=scale, batch=250)
    e_hat, g_hat = surrogate.predict(net, theta[2500:], scale)
    rmse = float((e_hat - E[2500:]).pow(2).mean().sqrt())
    rmse0 = float((e_hat0 - E[2500:]).pow(2).mean().sqrt())
    cos = float(torch.nn.functional.cosine_similarity(g_hat, G[2500:], dim=1).mean())
    print("local model: rmse %.4f (untrained %.4f, label std %.4f), grad cos %.3f" % (rmse, rmse0, E.std(), cos))
    # better than the constant predictor (the label spread) and than the untrained net
    assert rmse < 0.8 * float(E[2500:].std()) and rmse < 0.3 * rmse0
    assert cos > 0.5


def test_surrogate_loop_accounting_and_verification():
    """Every outer step is one accepted proposal or one exact Adam fallback,
    the history's evaluation count is the simulator's, and the last energy
    is the exact energy of the returned theta."""
    sim = surrogate.Simulator(8, 2, batch=64)
    theta, E, G = surrogate.generate(sim, 512, 9)
    scale = (float(E.mean()), float(E.std()))
    net = surrogate.MLP(sim.P, 128, 128, max_batch=512)
    surrogate.init_params(net, 2)
    surrogate.train(net, theta, E, G, epochs=3, scale=scale)
    theta0 = torch.tensor(W.theta_uniform(8, 1, sim.P)[0], device="cuda")
    sim.evals = 0
    th, hist, log = surrogate.optimize_surrogate(sim, net, scale, theta0, steps=25, lr=0.05, finetune=3)
    energies = [h[2] for h in hist]
    # an accepted proposal always lowers the verified energy; a fallback is one exact Adam step
    assert log["accepted"] + log["fallback"] == 25
    assert min(energies) < energies[0]
    assert hist[-1][1] == sim.evals >= 26
    e, _ = sim.energy_grad(th)
    assert abs(e - energies[-1]) < 1e-12


def test_trained_network_gains_over_the_loop_without_it():
    """The 16-qubit, 10-layer ansatz from the benchmark's theta_0, with the
    loop's default step size (lr 0.05).  Without the network every step of
    the loop is its exact Adam fallback, i.e. plain Adam at that step size;
    at equal exact evaluations the network's proposals reach a much lower
    energy (plain Adam at this step size settles near E - E0 = 1.33).  With
    a tuned step size plain Adam reaches the target faster than the loop,
    which the benchmark's comparison records."""
    sim = surrogate.Simulator(16, 10, batch=256)
    seed = 240619216
    theta, E, G = surrogate.generate(sim, 50000, seed)
    scale = (float(E.mean()), float(E.std()))
    net = surrogate.MLP(sim.P, 512, 512, max_batch=512)
    surrogate.init_params(net, seed + 1)
    surrogate.train(net, theta, E, G, epochs=30, scale=scale)
    del theta, E, G
    theta0 = torch.tensor(W.theta_uniform(seed + 2, 1, sim.P)[0], device="cuda")
    sim.evals = 0
    _, hs, log = surrogate.optimize_surrogate(sim, net, scale, theta0, steps=300, lr=0.05)
    evals = hs[-1][1]
    sim.evals = 0
    _, hp = surrogate.optimize_plain(sim, theta0, evals, 0.05)
    assert hp[-1][1] == evals
    e0 = surrogate.GROUND_E_TFIM16
    gap_s, gap_p = hs[-1][2] - e0, hp[-1][2] - e0
    print("after %d exact evaluations: loop with network E-E0 %.4f (%d accepted), plain Adam %.4f"
          % (evals, gap_s, log["accepted"], gap_p))
    assert gap_s < 0.75 * gap_p
