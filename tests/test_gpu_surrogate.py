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


def test_surrogate_loop_is_monotone_and_verified():
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
