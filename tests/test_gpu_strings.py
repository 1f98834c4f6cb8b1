"""The string family of the fitting layer and the learned proposal: a
Kirchhoff-Carrier string parameterised by theta = (T0^, EI^, L, d1^, d3^)
(fit.StringSetup), its autograd function through the GPU time loop and the
adjoint kernel (fit.StringFn), fitting with it, and a proposal network
trained on batched string simulations.  Inputs: seeded draws
(workloads.string_fit, the proposal priors); no data is read.

Bars: forward output to 1e-5 rel L2 against the FP64 oracle; the
theta-gradient, driven by the oracle's own dL/dy of the spectral-convergence
loss, to 1e-3 per component against the oracle's reverse recursion + chain
rule (oracle.params.string_theta_gradient)."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as OA
from oracle import losses as OL
from oracle import params as OP

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _setup(sf):
    from paper_2505_05940_amd import fit
    return fit.StringSetup(n_modes=sf["n_modes"], EAhat=sf["EAhat"], pluck=sf["pluck"], out=sf["out"],
                           proj_cells=sf["proj_cells"], fs=sf["fs"])


def test_stringfn_forward_and_gradient_against_oracle():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2505_05940_amd import fit
    sf = W.string_fit()
    st = _setup(sf)
    steps, fs = sf["n_steps"], sf["fs"]
    th0, tht = sf["theta0"], sf["theta_target"]
    _say(f"case: StringFn, 20-mode string, {steps} steps")
    y_o = OA.forward(OP.string_from_theta(sf, th0), steps, fs)[0]
    y_t = OA.forward(OP.string_from_theta(sf, tht), steps, fs)[0]
    ybar = OL.mrstft_loss_grad(y_o, y_t, log_term=False)
    g_o = OP.string_theta_gradient(sf, th0, steps, fs, ybar)
    theta = torch.tensor(th0[None], dtype=torch.float64, requires_grad=True)
    y = fit.StringFn.apply(theta, st, steps)
    e = float(np.linalg.norm(y[0].detach().double().cpu().numpy() - y_o) / np.linalg.norm(y_o))
    _say(f"  forward rel L2 {e:.2e}")
    assert e < 1e-5, e
    y.backward(torch.tensor(ybar, dtype=torch.float32, device="cuda").reshape(1, -1))
    g = theta.grad.numpy()[0]
    err = np.abs(g - g_o) / np.abs(g_o)
    _say(f"  gradient {g} / oracle {g_o}, rel err {err}")
    assert err.max() < 1e-3, err


def test_string_damping_fit():
    """fit.fit on a string with only d1^ and d3^ free, from 1.3 and 0.7 times
    the target, MR-STFT loss over 0.25 s: recovers both to 1e-3."""
    import torch
    from paper_2505_05940_amd import fit, modal
    sf = W.string_fit()
    st = _setup(sf)
    steps = sf["n_steps"]
    tgt = sf["theta_target"].copy()
    sim = modal.Sim([fit.string_instance(st, tgt)], sf["fs"])
    target = sim.run(steps).clone()
    sim.close()
    th0 = tgt.copy()
    th0[3] *= 1.3
    th0[4] *= 0.7
    _say("case: fit.fit, string damping d1^ and d3^, from (1.3, 0.7) x target")
    best, L, its, _ = fit.fit(target, th0, st, steps, iters=200, lr=0.02, tol=0.0, free=[3, 4])
    rel = np.abs(best[0][3:] / tgt[3:] - 1.0)
    _say(f"  best d1^, d3^ {best[0][3:]} target {tgt[3:]} rel {rel} loss {L[0]:.2e}")
    assert np.allclose(best[0][:3], th0[:3], rtol=1e-12, atol=0)
    assert rel.max() < 1e-3, rel


def test_string_proposal_beats_prior_centre():
    import torch
    from paper_2505_05940_amd import fit, proposal
    from paper_2505_05940_amd.mlp import MLP
    sf = W.string_fit(n_modes=12)  # as the benchmark's string proposal
    st = _setup(sf)
    base = sf["theta0"]
    steps, n_train, n_test = 8820, 32768, 128
    _say(f"case: string proposal, 12 modes, {n_train} sims x {steps} steps")
    th_train = proposal.sample_prior(np.random.default_rng(5), n_train, base, "string")
    X = proposal.features(proposal.simulate(st, th_train, steps))
    Z = torch.tensor(proposal.normalize(th_train, base, "string"), dtype=torch.float32, device="cuda")
    net = MLP(proposal.DIMS, max_batch=1024)
    net.init_params(seed=1)
    mse = proposal.train(net, X, Z, epochs=15)
    th_test = proposal.sample_prior(np.random.default_rng(50), n_test, base, "string")
    z = proposal.predict(net, proposal.features(proposal.simulate(st, th_test, steps)))
    err_prop = proposal.param_error(proposal.denormalize(z, base, "string"), th_test, base, "string")
    err_default = proposal.param_error(np.tile(proposal.prior_center(base, "string"), (n_test, 1)), th_test,
                                       base, "string")
    _say(f"  train mse {mse:.4f}; mean |z error| proposal {err_prop.mean():.3f}, "
         f"prior centre {err_default.mean():.3f}")
    assert np.isfinite(mse) and mse < 0.2
    assert err_prop.mean() < 0.5 * err_default.mean()
