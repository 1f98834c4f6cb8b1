"""What the learned proposal gains over the method without it: a network
trained on simulator output (batched dense path, hand-written MLP kernels)
maps held-out target sounds to parameters much closer to the truth than the
default initialisation (the prior centre) that plain fitting starts from.
Inputs: seeded draws from the proposal priors; no data is read."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_proposal_beats_prior_centre():
    import torch
    assert torch.cuda.is_available()
    from paper_2505_05940_amd import fit, proposal
    from paper_2505_05940_amd.mlp import MLP
    steps, n_train, n_test = 8820, 32768, 128
    setup = fit.PlateSetup(n_t=24, n_in=24)
    base = W.plate_fit(n_t=24)["theta0"]
    print(f"case: proposal 24/24 modes, {n_train} sims x {steps} steps", flush=True)
    th_train = proposal.sample_prior(np.random.default_rng(5), n_train, base)
    X = proposal.features(proposal.simulate(setup, th_train, steps))
    Z = torch.tensor(proposal.normalize(th_train, base), dtype=torch.float32, device="cuda")
    net = MLP(proposal.DIMS, max_batch=1024)
    net.init_params(seed=1)
    mse = proposal.train(net, X, Z, epochs=15)
    th_test = proposal.sample_prior(np.random.default_rng(50), n_test, base)
    z = proposal.predict(net, proposal.features(proposal.simulate(setup, th_test, steps)))
    err_prop = proposal.param_error(proposal.denormalize(z, base), th_test, base)
    err_default = proposal.param_error(np.tile(proposal.prior_center(base), (n_test, 1)), th_test, base)
    print(f"train mse {mse:.4f}; mean |z error| proposal {err_prop.mean():.3f}, "
          f"prior centre {err_default.mean():.3f}", flush=True)
    assert np.isfinite(mse) and mse < 0.2
    assert err_prop.mean() < 0.5 * err_default.mean()
    assert np.median(err_prop) < np.median(err_default)
