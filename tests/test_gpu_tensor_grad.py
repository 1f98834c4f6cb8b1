"""Gradient with respect to every coupling-tensor entry (modal_grad's g_H,
through the C ABI) against the FP64 oracle's reverse pass, and the tensor
replacement entry point (modal_set_tensor) against the oracle's forward loop.

The loss is a seeded linear functional L = sum_n g_n y_n, so both sides
differentiate the same scalar.  Bar: relative L2 error of each instance's
tensor gradient <= 1e-4 (that of the other gradients of modal_grad)."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as OA
from oracle import instances as OI
from oracle import simulate as OS

pytestmark = pytest.mark.gpu

TOL = 1e-4


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available()
    from paper_2505_05940_amd import modal, physics
    return modal, physics, torch


def _plates():
    a = W.plate_vk(n_t=14, n_in=11, family="sine", grid=None, n_steps=800)
    a["strike"]["amplitude"] = 3e-3
    b = W.plate_vk(n_t=70, n_in=6, family="sine", grid=None, n_steps=800)
    b["strike"]["amplitude"] = 2e-3
    return a, b


@pytest.mark.parametrize("max_wg,ckpt,waves", [(0, 0, 4), (3, 128, 4), (3, 300, 1)])
def test_tensor_gradient_matches_oracle(gpu, max_wg, ckpt, waves):
    modal, physics, torch = gpu
    wa, wb = _plates()
    wk = W.string_kc(n_modes=12)
    steps = 800
    pinsts = [physics.plate_instance(wa), physics.string_instance(wk), physics.plate_instance(wb)]
    oinsts = [OI.plate_instance(wa), OI.string_instance(wk), OI.plate_instance(wb)]
    rng = np.random.default_rng(11)
    g = rng.normal(size=(3, steps))
    for b in range(3):
        g[b] /= np.abs(oinsts[b]["x0"]).max()
    print(f"case: tensor grad vK 14/11 + KC 12 + vK 70/6, {steps} steps, max_wg={max_wg}, "
          f"ckpt={ckpt}, waves={waves}", flush=True)
    sim = modal.Sim(pinsts, 44100.0, flags=modal.FLAG_GRAD | modal.FLAG_SPLIT_ANY,
                    max_workgroups=max_wg, waves=waves)
    if max_wg:
        assert sim.info()["split_instances"] >= 1
    res = sim.grad(steps, torch.tensor(g, dtype=torch.float32, device="cuda"), ckpt_every=ckpt,
                   tensor=True)
    assert res["H"][1] is None
    for b in (0, 2):
        ref = OA.reverse(oinsts[b], steps, 44100.0, g[b].astype(np.float32).astype(float),
                         full_tensor=True)
        G = res["H"][b].double().cpu().numpy()
        assert G.shape == ref["H"].shape
        assert rel(G, ref["H"]) < TOL, (b, rel(G, ref["H"]))
        # the row-scale gradients are the tensor gradient contracted with H row by row
        assert rel(np.einsum("nij,nij->n", G, oinsts[b]["Ht"]), ref["row"]) < TOL
    # only the asked instances; a second call overwrites
    res2 = sim.grad(steps, torch.tensor(g, dtype=torch.float32, device="cuda"), ckpt_every=ckpt,
                    tensor=[False, False, True])
    assert res2["H"][0] is None
    assert torch.equal(res2["H"][2], res["H"][2])


def test_set_tensor_replaces_the_dynamics(gpu):
    modal, physics, torch = gpu
    wa, _ = _plates()
    steps = 600
    p = physics.plate_instance(wa)
    o = OI.plate_instance(wa)
    rng = np.random.default_rng(12)
    S = rng.uniform(0.5, 1.5, size=o["Ht"].shape)
    Hn = (o["Ht"] * (S + S.transpose(0, 2, 1)) / 2).astype(np.float32)
    sim = modal.Sim([p], 44100.0, flags=modal.FLAG_GRAD)
    sim.set_tensor(0, torch.tensor(Hn, device="cuda"))
    sim.reset()
    y = sim.run(steps).double().cpu().numpy()[0]
    ref = OS.run(dict(o, Ht=Hn.astype(float)), steps, 44100.0)
    assert rel(y, ref) < 1e-5
    # host memory too, back to the original
    sim.set_tensor(0, o["Ht"].astype(np.float32))
    sim.reset()
    y0 = sim.run(steps).double().cpu().numpy()[0]
    assert rel(y0, OS.run(dict(o), steps, 44100.0)) < 1e-5
    # an asymmetric tensor is refused, from either memory, and changes nothing
    Ha = Hn.copy()
    Ha[2, 1, 5] += np.abs(Hn).max()
    for src in (Ha, torch.tensor(Ha, device="cuda")):
        with pytest.raises(RuntimeError, match="symmetric"):
            sim.set_tensor(0, src)
    sim.reset()
    assert np.array_equal(sim.run(steps).double().cpu().numpy()[0], y0)


def test_tensor_fit_from_random_start(gpu):
    """The coupling-tensor fit (random normal symmetric start, Adam on the
    symmetric part of the tensor gradient) on a strongly struck small plate:
    its first loss is the oracle's loss at the start, and 80 iterations cut
    the loss more than tenfold (the FP64 oracle run of the same loop reaches
    0.012 from 0.34)."""
    modal, physics, torch = gpu
    from paper_2505_05940_amd import fit
    steps = 2000
    wl = W.plate_vk(n_t=6, n_in=4, family="sine", grid=None, n_steps=steps)
    wl["strike"]["amplitude"] = 1.5e-2
    p = physics.plate_instance(wl)
    o = OI.plate_instance(wl)
    target = OS.run(o, steps, 44100.0)
    rng = np.random.default_rng(0)
    R = rng.normal(size=o["Ht"].shape)
    H0 = (0.5 * (R + R.transpose(0, 2, 1)) * np.sqrt(2 * np.mean(o["Ht"] ** 2))).astype(np.float32)

    def mse(y, t):
        return ((y - t) ** 2).sum() / (t ** 2).sum()

    print("case: tensor fit 6/4 modes, 2000 steps, 80 iterations", flush=True)
    tt = torch.tensor(target, dtype=torch.float32, device="cuda")
    best_H, best_L, hist = fit.fit_tensor(p, tt, H0, steps, iters=80, lr=0.05, loss_fn=mse)
    y0 = OS.run(dict(o, Ht=H0.astype(float)), steps, 44100.0)
    L0 = float(np.sum((y0 - target) ** 2) / np.sum(target ** 2))
    assert abs(hist[0] - L0) < 1e-4 * L0, (hist[0], L0)
    assert best_L < 0.1 * hist[0], (best_L, hist[0])
    Hb = best_H.cpu().numpy()
    assert np.array_equal(Hb, Hb.transpose(0, 2, 1))


def test_tensor_fit_parallel_starts(gpu):
    """Several random starts as one batch: each start's first loss is the
    oracle's at that start, and the starts run independently (the batch's
    first start follows the single-start fit of the same start exactly)."""
    modal, physics, torch = gpu
    from paper_2505_05940_amd import fit
    steps = 1500
    wl = W.plate_vk(n_t=6, n_in=4, family="sine", grid=None, n_steps=steps)
    wl["strike"]["amplitude"] = 1.5e-2
    p = physics.plate_instance(wl)
    o = OI.plate_instance(wl)
    target = OS.run(o, steps, 44100.0)
    rng = np.random.default_rng(1)
    R = rng.normal(size=(3,) + o["Ht"].shape)
    H0 = (0.5 * (R + R.transpose(0, 1, 3, 2)) * np.sqrt(2 * np.mean(o["Ht"] ** 2))).astype(np.float32)

    def mse(y, t):
        return ((y - t) ** 2).sum() / (t ** 2).sum()

    print("case: tensor fit, 3 parallel starts, 1500 steps, 10 iterations", flush=True)
    tt = torch.tensor(target, dtype=torch.float32, device="cuda")
    hs = float(np.sqrt(np.mean(H0.astype(float) ** 2)))
    best_H, best_L, hist = fit.fit_tensor(p, tt, H0, steps, iters=10, lr=0.05, loss_fn=mse, h_scale=hs)
    assert best_H.shape == H0.shape and len(best_L) == 3 and len(hist) == 10
    for b in range(3):
        yb = OS.run(dict(o, Ht=H0[b].astype(float)), steps, 44100.0)
        Lb = float(np.sum((yb - target) ** 2) / np.sum(target ** 2))
        assert abs(hist[0][b] - Lb) < 1e-4 * Lb, (b, hist[0][b], Lb)
    # the same start alone (its own work partition, so sums in another order)
    _, _, h1 = fit.fit_tensor(p, tt, H0[0], steps, iters=10, lr=0.05, loss_fn=mse, h_scale=hs)
    assert np.allclose([h[0] for h in hist], h1, rtol=1e-4, atol=0), ([h[0] for h in hist], h1)
