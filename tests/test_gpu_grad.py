"""The reverse-mode gradient kernel (modal_grad, through the C ABI) against the
FP64 oracle's reverse recursion and against central differences.

The loss is a seeded linear functional L = sum_n g_n y_n (dL/dy = g), so both
sides differentiate exactly the same scalar.  Bar: relative L2 error of each
gradient vector <= 1e-4 against the oracle's reverse pass; 1e-3 against
central differences with a 1e-4 relative step taken on the FP64 oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as OA
from oracle import instances as OI

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


def _oracle_grads(oinst, steps, g, Hdot=None):
    r = OA.reverse(oinst, steps, 44100.0, g, Hdot=Hdot)
    om, ga = OA.sv_omega_gamma_grads(r, oinst["omega"], oinst["gamma"], 1 / 44100.0)
    return dict(omega=om, gamma=ga, c=r["c"], x0=r["x0"], xm1=r["xm1"], scale=r["scale"],
                theta=r["theta"], row=r["row"])


def _cases():
    wl_vk = W.plate_vk(n_t=14, n_in=11, family="sine", grid=None, n_steps=600)
    wl_vk["strike"]["amplitude"] = 3e-3
    wl_kc = W.string_kc(n_modes=12)
    return wl_vk, wl_kc


@pytest.mark.parametrize("max_wg,ckpt,waves", [(0, 0, 4), (3, 128, 4), (3, 128, 1), (0, 200, 1),
                                               (3, 128, 8), (0, 0, 8)])
def test_grad_matches_oracle(gpu, max_wg, ckpt, waves):
    modal, physics, torch = gpu
    wl_vk, wl_kc = _cases()
    steps = 600
    pinsts = [physics.plate_instance(wl_vk), physics.string_instance(wl_kc)]
    oinsts = [OI.plate_instance(wl_vk), OI.string_instance(wl_kc)]
    rng = np.random.default_rng(5)
    g = rng.normal(size=(2, steps))
    g[0] /= np.abs(oinsts[0]["x0"]).max()
    g[1] /= np.abs(oinsts[1]["x0"]).max()
    print(f"case: grad vK 14/11 + KC 12, {steps} steps, max_wg={max_wg}, ckpt={ckpt}, waves={waves}",
          flush=True)
    sim = modal.Sim(pinsts, 44100.0, flags=modal.FLAG_GRAD | modal.FLAG_SPLIT_ANY,
                    max_workgroups=max_wg, waves=waves)
    if max_wg:
        assert sim.info()["split_instances"] >= 1
    res = sim.grad(steps, torch.tensor(g, dtype=torch.float32, device="cuda"), ckpt_every=ckpt)
    for b in range(2):
        ref = _oracle_grads(oinsts[b], steps, g[b].astype(np.float32).astype(float))
        for k in ("omega", "gamma", "c", "x0", "xm1"):
            assert rel(res[k][b], ref[k]) < TOL, (b, k, rel(res[k][b], ref[k]))
        assert rel([res["scale"][b]], [ref["scale"]]) < TOL, (b, res["scale"][b], ref["scale"])
        if ref["row"] is not None:  # per-row scale gradients of the vK instance
            assert rel(res["row"][b], ref["row"]) < TOL, (b, rel(res["row"][b], ref["row"]))
    # the context is left at its initial state
    y1 = sim.run(50).cpu().numpy()
    sim.reset()
    assert np.array_equal(sim.run(50).cpu().numpy(), y1)


def test_tangent_direction(gpu):
    modal, physics, torch = gpu
    wl_vk, _ = _cases()
    steps = 400
    p = physics.plate_instance(wl_vk)
    o = OI.plate_instance(wl_vk)
    rng = np.random.default_rng(6)
    Hd = rng.normal(size=p["Ht"].shape)
    Hd = (0.5 * (Hd + Hd.transpose(0, 2, 1)) * np.abs(o["Ht"]).max()).astype(np.float32)
    g = rng.normal(size=(1, steps)) / np.abs(o["x0"]).max()
    sim = modal.Sim([p], 44100.0, flags=modal.FLAG_GRAD | modal.FLAG_SPLIT_ANY, max_workgroups=2)
    sim.set_tangent(0, Hd)
    res = sim.grad(steps, torch.tensor(g, dtype=torch.float32, device="cuda"), ckpt_every=150)
    ref = _oracle_grads(o, steps, g[0].astype(np.float32).astype(float), Hdot=Hd.astype(float))
    assert rel([res["theta"][0]], [ref["theta"]]) < TOL, (res["theta"][0], ref["theta"])
    assert rel(res["omega"][0], ref["omega"]) < TOL


def test_grad_matches_central_differences(gpu):
    """dL/domega_k of the GPU adjoint against central differences with the
    configured step (1e-4 relative) taken on the FP64 oracle: 1e-3.  The
    same differences of the GPU forward pass itself are limited by its FP32
    output samples (about 1e-3 here) and are held to 5e-3."""
    modal, physics, torch = gpu
    wl_vk, _ = _cases()
    steps = 600
    p = physics.plate_instance(wl_vk)
    o = OI.plate_instance(wl_vk)
    rng = np.random.default_rng(7)
    g = rng.normal(size=(1, steps)) / np.abs(p["x0"]).max()
    g32 = g[0].astype(np.float32).astype(float)
    gt = torch.tensor(g, dtype=torch.float32, device="cuda")
    sim = modal.Sim([p], 44100.0, flags=modal.FLAG_GRAD)
    res = sim.grad(steps, gt)
    for k in (0, 2, 4):  # components well above the FP32-output noise
        adj = res["omega"][0][k]
        h = 1e-4 * o["omega"][k]
        Lo, Lg = [], []
        for sgn in (1, -1):
            q = dict(o)
            q["omega"] = o["omega"].copy()
            q["omega"][k] += sgn * h
            Lo.append(float(g32 @ OA.forward(q, steps, 44100.0)[0]))
            qp = dict(p)
            qp["omega"] = p["omega"].copy()
            qp["omega"][k] += sgn * h
            y = modal.Sim([qp], 44100.0).run(steps).double().cpu().numpy()[0]
            Lg.append(float(g32 @ y))
        fd64 = (Lo[0] - Lo[1]) / (2 * h)
        fd32 = (Lg[0] - Lg[1]) / (2 * h)
        assert abs(fd64 - adj) < 1e-3 * abs(fd64), (k, fd64, adj)
        assert abs(fd32 - adj) < 5e-3 * abs(adj), (k, fd32, adj)


@pytest.mark.parametrize("max_wg", [0, 3])
def test_grad_reuses_the_checkpoints_of_forward_runs(gpu, max_wg):
    """A gradient context records checkpoints while it runs forward from step
    0; modal_grad with the same spacing then skips its own forward pass.  The
    result is bit-identical to the gradient of a fresh context, also when the
    run came in pieces, and a tensor replacement voids the recorded
    checkpoints."""
    modal, physics, torch = gpu
    wl_vk, wl_kc = _cases()
    steps = 1300
    pinsts = [physics.plate_instance(wl_vk), physics.string_instance(wl_kc)]
    rng = np.random.default_rng(9)
    g = torch.tensor(rng.normal(size=(2, steps)) * 1e3, dtype=torch.float32, device="cuda")
    print(f"case: checkpoint reuse, max_wg={max_wg}", flush=True)

    def fresh(insts):
        s = modal.Sim(insts, 44100.0, flags=modal.FLAG_GRAD | modal.FLAG_SPLIT_ANY, max_workgroups=max_wg)
        r = s.grad(steps, g)
        s.close()
        return r

    ref = fresh(pinsts)
    sim = modal.Sim(pinsts, 44100.0, flags=modal.FLAG_GRAD | modal.FLAG_SPLIT_ANY, max_workgroups=max_wg)
    sim.run(steps)
    a = sim.grad(steps, g)
    sim.run(300)
    sim.run(steps - 300)
    b = sim.grad(steps, g)
    for r in (a, b):
        for k in ("omega", "gamma", "c", "x0", "xm1", "row"):
            for i in range(2):
                assert np.array_equal(r[k][i], ref[k][i]), (k, i)
    # another spacing runs its own forward pass
    c = sim.grad(steps, g, ckpt_every=100)
    assert max(rel(c["omega"][i], ref["omega"][i]) for i in range(2)) < 1e-6
    # a new tensor after the run: the recorded checkpoints are not used
    H2 = (pinsts[0]["Ht"] * 0.8).astype(np.float32)
    sim.run(steps)
    sim.set_tensor(0, H2)
    d = sim.grad(steps, g)
    ref2 = fresh([dict(pinsts[0], Ht=H2), pinsts[1]])
    for k in ("omega", "x0", "row"):
        for i in range(2):
            assert np.array_equal(d[k][i], ref2[k][i]), (k, i)
    sim.close()
