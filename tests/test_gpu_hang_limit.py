"""The bounded wait of split instances: with a wait limit of 1 us, set from
the host through modal_desc.barrier_us, a slab wait gives up within a few
steps, every workgroup leaves its loop normally, and modal_run and
modal_grad report MODAL_EHANG; a context with the default limit then runs
as before (the device is left usable)."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _batch(physics):
    out = []
    for i, (nt, nin) in enumerate([(40, 40), (64, 30), (90, 90), (55, 20)]):
        wl = W.plate_vk(seed=400 + i, n_t=nt, n_in=nin, family="sine", grid=None, n_steps=3000)
        out.append(physics.plate_instance(wl))
    return out


def test_wait_limit_reports_ehang_and_leaves_the_device_usable():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2505_05940_amd import modal, physics
    insts = _batch(physics)
    kw = dict(flags=modal.FLAG_SPLIT_ANY, max_workgroups=24, waves=4)
    _say("case: 4 split plates, slab wait limit 1 us, modal_run")
    sim = modal.Sim(insts, 44100.0, barrier_us=1, **kw)
    assert sim.info()["split_instances"] >= 2, sim.info()
    with pytest.raises(modal.ModalError) as e:
        sim.run(3000)
    assert e.value.status == "EHANG"
    sim.close()
    _say("case: the same with modal_grad")
    g = modal.Sim(insts, 44100.0, barrier_us=1, flags=kw["flags"] | modal.FLAG_GRAD,
                  max_workgroups=24, waves=4)
    with pytest.raises(modal.ModalError) as e:
        g.grad(3000, torch.ones((len(insts), 3000), device="cuda"))
    assert e.value.status == "EHANG"
    g.close()
    _say("case: default limit afterwards, run twice, identical")
    ok = modal.Sim(insts, 44100.0, **kw)
    a = ok.run(3000).cpu().numpy()
    ok.reset()
    b = ok.run(3000).cpu().numpy()
    ok.close()
    assert np.isfinite(a).all() and np.array_equal(a, b)
