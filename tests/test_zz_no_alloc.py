"""modal_run_noalloc (the entry point for callers that cannot allocate device
memory) against modal_run on the same batches: two calls in a row, the
second on a smaller batch, with split instances so that the scratch counters
and partial forces are used.  Bar: the same launches, so bit-identical
outputs (and within 1e-5 relative L2 of each other in any case)."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _batch(modal, physics, seeds, n_t, n_in):
    out = []
    for i, s in enumerate(seeds):
        wl = W.plate_vk(seed=s, n_t=n_t[i], n_in=n_in[i], family="sine", grid=None, n_steps=2000)
        wl["strike"]["amplitude"] = 2e-3
        out.append(physics.plate_instance(wl))
    return out


def _pair(modal, insts, steps, chunk, max_wg):
    import torch
    kw = dict(flags=modal.FLAG_SPLIT_ANY, max_workgroups=max_wg, chunk_steps=chunk, waves=4)
    ref = modal.Sim(insts, 44100.0, **kw)
    na = modal.Sim(insts, 44100.0, **kw)
    assert na.info()["split_instances"] >= 1, na.info()
    y_ref = ref.run(steps).double().cpu().numpy()
    y = torch.full((len(insts), steps + 3), float("nan"), device="cuda")
    na.run_noalloc(steps, y)
    got = y[:, :steps].double().cpu().numpy()
    x_ref, xm_ref = ref.state()
    x, xm = na.state()
    ref.close()
    return na, got, y_ref, (x, xm), (x_ref, xm_ref)


def test_noalloc_matches_run_twice_smaller_second():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2505_05940_amd import modal, physics
    cases = [
        ("6 plates 40..90 modes, 1500 steps, chunks of 441", [301, 302, 303, 304, 305, 306],
         [40, 64, 90, 55, 73, 81], [40, 30, 90, 20, 73, 50], 1500, 441, 24),
        ("2 plates 33/48 modes, 700 steps, one launch", [311, 312], [33, 48], [33, 17], 700, 0, 6),
    ]
    for name, seeds, nt, nin, steps, chunk, mw in cases:
        _say(f"case: modal_run_noalloc vs modal_run, {name}")
        insts = _batch(modal, physics, seeds, nt, nin)
        na, got, y_ref, st, st_ref = _pair(modal, insts, steps, chunk, mw)
        for b in range(len(insts)):
            err = np.linalg.norm(got[b] - y_ref[b]) / np.linalg.norm(y_ref[b])
            assert err < 1e-5, (name, b, err)
        assert np.array_equal(got, y_ref), name
        assert np.array_equal(st[0], st_ref[0]) and np.array_equal(st[1], st_ref[1]), name
        # the context's own counters are brought up to date: modal_run
        # continues from where the scratch run stopped
        more = na.run(300).double().cpu().numpy()
        na.reset()
        whole = na.run(steps + 300).double().cpu().numpy()
        assert np.array_equal(more, whole[:, steps:]), name
        na.close()


def test_noalloc_rejects_other_paths():
    import torch
    from paper_2505_05940_amd import modal
    wl = W.linear_batch(seed=9, batch=4, n_modes=20, n_steps=500)
    sim = modal.Sim(wl["instances"], 44100.0)
    y = torch.empty((4, 500), device="cuda")
    with pytest.raises(modal.ModalError) as e:
        sim.run_noalloc(500, y)
    assert e.value.status == "ESTATE"
    sim.close()
