"""The autotuner: it times candidate launch shapes and the planner's
per-slab exchange cost on the actual batch and records the best under the
batch's key; modal_init then reads that plan from the cache file.  The
tuned context must equal a context given the same plan explicitly, bit for
bit, and the FP64 oracle to 1e-5 relative L2 per output signal."""
import json
import sys

import numpy as np
import pytest

import workloads as W
from oracle import instances as OI
from oracle import simulate as OS

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_tuned_shape_from_the_cache_is_parity_green(tmp_path):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2505_05940_amd import modal, physics, tune
    wls = []
    for i, (nt, nin) in enumerate([(30, 30), (52, 40), (90, 90), (64, 64), (45, 20), (77, 77)]):
        wl = W.plate_vk(seed=500 + i, n_t=nt, n_in=nin, family="sine", grid=None, n_steps=1500)
        wl["strike"]["amplitude"] = 2e-3
        wls.append(wl)
    insts = [physics.plate_instance(w) for w in wls]
    cache = str(tmp_path / "tune.json")
    _say("case: autotune of 6 plates over 3 shapes and 3 exchange costs, then a context from the cache")
    w, mw, sk = tune.autotune(insts, 44100.0, shapes=((4, 1), (1, 2), (4, 2)), samples=60, cache=cache,
                              log=_say, split_costs=(1, 32, 1024))
    key = modal.tune_key(insts, 44100.0)
    entry = json.load(open(cache))[key]
    assert (entry["waves"], entry["max_workgroups"], entry["split_cost_kb"]) == (w, mw, sk)
    assert tune.autotune(insts, 44100.0, cache=cache) == (w, mw, sk)  # served from the cache
    tuned = modal.Sim(insts, 44100.0, tune_cache=cache)
    explicit = modal.Sim(insts, 44100.0, waves=w, max_workgroups=mw, split_cost_kb=sk)
    default = modal.Sim(insts, 44100.0, tune_cache=str(tmp_path / "absent.json"))
    for k in ("workgroups", "units", "split_instances", "plan_makespan"):
        assert tuned.info()[k] == explicit.info()[k], k
    yt = tuned.run(1500).double().cpu().numpy()
    ye = explicit.run(1500).double().cpu().numpy()
    yd = default.run(1500).double().cpu().numpy()
    assert np.array_equal(yt, ye)
    for b, wl in enumerate(wls):
        ref = OS.run(OI.plate_instance(wl), 1500, wl["fs"])
        for y in (yt, yd):
            e = np.linalg.norm(y[b] - ref) / np.linalg.norm(ref)
            assert e < 1e-5, (b, e)
