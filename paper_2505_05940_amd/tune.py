"""Autotuner for the batched step kernel's launch shape.

The tunable is the number of co-resident workgroups the planner may use
(the work partition, slab sizes and packing follow from it).  Candidates are
multiples of the CU count; each is timed on the actual batch for a few
hundred samples with HIP events, and the best is cached in a JSON file keyed
by the device name and the batch's shapes.
"""
from __future__ import annotations

import hashlib
import json
import os

from . import modal

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_tune_cache.json")


def _key(insts, device):
    shapes = [(i["kind"], len(i["omega"]), int(i["Ht"].shape[0]) if i["kind"] == "vk" else 0)
              for i in insts]
    h = hashlib.sha256(json.dumps([device, shapes]).encode()).hexdigest()[:16]
    return h


def autotune(insts, fs, shapes=((4, 1), (4, 2), (4, 3), (1, 5), (1, 6), (1, 7), (1, 8)),
             samples=200, cache=CACHE, log=None):
    """Returns the best (waves per workgroup, max_workgroups) for this batch
    among `shapes` = (waves, workgroups per CU) pairs (cached)."""
    import torch
    props = torch.cuda.get_device_properties(0)
    cus = props.multi_processor_count
    key = _key(insts, props.name)
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        if key in table:
            return tuple(table[key]["best"])
    best, best_ms, trials = None, None, {}
    for waves, k in shapes:
        mw = k * cus
        sim = modal.Sim(insts, fs, flags=modal.FLAG_ASYNC, chunk_steps=samples, max_workgroups=mw,
                        waves=waves)
        y = torch.empty((len(insts), samples), device="cuda")
        sim.run(samples, out=y)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        sim.run(samples, out=y)
        b.record()
        torch.cuda.synchronize()
        sim.check()
        ms = a.elapsed_time(b) / samples
        trials[f"{waves}x{mw}"] = ms
        if log:
            log(f"autotune: {waves} waves x {mw} workgroups -> {ms:.3f} ms/sample")
        sim.close()
        if best_ms is None or ms < best_ms:
            best, best_ms = (waves, mw), ms
    table[key] = dict(best=list(best), ms_per_sample=best_ms, trials=trials)
    if cache:
        with open(cache, "w") as f:
            json.dump(table, f, indent=1)
    return best
