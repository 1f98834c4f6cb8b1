"""Autotuner for the step kernel's launch shape.

The tunables are the waves per workgroup and the number of co-resident
workgroups the planner may use (the work partition, slab sizes and packing
follow from them).  Each candidate (waves, workgroups per CU) is timed on the
actual batch for a few hundred samples with HIP events; the best is written
to a JSON file under the batch's key (``modal.tune_key``: a hash of the
device name and the batch's shapes), which ``modal_init`` reads when a
context is created with ``tune_cache`` set and no explicit launch shape:
    {"<key>": {"waves": W, "max_workgroups": M, "ms_per_sample": ...,
               "trials": {"WxM": ms, ...}}, ...}
"""
from __future__ import annotations

import json
import os

from . import modal

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_tune_cache.json")
SHAPES = ((4, 2), (4, 3), (8, 1), (8, 2), (1, 6), (1, 8))


def autotune(insts, fs, shapes=SHAPES, samples=200, cache=CACHE, log=None, flags=0):
    """The best (waves per workgroup, max_workgroups) for this batch among
    `shapes` = (waves, workgroups per CU) pairs, timed, and recorded in
    `cache` (a cached entry is returned without timing)."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    key = modal.tune_key(insts, fs, flags=flags)
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        if key in table:
            e = table[key]
            return e["waves"], e["max_workgroups"]
    best, best_ms, trials = None, None, {}
    for waves, k in shapes:
        mw = k * cus
        try:
            sim = modal.Sim(insts, fs, flags=flags | modal.FLAG_ASYNC, chunk_steps=samples,
                            max_workgroups=mw, waves=waves)
        except modal.ModalError as e:  # the shape does not fit this batch
            if log:
                log(f"autotune: {waves} waves x {mw} workgroups: {e}")
            continue
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
            log(f"autotune: {waves} waves x {mw} workgroups -> {ms:.4f} ms/sample")
        sim.close()
        if best_ms is None or ms < best_ms:
            best, best_ms = (waves, mw), ms
    if best is None:
        raise RuntimeError("autotune: no candidate launch shape fits the batch")
    table[key] = dict(waves=best[0], max_workgroups=best[1], ms_per_sample=best_ms, trials=trials)
    if cache:
        with open(cache, "w") as f:
            json.dump(table, f, indent=1)
    return best
