"""Autotuner for the step kernel's launch shape and work partition.

The tunables are the waves per workgroup, the number of co-resident
workgroups the planner may use, and the per-slab exchange cost the planner
charges a split instance (``split_cost_kb``), which decides which instances
are cut into row slabs and how the units are packed; the slab sizes and the
packing follow from them.  Each candidate (waves, workgroups per CU) is timed
on the actual batch for a few hundred samples with HIP events, then each
exchange cost with the best shape; the best is written to a JSON file under
the batch's key (``modal.tune_key``: a hash of the device name and the
batch's shapes), which ``modal_init`` reads when a context is created with
``tune_cache`` set and no explicit launch shape:
    {"<key>": {"waves": W, "max_workgroups": M, "split_cost_kb": S,
               "ms_per_sample": ..., "trials": {"WxM": ms, "WxM/S": ms, ...}}, ...}
"""
from __future__ import annotations

import json
import os

from . import modal

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_tune_cache.json")
SHAPES = ((4, 2), (4, 3), (8, 1), (8, 2), (1, 6), (1, 8))
SPLIT_COSTS_KB = (8, 16, 32, 64, 128)  # the planner's default is 32


def _time(insts, fs, flags, samples, log, **kw):
    """ms per sample of one candidate plan, or None if it does not fit."""
    import torch
    try:
        sim = modal.Sim(insts, fs, flags=flags | modal.FLAG_ASYNC, chunk_steps=samples, **kw)
    except modal.ModalError as e:  # the candidate does not fit this batch
        if log:
            log(f"autotune: {kw}: {e}")
        return None
    y = torch.empty((len(insts), samples), device="cuda")
    sim.run(samples, out=y)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    sim.run(samples, out=y)
    b.record()
    torch.cuda.synchronize()
    sim.check()
    sim.close()
    ms = a.elapsed_time(b) / samples
    if log:
        log(f"autotune: {kw} -> {ms:.4f} ms/sample")
    return ms


def autotune(insts, fs, shapes=SHAPES, samples=200, cache=CACHE, log=None, flags=0,
             split_costs=SPLIT_COSTS_KB):
    """The best (waves per workgroup, max_workgroups, split_cost_kb) for this
    batch: the shape among `shapes` = (waves, workgroups per CU) pairs, then
    the exchange cost among `split_costs` (KiB) with that shape, timed, and
    recorded in `cache` (a cached entry is returned without timing)."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    key = modal.tune_key(insts, fs, flags=flags)
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        if key in table:
            e = table[key]
            return e["waves"], e["max_workgroups"], e.get("split_cost_kb", 0)
    best, best_ms, trials = None, None, {}
    for waves, k in shapes:
        mw = k * cus
        ms = _time(insts, fs, flags, samples, log, max_workgroups=mw, waves=waves)
        if ms is None:
            continue
        trials[f"{waves}x{mw}"] = ms
        if best_ms is None or ms < best_ms:
            best, best_ms = (waves, mw, 0), ms
    if best is None:
        raise RuntimeError("autotune: no candidate launch shape fits the batch")
    for sk in split_costs:
        ms = _time(insts, fs, flags, samples, log, max_workgroups=best[1], waves=best[0], split_cost_kb=sk)
        if ms is None:
            continue
        trials[f"{best[0]}x{best[1]}/{sk}"] = ms
        if ms < best_ms:
            best, best_ms = (best[0], best[1], sk), ms
    # the optional cost is written before the trials: modal_init reads an
    # entry's fields up to its first closing brace
    table[key] = dict(waves=best[0], max_workgroups=best[1], split_cost_kb=best[2], ms_per_sample=best_ms,
                      trials=trials)
    if cache:
        with open(cache, "w") as f:
            json.dump(table, f, indent=1)
    return best
