"""The C ABI without a GPU: every declared symbol is exported, and argument
validation fails cleanly before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "modal.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(modal_[a-z_]+)\s*\(", src)))


def test_header_symbols_are_exported():
    from paper_2505_05940_amd import modal
    names = _declared()
    assert "modal_init" in names and "modal_run" in names
    for n in names:
        assert hasattr(modal.lib, n), n


def _inst(kind="linear", n=4, **kw):
    d = dict(kind=kind, omega=np.full(n, 2 * np.pi * 100.0), gamma=np.full(n, 1.0),
             x0=np.ones(n), xm1=np.ones(n), c=np.ones(n))
    d.update(kw)
    return d


@pytest.mark.parametrize("bad,code", [
    (dict(gamma=np.full(4, -1.0)), "EUNSTABLE"),
    (dict(gamma=np.zeros(4)), "EUNSTABLE"),
    (dict(omega=np.full(4, 2.01 * 44100.0)), "EUNSTABLE"),
    (dict(x0=np.array([1.0, np.nan, 0, 0])), "EINVAL"),
])
def test_validation_errors(bad, code):
    from paper_2505_05940_amd import modal
    with pytest.raises(modal.ModalError) as e:
        modal.Sim([_inst(**bad)], 44100.0, stream=0)
    assert e.value.status == code


def test_row_scale_must_be_finite():
    from paper_2505_05940_amd import modal
    H = np.zeros((2, 4, 4), np.float32)
    with pytest.raises(modal.ModalError) as e:
        modal.Sim([_inst(kind="vk", Ht=H, h_row_scale=np.array([1.0, np.inf]))], 44100.0, stream=0)
    assert e.value.status == "EINVAL"


def test_tf_rejects_overdamped_modes():
    from paper_2505_05940_amd import modal
    with pytest.raises(modal.ModalError) as e:
        modal.Sim([_inst(gamma=np.full(4, 1e4))], 44100.0, scheme="tf", stream=0)
    assert e.value.status == "EUNSTABLE"


def test_tension_needs_lambda():
    from paper_2505_05940_amd import modal
    with pytest.raises(modal.ModalError) as e:
        modal.Sim([_inst(kind="tension", lam=None, kappa=1.0)], 44100.0, stream=0)
    assert e.value.status == "EINVAL"


def test_sv_stability_boundary():
    """omega T above 2 puts an SV root outside the unit circle; validation
    rejects it on the host before any device call."""
    from paper_2505_05940_amd import modal
    with pytest.raises(modal.ModalError) as e:
        modal.Sim([_inst(omega=np.full(4, 2.0001 * 44100.0), gamma=np.zeros(4))], 44100.0, stream=0)
    assert e.value.status == "EUNSTABLE"


def test_plan_balances_the_batched_workload():
    """The partition of the 256-plate batch (shapes only, no tensors read):
    every instance is covered, no workgroup exceeds 1.15x the mean cost."""
    import workloads as W
    from paper_2505_05940_amd import modal
    wls = W.plate_batch()
    insts = [dict(kind="vk", omega=np.full(w["n_t"], 1e3), gamma=np.ones(w["n_t"]),
                  x0=np.zeros(w["n_t"]), xm1=np.zeros(w["n_t"]), c=np.ones(w["n_t"]),
                  n_in=w["n_in"]) for w in wls]
    for nb in (512, 2560, 4096):
        p = modal.plan(insts, nb)
        assert p["workgroups"] <= nb and p["units"] >= len(wls)
        assert p["makespan"] <= 1.15 * p["mean"], (nb, p)


def test_plan_splits_only_when_needed():
    """Small instances (tensor L2-resident) stay whole whatever the budget;
    a large one is cut into row slabs when workgroups are available."""
    from paper_2505_05940_amd import modal

    def inst(n):
        return dict(kind="vk", omega=np.full(n, 1e3), gamma=np.ones(n), x0=np.zeros(n),
                    xm1=np.zeros(n), c=np.ones(n), n_in=n)
    assert modal.plan([inst(40)], 8)["units"] == 1
    assert modal.plan([inst(40)] * 16, 1536)["units"] == 16
    assert modal.plan([inst(120)], 1)["units"] == 1
    p = modal.plan([inst(120)], 8)
    assert p["units"] == 8 and p["workgroups"] == 8


def test_split_cost_steers_the_plan():
    """The per-slab exchange cost the planner charges (modal_desc.split_cost_kb,
    the autotuner's knob): 0 is the default (32 KiB); another cost gives
    another partition, and a dearer one a costlier heaviest workgroup (its
    slabs carry the cost); a negative one is rejected."""
    import workloads as W
    from paper_2505_05940_amd import modal
    wls = W.plate_batch()
    insts = [dict(kind="vk", omega=np.full(w["n_t"], 1e3), gamma=np.ones(w["n_t"]),
                  x0=np.zeros(w["n_t"]), xm1=np.zeros(w["n_t"]), c=np.ones(w["n_t"]),
                  n_in=w["n_in"]) for w in wls]
    assert modal.plan(insts, 768) == modal.plan(insts, 768, split_cost_kb=32)
    cheap = modal.plan(insts, 768, split_cost_kb=1)
    dear = modal.plan(insts, 768, split_cost_kb=4096)
    assert dear != cheap and dear["makespan"] > cheap["makespan"], (cheap, dear)
    with pytest.raises(modal.ModalError) as e:
        modal.plan(insts, 768, split_cost_kb=-1)
    assert e.value.status == "EINVAL"
