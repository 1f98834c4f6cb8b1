"""The C++ FP64 oracle loop (oracle/cpp, used to time the oracle on all host
cores) against the Python oracle, plate by plate: the same parameters, mode
sets, coupling tensors, excitation and outputs."""
import numpy as np
import pytest

import workloads as W
from oracle import cpu_batch as CB
from oracle import instances as OI
from oracle import simulate as OS


@pytest.fixture(scope="module")
def lib():
    return CB.load(CB.compile_lib())


def _small_batch():
    return W.plate_batch(seed=41, batch=6, n_lo=4, n_hi=24)


def test_plate_pieces_match_the_python_oracle(lib):
    for wl in _small_batch():
        cpp = CB.plate(wl, lib)
        py = OI.plate_instance(wl)
        assert abs(cpp["Lx"] - py["Lx"]) < 1e-14 * py["Lx"] and abs(cpp["Ly"] - py["Ly"]) < 1e-14 * py["Ly"]
        for k in ("omega", "gamma", "c"):
            assert np.allclose(cpp[k], py[k], rtol=1e-13, atol=0), k
        assert np.allclose(cpp["x0"], py["x0"], rtol=1e-10, atol=1e-13 * np.abs(py["x0"]).max())
        assert np.abs(cpp["Ht"] - py["Ht"]).max() <= 1e-12 * np.abs(py["Ht"]).max()


def test_batch_outputs_match_the_python_oracle(lib):
    wls = _small_batch()
    y, t_build, t_loop, used = CB.run_batch(wls, 400, threads=2, lib=lib)
    assert used == 2 and t_build >= 0 and t_loop > 0
    for b, wl in enumerate(wls):
        ref = OS.run(OI.plate_instance(wl), 400, wl["fs"])
        assert np.linalg.norm(y[b] - ref) <= 1e-10 * np.linalg.norm(ref), b
