"""Python side of the C++ FP64 oracle loop for batches of von Karman plates
(``oracle/cpp/vk_batch_oracle.cpp``): the chain of ``instances.plate_instance``
(sine in-plane family, exact integrals) and ``simulate.run``, written again
as a plain C++ loop that runs the plates of a batch on all host cores, for
timing the oracle beside the GPU.

TEST INFRASTRUCTURE ONLY (tests/ and the CPU-baseline leg of bench.py).  It is
pinned to the Python oracle plate by plate (tests/test_oracle_cpp.py).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpp", "vk_batch_oracle.cpp")
LIB = os.path.join(HERE, "cpp", "libvk_batch_oracle.so")


def compile_lib(path: str = LIB) -> str:
    """g++ -O3 -march=native -fopenmp; returns the library path."""
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    subprocess.run(["g++", "-O3", "-march=native", "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC],
                   check=True, capture_output=True, text=True)
    os.replace(tmp, path)
    return path


def load(path: str = LIB):
    """The compiled library (compiled first if absent)."""
    if not os.path.exists(path):
        compile_lib(path)
    lib = C.CDLL(path)
    dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int32)
    lib.oracle_vk_plate.argtypes = [dp, ip, dp, dp, dp, dp, dp, dp]
    lib.oracle_vk_plate.restype = C.c_int
    lib.oracle_vk_batch.argtypes = [C.c_int, dp, ip, C.c_double, C.c_int, dp, C.c_int, dp]
    lib.oracle_vk_batch.restype = C.c_int
    return lib


def params(wl):
    """Parameter vectors of one batch plate (``workloads.plate_batch``)."""
    assert wl["inplane"] == "sine" and wl["grid"] is None and wl["damping"][0] == "affine_omega"
    st = wl["strike_rel"]
    d = np.array([wl["aspect"], wl["top_mode_hz"], wl["h"], wl["E"], wl["nu"], wl["rho"], wl["T0"],
                  wl["damping"][1], wl["damping"][2], st["xc"], st["yc"], st["amplitude"],
                  st["radius_rel"], wl["out_rel"][0], wl["out_rel"][1]], dtype=np.float64)
    i = np.array([wl["n_t"], wl["n_in"], wl["proj_grid"][0], wl["proj_grid"][1]], dtype=np.int32)
    return d, i


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def plate(wl, lib=None):
    """omega, gamma, x0, c [n_t], Ht [n_in, n_t, n_t], Lx, Ly of one plate."""
    lib = lib or load()
    d, i = params(wl)
    n, nin = wl["n_t"], wl["n_in"]
    out = {k: np.empty(n) for k in ("omega", "gamma", "x0", "c")}
    Ht = np.empty((nin, n, n))
    LL = np.empty(2)
    lib.oracle_vk_plate(_dp(d), i.ctypes.data_as(C.POINTER(C.c_int32)), _dp(out["omega"]),
                        _dp(out["gamma"]), _dp(out["x0"]), _dp(out["c"]), _dp(Ht), _dp(LL))
    return dict(out, Ht=Ht, Lx=LL[0], Ly=LL[1])


def run_batch(wls, n_steps, fs=44100.0, threads=0, lib=None):
    """Outputs [batch, n_steps] of every plate from rest, the build and loop
    wall times (s) and the OpenMP threads used."""
    lib = lib or load()
    ps = [params(w) for w in wls]
    d = np.ascontiguousarray(np.stack([p[0] for p in ps]))
    i = np.ascontiguousarray(np.stack([p[1] for p in ps]))
    y = np.empty((len(wls), n_steps))
    sec = np.empty(2)
    used = lib.oracle_vk_batch(len(wls), _dp(d), i.ctypes.data_as(C.POINTER(C.c_int32)), fs, n_steps,
                               _dp(y), threads, _dp(sec))
    return y, float(sec[0]), float(sec[1]), int(used)
