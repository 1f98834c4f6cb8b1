"""ctypes binding of libmodal.so (argument marshalling only).

Every step of the time loop runs in the library's HIP kernels; this module
converts numpy / torch arguments to the C structures of ``include/modal.h``.
Importing it without the built library raises immediately: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmodal.so")

KIND = {"linear": 0, "tension": 1, "vk": 2}
SCHEME = {"sv": 0, "tf": 1}
FLAG_ASYNC = 1
FLAG_GRAPH = 2
FLAG_GRAD = 4
FLAG_SPLIT_ANY = 8
FLAG_NO_SHARED = 16
FLAG_NO_BLOCK = 32
FLAG_RECURSE = 64

STATUS = {0: "OK", -1: "EINVAL", -2: "EUNSTABLE", -3: "ENOMEM", -4: "EHIP",
          -5: "ENONFINITE", -6: "ESTATE", -7: "EHANG"}

_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_ip = C.POINTER(C.c_int32)


class modal_instance(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_t", C.c_int32), ("n_in", C.c_int32),
                ("reserved", C.c_int32), ("omega", _dp), ("gamma", _dp), ("lam", _dp),
                ("kappa", C.c_double), ("H", _fp), ("x0", _dp), ("xm1", _dp),
                ("b_ext", _dp), ("e_ext", _fp), ("n_exc", C.c_int64), ("c_out", _dp),
                ("h_row_scale", _dp), ("mode_class", C.POINTER(C.c_uint8))]


class modal_desc(C.Structure):
    _fields_ = [("batch", C.c_int32), ("scheme", C.c_int32),
                ("inst", C.POINTER(modal_instance)), ("fs", C.c_double),
                ("flags", C.c_int32), ("max_workgroups", C.c_int32),
                ("chunk_steps", C.c_int32), ("waves", C.c_int32), ("barrier_us", C.c_int32),
                ("tune_cache", C.c_char_p), ("split_cost_kb", C.c_int32)]


class ModalError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2505_05940_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.modal_init.argtypes = [C.POINTER(vp), C.POINTER(modal_desc), vp]
    lib.modal_run.argtypes = [vp, C.c_int64, _fp, C.c_int64, vp]
    lib.modal_run_noalloc.argtypes = [vp, C.c_int64, _fp, C.c_int64, vp]
    lib.modal_check.argtypes = [vp, vp]
    lib.modal_reset.argtypes = [vp, vp]
    lib.modal_get_state.argtypes = [vp, _dp, _dp, vp]
    lib.modal_info.argtypes = [vp, C.POINTER(C.c_int64)]
    lib.modal_destroy.argtypes = [vp]
    lib.modal_destroy.restype = None
    lib.modal_last_error.restype = C.c_char_p
    lib.modal_grad.argtypes = [vp, C.c_int64, _fp, C.c_int64, C.c_int32, _dp, _dp, _dp, _dp, _dp,
                               _dp, _dp, _dp, C.POINTER(vp), vp]
    lib.modal_grad.restype = C.c_int
    lib.modal_set_tangent.argtypes = [vp, C.c_int32, _fp, vp]
    lib.modal_set_tangent.restype = C.c_int
    lib.modal_set_tensor.argtypes = [vp, C.c_int32, _fp, vp]
    lib.modal_set_tensor.restype = C.c_int
    lib.modal_plan.argtypes = [C.POINTER(modal_desc), C.c_int32, C.POINTER(C.c_int64)]
    lib.modal_plan.restype = C.c_int
    lib.modal_tune_key.argtypes = [C.POINTER(modal_desc), C.c_char_p, C.c_int32]
    lib.modal_tune_key.restype = C.c_int
    lib.modal_vk_coupling_sine.argtypes = [C.c_double, C.c_double, C.c_int32, _ip, _ip,
                                           C.c_int32, _ip, _ip, C.c_int32, C.c_int32,
                                           _dp, _fp, C.c_int32]
    lib.modal_tf_response.argtypes = [vp, vp, C.c_int32, vp, C.c_int32, vp, vp]
    lib.modal_tf_grad.argtypes = [vp, vp, C.c_int32, C.c_int32, vp, C.c_int32, vp, vp, vp]
    for f in ("modal_init", "modal_run", "modal_run_noalloc", "modal_check", "modal_reset", "modal_get_state",
              "modal_info", "modal_vk_coupling_sine", "modal_tf_response", "modal_tf_grad"):
        getattr(lib, f).restype = C.c_int
    return lib


lib = _load()


def _check(code):
    if code != 0:
        raise ModalError(code, lib.modal_last_error().decode())


def _d(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None:
        assert a.shape == (n,), (a.shape, n)
    return a


def _stream_handle(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(getattr(stream, "cuda_stream", stream)))


def vk_coupling_sine(Lx, Ly, m, q, a, b, scale_n, grid=None, threads=0):
    """Scaled sine-family coupling tensor [n_in, n_t, n_t] (float32) from the
    library's host builder; grid None = exact integrals."""
    m = np.ascontiguousarray(m, np.int32)
    q = np.ascontiguousarray(q, np.int32)
    a = np.ascontiguousarray(a, np.int32)
    b = np.ascontiguousarray(b, np.int32)
    sc = _d(scale_n, len(a))
    out = np.empty((len(a), len(m), len(m)), np.float32)
    nx, ny = (0, 0) if grid is None else grid
    _check(lib.modal_vk_coupling_sine(
        Lx, Ly, len(m), m.ctypes.data_as(_ip), q.ctypes.data_as(_ip), len(a),
        a.ctypes.data_as(_ip), b.ctypes.data_as(_ip), nx, ny,
        sc.ctypes.data_as(_dp), out.ctypes.data_as(_fp), threads))
    return out


def _build_desc(instances, fs, scheme="sv", flags=0, max_workgroups=0, chunk_steps=0,
                shapes_only=False, waves=0, barrier_us=0, tune_cache=None, split_cost_kb=0):
    """modal_desc for a list of instance dicts; returns (desc, keep-alive list, n_t list).
    With shapes_only (planning previews, which never read tensors) a vk
    instance may give "n_in" instead of "Ht"."""
    keep = []
    batch = len(instances)
    arr = (modal_instance * batch)()
    keep.append(arr)
    n_t = []
    for i, inst in enumerate(instances):
        n = len(inst["omega"])
        n_t.append(n)
        s = arr[i]
        s.kind = KIND[inst["kind"]]
        s.n_t = n
        s.reserved = 0
        for field, key in (("omega", "omega"), ("gamma", "gamma"), ("x0", "x0"),
                           ("xm1", "xm1"), ("c_out", "c")):
            a = _d(inst[key], n)
            keep.append(a)
            setattr(s, field, a.ctypes.data_as(_dp))
        if inst["kind"] == "tension":
            if inst.get("lam") is not None:
                a = _d(inst["lam"], n)
                keep.append(a)
                s.lam = a.ctypes.data_as(_dp)
            s.kappa = float(inst["kappa"])
        if inst["kind"] == "vk" and shapes_only and "Ht" not in inst:
            dummy = np.zeros(1, np.float32)
            keep.append(dummy)
            s.H = dummy.ctypes.data_as(_fp)
            s.n_in = int(inst["n_in"])
        elif inst["kind"] == "vk":
            H = inst["Ht"]
            if hasattr(H, "data_ptr"):
                assert H.dtype.itemsize == 4 and H.is_contiguous() and tuple(H.shape[1:]) == (n, n)
                s.H = C.cast(C.c_void_p(H.data_ptr()), _fp)
            else:
                H = np.ascontiguousarray(H, dtype=np.float32)
                assert H.ndim == 3 and H.shape[1:] == (n, n)
                s.H = H.ctypes.data_as(_fp)
            s.n_in = H.shape[0]
            keep.append(H)
            if inst.get("h_row_scale") is not None:
                sc = _d(inst["h_row_scale"], s.n_in)
                keep.append(sc)
                s.h_row_scale = sc.ctypes.data_as(_dp)
            if inst.get("mode_class") is not None:
                mc = np.ascontiguousarray(inst["mode_class"], dtype=np.uint8)
                assert mc.shape == (n,)
                keep.append(mc)
                s.mode_class = mc.ctypes.data_as(C.POINTER(C.c_uint8))
        else:
            s.n_in = 0
        if inst.get("e_ext") is not None:
            b = _d(inst["b_ext"], n)
            e = np.ascontiguousarray(inst["e_ext"], dtype=np.float32)
            keep += [b, e]
            s.b_ext = b.ctypes.data_as(_dp)
            s.e_ext = e.ctypes.data_as(_fp)
            s.n_exc = len(e)
    tc = None if tune_cache is None else os.fsencode(tune_cache)
    keep.append(tc)
    desc = modal_desc(batch=batch, scheme=SCHEME[scheme], inst=arr, fs=float(fs), flags=flags,
                      max_workgroups=max_workgroups, chunk_steps=chunk_steps, waves=waves,
                      barrier_us=barrier_us, tune_cache=tc, split_cost_kb=split_cost_kb)
    return desc, keep, n_t


def tune_key(instances, fs=44100.0, scheme="sv", flags=0):
    """The autotuner's cache key of a batch (``modal_tune_key``)."""
    desc, keep, _ = _build_desc(instances, fs, scheme, flags=flags, shapes_only=True)
    out = C.create_string_buffer(17)
    _check(lib.modal_tune_key(C.byref(desc), out, 17))
    return out.value.decode()


def plan(instances, n_workgroups, fs=44100.0, scheme="sv", flags=0, split_cost_kb=0):
    """Host-only preview of the work partition (``modal_plan``)."""
    desc, keep, _ = _build_desc(instances, fs, scheme, flags=flags, shapes_only=True,
                                split_cost_kb=split_cost_kb)
    out = (C.c_int64 * 4)()
    _check(lib.modal_plan(C.byref(desc), n_workgroups, out))
    return dict(units=out[0], workgroups=out[1], makespan=out[2], mean=out[3])


class Sim:
    """A batch of modal systems resident on the GPU (``modal_init``).

    ``instances``: list of dicts with keys kind ('linear' | 'tension' | 'vk'),
    omega, gamma, x0, xm1, c [n_t]; lam, kappa (tension); Ht float32
    [n_in, n_t, n_t] (vk, host numpy or a CUDA tensor) and optional
    h_row_scale [n_in] (the instance's tensor is h_row_scale[n] Ht[n];
    instances given the same Ht object share it, see ``modal_init``);
    optional mode_class [n_t] (uint8 0..3, the tensor's block structure);
    optional b_ext [n_t] and e_ext [n_exc] (float32).
    """

    def __init__(self, instances, fs, scheme="sv", flags=0, max_workgroups=0,
                 chunk_steps=0, stream=None, waves=0, barrier_us=0, tune_cache=None, split_cost_kb=0):
        self._ctx = C.c_void_p()
        self.batch = len(instances)
        desc, keep, self.n_t = _build_desc(instances, fs, scheme, flags, max_workgroups, chunk_steps,
                                           waves=waves, barrier_us=barrier_us, tune_cache=tune_cache,
                                           split_cost_kb=split_cost_kb)
        self._stream = stream
        _check(lib.modal_init(C.byref(self._ctx), C.byref(desc), _stream_handle(stream)))
        self.modes_total = sum(self.n_t)
        self.scheme = scheme
        self.n_in = [int(i["Ht"].shape[0]) if i["kind"] == "vk" else 0 for i in instances]
        self._row_off = np.concatenate([[0], np.cumsum(self.n_in)[:-1]]).astype(int)
        self.rows_total = int(sum(self.n_in))

    def run(self, n_steps, out=None):
        """Advance by n_steps; returns y [batch, n_steps] float32 on the GPU."""
        import torch
        if out is None:
            out = torch.empty((self.batch, n_steps), dtype=torch.float32, device="cuda")
        assert out.dtype == torch.float32 and out.is_cuda and out.shape[0] == self.batch
        assert out.stride(1) == 1 and out.shape[1] >= n_steps
        _check(lib.modal_run(self._ctx, n_steps, C.cast(C.c_void_p(out.data_ptr()), _fp),
                             out.stride(0), _stream_handle(self._stream)))
        return out

    def run_noalloc(self, n_steps, out):
        """``modal_run_noalloc``: like ``run`` into a caller-given buffer, with
        no device allocation in the call."""
        import torch
        assert out.dtype == torch.float32 and out.is_cuda and out.shape[0] == self.batch
        assert out.stride(1) == 1 and out.shape[1] >= n_steps
        _check(lib.modal_run_noalloc(self._ctx, n_steps, C.cast(C.c_void_p(out.data_ptr()), _fp),
                                     out.stride(0), _stream_handle(self._stream)))
        return out

    def check(self):
        _check(lib.modal_check(self._ctx, _stream_handle(self._stream)))

    def set_tangent(self, b, Hd):
        """Tangent tensor dHt/dtheta of instance b (float32 [n_in, n_t, n_t])."""
        if hasattr(Hd, "data_ptr"):
            ptr = C.cast(C.c_void_p(Hd.data_ptr()), _fp)
            keep = Hd
        else:
            keep = np.ascontiguousarray(Hd, dtype=np.float32)
            ptr = keep.ctypes.data_as(_fp)
        _check(lib.modal_set_tangent(self._ctx, b, ptr, _stream_handle(self._stream)))
        del keep

    def set_tensor(self, b, H):
        """Replace the coupling tensor of VK instance b (float32 [n_in, n_t, n_t],
        CUDA tensor or host array)."""
        if hasattr(H, "data_ptr"):
            assert H.dtype.itemsize == 4 and H.is_contiguous()
            ptr = C.cast(C.c_void_p(H.data_ptr()), _fp)
            keep = H
        else:
            keep = np.ascontiguousarray(H, dtype=np.float32)
            ptr = keep.ctypes.data_as(_fp)
        _check(lib.modal_set_tensor(self._ctx, b, ptr, _stream_handle(self._stream)))
        del keep

    def grad(self, n_steps, dL_dy, ckpt_every=0, tensor=False):
        """Reverse-mode gradient of L over the first n_steps outputs from the
        initial state; dL_dy is a CUDA float32 tensor [batch, >= n_steps].
        Returns per-instance lists of numpy arrays (omega, gamma, c, x0, xm1,
        and row = dL/dlog s_n per in-plane row of a vk instance) and [batch]
        arrays (scale = dL/dlog s, theta).  tensor=True (or a list of booleans
        per instance) adds H: per instance a CUDA float32 tensor
        [n_in, n_t, n_t] with dL/dHt entry by entry (None where not asked or
        not vk)."""
        assert dL_dy.is_cuda and dL_dy.dtype.itemsize == 4 and dL_dy.stride(1) == 1
        M = self.modes_total
        out = {k: np.zeros(M) for k in ("omega", "gamma", "c", "x0", "xm1")}
        scale = np.zeros(self.batch)
        theta = np.zeros(self.batch)
        row = np.zeros(max(1, self.rows_total))
        gH = [None] * self.batch
        ptrs = None
        if tensor:
            import torch
            want = tensor if isinstance(tensor, (list, tuple)) else [True] * self.batch
            for b in range(self.batch):
                if want[b] and self.n_in[b] > 0:
                    gH[b] = torch.empty((self.n_in[b], self.n_t[b], self.n_t[b]), dtype=torch.float32,
                                        device=dL_dy.device)
            ptrs = (C.c_void_p * self.batch)(*[(g.data_ptr() if g is not None else None) for g in gH])
        _check(lib.modal_grad(self._ctx, n_steps, C.cast(C.c_void_p(dL_dy.data_ptr()), _fp),
                              dL_dy.stride(0), ckpt_every,
                              *(out[k].ctypes.data_as(_dp) for k in ("omega", "gamma", "c", "x0", "xm1")),
                              scale.ctypes.data_as(_dp), theta.ctypes.data_as(_dp),
                              row.ctypes.data_as(_dp), ptrs, _stream_handle(self._stream)))
        splits = np.cumsum(self.n_t)[:-1]
        res = {k: np.split(v, splits) for k, v in out.items()}
        res["scale"] = scale
        res["theta"] = theta
        res["row"] = [row[o:o + n] if n else np.zeros(0) for o, n in zip(self._row_off, self.n_in)]
        if tensor:
            res["H"] = gH
        return res

    def reset(self):
        _check(lib.modal_reset(self._ctx, _stream_handle(self._stream)))

    def state(self):
        x = np.empty(self.modes_total)
        xm = np.empty(self.modes_total)
        _check(lib.modal_get_state(self._ctx, x.ctypes.data_as(_dp), xm.ctypes.data_as(_dp),
                                   _stream_handle(self._stream)))
        return x, xm

    def info(self):
        v = (C.c_int64 * 15)()
        _check(lib.modal_info(self._ctx, v))
        keys = ("workgroups", "units", "split_instances", "coupling_bytes_per_step",
                "padded_bytes_per_step", "steps", "lds_bytes", "workgroups_per_cu",
                "plan_makespan", "plan_mean", "path", "flops_per_step", "blocked_instances",
                "dense_bytes_per_step", "resident_floats")
        out = dict(zip(keys, list(v)))
        out["shared"] = int(out["path"] == 1)  # 0 recursion, 1 shared tensor, 2 linear closed form
        return out

    def close(self):
        if self._ctx:
            lib.modal_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
