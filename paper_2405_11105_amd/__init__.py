"""Localized EVD clutter filter for AMD MI355X -- Python binding of ``liblcf.so``.

Thin ctypes layer over the C ABI in ``include/lcf.h``: it marshals torch device
tensors (memory) and the current HIP stream into the library calls. Every step
of the filter runs in the library's HIP kernels; there is no fallback path, and
the calls raise if the shared library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "liblcf.so")

PREC_FP32, PREC_BF16X3 = 0, 1
CUT_FIXED_K, CUT_KNEE, CUT_EXPLICIT, CUT_MLP, CUT_MEDIAN, CUT_SLOPE, CUT_POWER, CUT_NCC = 0, 1, 2, 3, 4, 5, 6, 7
ABI_VERSION = 6
SHAPE_HARD, SHAPE_SIGMOID = 0, 1
PD_EQ13, PD_SUM, PD_EQ13_COMPENSATED = 0, 1, 2
OPT_SCHEDULE, OPT_MAX_SWEEPS, OPT_USE_GRAPH, OPT_SUBSPACE_IT, OPT_STAGE_TIMING, OPT_AUTOTUNE, OPT_EVD = 1, 2, 3, 4, 5, 6, 7
OPT_MLP_GATE = 8
EVD_TRIDIAGONAL, EVD_JACOBI = 0, 1
STAGES = ["windows", "gram1", "gram1_reduce", "tissue", "gram2", "gram2_reduce", "assemble", "evd",
          "rules", "mlp", "projector", "reproj", "evd_vectors", "ncc", "cov_stream"]
FLAG_NONPOSITIVE, FLAG_NONFINITE, FLAG_NO_CONVERGE, FLAG_MLP_FALLBACK, FLAG_EVD_JACOBI = 1, 2, 4, 8, 16

STATUS = {0: "LCF_OK", 1: "LCF_ERR_INVALID_ARG", 2: "LCF_ERR_UNSUPPORTED", 3: "LCF_ERR_OUT_OF_MEMORY",
          4: "LCF_ERR_DEVICE", 5: "LCF_ERR_NONFINITE_INPUT", 6: "LCF_ERR_NO_CONVERGENCE", 7: "LCF_ERR_MODEL",
          8: "LCF_ERR_SCRATCH_LIMIT"}
NOALLOC_SCRATCH_BYTES = 192 * 1024 * 1024


class LcfError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS.get(status, status)}")
        self.status = status


class Geometry(C.Structure):
    _fields_ = [("ny", C.c_int32), ("nx", C.c_int32), ("nt", C.c_int32), ("gy", C.c_int32),
                ("gx", C.c_int32), ("reserved", C.c_int32), ("sigma_frac", C.c_double),
                ("trunc_sigmas", C.c_double)]


class ThresholdC(C.Structure):
    _fields_ = [("cut", C.c_int32), ("shape", C.c_int32), ("pd_mode", C.c_int32), ("k_fixed", C.c_int32),
                ("beta_knee", C.c_double), ("knee_max_frac", C.c_double), ("beta_sigmoid", C.c_double),
                ("deflate_rho", C.c_double), ("explicit_w", C.c_void_p), ("beta_median", C.c_double),
                ("slope_thr", C.c_double), ("beta_power", C.c_double)]


class DiagC(C.Structure):
    _fields_ = [("eigvals", C.c_void_p), ("weights", C.c_void_p), ("k", C.c_void_p), ("sweeps", C.c_void_p),
                ("flags", C.c_void_p), ("alpha", C.c_void_p), ("cov", C.c_void_p), ("eigvecs", C.c_void_p),
                ("rank", C.c_void_p), ("curve", C.c_void_p), ("mlp_gate", C.c_void_p)]


@dataclass
class Threshold:
    """Thresholding rule; field meanings follow ``lcf_threshold``."""
    cut: int = CUT_FIXED_K
    shape: int = SHAPE_HARD
    pd_mode: int = PD_EQ13
    k_fixed: int = 4
    beta_knee: float = 1.0
    knee_max_frac: float = 0.5
    beta_sigmoid: float = 2.0
    deflate_rho: float = 1e-5
    beta_median: float = 1.43      # the scaling factor of the paper's Fig. 2a example
    slope_thr: float = 1.1         # the slope threshold of the paper's Fig. 2c example
    beta_power: float = 2.0        # the order of the paper's Fig. 2g example

    def to_c(self, explicit_ptr: int = 0) -> ThresholdC:
        return ThresholdC(self.cut, self.shape, self.pd_mode, self.k_fixed, self.beta_knee,
                          self.knee_max_frac, self.beta_sigmoid, self.deflate_rho, explicit_ptr or None,
                          self.beta_median, self.slope_thr, self.beta_power)


_lib = None


def load():
    """Load liblcf.so (built by ``build.py``); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.lcf_create.argtypes = [i32, C.POINTER(vp)]
    lib.lcf_destroy.argtypes = [vp]
    lib.lcf_set_option.argtypes = [vp, i32, i64]
    lib.lcf_validate.argtypes = [C.POINTER(Geometry), C.POINTER(ThresholdC), i32]
    lib.lcf_filter.argtypes = [vp, C.POINTER(Geometry), C.POINTER(ThresholdC), i32, vp, vp, vp,
                               C.POINTER(DiagC), vp]
    lib.lcf_filter_noalloc.argtypes = lib.lcf_filter.argtypes
    lib.lcf_filter_batch.argtypes = [vp, i32, C.POINTER(Geometry), C.POINTER(ThresholdC), i32,
                                     C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), vp]
    lib.lcf_heevd_batched.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp]
    lib.lcf_stream_create.argtypes = [vp, C.POINTER(Geometry), C.POINTER(ThresholdC), i32, C.POINTER(vp)]
    lib.lcf_stream_push.argtypes = [vp, vp, i32, vp, vp, C.POINTER(DiagC), vp]
    lib.lcf_stream_destroy.argtypes = [vp]
    lib.lcf_sync.argtypes = [vp, vp]
    lib.lcf_stage_time.argtypes = [vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_int64), i32]
    lib.lcf_mlp_init.argtypes = [vp, C.c_uint64]
    lib.lcf_mlp_set_params.argtypes = [vp, vp, i64]
    lib.lcf_mlp_get_params.argtypes = [vp, vp, i64]
    lib.lcf_mlp_get_grads.argtypes = [vp, vp, i64]
    lib.lcf_mlp_save.argtypes = [vp, C.c_char_p]
    lib.lcf_mlp_load.argtypes = [vp, C.c_char_p]
    lib.lcf_mlp_infer.argtypes = [vp, vp, vp, i32, vp]
    lib.lcf_mlp_train_step.argtypes = [vp, vp, vp, i32, C.c_float, vp, vp]
    lib.lcf_tune_save.argtypes = [vp, C.c_char_p]
    lib.lcf_tune_load.argtypes = [vp, C.c_char_p]
    lib.lcf_status_str.argtypes = [i32]
    lib.lcf_status_str.restype = C.c_char_p
    for name in ("lcf_create", "lcf_destroy", "lcf_set_option", "lcf_validate", "lcf_filter", "lcf_filter_noalloc",
                 "lcf_filter_batch", "lcf_heevd_batched", "lcf_sync", "lcf_abi_version",
                 "lcf_stream_create", "lcf_stream_push", "lcf_stream_destroy",
                 "lcf_stage_time",
                 "lcf_mlp_init", "lcf_mlp_set_params", "lcf_mlp_get_params", "lcf_mlp_get_grads", "lcf_mlp_save",
                 "lcf_mlp_load", "lcf_mlp_infer", "lcf_mlp_train_step", "lcf_tune_save", "lcf_tune_load"):
        getattr(lib, name).restype = i32
    if lib.lcf_abi_version() != ABI_VERSION:
        raise RuntimeError(f"{LIB_PATH}: ABI version {lib.lcf_abi_version()}, the binding needs {ABI_VERSION}")
    _lib = lib
    return lib


def _check(st: int, what: str):
    if st != 0:
        raise LcfError(st, what)


def geometry(ny, nx, nt, gy, gx, sigma_frac=1.0 / 3.0, trunc_sigmas=6.0) -> Geometry:
    return Geometry(ny, nx, nt, gy, gx, 0, sigma_frac, trunc_sigmas)


def validate(geo: Geometry, thr: Threshold, precision: int = PREC_FP32) -> int:
    """Host-only argument check; returns the lcf_status code."""
    lib = load()
    tc = thr.to_c(1 if thr.cut == CUT_EXPLICIT else 0)
    return int(lib.lcf_validate(C.byref(geo), C.byref(tc), precision))


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(None)


def _diag_buffers(nd, nt, dev, cut, want, cov=False):
    """Device buffers for lcf_diag (dict of torch tensors) and the C struct, or (None, None)."""
    if not want:
        return None, None
    import torch
    dg = dict(eigvals=torch.empty((nd, nt), dtype=torch.float64, device=dev),
              weights=torch.empty((nd, nt), dtype=torch.float32, device=dev),
              k=torch.empty(nd, dtype=torch.int32, device=dev),
              sweeps=torch.empty(nd, dtype=torch.int32, device=dev),
              flags=torch.empty(nd, dtype=torch.int32, device=dev),
              alpha=torch.empty(nd, dtype=torch.float64, device=dev),
              rank=torch.empty(nd, dtype=torch.int32, device=dev))
    if cut == CUT_NCC:
        dg["curve"] = torch.empty((nd, nt), dtype=torch.float64, device=dev)
    if cut == CUT_MLP:
        dg["mlp_gate"] = torch.empty(nd, dtype=torch.float64, device=dev)
    if cov:
        dg["cov"] = torch.empty((nd, nt, nt), dtype=torch.complex128, device=dev)
        dg["eigvecs"] = torch.empty((nd, nt, nt), dtype=torch.complex128, device=dev)
    dgc = DiagC(*(_ptr(dg.get(n)) for n in ("eigvals", "weights", "k", "sweeps", "flags", "alpha",
                                            "cov", "eigvecs", "rank", "curve", "mlp_gate")))
    return dg, dgc


class Context:
    """An lcf_context on one device (options: schedule, max_sweeps, use_graph, autotune)."""

    def __init__(self, device: int = 0, schedule: int = 0, max_sweeps: int = 30, use_graph: int = 0,
                 autotune: int = 0):
        lib = load()
        h = C.c_void_p()
        _check(lib.lcf_create(device, C.byref(h)), "lcf_create")
        self._h = h
        self.device = device
        self.options = {OPT_MLP_GATE: 100}      # values set through this object (library defaults otherwise)
        self.set_option(OPT_SCHEDULE, schedule)
        self.set_option(OPT_MAX_SWEEPS, max_sweeps)
        self.set_option(OPT_USE_GRAPH, use_graph)
        self.set_option(OPT_AUTOTUNE, autotune)

    def tune_save(self, path: str):
        _check(load().lcf_tune_save(self._h, path.encode()), "lcf_tune_save")

    def tune_load(self, path: str):
        _check(load().lcf_tune_load(self._h, path.encode()), "lcf_tune_load")

    def set_option(self, opt: int, value: int):
        _check(load().lcf_set_option(self._h, opt, int(value)), "lcf_set_option")
        self.options[opt] = int(value)

    def close(self):
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            _check(load().lcf_destroy(h), "lcf_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self) -> int:
        return int(load().lcf_sync(self._h, _stream()))

    def stage_times(self, reset: bool = False) -> dict:
        """{stage name: (total device ms, launches)} accumulated with OPT_STAGE_TIMING on."""
        out = {}
        lib = load()
        for i, name in enumerate(STAGES):
            ms, n = C.c_double(), C.c_int64()
            _check(lib.lcf_stage_time(self._h, i, C.byref(ms), C.byref(n), 0), "lcf_stage_time")
            out[name] = (ms.value, n.value)
        if reset:
            _check(lib.lcf_stage_time(self._h, 0, None, None, 1), "lcf_stage_time")
        return out

    def filter(self, iq, gy: int, gx: int, thr: Threshold, precision: int = PREC_FP32,
               sigma_frac: float = 1.0 / 3.0, trunc_sigmas: float = 6.0, iq_out: bool = True,
               diag: bool = False, diag_cov: bool = False, explicit_w=None, out=None, noalloc: bool = False):
        """Filter one packet ``iq`` (torch complex64 on the GPU, [nt][ny][nx]).

        ``noalloc`` calls ``lcf_filter_noalloc`` (the library's fixed device
        block instead of its arena; pass ``out`` to allocate nothing here either).
        Returns (iq_out or None, pd, diag dict or None)."""
        import torch
        assert iq.is_cuda and iq.dtype == torch.complex64 and iq.is_contiguous() and iq.dim() == 3
        nt, ny, nx = iq.shape
        dev = iq.device
        geo = geometry(ny, nx, nt, gy, gx, sigma_frac, trunc_sigmas)
        if out is None:
            pd = torch.empty((ny, nx), dtype=torch.float32, device=dev)
            io = torch.empty_like(iq) if iq_out else None
        else:
            io, pd = out
        ew = None
        if thr.cut == CUT_EXPLICIT:
            ew = explicit_w.to(device=dev, dtype=torch.float32).contiguous()
        tc = thr.to_c(ew.data_ptr() if ew is not None else 0)
        dg, dgc = _diag_buffers(nd=gy * gx, nt=nt, dev=dev, cut=thr.cut, want=diag or diag_cov, cov=diag_cov)
        fn = load().lcf_filter_noalloc if noalloc else load().lcf_filter
        st = fn(self._h, C.byref(geo), C.byref(tc), precision, _ptr(iq), _ptr(io), _ptr(pd),
                C.byref(dgc) if dgc is not None else None, _stream())
        _check(st, "lcf_filter_noalloc" if noalloc else "lcf_filter")
        return io, pd, dg

    def filter_batch(self, iqs: Sequence, grids: Sequence, thr: Threshold, precision: int = PREC_FP32,
                     sigma_frac: float = 1.0 / 3.0, trunc_sigmas: float = 6.0, iq_out: bool = False,
                     outs=None, explicit_w=None):
        """Filter several packets of any shapes in one call. Returns (iq_outs, pds).

        With CUT_EXPLICIT, ``explicit_w`` is a list of per-packet [nd][nt] weight
        tensors; they are passed to the library back to back in call order."""
        import torch
        n = len(iqs)
        geos = (Geometry * n)()
        ip = (C.c_void_p * n)()
        op = (C.c_void_p * n)()
        pp = (C.c_void_p * n)()
        pds, ios = [], []
        for i, (iq, (gy, gx)) in enumerate(zip(iqs, grids)):
            assert iq.is_cuda and iq.dtype == torch.complex64 and iq.is_contiguous()
            nt, ny, nx = iq.shape
            geos[i] = geometry(ny, nx, nt, gy, gx, sigma_frac, trunc_sigmas)
            if outs is None:
                pd = torch.empty((ny, nx), dtype=torch.float32, device=iq.device)
                io = torch.empty_like(iq) if iq_out else None
            else:
                io, pd = outs[i]
            pds.append(pd)
            ios.append(io)
            ip[i] = iq.data_ptr()
            op[i] = io.data_ptr() if io is not None else None
            pp[i] = pd.data_ptr()
        ew = None
        if thr.cut == CUT_EXPLICIT and explicit_w is not None:
            ew = torch.cat([w.reshape(-1).to(device=iqs[0].device, dtype=torch.float32) for w in explicit_w])
        tc = thr.to_c(ew.data_ptr() if ew is not None else 0)
        st = load().lcf_filter_batch(self._h, n, geos, C.byref(tc), precision, ip, op, pp, _stream())
        _check(st, "lcf_filter_batch")
        return ios, pds

    # ---- learned weights
    MLP_NPARAM = 131712

    def mlp_init(self, seed: int = 0):
        _check(load().lcf_mlp_init(self._h, int(seed)), "lcf_mlp_init")

    def mlp_set_params(self, vec):
        import numpy as np
        v = np.ascontiguousarray(vec, dtype=np.float32)
        _check(load().lcf_mlp_set_params(self._h, v.ctypes.data, v.size), "lcf_mlp_set_params")

    def mlp_get_params(self):
        import numpy as np
        v = np.empty(self.MLP_NPARAM, dtype=np.float32)
        _check(load().lcf_mlp_get_params(self._h, v.ctypes.data, v.size), "lcf_mlp_get_params")
        return v

    def mlp_get_grads(self):
        import numpy as np
        v = np.empty(self.MLP_NPARAM, dtype=np.float32)
        _check(load().lcf_mlp_get_grads(self._h, v.ctypes.data, v.size), "lcf_mlp_get_grads")
        return v

    def mlp_save(self, path: str):
        _check(load().lcf_mlp_save(self._h, path.encode()), "lcf_mlp_save")

    def mlp_load(self, path: str):
        _check(load().lcf_mlp_load(self._h, path.encode()), "lcf_mlp_load")

    def mlp_infer(self, lam):
        """lam: torch float64 [b][128] on the GPU (descending). Returns float32 weights [b][128]."""
        import torch
        assert lam.is_cuda and lam.dtype == torch.float64 and lam.is_contiguous() and lam.shape[1] == 128
        w = torch.empty(lam.shape, dtype=torch.float32, device=lam.device)
        _check(load().lcf_mlp_infer(self._h, _ptr(lam), _ptr(w), lam.shape[0], _stream()), "lcf_mlp_infer")
        return w

    def mlp_train_step(self, lam, target, lr: float, loss_out=None):
        _check(load().lcf_mlp_train_step(self._h, _ptr(lam), _ptr(target), lam.shape[0], float(lr),
                                         _ptr(loss_out), _stream()), "lcf_mlp_train_step")

    def heevd(self, a, vectors: bool = True):
        """Batched Hermitian EVD of a (torch complex128 [n][nt][nt] on the GPU).
        Returns (w descending [n][nt] float64, v [n][nt][nt] or None, sweeps [n])."""
        import torch
        assert a.is_cuda and a.dtype == torch.complex128 and a.is_contiguous() and a.dim() == 3
        n, nt, _ = a.shape
        w = torch.empty((n, nt), dtype=torch.float64, device=a.device)
        v = torch.empty_like(a) if vectors else None
        sw = torch.empty(n, dtype=torch.int32, device=a.device)
        st = load().lcf_heevd_batched(self._h, n, nt, _ptr(a), _ptr(w), _ptr(v), _ptr(sw), _stream())
        _check(st, "lcf_heevd_batched")
        return w, v, sw


class Stream:
    """An lcf_stream: sliding packets of one geometry through one context
    (``lcf_stream_create`` / ``lcf_stream_push`` / ``lcf_stream_destroy``)."""

    def __init__(self, ctx: Context, ny: int, nx: int, nt: int, gy: int, gx: int, thr: Threshold,
                 precision: int = PREC_FP32, sigma_frac: float = 1.0 / 3.0, trunc_sigmas: float = 6.0,
                 explicit_w=None):
        lib = load()
        self.ctx = ctx
        self.geo = geometry(ny, nx, nt, gy, gx, sigma_frac, trunc_sigmas)
        self.thr = thr
        self._ew = explicit_w            # kept alive: the library keeps the pointer
        tc = thr.to_c(explicit_w.data_ptr() if explicit_w is not None else 0)
        h = C.c_void_p()
        _check(lib.lcf_stream_create(ctx._h, C.byref(self.geo), C.byref(tc), precision, C.byref(h)),
               "lcf_stream_create")
        self._h = h

    def push(self, iq, hop: int, iq_out: bool = True, diag: bool = False, out=None):
        """Filter the current packet ``iq`` (torch complex64 [nt][ny][nx] on the GPU)
        whose first nt - hop frames are the previous packet's last ones.
        Returns (iq_out or None, pd, diag dict or None)."""
        import torch
        assert iq.is_cuda and iq.dtype == torch.complex64 and iq.is_contiguous() and iq.dim() == 3
        nt, ny, nx = iq.shape
        assert (nt, ny, nx) == (self.geo.nt, self.geo.ny, self.geo.nx)
        if out is None:
            pd = torch.empty((ny, nx), dtype=torch.float32, device=iq.device)
            io = torch.empty_like(iq) if iq_out else None
        else:
            io, pd = out
        dg, dgc = _diag_buffers(self.geo.gy * self.geo.gx, nt, iq.device, self.thr.cut, diag)
        st = load().lcf_stream_push(self._h, _ptr(iq), int(hop), _ptr(io), _ptr(pd),
                                    C.byref(dgc) if dgc is not None else None, _stream())
        _check(st, "lcf_stream_push")
        return io, pd, dg

    def close(self):
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            _check(load().lcf_stream_destroy(h), "lcf_stream_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

