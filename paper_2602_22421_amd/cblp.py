"""Python binding of libcblp.so (ctypes; argument marshalling only).

Every function named like an entry point of ``include/cblp.h`` passes torch
device tensors through as raw pointers together with torch's current HIP
stream; all arithmetic of the method runs in the library's HIP kernels.  The
library must be built (``python paper_2602_22421_amd/csrc/build.py`` or
``__graft_entry__.build()``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcblp.so")

CBLP_OK, CBLP_EINVAL, CBLP_ENOMEM, CBLP_EHIP, CBLP_ENONFINITE, CBLP_ENOTCONVERGED = range(6)
CBLP_F32, CBLP_F64 = 1, 2
SPFOM_STEP_CONST, SPFOM_STEP_POLYAK = 0, 1
SPFOM_BOUND_GLOBAL, SPFOM_BOUND_SEGMENT = 0, 1
NTRACE = 10
TRACE_COLS = ("D", "P", "Z", "eta2", "infeas", "dbest", "lb", "gap", "step", "theta")
EXPORTS = ("cblp_create", "cblp_destroy", "spfom_reset", "spfom_iterate", "spfom_solve",
           "cblp_gap", "cblp_sales", "cblp_launch_info", "cblp_timing", "cblp_timing_read",
           "spfom_minibatch", "cblp_recover", "cblp_gap_static", "cblp_gap_static_max_products",
           "cblp_last_error", "cblp_batch_create", "cblp_batch_destroy", "spfom_batch_iterate",
           "spfom_batch_solve", "cblp_batch_tune", "cblp_batch_tune_cached", "cblp_batch_info",
           "cblp_batch_select", "cblp_refresh", "cblp_batch_mask", "cblp_batch_persistent",
           "gosim_lp_inputs",
           "gosim_period", "gosim_run",
           "wsnet_num_params", "wsnet_create", "wsnet_destroy", "wsnet_params", "wsnet_features",
           "wsnet_forward", "wsnet_gradients", "wsnet_train_step", "wsnet_train_epochs",
           "wsnet_targets", "wsnet_predict", "wsnet_start")


class SpfomParams(ctypes.Structure):
    _fields_ = [("rule", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("tau", ctypes.c_double), ("tau_vec", ctypes.c_void_p),
                ("gamma", ctypes.c_double), ("mu", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iters", ctypes.c_int64),
                ("bound", ctypes.c_int32), ("tau_decay", ctypes.c_double),
                ("decay_every", ctypes.c_int64)]


class SpfomStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("trace", ctypes.c_double * NTRACE),
                ("seconds", ctypes.c_double), ("status", ctypes.c_int32)]

    def as_dict(self):
        d = {k: float(self.trace[i]) for i, k in enumerate(TRACE_COLS)}
        d.update(iters=int(self.iters), seconds=float(self.seconds), status=int(self.status))
        return d


class CblpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cblp error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = _LIB_PATH) -> ctypes.CDLL:
    """Load libcblp.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2602_22421_amd/csrc/build.py")
    lib = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.cblp_create.restype = ctypes.c_int
    lib.cblp_create.argtypes = [ctypes.POINTER(vp), i64, i64, i64, vp, vp, vp, vp, vp, vp, vp,
                                vp, vp, vp, vp, i32, vp]
    lib.cblp_destroy.restype = None
    lib.cblp_destroy.argtypes = [vp]
    lib.spfom_reset.restype = ctypes.c_int
    lib.spfom_reset.argtypes = [vp, vp]
    lib.spfom_iterate.restype = ctypes.c_int
    lib.spfom_iterate.argtypes = [vp, vp, ctypes.POINTER(SpfomParams), i64, vp,
                                  ctypes.POINTER(SpfomStats), vp]
    lib.cblp_gap_static.restype = ctypes.c_int
    lib.cblp_gap_static.argtypes = [i64, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, i32,
                                    vp, vp, vp, vp]
    lib.cblp_gap_static_max_products.restype = i64
    lib.cblp_gap_static_max_products.argtypes = []
    lib.cblp_recover.restype = ctypes.c_int
    lib.cblp_recover.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.spfom_minibatch.restype = ctypes.c_int
    lib.spfom_minibatch.argtypes = [vp, vp, ctypes.POINTER(SpfomParams), vp, i64, i64, vp, vp]
    lib.spfom_solve.restype = ctypes.c_int
    lib.spfom_solve.argtypes = [vp, vp, ctypes.POINTER(SpfomParams), ctypes.POINTER(SpfomStats), vp]
    lib.cblp_gap.restype = ctypes.c_int
    lib.cblp_gap.argtypes = [vp, vp, ctypes.POINTER(SpfomStats), vp]
    lib.cblp_sales.restype = ctypes.c_int
    lib.cblp_sales.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.cblp_launch_info.restype = ctypes.c_int
    lib.cblp_launch_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                     ctypes.POINTER(i32), ctypes.POINTER(i32),
                                     ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_int64)]
    lib.cblp_timing.restype = ctypes.c_int
    lib.cblp_timing.argtypes = [vp, i32]
    lib.cblp_timing_read.restype = ctypes.c_int
    lib.cblp_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int64), vp]
    pp = ctypes.POINTER(vp)
    lib.cblp_batch_create.restype = ctypes.c_int
    lib.cblp_batch_create.argtypes = [pp, i32, pp, vp]
    lib.cblp_batch_destroy.restype = None
    lib.cblp_batch_destroy.argtypes = [vp]
    lib.spfom_batch_iterate.restype = ctypes.c_int
    lib.spfom_batch_iterate.argtypes = [vp, pp, pp, ctypes.POINTER(SpfomParams), i64, vp, vp]
    lib.spfom_batch_solve.restype = ctypes.c_int
    lib.spfom_batch_solve.argtypes = [vp, pp, pp, ctypes.POINTER(SpfomParams),
                                      ctypes.POINTER(SpfomStats), vp]
    lib.cblp_batch_tune.restype = ctypes.c_int
    lib.cblp_batch_tune.argtypes = [vp, pp, pp, ctypes.POINTER(SpfomParams), i32,
                                    ctypes.POINTER(i32), vp]
    lib.cblp_batch_tune_cached.restype = ctypes.c_int
    lib.cblp_batch_tune_cached.argtypes = [vp, pp, pp, ctypes.POINTER(SpfomParams), i32,
                                           ctypes.c_char_p, ctypes.POINTER(i32),
                                           ctypes.POINTER(i32), vp]
    lib.cblp_batch_info.restype = ctypes.c_int
    lib.cblp_batch_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                    ctypes.POINTER(i32)]
    lib.cblp_batch_select.restype = ctypes.c_int
    lib.cblp_batch_select.argtypes = [vp, i32]
    lib.cblp_refresh.restype = ctypes.c_int
    lib.cblp_refresh.argtypes = [vp, vp]
    lib.cblp_batch_mask.restype = ctypes.c_int
    lib.cblp_batch_mask.argtypes = [vp, vp]
    lib.cblp_batch_persistent.restype = ctypes.c_int
    lib.cblp_batch_persistent.argtypes = [vp, i32]
    lib.gosim_lp_inputs.restype = ctypes.c_int
    lib.gosim_lp_inputs.argtypes = [i32, i64, vp, i64, ctypes.c_double, vp, vp, vp, vp, i32, vp]
    lib.gosim_period.restype = ctypes.c_int
    lib.gosim_period.argtypes = [i32, i64, i64, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, i32, vp]
    lib.gosim_run.restype = ctypes.c_int
    lib.gosim_run.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp, ctypes.POINTER(SpfomParams),
                              ctypes.c_double, vp, vp, vp, vp, vp, vp]
    lib.cblp_last_error.restype = ctypes.c_char_p
    lib.cblp_last_error.argtypes = []
    lib.wsnet_num_params.restype = i64
    lib.wsnet_num_params.argtypes = []
    lib.wsnet_create.restype = ctypes.c_int
    lib.wsnet_create.argtypes = [ctypes.POINTER(vp), ctypes.c_uint64, vp]
    lib.wsnet_destroy.restype = None
    lib.wsnet_destroy.argtypes = [vp]
    lib.wsnet_params.restype = ctypes.c_int
    lib.wsnet_params.argtypes = [vp, vp, vp, vp]
    lib.wsnet_features.restype = ctypes.c_int
    lib.wsnet_features.argtypes = [vp, vp, vp]
    lib.wsnet_forward.restype = ctypes.c_int
    lib.wsnet_forward.argtypes = [vp, vp, i64, vp, vp]
    lib.wsnet_gradients.restype = ctypes.c_int
    lib.wsnet_gradients.argtypes = [vp, vp, vp, i64, vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.wsnet_train_step.restype = ctypes.c_int
    lib.wsnet_train_step.argtypes = [vp, vp, vp, i64, ctypes.c_float,
                                     ctypes.POINTER(ctypes.c_double), vp]
    lib.wsnet_train_epochs.restype = ctypes.c_int
    lib.wsnet_train_epochs.argtypes = [vp, vp, vp, i64, i64, i32, ctypes.c_float, ctypes.c_uint64,
                                       vp, vp]
    lib.wsnet_targets.restype = ctypes.c_int
    lib.wsnet_targets.argtypes = [vp, vp, vp, vp]
    lib.wsnet_predict.restype = ctypes.c_int
    lib.wsnet_predict.argtypes = [vp, vp, vp, vp]
    lib.wsnet_start.restype = ctypes.c_int
    lib.wsnet_start.argtypes = [vp, vp, vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double), vp]
    _lib = lib
    return lib


def last_error() -> str:
    return load().cblp_last_error().decode()


def _check(rc: int, allow=()):
    if rc != CBLP_OK and rc not in allow:
        raise CblpError(rc, last_error())
    return rc


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


# ------------------------------------------------------------------ raw ABI

def cblp_create(L, n, m, seg_ptr, prod_idx, v, w, v0, lam, r, a_ptr, a_idx, a_val, c,
                dtype: int, stream=None) -> int:
    h = ctypes.c_void_p()
    _check(load().cblp_create(ctypes.byref(h), int(L), int(n), int(m), _ptr(seg_ptr),
                              _ptr(prod_idx), _ptr(v), _ptr(w), _ptr(v0), _ptr(lam), _ptr(r),
                              _ptr(a_ptr), _ptr(a_idx), _ptr(a_val), _ptr(c), int(dtype),
                              _stream(stream)))
    return h.value


def cblp_destroy(h) -> None:
    if h:
        load().cblp_destroy(ctypes.c_void_p(h))


def spfom_reset(h, stream=None) -> None:
    _check(load().spfom_reset(ctypes.c_void_p(h), _stream(stream)))


def cblp_refresh(h, stream=None) -> None:
    _check(load().cblp_refresh(ctypes.c_void_p(h), _stream(stream)))


def spfom_iterate(h, eta, params: SpfomParams, iters: int, trace: Optional[np.ndarray] = None,
                  stats: Optional[SpfomStats] = None, stream=None) -> None:
    tp = None
    if trace is not None:
        assert trace.dtype == np.float64 and trace.flags.c_contiguous
        assert trace.shape == (iters, NTRACE)
        tp = ctypes.c_void_p(trace.ctypes.data)
    _check(load().spfom_iterate(ctypes.c_void_p(h), _ptr(eta), ctypes.byref(params), int(iters),
                                tp, None if stats is None else ctypes.byref(stats),
                                _stream(stream)))


def spfom_minibatch(h, eta, params: SpfomParams, batch, iters: int,
                    trace: Optional[np.ndarray] = None, stream=None) -> None:
    """batch: int32 device tensor [iters, B] of segment ids."""
    assert batch.dtype == torch.int32 and batch.is_contiguous() and batch.dim() == 2
    assert batch.shape[0] == iters
    tp = None
    if trace is not None:
        assert trace.dtype == np.float64 and trace.flags.c_contiguous
        assert trace.shape == (iters, NTRACE)
        tp = ctypes.c_void_p(trace.ctypes.data)
    _check(load().spfom_minibatch(ctypes.c_void_p(h), _ptr(eta), ctypes.byref(params),
                                  _ptr(batch), int(batch.shape[1]), int(iters), tp,
                                  _stream(stream)))


def spfom_solve(h, eta, params: SpfomParams, stream=None) -> SpfomStats:
    st = SpfomStats()
    _check(load().spfom_solve(ctypes.c_void_p(h), _ptr(eta), ctypes.byref(params),
                              ctypes.byref(st), _stream(stream)), allow=(CBLP_ENOTCONVERGED,))
    return st


def cblp_gap(h, eta, stream=None) -> SpfomStats:
    st = SpfomStats()
    _check(load().cblp_gap(ctypes.c_void_p(h), _ptr(eta), ctypes.byref(st), _stream(stream)))
    return st


def cblp_sales(h, eta, S_out=None, u_out=None, seg_R_out=None, s_out=None, stream=None) -> None:
    _check(load().cblp_sales(ctypes.c_void_p(h), _ptr(eta), _ptr(S_out), _ptr(u_out),
                             _ptr(seg_R_out), _ptr(s_out), _stream(stream)))


SEG_KERNELS = ("f32-three-part-lds-prices", "f32-three-part-split-prices-ids16",
               "f32-three-part-split-prices-ids32", "f64-8-lane-ids16", "f64-8-lane-ids32")


def cblp_gap_static(prob: "Problem", eta, S_out, bounds, stream=None) -> None:
    """The allocation-free pass over prob's device arrays (not its handle)."""
    _check(load().cblp_gap_static(prob.L, prob.n, prob.m, _ptr(prob.seg_ptr), _ptr(prob.idx),
                                  _ptr(prob.v), _ptr(prob.w), _ptr(prob.v0), _ptr(prob.lam),
                                  _ptr(prob.r), _ptr(prob.a_ptr), _ptr(prob.a_idx),
                                  _ptr(prob.a_val), _ptr(prob.c),
                                  CBLP_F32 if prob.dtype == torch.float32 else CBLP_F64,
                                  _ptr(eta), _ptr(S_out), _ptr(bounds), _stream(stream)))


def cblp_gap_static_max_products() -> int:
    return int(load().cblp_gap_static_max_products())


def cblp_recover(h, y, rank, alpha, alpha0, stream=None) -> None:
    _check(load().cblp_recover(ctypes.c_void_p(h), _ptr(y), _ptr(rank), _ptr(alpha),
                               _ptr(alpha0), _stream(stream)))


def cblp_launch_info(h) -> dict:
    g, b, b64 = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    f, k = ctypes.c_int32(), ctypes.c_int32()
    e = ctypes.c_int64()
    _check(load().cblp_launch_info(ctypes.c_void_p(h), ctypes.byref(g), ctypes.byref(b),
                                   ctypes.byref(b64), ctypes.byref(f), ctypes.byref(k),
                                   ctypes.byref(e)))
    return {"seg_grid": g.value, "lds_bins": b.value, "lds_bins64": b64.value,
            "fx_bits": f.value, "kernel": SEG_KERNELS[k.value], "slot_entries": e.value}


def cblp_timing(h, enable: bool) -> None:
    _check(load().cblp_timing(ctypes.c_void_p(h), int(bool(enable))))


def cblp_timing_read(h, stream=None):
    """Returns ((segment_ms, dual_ms), (segment_launches, dual_launches))."""
    ms = (ctypes.c_double * 2)()
    n = (ctypes.c_int64 * 2)()
    _check(load().cblp_timing_read(ctypes.c_void_p(h), ms, n, _stream(stream)))
    return (ms[0], ms[1]), (n[0], n[1])


# ------------------------------------------------------------------ convenience

def make_params(*, rule: int = SPFOM_STEP_CONST, check_every: int = 10, tau: float = 1.0,
                tau_vec: Optional[torch.Tensor] = None, gamma: float = 1.0, mu: float = 0.0,
                tol: float = 1e-4, max_iters: int = 10000,
                bound: int = SPFOM_BOUND_GLOBAL, tau_decay: float = 1.0,
                decay_every: int = 1) -> SpfomParams:
    p = SpfomParams(int(rule), int(check_every), float(tau),
                    None if tau_vec is None else tau_vec.data_ptr(), float(gamma), float(mu),
                    float(tol), int(max_iters), int(bound), float(tau_decay), int(decay_every))
    p._keep = tau_vec  # keep the tensor alive with the struct
    return p


class Problem:
    """An instance uploaded to the current device plus its solver handle.

    ``inst`` is any object with the fields of
    ``paper_2602_22421_amd.instances.Instance``; its real arrays are converted
    to ``dtype`` (torch.float32 or torch.float64) on the device."""

    def __init__(self, inst, dtype=torch.float32, device="cuda"):
        self.dtype = dtype
        self.device = torch.device(device)
        npdt = np.float32 if dtype == torch.float32 else np.float64
        dev = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(self.device)
        self.L, self.n, self.m = int(inst.L), int(inst.n), int(inst.m)
        self.seg_ptr = dev(inst.seg_ptr, np.int64)
        self.idx = dev(inst.idx, np.int32)
        self.v, self.w = dev(inst.v, npdt), dev(inst.w, npdt)
        self.v0, self.lam = dev(inst.v0, npdt), dev(inst.lam, npdt)
        self.r, self.c = dev(inst.r, npdt), dev(inst.c, npdt)
        if inst.a_ptr is None:
            self.a_ptr = self.a_idx = self.a_val = None
        else:
            self.a_ptr = dev(inst.a_ptr, np.int64)
            self.a_idx = dev(inst.a_idx, np.int32)
            self.a_val = dev(inst.a_val, npdt)
        self.nnz = int(inst.seg_ptr[-1])
        self.h = cblp_create(self.L, self.n, self.m, self.seg_ptr, self.idx, self.v, self.w,
                             self.v0, self.lam, self.r, self.a_ptr, self.a_idx, self.a_val,
                             self.c, CBLP_F32 if dtype == torch.float32 else CBLP_F64)

    def close(self):
        if getattr(self, "h", None):
            cblp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def zeros_eta(self) -> torch.Tensor:
        return torch.zeros(self.m, dtype=self.dtype, device=self.device)

    def tensor(self, a) -> torch.Tensor:
        return torch.as_tensor(np.asarray(a), dtype=self.dtype).to(self.device)

    def reset(self):
        spfom_reset(self.h)

    def refresh(self, v=None, w=None, c=None):
        """New attractions and capacities (numpy arrays or tensors) written into
        this Problem's device arrays in place, then re-read by the handle."""
        for dst, src in ((self.v, v), (self.w, w), (self.c, c)):
            if src is not None:
                dst.copy_(torch.as_tensor(np.asarray(src) if not isinstance(src, torch.Tensor)
                                          else src, dtype=self.dtype))
        cblp_refresh(self.h)

    def iterate(self, eta: torch.Tensor, iters: int, params: SpfomParams, trace: bool = True):
        tr = np.zeros((int(iters), NTRACE)) if trace else None
        st = SpfomStats()
        spfom_iterate(self.h, eta, params, iters, tr, st)
        return tr, st

    def solve(self, eta: torch.Tensor, params: SpfomParams) -> SpfomStats:
        return spfom_solve(self.h, eta, params)

    def recover(self, y: torch.Tensor):
        """Nested assortments and their probabilities behind per-entry sales
        y [nnz] (float64 device tensor): (rank, alpha, alpha0)."""
        assert y.dtype == torch.float64 and y.numel() == self.nnz
        rank = torch.empty(self.nnz, dtype=torch.int32, device=self.device)
        alpha = torch.empty(self.nnz, dtype=torch.float64, device=self.device)
        alpha0 = torch.empty(self.L, dtype=torch.float64, device=self.device)
        cblp_recover(self.h, y.contiguous(), rank, alpha, alpha0)
        return rank, alpha, alpha0

    def minibatch(self, eta: torch.Tensor, batch, params: SpfomParams, trace: bool = True):
        """Stochastic minibatch iterations over the rows of batch ([iters, B]
        segment ids, numpy or a device int32 tensor)."""
        if not isinstance(batch, torch.Tensor):
            batch = torch.from_numpy(np.ascontiguousarray(batch, dtype=np.int32)).to(self.device)
        iters = int(batch.shape[0])
        tr = np.zeros((iters, NTRACE)) if trace else None
        spfom_minibatch(self.h, eta, params, batch, iters, tr)
        return tr

    def gap(self, eta: torch.Tensor) -> dict:
        return cblp_gap(self.h, eta).as_dict()

    def sales(self, eta: torch.Tensor, seg_R: bool = False, entries: bool = False):
        """(S, u, R) at fixed eta; with entries=True also the per-entry sales
        s [nnz] in the instance's CSR order, as a fourth value."""
        S = torch.zeros(self.n, dtype=torch.float64, device=self.device)
        u = torch.zeros(self.m, dtype=torch.float64, device=self.device)
        R = torch.zeros(self.L, dtype=self.dtype, device=self.device) if seg_R else None
        s = torch.zeros(self.nnz, dtype=torch.float64, device=self.device) if entries else None
        cblp_sales(self.h, eta, S, u, R, s)
        return (S, u, R, s) if entries else (S, u, R)


# ------------------------------------------------------------------ batches

def _ptr_array(tensors):
    arr = (ctypes.c_void_p * len(tensors))()
    for q, t in enumerate(tensors):
        arr[q] = None if t is None else t.data_ptr()
    return arr


def cblp_batch_create(handles, stream=None) -> int:
    hs = (ctypes.c_void_p * len(handles))(*handles)
    b = ctypes.c_void_p()
    _check(load().cblp_batch_create(ctypes.byref(b), len(handles), hs, _stream(stream)))
    return b.value


def cblp_batch_destroy(b) -> None:
    if b:
        load().cblp_batch_destroy(ctypes.c_void_p(b))


def spfom_batch_iterate(b, etas, tau_vecs, params: SpfomParams, iters: int, rows=None,
                        stream=None) -> None:
    tv = None if tau_vecs is None else _ptr_array(tau_vecs)
    rp = None if rows is None else ctypes.c_void_p(rows.ctypes.data)
    _check(load().spfom_batch_iterate(ctypes.c_void_p(b), _ptr_array(etas), tv,
                                      ctypes.byref(params), int(iters), rp, _stream(stream)))


def spfom_batch_solve(b, etas, tau_vecs, params: SpfomParams, stream=None):
    outs = (SpfomStats * len(etas))()
    tv = None if tau_vecs is None else _ptr_array(tau_vecs)
    _check(load().spfom_batch_solve(ctypes.c_void_p(b), _ptr_array(etas), tv,
                                    ctypes.byref(params), outs, _stream(stream)),
           allow=(CBLP_ENOTCONVERGED, CBLP_ENONFINITE))
    return [o.as_dict() for o in outs]


def cblp_batch_tune_cached(b, etas, tau_vecs, params: SpfomParams, iters: int, cache_path: str,
                           stream=None):
    chosen, ipb = ctypes.c_int32(), ctypes.c_int32()
    tv = None if tau_vecs is None else _ptr_array(tau_vecs)
    _check(load().cblp_batch_tune_cached(ctypes.c_void_p(b), _ptr_array(etas), tv,
                                         ctypes.byref(params), int(iters),
                                         os.fsencode(cache_path), ctypes.byref(chosen),
                                         ctypes.byref(ipb), _stream(stream)))
    return chosen.value, ipb.value


def cblp_batch_tune(b, etas, tau_vecs, params: SpfomParams, iters: int, stream=None) -> int:
    chosen = ctypes.c_int32()
    tv = None if tau_vecs is None else _ptr_array(tau_vecs)
    _check(load().cblp_batch_tune(ctypes.c_void_p(b), _ptr_array(etas), tv, ctypes.byref(params),
                                  int(iters), ctypes.byref(chosen), _stream(stream)))
    return chosen.value


def cblp_batch_select(b, variant: int) -> None:
    _check(load().cblp_batch_select(ctypes.c_void_p(b), int(variant)))


def cblp_batch_persistent(b, mode: int) -> None:
    _check(load().cblp_batch_persistent(ctypes.c_void_p(b), int(mode)))


def cblp_batch_mask(b, take_part=None) -> None:
    arr = None
    if take_part is not None:
        arr = np.ascontiguousarray(np.asarray(take_part) != 0, dtype=np.int32)
    _check(load().cblp_batch_mask(ctypes.c_void_p(b),
                                  None if arr is None else arr.ctypes.data_as(ctypes.c_void_p)))


def cblp_batch_info(b) -> dict:
    it, g, v = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load().cblp_batch_info(ctypes.c_void_p(b), ctypes.byref(it), ctypes.byref(g),
                                  ctypes.byref(v)))
    return {"items": it.value, "grid": g.value, "variant": v.value}


class Batch:
    """Several Problems advanced together (the Problems must outlive the batch
    and must not be iterated on their own while it exists)."""

    def __init__(self, problems):
        self.problems = list(problems)
        self.b = cblp_batch_create([p.h for p in self.problems])

    def close(self):
        if getattr(self, "b", None):
            cblp_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def iterate(self, etas, iters: int, params: SpfomParams, tau_vecs=None):
        rows = np.zeros((len(self.problems), NTRACE))
        spfom_batch_iterate(self.b, etas, tau_vecs, params, iters, rows)
        return rows

    def solve(self, etas, params: SpfomParams, tau_vecs=None):
        return spfom_batch_solve(self.b, etas, tau_vecs, params)

    def tune(self, etas, params: SpfomParams, iters: int = 5, tau_vecs=None) -> int:
        return cblp_batch_tune(self.b, etas, tau_vecs, params, iters)

    def tune_cached(self, etas, params: SpfomParams, cache_path: str, iters: int = 5,
                    tau_vecs=None):
        """(variant, items per block) from the tuning cache, or tuned and stored."""
        return cblp_batch_tune_cached(self.b, etas, tau_vecs, params, iters, cache_path)

    def info(self) -> dict:
        return cblp_batch_info(self.b)

    def persistent(self, mode: int) -> None:
        """-1: one launch per solve for small batches (default), 0: never, 1: always."""
        cblp_batch_persistent(self.b, mode)

    def select(self, variant: int) -> None:
        cblp_batch_select(self.b, variant)

    def mask(self, take_part=None) -> None:
        cblp_batch_mask(self.b, take_part)


# ------------------------------------------------- bid-price policy simulation

def _dt(t: torch.Tensor) -> int:
    return CBLP_F32 if t.dtype == torch.float32 else CBLP_F64


def gosim_lp_inputs(inv, periods_left: int, tau0: float, r, c, tau, eta=None,
                    stream=None) -> None:
    """inv [runs, n] int64, r/c/tau/eta [runs, n] (one dtype), device tensors."""
    runs, n = r.shape
    assert inv.dtype == torch.int64 and inv.shape == r.shape and c.dtype == tau.dtype == r.dtype
    assert eta is None or (eta.dtype == r.dtype and eta.shape == r.shape)
    _check(load().gosim_lp_inputs(int(runs), int(n), _ptr(inv), int(periods_left), float(tau0),
                                  _ptr(r), _ptr(c), _ptr(tau), _ptr(eta), _dt(r), _stream(stream)))


def gosim_period(K: int, eta, r, prefs, u, inv, offer, sales, revenue, in_stock=None,
                 stream=None) -> None:
    """eta/r [runs, n], prefs [runs, N, n] (one dtype), u [runs, N] float64,
    inv/sales [runs, n] int64, offer [runs, K] int32, revenue [runs] float64."""
    runs, N, n = prefs.shape
    assert eta.dtype == r.dtype == prefs.dtype and u.dtype == torch.float64
    assert inv.dtype == sales.dtype == torch.int64 and offer.dtype == torch.int32
    assert offer.shape == (runs, K) and sales.shape == (runs, n) and u.shape == (runs, N)
    _check(load().gosim_period(int(runs), int(N), int(n), int(K), _ptr(eta), _ptr(r), _ptr(prefs),
                               _ptr(u), _ptr(inv), _ptr(offer), _ptr(sales), _ptr(revenue),
                               _ptr(in_stock), _dt(r), _stream(stream)))


def gosim_run(b, periods: int, K: int, prefs, u, r, inv, eta, tau_work, params: SpfomParams,
              tau0: float, offers, sales, revenue, lp_iters: Optional[np.ndarray] = None,
              lp_gap: Optional[np.ndarray] = None, stream=None) -> None:
    lp = gp = None
    if lp_iters is not None:
        assert lp_iters.dtype == np.int64 and lp_iters.flags.c_contiguous
        lp = ctypes.c_void_p(lp_iters.ctypes.data)
    if lp_gap is not None:
        assert lp_gap.dtype == np.float64 and lp_gap.flags.c_contiguous
        gp = ctypes.c_void_p(lp_gap.ctypes.data)
    _check(load().gosim_run(ctypes.c_void_p(b), int(periods), int(K), _ptr(prefs), _ptr(u), _ptr(r),
                            _ptr(inv), _ptr(eta), _ptr(tau_work), ctypes.byref(params), float(tau0),
                            _ptr(offers), _ptr(sales), _ptr(revenue), lp, gp, _stream(stream)))


class GoSim:
    """The GO bid-price policy on a market (``instances.Market``) for all its
    runs: one handle per run over shared structure arrays and one
    [runs, N, n] preference work buffer, batched together."""

    def __init__(self, market, dtype=torch.float32, device="cuda"):
        self.dtype, self.device = dtype, torch.device(device)
        npdt = np.float32 if dtype == torch.float32 else np.float64
        dev = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(self.device)
        R, T, N, n = market.runs, market.periods, market.customers, market.n
        self.runs, self.periods, self.N, self.n = R, T, N, n
        self.r = dev(market.r, npdt)
        self.inv0 = np.ascontiguousarray(market.inv0, dtype=np.int64)
        self.prefs = dev(market.prefs, npdt)
        self.u = dev(market.u, np.float64)
        self.seg_ptr = dev(np.arange(N + 1) * n, np.int64)
        self.idx = dev(np.tile(np.arange(n), N), np.int32)
        self.w = torch.zeros(N * n, dtype=dtype, device=self.device)
        self.v0 = torch.ones(N, dtype=dtype, device=self.device)
        self.lam = torch.ones(N, dtype=dtype, device=self.device)
        self.v = self.prefs[0].clone() if T else torch.ones(R, N, n, dtype=dtype, device=self.device)
        self.c = torch.zeros(R, n, dtype=dtype, device=self.device)
        self.tau = torch.ones(R, n, dtype=dtype, device=self.device)
        self.handles = []
        try:
            for q in range(R):
                self.handles.append(cblp_create(N, n, n, self.seg_ptr, self.idx, self.v[q], self.w,
                                                self.v0, self.lam, self.r[q], None, None, None,
                                                self.c[q], _dt(self.r)))
            self.b = cblp_batch_create(self.handles)
        except Exception:
            self.close()
            raise

    def close(self):
        if getattr(self, "b", None):
            cblp_batch_destroy(self.b)
            self.b = None
        for h in getattr(self, "handles", []):
            cblp_destroy(h)
        self.handles = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, K: int, params: SpfomParams, tau0: float, eta=None):
        """All periods from the initial stock; returns a dict of offers
        [T, runs, K], sales [T, runs, n], revenue [T, runs], lp_iters and
        lp_gap [T, runs] (numpy), the final stock and the final duals
        (tensors)."""
        T, R, n = self.periods, self.runs, self.n
        inv = torch.from_numpy(self.inv0.copy()).to(self.device)
        eta = torch.zeros(R, n, dtype=self.dtype, device=self.device) if eta is None else eta
        offers = torch.empty(T, R, K, dtype=torch.int32, device=self.device)
        sales = torch.empty(T, R, n, dtype=torch.int64, device=self.device)
        revenue = torch.empty(T, R, dtype=torch.float64, device=self.device)
        lp = np.zeros((T, R), dtype=np.int64)
        gap = np.zeros((T, R))
        gosim_run(self.b, T, K, self.prefs, self.u, self.r, inv, eta, self.tau, params, tau0,
                  offers, sales, revenue, lp, gap)
        return {"offers": offers.cpu().numpy(), "sales": sales.cpu().numpy(),
                "revenue": revenue.cpu().numpy(), "lp_iters": lp, "lp_gap": gap, "inv": inv,
                "eta": eta}


# ------------------------------------------------------------ learned warm start

def wsnet_num_params() -> int:
    return int(load().wsnet_num_params())


def wsnet_create(seed: int = 0, stream=None) -> int:
    w = ctypes.c_void_p()
    _check(load().wsnet_create(ctypes.byref(w), ctypes.c_uint64(seed), _stream(stream)))
    return w.value


def wsnet_destroy(w) -> None:
    if w:
        load().wsnet_destroy(ctypes.c_void_p(w))


def wsnet_params(w, get: Optional[np.ndarray] = None, set: Optional[np.ndarray] = None,
                 stream=None) -> None:
    for a in (get, set):
        if a is not None:
            assert a.dtype == np.float32 and a.flags.c_contiguous
            assert a.size == wsnet_num_params()
    _check(load().wsnet_params(ctypes.c_void_p(w),
                               None if get is None else get.ctypes.data_as(ctypes.c_void_p),
                               None if set is None else set.ctypes.data_as(ctypes.c_void_p),
                               _stream(stream)))


def wsnet_features(h, X: torch.Tensor, stream=None) -> None:
    assert X.dtype == torch.float32 and X.is_contiguous()
    _check(load().wsnet_features(ctypes.c_void_p(h), _ptr(X), _stream(stream)))


def wsnet_forward(w, X: torch.Tensor, y: torch.Tensor, stream=None) -> None:
    assert X.dtype == torch.float32 and y.dtype == torch.float32 and X.shape[1] == 4
    assert X.is_contiguous() and y.numel() >= X.shape[0]
    _check(load().wsnet_forward(ctypes.c_void_p(w), _ptr(X), X.shape[0], _ptr(y),
                                _stream(stream)))


def wsnet_gradients(w, X: torch.Tensor, Y: torch.Tensor, grads: Optional[torch.Tensor] = None,
                    stream=None) -> float:
    assert X.dtype == torch.float32 and Y.dtype == torch.float32 and X.shape[1] == 4
    assert X.is_contiguous() and Y.numel() == X.shape[0]
    if grads is not None:
        assert grads.dtype == torch.float32 and grads.numel() == wsnet_num_params()
    loss = ctypes.c_double()
    _check(load().wsnet_gradients(ctypes.c_void_p(w), _ptr(X), _ptr(Y), X.shape[0], _ptr(grads),
                                  ctypes.byref(loss), _stream(stream)))
    return loss.value


def wsnet_train_step(w, X: torch.Tensor, Y: torch.Tensor, lr: float, want_loss: bool = False,
                     stream=None) -> Optional[float]:
    assert X.dtype == torch.float32 and Y.dtype == torch.float32 and X.shape[1] == 4
    assert X.is_contiguous() and Y.numel() == X.shape[0]
    loss = ctypes.c_double()
    _check(load().wsnet_train_step(ctypes.c_void_p(w), _ptr(X), _ptr(Y), X.shape[0],
                                   ctypes.c_float(lr), ctypes.byref(loss) if want_loss else None,
                                   _stream(stream)))
    return loss.value if want_loss else None


def wsnet_train_epochs(w, X: torch.Tensor, Y: torch.Tensor, batch: int, epochs: int, lr: float,
                       seed: int = 0, stream=None) -> np.ndarray:
    assert X.dtype == torch.float32 and Y.dtype == torch.float32 and X.shape[1] == 4
    assert X.is_contiguous() and Y.is_contiguous() and Y.numel() == X.shape[0]
    losses = np.zeros(max(int(epochs), 1))
    _check(load().wsnet_train_epochs(ctypes.c_void_p(w), _ptr(X), _ptr(Y), X.shape[0], int(batch),
                                     int(epochs), ctypes.c_float(lr), ctypes.c_uint64(seed),
                                     losses.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
    return losses[:int(epochs)]


def wsnet_targets(h, eta: torch.Tensor, Y: torch.Tensor, stream=None) -> None:
    assert Y.dtype == torch.float32 and Y.is_contiguous()
    _check(load().wsnet_targets(ctypes.c_void_p(h), _ptr(eta), _ptr(Y), _stream(stream)))


def wsnet_predict(w, h, eta: torch.Tensor, stream=None) -> None:
    _check(load().wsnet_predict(ctypes.c_void_p(w), ctypes.c_void_p(h), _ptr(eta),
                                _stream(stream)))


def wsnet_start(w, h, eta: torch.Tensor, stream=None) -> dict:
    used = ctypes.c_int32()
    dp, d0 = ctypes.c_double(), ctypes.c_double()
    _check(load().wsnet_start(ctypes.c_void_p(w), ctypes.c_void_p(h), _ptr(eta), ctypes.byref(used),
                              ctypes.byref(dp), ctypes.byref(d0), _stream(stream)))
    return {"used": bool(used.value), "D_pred": dp.value, "D0": d0.value}


class WarmStartNet:
    """The warm-start network (owns its device parameters)."""

    def __init__(self, seed: int = 0):
        self.w = wsnet_create(seed)

    def close(self):
        if getattr(self, "w", None):
            wsnet_destroy(self.w)
            self.w = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def params(self) -> np.ndarray:
        out = np.empty(wsnet_num_params(), np.float32)
        wsnet_params(self.w, get=out)
        return out

    @params.setter
    def params(self, p) -> None:
        wsnet_params(self.w, set=np.ascontiguousarray(p, dtype=np.float32))

    def forward(self, X: torch.Tensor) -> torch.Tensor:
        y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        wsnet_forward(self.w, X, y)
        return y

    def gradients(self, X: torch.Tensor, Y: torch.Tensor):
        g = torch.empty(wsnet_num_params(), dtype=torch.float32, device=X.device)
        loss = wsnet_gradients(self.w, X, Y, g)
        return loss, g

    def train_step(self, X: torch.Tensor, Y: torch.Tensor, lr: float, want_loss=False):
        return wsnet_train_step(self.w, X, Y, lr, want_loss)

    def train(self, X: torch.Tensor, Y: torch.Tensor, *, epochs: int, batch: int, lr: float,
              seed: int = 0) -> np.ndarray:
        return wsnet_train_epochs(self.w, X, Y, batch, epochs, lr, seed)

    def predict(self, prob: "Problem") -> torch.Tensor:
        eta = prob.zeros_eta()
        wsnet_predict(self.w, prob.h, eta)
        return eta

    def start(self, prob: "Problem"):
        """The warm start with its cold fallback (decided in the library):
        returns (eta, info) with info = {used, D_pred, D0}."""
        eta = prob.zeros_eta()
        info = wsnet_start(self.w, prob.h, eta)
        return eta, info


def targets(prob: "Problem", eta: torch.Tensor) -> torch.Tensor:
    """What the network predicts for each dual's row ([m]; m = n for A = I)."""
    Y = torch.empty(prob.m, dtype=torch.float32, device=prob.device)
    wsnet_targets(prob.h, eta, Y)
    return Y


def features(prob: "Problem") -> torch.Tensor:
    """Features of each dual's row ([m, 4]: per product for A = I, per resource otherwise)."""
    X = torch.empty((prob.m, 4), dtype=torch.float32, device=prob.device)
    wsnet_features(prob.h, X)
    return X
