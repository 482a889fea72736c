"""FP64 CPU oracle for full-batch SPFOM (test infrastructure only).

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
use this package; the solver library never imports, links or runs it.  The
arithmetic lives in ``spfom_oracle.c`` (plain C, FP64, compiled with gcc);
this module marshals numpy arrays through ctypes.  ``lp`` formulates the
sales-based and choice-based LPs for an independent LP solver and ``mlp``
holds the warm-start network's FP64 reference.  (The paper's own greedy inner
solve with golden-section search is restated as a cross-check in
``tests/test_oracle_pins.py``.)

Every function here has a pin in ``tests/test_oracle_*.py`` except the ones
the header of ``spfom_oracle.c`` marks as the build's own readings (the
certified gap and the Polyak step), which are pinned by the LP optimum they
must bracket.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spfom_oracle.c")
_LIB = os.path.join(_HERE, "libspfom_oracle.so")
NTRACE = 10
TRACE_COLS = ("D", "P", "Z", "eta2", "infeas", "dbest", "lb", "gap", "step", "theta")
RULE_CONST, RULE_POLYAK = 0, 1

_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_int64)
_ip = ctypes.POINTER(ctypes.c_int32)


class _Inst(ctypes.Structure):
    _fields_ = [("L", _i64), ("n", _i64), ("m", _i64), ("seg_ptr", _lp),
                ("idx", _ip), ("v", _dp), ("w", _dp), ("v0", _dp), ("lam", _dp),
                ("r", _dp), ("c", _dp), ("a_ptr", _lp), ("a_idx", _ip),
                ("a_val", _dp)]


class _Params(ctypes.Structure):
    _fields_ = [("rule", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("perseg", ctypes.c_int32), ("gamma", ctypes.c_double), ("mu", ctypes.c_double),
                ("tau", _dp), ("tau_decay", ctypes.c_double), ("decay_every", _i64)]


class _State(ctypes.Structure):
    _fields_ = [("t", _i64), ("t0", _i64), ("cnt", _i64), ("dbest", ctypes.c_double),
                ("lb", ctypes.c_double), ("sum_p", ctypes.c_double), ("sum_u", _dp),
                ("sum_pl", _dp)]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                        "-ffp-contract=off", _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        lib.orc_segment.restype = _i64
        lib.orc_segment.argtypes = [_i64, _dp, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                    _dp, _dp, _dp]
        lib.orc_pass.restype = ctypes.c_int
        lib.orc_pass.argtypes = [ctypes.POINTER(_Inst), _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                 _dp, _dp]
        lib.orc_state_reset.restype = None
        lib.orc_state_reset.argtypes = [ctypes.POINTER(_State), _i64]
        lib.orc_state_clear_segments.restype = None
        lib.orc_state_clear_segments.argtypes = [ctypes.POINTER(_State), _i64]
        lib.orc_iterate.restype = ctypes.c_int
        lib.orc_iterate.argtypes = [ctypes.POINTER(_Inst), ctypes.POINTER(_Params),
                                    ctypes.POINTER(_State), _i64, _dp, _dp]
        lib.orc_minibatch.restype = ctypes.c_int
        lib.orc_minibatch.argtypes = [ctypes.POINTER(_Inst), ctypes.POINTER(_Params), _i64, _i64,
                                      _ip, _dp, _dp, _dp]
        _lib = lib
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class _Bound:
    """Instance arrays promoted to FP64 and kept alive for the C side."""

    def __init__(self, inst):
        self.seg_ptr = np.ascontiguousarray(inst.seg_ptr, dtype=np.int64)
        self.idx = np.ascontiguousarray(inst.idx, dtype=np.int32)
        self.v, self.w = _f64(inst.v), _f64(inst.w)
        self.v0, self.lam = _f64(inst.v0), _f64(inst.lam)
        self.r, self.c = _f64(inst.r), _f64(inst.c)
        self.a_ptr = None if inst.a_ptr is None else np.ascontiguousarray(inst.a_ptr, dtype=np.int64)
        self.a_idx = None if inst.a_idx is None else np.ascontiguousarray(inst.a_idx, dtype=np.int32)
        self.a_val = _f64(inst.a_val)
        self.L, self.n, self.m = int(inst.L), int(inst.n), int(inst.m)
        self.s = _Inst(self.L, self.n, self.m, self.seg_ptr.ctypes.data_as(_lp),
                       self.idx.ctypes.data_as(_ip), _d(self.v), _d(self.w), _d(self.v0),
                       _d(self.lam), _d(self.r), _d(self.c),
                       None if self.a_ptr is None else self.a_ptr.ctypes.data_as(_lp),
                       None if self.a_idx is None else self.a_idx.ctypes.data_as(_ip),
                       _d(self.a_val))


def segment_response(rho, v, w, v0: float, lam: float):
    """Exact best response of one segment.  Returns (R*, D_l, sales)."""
    rho, v, w = _f64(rho), _f64(v), _f64(w)
    k = rho.shape[0]
    s = np.zeros(k)
    R = ctypes.c_double()
    D = ctypes.c_double()
    q = _load().orc_segment(k, _d(rho), _d(v), _d(w), float(v0), float(lam),
                            ctypes.byref(R), ctypes.byref(D), _d(s))
    if q < 0:
        raise MemoryError("oracle segment solve")
    return R.value, D.value, s


def best_response(inst, eta):
    """One pass at fixed eta: every segment's exact best response."""
    b = _Bound(inst)
    eta = _f64(eta)
    out = dict(rho=np.zeros(b.n), S=np.zeros(b.n), u=np.zeros(b.m), seg_R=np.zeros(b.L),
               seg_p=np.zeros(b.L), sales=np.zeros(int(b.seg_ptr[-1])))
    Z = ctypes.c_double()
    P = ctypes.c_double()
    rc = _load().orc_pass(ctypes.byref(b.s), _d(eta), _d(out["rho"]), _d(out["S"]),
                          _d(out["u"]), _d(out["seg_R"]), _d(out["seg_p"]),
                          _d(out["sales"]), ctypes.byref(Z), ctypes.byref(P))
    if rc:
        raise MemoryError("oracle pass")
    out["Z"], out["P"] = Z.value, P.value
    out["D"] = float(np.dot(b.c, eta)) + Z.value
    return out


def dual_value(inst, eta) -> float:
    """D(eta) = c . eta + sum_l lambda_l R*_l(eta)."""
    return best_response(inst, eta)["D"]


class Solver:
    """Full-batch SPFOM iterations with the certified-gap state."""

    def __init__(self, inst, *, tau=None, rule: int = RULE_CONST, gamma: float = 1.0,
                 mu: float = 0.0, check_every: int = 10, perseg: bool = False,
                 tau_decay: float = 1.0, decay_every: int = 1):
        self.b = _Bound(inst)
        m = self.b.m
        if tau is None:
            tau = np.ones(m)
        tau = np.broadcast_to(np.asarray(tau, dtype=np.float64), (m,)).copy()
        self.tau = tau
        self.prm = _Params(int(rule), int(check_every), int(bool(perseg)), float(gamma),
                           float(mu), _d(self.tau), float(tau_decay), int(decay_every))
        self.sum_u = np.zeros(max(m, 1))
        self.sum_pl = np.zeros(max(self.b.L, 1))
        self.st = _State(0, 0, 0, 0.0, 0.0, 0.0, _d(self.sum_u), _d(self.sum_pl))
        self.reset()

    def reset(self):
        _load().orc_state_reset(ctypes.byref(self.st), self.b.m)
        _load().orc_state_clear_segments(ctypes.byref(self.st), self.b.L)

    @property
    def t(self) -> int:
        return int(self.st.t)

    def iterate(self, eta, iters: int, trace: bool = True):
        """Advance `iters` iterations from eta; returns (eta, trace[iters, 10])."""
        eta = np.array(eta, dtype=np.float64, copy=True)
        tr = np.zeros((int(iters), NTRACE)) if trace else None
        rc = _load().orc_iterate(ctypes.byref(self.b.s), ctypes.byref(self.prm),
                                 ctypes.byref(self.st), int(iters), _d(eta), _d(tr))
        if rc:
            raise MemoryError("oracle iterate")
        return eta, tr

    def solve(self, eta0, tol: float, max_iters: int):
        """Iterate in blocks of check_every until the certified gap <= tol."""
        eta = np.array(eta0, dtype=np.float64, copy=True)
        K = int(self.prm.check_every)
        last = None
        while self.t < max_iters:
            eta, tr = self.iterate(eta, min(K, max_iters - self.t))
            last = tr[-1]
            if self.t % K == 0 and last[7] <= tol:
                return eta, last, True
        return eta, last, False


class Minibatch:
    """Stochastic minibatch SPFOM (Algorithm 2; Algorithm 3 with k B < L):
    the per-segment sales y persist; each iteration re-solves the segments of
    one row of ``batch`` and steps the duals with the sales of all segments."""

    def __init__(self, inst, *, tau=None, mu: float = 0.0, y0=None):
        self.b = _Bound(inst)
        m = self.b.m
        tau = np.ones(m) if tau is None else tau
        self.tau = np.broadcast_to(np.asarray(tau, dtype=np.float64), (m,)).copy()
        self.prm = _Params(RULE_CONST, 1, 0, 1.0, float(mu), _d(self.tau), 1.0, 1)
        nnz = int(self.b.seg_ptr[-1])
        self.y = np.zeros(nnz) if y0 is None else np.array(y0, dtype=np.float64, copy=True)

    def iterate(self, eta, batch):
        """Run len(batch) iterations; batch [iters, B] int segment ids (distinct
        within a row).  Returns (eta, trace[iters, 10])."""
        batch = np.ascontiguousarray(batch, dtype=np.int32)
        iters, B = batch.shape
        if iters and (batch.min() < 0 or batch.max() >= self.b.L):
            raise ValueError("segment id out of range")
        eta = np.array(eta, dtype=np.float64, copy=True)
        tr = np.zeros((iters, NTRACE))
        rc = _load().orc_minibatch(ctypes.byref(self.b.s), ctypes.byref(self.prm), iters, B,
                                   batch.ctypes.data_as(_ip), _d(self.y), _d(eta), _d(tr))
        if rc:
            raise MemoryError("oracle minibatch")
        return eta, tr


def recover(inst, y):
    """SBLP -> CBLP recovery (the nested sets of Section 4.4) from per-entry
    sales y [nnz]: returns (rank [nnz] int32, alpha [nnz], alpha0 [L]); entry
    e's alpha is the probability of offering the entries of its segment
    ranked at most rank[e], alpha0 that of the empty set."""
    b = _Bound(inst)
    y = np.ascontiguousarray(y, dtype=np.float64)
    nnz = int(b.seg_ptr[-1])
    rank = np.zeros(nnz, dtype=np.int32)
    alpha = np.zeros(nnz)
    alpha0 = np.zeros(b.L)
    lib = _load()
    if not hasattr(lib, "_rec_set"):
        lib.orc_recover.restype = ctypes.c_int
        lib.orc_recover.argtypes = [ctypes.POINTER(_Inst), _dp, _ip, _dp, _dp]
        lib._rec_set = True
    if lib.orc_recover(ctypes.byref(b.s), _d(y), rank.ctypes.data_as(_ip), _d(alpha), _d(alpha0)):
        raise MemoryError("oracle recover")
    return rank, alpha, alpha0
