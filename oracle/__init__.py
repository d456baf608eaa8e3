"""CPU oracle for aggregate risk analysis -- TEST INFRASTRUCTURE ONLY.

Plain C (ara_oracle.c, binary64, built with -ffp-contract=off) driven through
ctypes.  Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the product library never does, and the two
share no code.  See ara_oracle.c for the readings of the paper it implements.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ara_oracle.c")
LIB = os.path.join(HERE, "libara_oracle.so")

_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_F64 = ctypes.c_double


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP for the optional all-core trial split)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        lib = ctypes.CDLL(LIB)
        lib.oracle_build_tables.argtypes = [_I32, _I32, _P, _P, _P, _P]
        lib.oracle_forward.argtypes = [_I32, _I32, _P, _I64, _P, _P, _I32, _P, _P, _P, _P,
                                       _I64, _I64, _I32, _P, _P, _P, _P, _P, _P]
        lib.oracle_tail_count.argtypes = [_I64, _F64]
        lib.oracle_tail_count.restype = _I64
        lib.oracle_metrics.argtypes = [_P, _I32, _I64, _F64, _P]
        lib.oracle_metric_weights.argtypes = [_P, _I32, _I64, _F64, _P]
        lib.oracle_backward.argtypes = [_I32, _I32, _P, _I64, _P, _P, _I32, _P, _P, _P, _P,
                                        _I64, _I64, _I32, _P, _I32, _P, _P]
        lib.oracle_num_threads_available.restype = _I32
        lib.oracle_philox4x32_10.argtypes = [_P, _P, _P]
        lib.oracle_su_draw.argtypes = [_F64, _F64, ctypes.c_uint64, _I64, _I32]
        lib.oracle_su_draw.restype = _F64
        lib.oracle_forward_su.argtypes = [_I32, _I32, _P, _P, _I64, _P, _P, _I32, _P, _P, _P, _P,
                                          ctypes.c_uint64, _I64, _I64, _I32, _P, _P]
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def build_tables(elts) -> np.ndarray:
    """Dense direct-access binary32 tables [n_elts, catalog] (0 = absent)."""
    lib = _load()
    out = np.empty((elts.n_elts, elts.catalog), dtype=np.float32)
    ro, ri, rl = _c(elts.rec_off, np.int64), _c(elts.rec_ids, np.int32), _c(elts.rec_loss, np.float32)
    rc = lib.oracle_build_tables(elts.n_elts, elts.catalog, _ptr(ro), _ptr(ri), _ptr(rl), _ptr(out))
    if rc != 0:
        raise OracleError(f"oracle_build_tables status {rc}")
    return out


def forward(tables: np.ndarray, yet, layers, elt_terms, layer_terms=None, t0: int = 0,
            t1: Optional[int] = None, n_threads: int = 1, want_yelt: bool = False):
    """Literal Algorithm 1.  Returns dict(ylt, s_pre, hits, ylt_closed), each
    [n_layers, t1-t0]; with want_yelt also yelt [n_layers, occurrences in the
    trial range] (per-occurrence losses, storage order) and occ_max
    [n_layers, t1-t0]."""
    lib = _load()
    t1 = yet.n_trials if t1 is None else t1
    nl = layers.n_layers
    layer_terms = layers.terms if layer_terms is None else layer_terms
    n = t1 - t0
    ylt = np.empty((nl, n), np.float64)
    s_pre = np.empty((nl, n), np.float64)
    hits = np.empty((nl, n), np.int32)
    closed = np.empty((nl, n), np.float64)
    nocc = int(yet.offsets[t1] - yet.offsets[t0])
    yelt = np.empty((nl, nocc), np.float64) if want_yelt else None
    occ_max = np.empty((nl, n), np.float64) if want_yelt else None
    tb = _c(tables, np.float32)
    off, ids = _c(yet.offsets, np.int64), _c(yet.ids, np.int32)
    lo, le = _c(layers.elt_off, np.int32), _c(layers.elt_ids, np.int32)
    et, lt = _c(elt_terms, np.float64), _c(layer_terms, np.float64)
    rc = lib.oracle_forward(tb.shape[0], tb.shape[1], _ptr(tb), yet.n_trials, _ptr(off), _ptr(ids),
                            nl, _ptr(lo), _ptr(le), _ptr(et), _ptr(lt), t0, t1, n_threads,
                            _ptr(ylt), _ptr(s_pre), _ptr(hits), _ptr(closed),
                            _ptr(yelt) if want_yelt else None, _ptr(occ_max) if want_yelt else None)
    if rc != 0:
        raise OracleError(f"oracle_forward status {rc}")
    out = dict(ylt=ylt, s_pre=s_pre, hits=hits, ylt_closed=closed)
    if want_yelt:
        out.update(yelt=yelt, occ_max=occ_max)
    return out


def tail_count(n: int, p: float) -> int:
    return int(_load().oracle_tail_count(n, p))


def metrics(ylt: np.ndarray, p: float) -> np.ndarray:
    """[n_layers, 3] = (AAL, PML_p, TVaR_p) per layer row of ylt."""
    lib = _load()
    y = _c(np.atleast_2d(ylt), np.float64)
    out = np.empty((y.shape[0], 3), np.float64)
    rc = lib.oracle_metrics(_ptr(y), y.shape[0], y.shape[1], p, _ptr(out))
    if rc != 0:
        raise OracleError(f"oracle_metrics status {rc}")
    return out


def metric_weights(ylt: np.ndarray, p: float) -> np.ndarray:
    """[3, n_layers, n] = dAAL/dY, dPML/dY, dTVaR/dY."""
    lib = _load()
    y = _c(np.atleast_2d(ylt), np.float64)
    w = np.empty((3,) + y.shape, np.float64)
    rc = lib.oracle_metric_weights(_ptr(y), y.shape[0], y.shape[1], p, _ptr(w))
    if rc != 0:
        raise OracleError(f"oracle_metric_weights status {rc}")
    return w


def backward(tables: np.ndarray, yet, layers, elt_terms, layer_terms, cot: np.ndarray,
             t0: int = 0, t1: Optional[int] = None, n_threads: int = 1):
    """Reverse sweep.  cot: [n_cot, n_layers, t1-t0].  Returns
    (grad_elt [n_cot, n_elts, 3], grad_layer [n_cot, n_layers, 4]).
    n_threads > 1 splits the trials into contiguous shares summed in order."""
    lib = _load()
    t1 = yet.n_trials if t1 is None else t1
    cot = _c(cot, np.float64)
    if cot.ndim == 2:
        cot = cot[None]
    nc = cot.shape[0]
    nl = layers.n_layers
    tb = _c(tables, np.float32)
    ge = np.empty((nc, tb.shape[0], 3), np.float64)
    gl = np.empty((nc, nl, 4), np.float64)
    off, ids = _c(yet.offsets, np.int64), _c(yet.ids, np.int32)
    lo, le = _c(layers.elt_off, np.int32), _c(layers.elt_ids, np.int32)
    et, lt = _c(elt_terms, np.float64), _c(layer_terms, np.float64)
    rc = lib.oracle_backward(tb.shape[0], tb.shape[1], _ptr(tb), yet.n_trials, _ptr(off), _ptr(ids),
                             nl, _ptr(lo), _ptr(le), _ptr(et), _ptr(lt), t0, t1, nc, _ptr(cot),
                             n_threads, _ptr(ge), _ptr(gl))
    if rc != 0:
        raise OracleError(f"oracle_backward status {rc}")
    return ge, gl


def philox4x32_10(ctr, key) -> np.ndarray:
    """One Philox4x32-10 block (uint32 [4]) of counter ctr[4] under key[2]."""
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.empty(4, np.uint32)
    _load().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def su_draw(mu: float, sigma: float, seed: int, occ: int, elt: int) -> float:
    """The loss drawn for occurrence `occ` in ELT `elt` (reading R10/R11)."""
    return float(_load().oracle_su_draw(float(mu), float(sigma), int(seed), int(occ), int(elt)))


def build_sigma_tables(elts, rec_sigma) -> np.ndarray:
    """Dense binary32 standard deviations [n_elts, catalog], laid out like
    the loss tables (0 where the ELT has no record)."""
    lib = _load()
    out = np.empty((elts.n_elts, elts.catalog), dtype=np.float32)
    ro, ri, rs = _c(elts.rec_off, np.int64), _c(elts.rec_ids, np.int32), _c(rec_sigma, np.float32)
    rc = lib.oracle_build_tables(elts.n_elts, elts.catalog, _ptr(ro), _ptr(ri), _ptr(rs), _ptr(out))
    if rc != 0:
        raise OracleError(f"oracle_build_tables (sigma) status {rc}")
    return out


def forward_su(tables: np.ndarray, sigma_tables: np.ndarray, yet, layers, elt_terms, layer_terms, seed: int,
               t0: int = 0, t1: Optional[int] = None, n_threads: int = 1):
    """Algorithm 1 with secondary uncertainty (readings R10/R11).  Returns
    dict(ylt, s_pre), each [n_layers, t1-t0]."""
    lib = _load()
    t1 = yet.n_trials if t1 is None else t1
    nl = layers.n_layers
    n = t1 - t0
    ylt = np.empty((nl, n), np.float64)
    s_pre = np.empty((nl, n), np.float64)
    tb, sg = _c(tables, np.float32), _c(sigma_tables, np.float32)
    off, ids = _c(yet.offsets, np.int64), _c(yet.ids, np.int32)
    lo, le = _c(layers.elt_off, np.int32), _c(layers.elt_ids, np.int32)
    et, lt = _c(elt_terms, np.float64), _c(layer_terms, np.float64)
    rc = lib.oracle_forward_su(tb.shape[0], tb.shape[1], _ptr(tb), _ptr(sg), yet.n_trials, _ptr(off), _ptr(ids),
                               nl, _ptr(lo), _ptr(le), _ptr(et), _ptr(lt), int(seed), t0, t1, n_threads,
                               _ptr(ylt), _ptr(s_pre))
    if rc != 0:
        raise OracleError(f"oracle_forward_su status {rc}")
    return {"ylt": ylt, "s_pre": s_pre}


def num_threads_available() -> int:
    return int(_load().oracle_num_threads_available())


class use_library:
    """Temporarily route every call through another build of ara_oracle.c
    (used by the mutation tests, which compile deliberately broken copies)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self._saved = _load()
        _lib = None
        saved_lib = LIB
        globals()["LIB"] = self.path
        try:
            _load()
        finally:
            globals()["LIB"] = saved_lib
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved
        return False
