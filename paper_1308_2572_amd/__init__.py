"""Python binding of libara.so, the MI355X aggregate-risk-analysis library.

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in include/ara.h.  PyTorch supplies device
memory (caller-owned workspaces) and the current HIP stream.  The binding
refuses to run without the compiled library; there is no CPU fallback.

Functions named ``ara_*`` are one-to-one wrappers of the C entry points (they
take raw integers/pointers and raise AraError on a non-zero status); the
classes and functions below them hold tensors alive and size workspaces.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libara.so")

ARA_OK, ARA_E_INVAL, ARA_E_RANGE, ARA_E_DUP, ARA_E_NOSPACE, ARA_E_HIP, ARA_E_LIMIT, ARA_E_BUSY = range(8)
ARA_F_EMIT_HITS = 1
ARA_F_FP32_ACCUM = 2
PREP_TRANSPOSED = 1          # ARA_PREP_TRANSPOSED
PREP_TRIAL_MAJOR = 2         # ARA_PREP_TRIAL_MAJOR
PREP_POSITIONS = 4           # ARA_PREP_POSITIONS
ARA_MAX_COTANGENTS = 4
ARA_MAX_LAYERS = 65535

_c_i32, _c_i64, _c_u32, _c_f64, _c_p, _c_sz = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double,
                                               ctypes.c_void_p, ctypes.c_size_t)


class AraError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class ara_yet(ctypes.Structure):
    _fields_ = [("n_trials", _c_i64), ("nnz", _c_i64), ("catalog", _c_i32), ("range_bits", _c_i32),
                ("n_ranges", _c_i32), ("groups", _c_i32), ("trials_per_group", _c_i32),
                ("trials_per_block", _c_i32), ("n_blocks", _c_i32), ("max_occ", _c_i32),
                ("n_codes", _c_i64), ("code", _c_p), ("seg_base", _c_p), ("seg_run", _c_p), ("lane_start", _c_p),
                ("n_slices", _c_i32), ("reserved", _c_i32), ("slice_trials", _c_i64), ("tr_off", _c_p),
                ("tr_ent", _c_p), ("t_off", _c_p), ("t_ids", _c_p), ("t_cnt", _c_p), ("pos", _c_p)]


class ara_tables(ctypes.Structure):
    _fields_ = [("n_elts", _c_i32), ("catalog", _c_i32), ("words", _c_i32), ("reserved", _c_i32),
                ("loss", _c_p), ("present", _c_p)]


class ara_layers(ctypes.Structure):
    _fields_ = [("n_layers", _c_i32), ("reserved", _c_i32), ("elt_off", _c_p), ("elt_ids", _c_p)]


class ara_quote(ctypes.Structure):
    _fields_ = [("n_elts", _c_i32), ("want_grad", _c_i32), ("elt_ids", _c_p), ("layer_terms", _c_f64 * 4),
                ("trial_begin", _c_i64), ("trial_end", _c_i64), ("p", _c_f64)]


class ara_quote_result(ctypes.Structure):
    _fields_ = [("status", _c_i32), ("n_elts", _c_i32), ("metrics", _c_f64 * 3), ("grad_layer", (_c_f64 * 4) * 3),
                ("grad_elt", _c_p), ("t_submit_ms", _c_f64), ("t_admit_ms", _c_f64), ("t_done_ms", _c_f64)]


_P = ctypes.POINTER
_SIGNATURES = {
    "ara_status_string": (ctypes.c_char_p, [_c_i32]),
    "ara_last_error": (ctypes.c_char_p, []),
    "ara_abi_version": (_c_i32, []),
    "ara_check_device_error": (_c_i32, [_c_p, _c_p]),
    "ara_yet_prepare_bytes": (_c_i32, [_c_i64, _c_i64, _c_i32, _c_u32, _P(_c_sz)]),
    "ara_yet_prepare": (_c_i32, [_c_p, _c_p, _c_i64, _c_i32, _c_u32, _c_p, _c_sz, _c_p, _P(ara_yet)]),
    "ara_build_elt_tables_bytes": (_c_i32, [_c_i32, _c_i32, _P(_c_sz)]),
    "ara_build_elt_tables": (_c_i32, [_c_i32, _c_i32, _c_p, _c_p, _c_p, _c_p, _c_sz, _c_p, _P(ara_tables)]),
    "ara_ylt_workspace_bytes": (_c_i32, [_P(ara_tables), _P(ara_yet), _P(ara_layers), _c_u32, _P(_c_sz)]),
    "ara_ylt_forward": (_c_i32, [_P(ara_tables), _P(ara_yet), _P(ara_layers), _c_p, _c_p, _c_i64, _c_i64, _c_u32,
                                 _c_p, _c_p, _c_p, _c_p, _c_sz, _c_p]),
    "ara_ylt_forward_noalloc": (_c_i32, [_P(ara_tables), _P(ara_yet), _P(ara_layers), _c_p, _c_p, _c_i64, _c_i64,
                                         _c_u32, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "ara_yelt_workspace_bytes": (_c_i32, [_P(ara_tables), _P(ara_layers), _P(_c_sz)]),
    "ara_yelt_forward": (_c_i32, [_P(ara_tables), _c_p, _c_p, _c_i64, _P(ara_layers), _c_p, _c_p, _c_i64, _c_i64,
                                  _c_i64, _c_i64, _c_p, _c_p, _c_p, _c_sz, _c_p]),
    "ara_build_elt_sigma": (_c_i32, [_P(ara_tables), _c_p, _c_p, _c_p, _c_p, _c_p]),
    "ara_su_workspace_bytes": (_c_i32, [_P(ara_tables), _P(ara_layers), _c_p, _P(_c_sz)]),
    "ara_ylt_forward_su": (_c_i32, [_P(ara_tables), _c_p, _P(ara_yet), _P(ara_layers), _c_p, _c_p, _c_p,
                                    ctypes.c_uint64, _c_i64, _c_i64, _c_p, _c_p, _c_p, _c_sz, _c_p]),
    "ara_metrics_workspace_bytes": (_c_i32, [_c_i32, _c_i64, _P(_c_sz)]),
    "ara_metrics": (_c_i32, [_c_p, _c_i32, _c_i64, _c_f64, _c_p, _c_p, _c_p, _c_sz, _c_p]),
    "ara_metrics_vjp": (_c_i32, [_c_p, _c_i32, _c_i64, _c_p, _c_p, _c_p]),
    "ara_server_arena_bytes": (_c_i32, [_P(ara_tables), _P(ara_yet), _c_i32, _P(_c_sz)]),
    "ara_server_create": (_c_i32, [_P(ara_tables), _P(ara_yet), _c_p, _c_p, _c_sz, _c_i32, _P(_c_p)]),
    "ara_server_submit": (_c_i32, [_c_p, _P(ara_quote), _P(_c_i64)]),
    "ara_server_poll": (_c_i32, [_c_p, _c_i64, _P(ara_quote_result)]),
    "ara_server_wait": (_c_i32, [_c_p, _c_i64, _P(ara_quote_result)]),
    "ara_server_cancel": (_c_i32, [_c_p, _c_i64]),
    "ara_server_stats": (_c_i32, [_c_p, _P(_c_i64)]),
    "ara_server_destroy": (_c_i32, [_c_p]),
    "ara_profile_enable": (_c_i32, [_c_i32]),
    "ara_profile_enable_kinds": (_c_i32, [ctypes.c_uint32]),
    "ara_profile_read": (_c_i32, [_c_i32, _P(_c_f64), _P(_c_i64)]),
    "ara_profile_reset": (_c_i32, []),
    "ara_ylt_backward_workspace_bytes": (_c_i32, [_P(ara_tables), _P(ara_yet), _P(ara_layers), _c_i32, _P(_c_sz)]),
    "ara_ylt_backward": (_c_i32, [_P(ara_tables), _P(ara_yet), _P(ara_layers), _c_p, _c_p, _c_i64, _c_i64, _c_p,
                                  _c_i32, _c_p, _c_p, _c_p, _c_p, _c_sz, _c_p]),
}

_lib = None


def library() -> ctypes.CDLL:
    """Load libara.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1308_2572_amd.build` "
                              f"(the HIP library is required; there is no CPU path)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int, what: str) -> None:
    if rc != ARA_OK:
        lib = library()
        raise AraError(rc, f"{what}: {lib.ara_status_string(rc).decode()} ({lib.ara_last_error().decode()})")


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return t.data_ptr() or None


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


# --------------------------------------------------------------------------
# resident inputs
# --------------------------------------------------------------------------

class PreparedYet:
    """A YET laid out on the device by ara_yet_prepare (keeps its buffer alive)."""

    def __init__(self, offsets: torch.Tensor, ids: torch.Tensor, catalog: int, transposed: bool = True,
                 trial_major: Optional[bool] = None, positions: bool = False):
        """transposed: also build the event-major copy that the backward
        needs (ARA_PREP_TRANSPOSED); leave it off for forward-only use.
        trial_major: also keep a trial-major copy (ARA_PREP_TRIAL_MAJOR), with
        which the backward of the metrics reads only the trials whose weight
        differs from the common one; on by default with `transposed`.
        positions: also store each occurrence's position in its trial
        (ARA_PREP_POSITIONS), which the secondary-uncertainty forward needs."""
        lib = library()
        if offsets.dtype != torch.int64 or ids.dtype != torch.int32:
            raise ValueError("offsets must be int64 and ids int32")
        n_trials = offsets.numel() - 1
        nnz = ids.numel()
        trial_major = transposed if trial_major is None else trial_major
        flags = ((PREP_TRANSPOSED if transposed else 0) | (PREP_TRIAL_MAJOR if trial_major else 0)
                 | (PREP_POSITIONS if positions else 0))
        nb = _c_sz()
        _check(lib.ara_yet_prepare_bytes(n_trials, nnz, catalog, flags, ctypes.byref(nb)), "ara_yet_prepare_bytes")
        self.device = offsets.device
        self.buf = _workspace(nb.value, self.device)
        self.handle = ara_yet()
        _check(lib.ara_yet_prepare(_dptr(offsets), _dptr(ids), n_trials, catalog, flags, _dptr(self.buf),
                                   self.buf.numel(), _stream(), ctypes.byref(self.handle)), "ara_yet_prepare")
        self.n_trials = n_trials
        self.catalog = catalog
        self.transposed = transposed
        self.positions = positions

    @classmethod
    def from_numpy(cls, yet, device="cuda", transposed: bool = True, trial_major: Optional[bool] = None,
                   positions: bool = False):
        off = torch.from_numpy(np.ascontiguousarray(yet.offsets, np.int64)).to(device)
        ids = torch.from_numpy(np.ascontiguousarray(yet.ids, np.int32)).to(device)
        out = cls(off, ids, int(yet.catalog), transposed=transposed, trial_major=trial_major, positions=positions)
        return out


class EltTables:
    """Direct-access ELT tables built on the device by ara_build_elt_tables."""

    def __init__(self, rec_off: torch.Tensor, rec_ids: torch.Tensor, rec_loss: torch.Tensor, catalog: int):
        lib = library()
        n_elts = rec_off.numel() - 1
        nb = _c_sz()
        _check(lib.ara_build_elt_tables_bytes(n_elts, catalog, ctypes.byref(nb)), "ara_build_elt_tables_bytes")
        self.device = rec_off.device
        self.buf = _workspace(nb.value, self.device)
        self.handle = ara_tables()
        _check(lib.ara_build_elt_tables(n_elts, catalog, _dptr(rec_off), _dptr(rec_ids), _dptr(rec_loss),
                                        _dptr(self.buf), self.buf.numel(), _stream(), ctypes.byref(self.handle)),
               "ara_build_elt_tables")
        self.n_elts = n_elts
        self.catalog = catalog
        # the CSR is kept for the standard-deviation tables of secondary uncertainty
        self.rec_off = rec_off
        self.rec_ids = rec_ids
        off_h = rec_off.cpu().numpy().astype(np.int64)
        self.records = np.ascontiguousarray(off_h[1:] - off_h[:-1], dtype=np.int64)

    @classmethod
    def from_numpy(cls, elts, device="cuda"):
        return cls(torch.from_numpy(np.ascontiguousarray(elts.rec_off, np.int64)).to(device),
                   torch.from_numpy(np.ascontiguousarray(elts.rec_ids, np.int32)).to(device),
                   torch.from_numpy(np.ascontiguousarray(elts.rec_loss, np.float32)).to(device),
                   int(elts.catalog))


class SigmaTables:
    """Standard deviations of the ELT records (secondary uncertainty), dense
    binary32 [n_elts, catalog] on the device, built by ara_build_elt_sigma."""

    def __init__(self, tables: EltTables, rec_sigma: torch.Tensor):
        lib = library()
        rec_sigma = rec_sigma.to(device=tables.device, dtype=torch.float32).contiguous()
        self.sigma = torch.empty((tables.n_elts, tables.catalog), dtype=torch.float32, device=tables.device)
        _check(lib.ara_build_elt_sigma(ctypes.byref(tables.handle), _dptr(tables.rec_off), _dptr(tables.rec_ids),
                                       _dptr(rec_sigma), _dptr(self.sigma), _stream()), "ara_build_elt_sigma")

    @classmethod
    def from_numpy(cls, tables: EltTables, rec_sigma):
        return cls(tables, torch.from_numpy(np.ascontiguousarray(rec_sigma, np.float32)))


class Layers:
    """Host-side layer structure (ELT lists in listed order)."""

    def __init__(self, elt_off, elt_ids):
        self.elt_off = np.ascontiguousarray(elt_off, dtype=np.int32)
        self.elt_ids = np.ascontiguousarray(elt_ids, dtype=np.int32)
        self.handle = ara_layers(int(self.elt_off.shape[0] - 1), 0,
                                 self.elt_off.ctypes.data_as(_c_p), self.elt_ids.ctypes.data_as(_c_p))

    @property
    def n_layers(self) -> int:
        return int(self.elt_off.shape[0] - 1)


# --------------------------------------------------------------------------
# computations
# --------------------------------------------------------------------------

def yelt_forward(tables: EltTables, offsets: torch.Tensor, ids: torch.Tensor, layers: Layers,
                 elt_terms: torch.Tensor, layer_terms: torch.Tensor, trial_begin: int = 0,
                 trial_end: Optional[int] = None, check: bool = False):
    """Per-occurrence losses over the trial-major YET (device int64 offsets,
    int32 ids, storage order).  Returns (yelt [n_layers, occurrences in the
    range], occ_max [n_layers, n])."""
    lib = library()
    if offsets.dtype != torch.int64 or ids.dtype != torch.int32:
        raise ValueError("offsets must be int64 and ids int32")
    n_trials = offsets.numel() - 1
    trial_end = n_trials if trial_end is None else trial_end
    if not (0 <= trial_begin <= trial_end <= n_trials):
        raise AraError(ARA_E_RANGE, "trial range outside the YET")
    n = trial_end - trial_begin
    L = layers.n_layers
    dev = offsets.device
    occ_begin = int(offsets[trial_begin].item())
    occ_count = int(offsets[trial_end].item()) - occ_begin
    nb = _c_sz()
    _check(lib.ara_yelt_workspace_bytes(ctypes.byref(tables.handle), ctypes.byref(layers.handle), ctypes.byref(nb)),
           "ara_yelt_workspace_bytes")
    ws = _workspace(nb.value, dev)
    yelt = torch.empty((L, max(occ_count, 0)), dtype=torch.float64, device=dev)
    occ_max = torch.empty((L, n), dtype=torch.float64, device=dev)
    et = elt_terms.to(device=dev, dtype=torch.float64).contiguous()
    lt = layer_terms.to(device=dev, dtype=torch.float64).contiguous()
    _check(lib.ara_yelt_forward(ctypes.byref(tables.handle), _dptr(offsets), _dptr(ids), n_trials,
                                ctypes.byref(layers.handle), _dptr(et), _dptr(lt), trial_begin, trial_end,
                                occ_begin, occ_count, _dptr(yelt), _dptr(occ_max), _dptr(ws), ws.numel(),
                                _stream()), "ara_yelt_forward")
    if check:
        _check(lib.ara_check_device_error(_dptr(ws), _stream()), "ara_yelt_forward (device)")
    return yelt, occ_max


def ylt_forward_su(tables: EltTables, sigma: SigmaTables, yet: PreparedYet, layers: Layers,
                   elt_terms: torch.Tensor, layer_terms: torch.Tensor, seed: int, trial_begin: int = 0,
                   trial_end: Optional[int] = None, want_s_pre: bool = True, check: bool = False):
    """Algorithm 1 with secondary uncertainty (a lognormal draw per occurrence
    and ELT) over a YET prepared with positions.  Returns (ylt, s_pre or
    None), each [n_layers, n]."""
    lib = library()
    trial_end = yet.n_trials if trial_end is None else trial_end
    if not (0 <= trial_begin <= trial_end <= yet.n_trials):
        raise AraError(ARA_E_RANGE, "trial range outside the YET")
    n = trial_end - trial_begin
    L = layers.n_layers
    dev = yet.device
    rec = tables.records
    nb = _c_sz()
    _check(lib.ara_su_workspace_bytes(ctypes.byref(tables.handle), ctypes.byref(layers.handle),
                                      rec.ctypes.data_as(_c_p), ctypes.byref(nb)), "ara_su_workspace_bytes")
    ws = _workspace(nb.value, dev)
    ylt = torch.empty((L, n), dtype=torch.float64, device=dev)
    s_pre = torch.empty((L, n), dtype=torch.float64, device=dev) if want_s_pre else None
    et = elt_terms.to(device=dev, dtype=torch.float64).contiguous()
    lt = layer_terms.to(device=dev, dtype=torch.float64).contiguous()
    _check(lib.ara_ylt_forward_su(ctypes.byref(tables.handle), _dptr(sigma.sigma), ctypes.byref(yet.handle),
                                  ctypes.byref(layers.handle), rec.ctypes.data_as(_c_p), _dptr(et), _dptr(lt),
                                  int(seed) & 0xFFFFFFFFFFFFFFFF, trial_begin, trial_end, _dptr(ylt), _dptr(s_pre),
                                  _dptr(ws), ws.numel(), _stream()), "ara_ylt_forward_su")
    if check:
        _check(lib.ara_check_device_error(_dptr(ws), _stream()), "ara_ylt_forward_su (device)")
    return ylt, s_pre


def ylt_forward(tables: EltTables, yet: PreparedYet, layers: Layers, elt_terms: torch.Tensor,
                layer_terms: torch.Tensor, trial_begin: int = 0, trial_end: Optional[int] = None,
                want_s_pre: bool = True, want_hits: bool = False, check: bool = False, fp32_accum: bool = False):
    """Returns (ylt, s_pre or None, hits or None), each [n_layers, n].
    fp32_accum: binary32 occurrence values and trial totals (ARA_F_FP32_ACCUM)."""
    lib = library()
    trial_end = yet.n_trials if trial_end is None else trial_end
    n = trial_end - trial_begin
    L = layers.n_layers
    dev = yet.device
    flags = (ARA_F_EMIT_HITS if want_hits else 0) | (ARA_F_FP32_ACCUM if fp32_accum else 0)
    nb = _c_sz()
    _check(lib.ara_ylt_workspace_bytes(ctypes.byref(tables.handle), ctypes.byref(yet.handle),
                                       ctypes.byref(layers.handle), flags, ctypes.byref(nb)), "ara_ylt_workspace_bytes")
    ws = _workspace(nb.value, dev)
    ylt = torch.empty((L, n), dtype=torch.float64, device=dev)
    s_pre = torch.empty((L, n), dtype=torch.float64, device=dev) if want_s_pre else None
    hits = torch.empty((L, n), dtype=torch.int32, device=dev) if want_hits else None
    et = elt_terms.to(device=dev, dtype=torch.float64).contiguous()
    lt = layer_terms.to(device=dev, dtype=torch.float64).contiguous()
    _check(lib.ara_ylt_forward(ctypes.byref(tables.handle), ctypes.byref(yet.handle), ctypes.byref(layers.handle),
                               _dptr(et), _dptr(lt), trial_begin, trial_end, flags, _dptr(ylt), _dptr(s_pre),
                               _dptr(hits), _dptr(ws), ws.numel(), _stream()), "ara_ylt_forward")
    if check:
        _check(lib.ara_check_device_error(_dptr(ws), _stream()), "ara_ylt_forward (device)")
    return ylt, s_pre, hits


def ylt_forward_noalloc(tables: EltTables, yet: PreparedYet, layers: Layers, elt_terms: torch.Tensor,
                        layer_terms: torch.Tensor, ylt: torch.Tensor, s_pre: Optional[torch.Tensor] = None,
                        hits: Optional[torch.Tensor] = None, status: Optional[torch.Tensor] = None,
                        trial_begin: int = 0, trial_end: Optional[int] = None, fp32_accum: bool = False) -> None:
    """ara_ylt_forward_noalloc into caller tensors (ylt, s_pre, hits: [n_layers,
    n]; status: one device int32 or None): the library's own scratch serves as
    the workspace.  Terms must already be contiguous binary64 on the device."""
    lib = library()
    trial_end = yet.n_trials if trial_end is None else trial_end
    flags = (ARA_F_EMIT_HITS if hits is not None else 0) | (ARA_F_FP32_ACCUM if fp32_accum else 0)
    _check(lib.ara_ylt_forward_noalloc(ctypes.byref(tables.handle), ctypes.byref(yet.handle),
                                       ctypes.byref(layers.handle), _dptr(elt_terms), _dptr(layer_terms), trial_begin,
                                       trial_end, flags, _dptr(ylt), _dptr(s_pre), _dptr(hits), _dptr(status),
                                       _stream()), "ara_ylt_forward_noalloc")


def metrics(ylt: torch.Tensor, p: float, want_weights: bool = False):
    """Returns (out [n_layers, 3] = AAL, PML, TVaR; weights [3, n_layers, n] or None)."""
    lib = library()
    ylt = ylt.contiguous()
    L, n = ylt.shape
    nb = _c_sz()
    _check(lib.ara_metrics_workspace_bytes(L, n, ctypes.byref(nb)), "ara_metrics_workspace_bytes")
    ws = _workspace(nb.value, ylt.device)
    out = torch.empty((L, 3), dtype=torch.float64, device=ylt.device)
    w = torch.empty((3, L, n), dtype=torch.float64, device=ylt.device) if want_weights else None
    _check(lib.ara_metrics(_dptr(ylt), L, n, float(p), _dptr(out), _dptr(w), _dptr(ws), ws.numel(), _stream()),
           "ara_metrics")
    return out, w


def metrics_vjp(weights: torch.Tensor, grad_out: torch.Tensor) -> torch.Tensor:
    lib = library()
    _, L, n = weights.shape
    g = grad_out.to(dtype=torch.float64).contiguous()
    out = torch.empty((L, n), dtype=torch.float64, device=weights.device)
    _check(lib.ara_metrics_vjp(_dptr(weights), L, n, _dptr(g), _dptr(out), _stream()), "ara_metrics_vjp")
    return out


def ylt_backward(tables: EltTables, yet: PreparedYet, layers: Layers, elt_terms: torch.Tensor,
                 layer_terms: torch.Tensor, s_pre: torch.Tensor, grad_ylt: torch.Tensor, trial_begin: int = 0,
                 trial_end: Optional[int] = None) -> Tuple[torch.Tensor, torch.Tensor]:
    """grad_ylt: [n_cot, n_layers, n] (or [n_layers, n]).  Returns
    (grad_elt [n_cot, n_elts, 3], grad_layer [n_cot, n_layers, 4])."""
    lib = library()
    trial_end = yet.n_trials if trial_end is None else trial_end
    squeeze = grad_ylt.dim() == 2
    g = (grad_ylt[None] if squeeze else grad_ylt).to(dtype=torch.float64).contiguous()
    n_cot = g.shape[0]
    dev = yet.device
    nb = _c_sz()
    _check(lib.ara_ylt_backward_workspace_bytes(ctypes.byref(tables.handle), ctypes.byref(yet.handle),
                                                ctypes.byref(layers.handle), n_cot, ctypes.byref(nb)),
           "ara_ylt_backward_workspace_bytes")
    ws = _workspace(nb.value, dev)
    ge = torch.empty((n_cot, tables.n_elts, 3), dtype=torch.float64, device=dev)
    gl = torch.empty((n_cot, layers.n_layers, 4), dtype=torch.float64, device=dev)
    et = elt_terms.to(device=dev, dtype=torch.float64).contiguous()
    lt = layer_terms.to(device=dev, dtype=torch.float64).contiguous()
    _check(lib.ara_ylt_backward(ctypes.byref(tables.handle), ctypes.byref(yet.handle), ctypes.byref(layers.handle),
                                _dptr(et), _dptr(lt), trial_begin, trial_end, _dptr(s_pre.contiguous()), n_cot,
                                _dptr(g), _dptr(ge), _dptr(gl), _dptr(ws), ws.numel(), _stream()), "ara_ylt_backward")
    if squeeze:
        return ge[0], gl[0]
    return ge, gl


PROF_OCC, PROF_FWD, PROF_METRICS, PROF_BWD, PROF_BWD_RED, PROF_YELT, PROF_SU = range(7)


def profile_enable(on: bool = True, kinds=None) -> None:
    """Record HIP-event timings of every kind (or only of `kinds`, a list of
    PROF_* values); on=False stops."""
    if kinds is None or not on:
        _check(library().ara_profile_enable(1 if on else 0), "ara_profile_enable")
    else:
        mask = 0
        for k in kinds:
            mask |= 1 << int(k)
        _check(library().ara_profile_enable_kinds(mask), "ara_profile_enable_kinds")


def profile_reset() -> None:
    _check(library().ara_profile_reset(), "ara_profile_reset")


def profile_read(kind: int) -> Tuple[float, int]:
    """(total milliseconds, launches) recorded for one kernel kind."""
    ms, n = _c_f64(), _c_i64()
    _check(library().ara_profile_read(kind, ctypes.byref(ms), ctypes.byref(n)), "ara_profile_read")
    return ms.value, n.value


# --------------------------------------------------------------------------
# quote server
# --------------------------------------------------------------------------

class QuoteServer:
    """Continuous-batching quote server over a resident YET and ELT set (the
    scheduler runs in libara.so; this object owns the device arena)."""

    def __init__(self, tables: EltTables, yet: PreparedYet, elt_terms: torch.Tensor, arena_bytes: Optional[int] = None,
                 quotes_with_grad: int = 16, max_slots: int = 64):
        lib = library()
        if arena_bytes is None:
            nb = _c_sz()
            _check(lib.ara_server_arena_bytes(ctypes.byref(tables.handle), ctypes.byref(yet.handle), quotes_with_grad,
                                              ctypes.byref(nb)), "ara_server_arena_bytes")
            arena_bytes = nb.value
        self.tables, self.yet = tables, yet
        self.elt_terms = elt_terms.to(device=yet.device, dtype=torch.float64).contiguous()
        self.arena = _workspace(arena_bytes, yet.device)
        torch.cuda.synchronize(yet.device)
        self.handle = ctypes.c_void_p()
        _check(lib.ara_server_create(ctypes.byref(tables.handle), ctypes.byref(yet.handle), _dptr(self.elt_terms),
                                     _dptr(self.arena), self.arena.numel(), max_slots, ctypes.byref(self.handle)),
               "ara_server_create")
        self._keep = {}

    def submit(self, elt_ids, layer_terms, trial_begin: int, trial_end: int, p: float = 0.99,
               want_grad: bool = False) -> int:
        ids = np.ascontiguousarray(elt_ids, dtype=np.int32)
        q = ara_quote(int(ids.shape[0]), 1 if want_grad else 0, ids.ctypes.data_as(_c_p),
                      (_c_f64 * 4)(*[float(v) for v in layer_terms]), int(trial_begin), int(trial_end), float(p))
        t = _c_i64()
        _check(library().ara_server_submit(self.handle, ctypes.byref(q), ctypes.byref(t)), "ara_server_submit")
        self._keep[t.value] = (int(ids.shape[0]), bool(want_grad))
        return t.value

    def _result(self, ticket: int, blocking: bool):
        n_elts, want_grad = self._keep[ticket]
        ge = np.zeros((3, n_elts, 3), np.float64)
        r = ara_quote_result()
        r.grad_elt = ge.ctypes.data_as(_c_p) if want_grad else None
        lib = library()
        rc = lib.ara_server_wait(self.handle, ticket, ctypes.byref(r)) if blocking else \
            lib.ara_server_poll(self.handle, ticket, ctypes.byref(r))
        if rc == ARA_E_BUSY:
            return None
        del self._keep[ticket]
        _check(rc, "ara_server_wait" if blocking else "ara_server_poll")
        out = {"metrics": np.array(r.metrics[:]), "t_submit_ms": r.t_submit_ms, "t_admit_ms": r.t_admit_ms,
               "t_done_ms": r.t_done_ms}
        if want_grad:
            out["grad_layer"] = np.array([r.grad_layer[m][:] for m in range(3)])
            out["grad_elt"] = ge
        return out

    def wait(self, ticket: int):
        return self._result(ticket, True)

    def poll(self, ticket: int):
        return self._result(ticket, False)

    def cancel(self, ticket: int) -> bool:
        rc = library().ara_server_cancel(self.handle, ticket)
        if rc == ARA_E_BUSY:
            return False
        _check(rc, "ara_server_cancel")
        return True

    def stats(self):
        st = (_c_i64 * 9)()
        _check(library().ara_server_stats(self.handle, st), "ara_server_stats")
        keys = ["iterations", "packed_launches", "max_quotes_per_launch", "queued", "active", "free_arena_bytes",
                "items", "shared_block_items", "max_finished_per_launch"]
        return dict(zip(keys, list(st)))

    def close(self):
        if self.handle:
            library().ara_server_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------
# autograd
# --------------------------------------------------------------------------

class YLT(torch.autograd.Function):
    """ylt = YLT.apply(elt_terms, layer_terms, engine) with engine = (tables, yet, layers, t0, t1)."""

    @staticmethod
    def forward(ctx, elt_terms, layer_terms, engine):
        tables, yet, layers, t0, t1 = engine
        ylt, s_pre, _ = ylt_forward(tables, yet, layers, elt_terms, layer_terms, t0, t1, want_s_pre=True)
        ctx.engine = engine
        ctx.save_for_backward(elt_terms, layer_terms, s_pre)
        return ylt

    @staticmethod
    def backward(ctx, grad_ylt):
        elt_terms, layer_terms, s_pre = ctx.saved_tensors
        tables, yet, layers, t0, t1 = ctx.engine
        ge, gl = ylt_backward(tables, yet, layers, elt_terms, layer_terms, s_pre, grad_ylt, t0, t1)
        return ge.to(elt_terms.dtype), gl.to(layer_terms.dtype), None


class Metrics(torch.autograd.Function):
    """out = Metrics.apply(ylt, p): [n_layers, 3] = (AAL, PML_p, TVaR_p)."""

    @staticmethod
    def forward(ctx, ylt, p):
        out, w = metrics(ylt, p, want_weights=True)
        ctx.save_for_backward(w)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        (w,) = ctx.saved_tensors
        return metrics_vjp(w, grad_out), None


__all__ = [
    "AraError", "PreparedYet", "EltTables", "SigmaTables", "Layers", "ylt_forward", "ylt_forward_su", "yelt_forward",
    "metrics", "metrics_vjp", "ylt_backward",
    "YLT", "Metrics", "QuoteServer", "library", "ara_yet", "ara_tables", "ara_layers", "ARA_F_EMIT_HITS", "ARA_F_FP32_ACCUM",
]
