"""Host-side checks of the C ABI: the library loads, exports every function
include/ara.h declares, and rejects bad arguments before any device work.
No compute call reaches a GPU here."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ara.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ara_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def ara():
    import paper_1308_2572_amd as ara
    ara.library()
    return ara


def test_every_declared_symbol_is_exported(ara):
    lib = ara.library()
    names = declared_functions()
    assert len(names) >= 14
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    # and the binding wraps each of them with a signature
    from paper_1308_2572_amd import _SIGNATURES
    assert sorted(_SIGNATURES) == names


def test_status_strings(ara):
    lib = ara.library()
    assert lib.ara_status_string(0) == b"ok"
    assert b"duplicate" in lib.ara_status_string(3)
    assert lib.ara_status_string(99) == b"unknown status"
    assert lib.ara_abi_version() == 2


def test_profile_controls(ara):
    """Recording by kind: known kinds are accepted (nothing is recorded
    without device work), unknown bits are refused, and reads of a kind
    with no launches give zero."""
    lib = ara.library()
    assert lib.ara_profile_enable_kinds(1 << ara.PROF_FWD) == 0
    assert lib.ara_profile_enable_kinds(0xFF) == 0
    assert lib.ara_profile_enable_kinds(1 << 8) == 1
    assert b"unknown kind" in lib.ara_last_error()
    assert lib.ara_profile_enable(0) == 0
    assert lib.ara_profile_reset() == 0
    ms, n = ctypes.c_double(), ctypes.c_int64()
    assert lib.ara_profile_read(ara.PROF_METRICS, ctypes.byref(ms), ctypes.byref(n)) == 0
    assert ms.value == 0.0 and n.value == 0
    assert lib.ara_profile_read(8, ctypes.byref(ms), ctypes.byref(n)) == 1


def test_size_queries(ara):
    lib = ara.library()
    nb = ctypes.c_size_t()
    assert lib.ara_yet_prepare_bytes(1000, 1_000_000, 200_000, 0, ctypes.byref(nb)) == 0
    assert nb.value >= 4 * 1_000_000
    plain = nb.value
    assert lib.ara_yet_prepare_bytes(1000, 1_000_000, 200_000, ara.PREP_TRANSPOSED, ctypes.byref(nb)) == 0
    assert nb.value >= plain + 4 * 1_000_000 + 8 * (8 * 200_000 + 1)     # event-major entries and list offsets
    tr = nb.value
    # the trial-major copy adds the offsets and the IDs once more
    assert lib.ara_yet_prepare_bytes(1000, 1_000_000, 200_000, ara.PREP_TRANSPOSED | ara.PREP_TRIAL_MAJOR,
                                     ctypes.byref(nb)) == 0
    assert nb.value >= tr + 4 * 1_000_000 + 8 * 1001
    # positions add one 16-bit word per code slot and a copy of the offsets
    assert lib.ara_yet_prepare_bytes(1000, 1_000_000, 200_000, ara.PREP_POSITIONS, ctypes.byref(nb)) == 0
    assert nb.value >= plain + 2 * 1_000_000 + 8 * 1001
    assert lib.ara_yet_prepare_bytes(1000, 1_000_000, 200_000, 8, ctypes.byref(nb)) == 1   # unknown flag
    assert lib.ara_build_elt_tables_bytes(15, 2_000_000, ctypes.byref(nb)) == 0
    assert nb.value >= 15 * 2_000_000 * 4
    assert lib.ara_metrics_workspace_bytes(2, 1000, ctypes.byref(nb)) == 0
    assert nb.value >= 2 * 1000 * 8
    assert lib.ara_yet_prepare_bytes(10, 10, 1 << 27, 0, ctypes.byref(nb)) == 6       # beyond the catalogue limit
    assert lib.ara_yet_prepare_bytes(-1, 10, 100, 0, ctypes.byref(nb)) == 1


def test_argument_validation_before_device_work(ara):
    lib = ara.library()
    # p outside (0, 1)
    assert lib.ara_metrics(None, 1, 10, 1.5, None, None, None, 0, None) == 1
    assert b"p must" in lib.ara_last_error()
    # layer referring to an ELT that does not exist
    tables = ara.ara_tables(n_elts=2, catalog=100, words=4)
    yet = ara.ara_yet(n_trials=10, catalog=100, range_bits=15, groups=16)
    lay = ara.Layers([0, 2], [0, 5])
    nb = ctypes.c_size_t()
    assert lib.ara_ylt_workspace_bytes(ctypes.byref(tables), ctypes.byref(yet), ctypes.byref(lay.handle), 0,
                                       ctypes.byref(nb)) == 2
    # too many ELTs in one layer
    lay = ara.Layers([0, 130], np.zeros(130, np.int32))
    assert lib.ara_ylt_workspace_bytes(ctypes.byref(tables), ctypes.byref(yet), ctypes.byref(lay.handle), 0,
                                       ctypes.byref(nb)) == 6
    # more layers than one launch grid holds rows for
    L = ara.ARA_MAX_LAYERS + 1
    lay = ara.Layers(np.arange(L + 1, dtype=np.int32), np.zeros(L, np.int32))
    assert lib.ara_ylt_workspace_bytes(ctypes.byref(tables), ctypes.byref(yet), ctypes.byref(lay.handle), 0,
                                       ctypes.byref(nb)) == 6
    assert b"ARA_MAX_LAYERS" in lib.ara_last_error()
    assert lib.ara_metrics(None, L, 10, 0.99, None, None, None, 0, None) == 6
    assert lib.ara_metrics_vjp(None, L, 10, None, None, None) == 6
    # mismatched catalogues
    yet2 = ara.ara_yet(n_trials=10, catalog=101, range_bits=15, groups=16)
    lay = ara.Layers([0, 1], [0])
    assert lib.ara_ylt_workspace_bytes(ctypes.byref(tables), ctypes.byref(yet2), ctypes.byref(lay.handle), 0,
                                       ctypes.byref(nb)) == 1
    # the two known flags are accepted alone and together; any other bit is not
    for fl in (ara.ARA_F_EMIT_HITS, ara.ARA_F_FP32_ACCUM, ara.ARA_F_EMIT_HITS | ara.ARA_F_FP32_ACCUM):
        assert lib.ara_ylt_workspace_bytes(ctypes.byref(tables), ctypes.byref(yet), ctypes.byref(lay.handle), fl,
                                           ctypes.byref(nb)) == 0
    # unknown flag, and hits without the flag
    for fl in (4, 8, 1 << 31):
        assert lib.ara_ylt_workspace_bytes(ctypes.byref(tables), ctypes.byref(yet), ctypes.byref(lay.handle), fl,
                                           ctypes.byref(nb)) == 1
    assert lib.ara_ylt_forward(ctypes.byref(tables), ctypes.byref(yet), ctypes.byref(lay.handle), None, None, 0, 5,
                               0, None, None, ctypes.c_void_p(16), None, 0, None) == 1
    # trial range outside the YET
    assert lib.ara_ylt_forward(ctypes.byref(tables), ctypes.byref(yet), ctypes.byref(lay.handle), None, None, 0, 11,
                               0, None, None, None, None, 0, None) == 2
    # the backward needs the event-major copy of the YET
    assert lib.ara_ylt_backward_workspace_bytes(ctypes.byref(tables), ctypes.byref(yet), ctypes.byref(lay.handle), 1,
                                                ctypes.byref(nb)) == 1
    assert b"ARA_PREP_TRANSPOSED" in lib.ara_last_error()


def test_forward_lds_plan_limits(ara):
    """The forward workgroup's LDS holds the per-trial totals (and hit
    counts), the range table and the segment windows, and the rest is one
    range's table slice.  At the largest catalogue (2048 ranges) with blocks
    of 4096 trials and hit counts nothing is left: the size query and the
    forward refuse with ARA_E_LIMIT before any device work, instead of a
    wrapped-around size.  Blocks of 3744 trials (234 per group) still do
    not fit with hit counts; 3728 do, and so does every size without them."""
    lib = ara.library()
    cat = 1 << 26
    tables = ara.ara_tables(n_elts=2, catalog=cat, words=cat // 32)
    lay = ara.Layers([0, 2], [0, 1])
    nb = ctypes.c_size_t()

    def query(tb, flags):
        yet = ara.ara_yet(n_trials=4 * tb, catalog=cat, range_bits=15, groups=16, trials_per_group=tb // 16,
                          trials_per_block=tb, n_blocks=4, n_ranges=2048)
        return lib.ara_ylt_workspace_bytes(ctypes.byref(tables), ctypes.byref(yet), ctypes.byref(lay.handle),
                                           flags, ctypes.byref(nb)), yet

    H, F = ara.ARA_F_EMIT_HITS, ara.ARA_F_FP32_ACCUM
    rc, yet = query(4096, H)
    assert rc == 6 and b"no LDS" in lib.ara_last_error()
    assert lib.ara_ylt_forward(ctypes.byref(tables), ctypes.byref(yet), ctypes.byref(lay.handle), ctypes.c_void_p(256),
                               ctypes.c_void_p(256), 0, 10, H, ctypes.c_void_p(256), None, ctypes.c_void_p(256),
                               ctypes.c_void_p(256), 1 << 40, None) == 6
    assert query(16 * 234, H)[0] == 6
    assert query(16 * 233, H)[0] == 0
    for fl in (0, F, H | F):
        assert query(4096, fl)[0] == 0, fl
    assert query(16 * 123, H)[0] == 0          # blocks of 1M trials on 256 CUs


def test_secondary_uncertainty_queries_and_validation(ara):
    lib = ara.library()
    tables = ara.ara_tables(n_elts=3, catalog=200_000, words=6250)
    lay = ara.Layers([0, 2, 3], [0, 2, 1])
    rec = np.array([1000, 50, 20_000], np.int64)
    nb = ctypes.c_size_t()
    assert lib.ara_su_workspace_bytes(ctypes.byref(tables), ctypes.byref(lay.handle), rec.ctypes.data_as(ctypes.c_void_p),
                                      ctypes.byref(nb)) == 0
    small = nb.value
    assert small >= (1000 + 20_000 + 50) * 32                       # one 32-byte entry per (event, ELT) pair
    rec2 = np.array([1000, 50, 90_000], np.int64)
    assert lib.ara_su_workspace_bytes(ctypes.byref(tables), ctypes.byref(lay.handle),
                                      rec2.ctypes.data_as(ctypes.c_void_p), ctypes.byref(nb)) == 0
    assert nb.value >= small + 70_000 * 32
    bad = np.array([1000, -1, 5], np.int64)
    assert lib.ara_su_workspace_bytes(ctypes.byref(tables), ctypes.byref(lay.handle),
                                      bad.ctypes.data_as(ctypes.c_void_p), ctypes.byref(nb)) == 1
    assert lib.ara_su_workspace_bytes(ctypes.byref(tables), ctypes.byref(lay.handle), None, ctypes.byref(nb)) == 1
    # a YET handle as ara_yet_prepare fills it (host-only stand-in: no device work happens below)
    fake = ctypes.c_void_p(256)
    yet = ara.ara_yet(n_trials=10, nnz=100, catalog=200_000, range_bits=15, n_ranges=7, groups=16,
                      trials_per_group=1, trials_per_block=16, n_blocks=1, code=fake, pos=fake, t_off=fake)
    recp = rec.ctypes.data_as(ctypes.c_void_p)

    def su(yet_, t0, t1, ws, nbytes, records=recp, ptr=None):
        return lib.ara_ylt_forward_su(ctypes.byref(tables), ptr, ctypes.byref(yet_), ctypes.byref(lay.handle), records,
                                      ptr, ptr, 7, t0, t1, ptr, None, ws, nbytes, None)
    # trial range outside the YET, null workspace, null records: all before any device work
    assert su(yet, 0, 11, fake, 1 << 30) == 2
    assert su(yet, 0, 10, None, 1 << 30) == 1
    assert su(yet, 0, 10, fake, 1 << 30, records=None) == 1
    # a workspace smaller than the query
    assert su(yet, 0, 10, fake, 4096, ptr=fake) == 4
    # a YET prepared without positions, or over another catalogue
    nopos = ara.ara_yet(n_trials=10, nnz=100, catalog=200_000, range_bits=15, n_ranges=7, groups=16, code=fake)
    assert su(nopos, 0, 10, fake, 1 << 30, ptr=fake) == 1
    other = ara.ara_yet(n_trials=10, nnz=100, catalog=100_000, range_bits=15, n_ranges=4, groups=16, code=fake,
                        pos=fake, t_off=fake)
    assert su(other, 0, 10, fake, 1 << 30, ptr=fake) == 1
    assert lib.ara_build_elt_sigma(ctypes.byref(tables), None, None, None, None, None) == 1


def test_product_refuses_to_run_without_library(tmp_path, monkeypatch):
    import paper_1308_2572_amd as ara
    monkeypatch.setattr(ara, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(ara, "_lib", None)
    with pytest.raises(ImportError):
        ara.library()


def test_product_does_not_import_oracle():
    src_dir = os.path.join(ROOT, "paper_1308_2572_amd")
    for dirpath, _, files in os.walk(src_dir):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "ara_oracle" not in text, f
