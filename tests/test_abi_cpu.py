"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_1501_06561_amd import fdsketch as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "fdsketch.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M))


def test_library_exports_every_declared_symbol():
    L = F.lib()
    decl = _declared()
    assert decl, "no declarations parsed"
    assert decl == set(F.EXPORTS), decl ^ set(F.EXPORTS)
    for name in decl:
        assert hasattr(L, name), name
    assert b"gfx950" in L.fdsk_version()


@pytest.mark.parametrize("cfg,code", [
    (dict(d=0, l=4), -1),
    (dict(d=10, l=0), -1),
    (dict(d=10, l=8, buffer_rows=5), -1),
    (dict(d=10, l=600), -6),                 # 2l > 1024
    (dict(d=10, l=8, variant=7), -1),
    (dict(d=10, l=8, variant=6), -1),
    (dict(d=10, l=8, variant=4), -1),                  # SSD needs buffer_rows == l
    (dict(d=10, l=8, variant=4, buffer_rows=12), -1),
    (dict(d=10, l=1, variant=4, buffer_rows=1), -1),   # SSD needs l >= 2
    (dict(d=10, l=8, variant=2, alpha=0.0), -1),
    (dict(d=10, l=8, variant=3, alpha=1.5), -1),
    (dict(d=10, l=8, flags=6), -1),
    (dict(d=10, l=8, precision=4), -1),
    (dict(d=10, l=8, precision=1), -6),      # one BF16 pass: fdsk_gram only
    (dict(d=70000, l=8), -1),
])
def test_create_rejects_bad_config(cfg, code):
    c = F.FdskConfig(cfg.get("d", 10), cfg.get("l", 4), cfg.get("buffer_rows", 0),
                     cfg.get("variant", 0), cfg.get("alpha", 0.2), cfg.get("precision", 0),
                     cfg.get("flags", 0))
    h = ctypes.c_void_p()
    rc = F.lib().sketch_create(ctypes.byref(c), None, ctypes.byref(h))
    assert rc == code
    assert not h.value
    assert F.lib().sketch_last_error(None)


@pytest.mark.parametrize("cfg,code", [
    (dict(variant=4, buffer_rows=8), -6),      # SSD: single sketches only
    (dict(variant=5), -6),                     # CFD: single sketches only
    (dict(variant=6), -1),
    (dict(precision=3), -6),                   # FP8 Gram: single sketches only
    (dict(precision=1), -6),                   # one BF16 pass: fdsk_gram only
    (dict(l=200), -6),                         # 400 buffer rows > 256
    (dict(flags=1), -1),                       # flags differ between the sketches
    (dict(flags=2), -6),                       # Jacobi: single sketches only
])
def test_batch_create_rejects_bad_config(cfg, code):
    good = F.FdskConfig(64, 8, 0, 0, 0.2, 0, 0)
    bad = F.FdskConfig(cfg.get("d", 64), cfg.get("l", 8), cfg.get("buffer_rows", 0),
                       cfg.get("variant", 0), cfg.get("alpha", 0.2), cfg.get("precision", 0),
                       cfg.get("flags", 0))
    arr = (F.FdskConfig * 2)(good, bad)
    h = ctypes.c_void_p()
    rc = F.lib().sketch_batch_create(2, arr, None, ctypes.byref(h))
    assert rc == code
    assert not h.value
    assert F.lib().sketch_batch_last_error(None)


def test_null_handles_are_rejected():
    L = F.lib()
    rep = F.FdskReport()
    assert L.sketch_append_rows(None, None, 1, 1, 0, 0) == -1
    assert L.sketch_finalize(None, None, 1, 0, 0, None) == -1
    assert L.sketch_merge(None, None) == -1
    assert L.sketch_stats(None, ctypes.byref(rep)) == -1
    L.sketch_destroy(None)


def test_batch_null_handles_are_rejected():
    L = F.lib()
    assert L.sketch_batch_reset(None) == -1
    assert L.sketch_batch_profile(None, ctypes.byref(F.FdskProfile())) == -1
    L.sketch_batch_destroy(None)


def test_struct_layouts_match_header():
    assert ctypes.sizeof(F.FdskProfile) == 9 * 8 * 3
    assert ctypes.sizeof(F.FdskConfig) == 40
    assert ctypes.sizeof(F.FdskReport) == 9 * 8 + 2 * 8 + 4 * 4 + 8


@pytest.mark.parametrize("kind,d,l,s,code", [
    (7, 10, 8, 4, -1),        # unknown kind
    (0, 0, 8, 4, -1),         # d = 0
    (2, 10, 0, 4, -1),        # l = 0
    (1, 10, 10, 4, -1),       # OSNAP: s must divide l
    (1, 10, 8, 9, -1),        # OSNAP: s <= 8
])
def test_rsketch_create_rejects_bad_arguments(kind, d, l, s, code):
    h = ctypes.c_void_p()
    rc = F.lib().rsketch_create(kind, d, l, s, ctypes.c_uint64(0), None, ctypes.byref(h))
    assert rc == code
    assert not h.value
    assert F.lib().rsketch_last_error(None)
