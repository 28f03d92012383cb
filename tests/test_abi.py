"""The C-ABI library loads and exports every entry point include/dbl.h declares (no GPU needed)."""
import ctypes
import os
import re

import paper_2101_09441_amd as dbl
from paper_2101_09441_amd.binding import DblOptions

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "dbl.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dbl_[a-z_]+)\s*\(", text)))


def test_header_declares_what_the_binding_expects():
    assert _declared() == sorted(dbl.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = dbl.load_library()
    for name in _declared():
        assert hasattr(lib, name), name


def test_host_only_entry_points():
    lib = dbl.load_library()
    opt = DblOptions()
    lib.dbl_default_options(ctypes.byref(opt))
    assert opt.num_landmarks == 64 and opt.bl_bits == 64
    assert abs(opt.slack_fraction - 0.25) < 1e-7 and opt.slack_min == 4
    assert lib.dbl_status_str(dbl.DBL_ERR_VERTEX_RANGE) == b"vertex id out of range"
    assert lib.dbl_num_vertices(None) == 0
    out = ctypes.c_void_p(123)
    # invalid arguments are rejected before any device work
    assert lib.dbl_build(0, 0, None, None, None, None, ctypes.byref(out)) == dbl.DBL_ERR_INVALID_ARG
    assert out.value is None
    bad = DblOptions()
    lib.dbl_default_options(ctypes.byref(bad))
    bad.bl_bits = 48
    assert lib.dbl_build(4, 0, None, None, ctypes.byref(bad), None,
                         ctypes.byref(out)) == dbl.DBL_ERR_INVALID_ARG
    assert opt.row_fill == 0
    lib.dbl_default_options(ctypes.byref(bad))
    bad.row_fill = 3
    assert lib.dbl_build(4, 0, None, None, ctypes.byref(bad), None,
                         ctypes.byref(out)) == dbl.DBL_ERR_INVALID_ARG
    assert lib.dbl_insert_edges(None, 1, None, None, None) == dbl.DBL_ERR_INVALID_ARG
    assert lib.dbl_query_batch(None, 1, None, None, None, None) == dbl.DBL_ERR_INVALID_ARG
    assert lib.dbl_query_batch_noalloc(None, 1, None, None, None,
                                       None) == dbl.DBL_ERR_INVALID_ARG
