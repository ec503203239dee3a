"""The C-ABI library builds, loads and exports every entry point that
include/qhp.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "qhp.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(qhp_\w+)\s*\(", text, re.M)))


def test_header_declares_the_verbs():
    names = declared_symbols()
    for verb in ("qhp_create", "qhp_mesh", "qhp_assemble", "qhp_set_incident", "qhp_step", "qhp_run",
                 "qhp_history_sum", "qhp_destroy"):
        assert verb in names


def test_library_exports_every_declared_symbol():
    import paper_2312_06367_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("libqhp.so not built")
    L = ctypes.CDLL(pkg.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(L, name), name
    assert set(declared_symbols()) == set(pkg.EXPORTS)


def test_batch_tile_shape_counts():
    """qhp_batch_variants is host logic: six history tile shapes for FP32 or
    FP32-block/FP64-sum batches with 2, 4 or 8 right-hand sides, one where
    there is no choice, none for unsupported precisions or counts."""
    import paper_2312_06367_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("libqhp.so not built")
    for p in ("f32", "f32a"):
        for n in (2, 4, 8):
            assert pkg.batch_variants(p, n) == 6
        assert pkg.batch_variants(p, 1) == 1
        assert pkg.batch_variants(p, 3) == 0
    assert pkg.batch_variants("f64", 8) == 1
    assert pkg.batch_variants("bf16", 4) == 0
    assert pkg.batch_variants("i8x4", 8) == 0
