"""The C-ABI library loads and exports every entry point declared in include/krig.h (no GPU calls)."""
import os
import re
import ctypes

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "krig.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(krig_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("krig_plan_create", "krig_weights", "krig_scatter", "krig_predict", "krig_predict_adjoint",
              "krig_csim", "krig_solve", "krig_convolve"):
        assert s in syms


def test_library_exports_every_declared_symbol(krig):
    lib = ctypes.CDLL(krig.LIB_PATH)
    for s in declared_symbols():
        assert hasattr(lib, s), s
    assert set(declared_symbols()) <= set(krig.EXPORTS)


def test_argument_errors_are_reported_without_a_gpu(krig):
    lib = krig.load_library()
    # NULL plan / NULL output pointer are rejected on the host before any device work
    assert lib.krig_plan_destroy(None) == -1
    assert lib.krig_plan_create(None, None, None, 0, None, 1, None) == -1
    assert lib.krig_strerror(-2) == b"site outside the prediction grid"
