"""The C-ABI library loads and exports every symbol the headers declare (no GPU needed).

Only host-side behaviour is exercised here: workspace sizing and argument validation,
which reject bad input before any HIP call.
"""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        names |= set(re.findall(r"OF_API\s+[^;(]*?\b(of_\w+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    import paper_1306_2461_amd as ofmi
    return ofmi.load()


def test_headers_declare_entry_points():
    names = _declared()
    for n in ("of_plan_create", "of_compute", "of_plan_destroy", "of_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    from paper_1306_2461_amd import _binding
    assert set(_declared()) <= set(_binding.SIGNATURES), "binding lacks a declared entry point"


def test_workspace_bytes_and_validation(lib):
    # 2 pyramids of levels >= 1 (FP32) + 4 level-0 flow planes, each 256-byte aligned
    def a(x):
        return (x + 255) // 256 * 256
    H, W = 100, 70
    sizes = [(50, 35), (25, 18)]
    expect = sum(2 * a(h * w * 4) for h, w in sizes) + 4 * a(H * W * 4)
    assert lib.of_plan_workspace_bytes(H, W, 3, 4, 4, 0) == expect
    expect16 = sum(2 * a(h * w * 2) for h, w in sizes) + 4 * a(H * W * 4)
    assert lib.of_plan_workspace_bytes(H, W, 3, 4, 4, 1) == expect16
    for bad in [(0, 5, 1, 1, 1, 0), (5, 5, 0, 1, 1, 0), (4, 4, 4, 1, 1, 0), (64, 64, 2, -1, 1, 0),
                (64, 64, 2, 99, 1, 0), (64, 64, 2, 2, -1, 0), (64, 64, 2, 2, 1, 64)]:
        assert lib.of_plan_workspace_bytes(*bad) == 0
    # OF_FLAG_NORMALIZE adds two level-0 float32 planes; the Gaussian window needs nothing more
    assert lib.of_plan_workspace_bytes(H, W, 3, 4, 4, 8) == expect + 2 * a(H * W * 4)
    assert lib.of_plan_workspace_bytes(H, W, 3, 4, 4, 16) == expect
    # OF_FLAG_GRAPH changes the launch mode only
    assert lib.of_plan_workspace_bytes(H, W, 3, 4, 4, 32) == expect
    # the plan-only flags are refused by batches and servers
    import ctypes
    hs, ws = (ctypes.c_int * 1)(H), (ctypes.c_int * 1)(W)
    assert lib.of_batch_workspace_bytes(1, hs, ws, 3, 4, 4, 0) > 0
    for f in (8, 16, 32):
        assert lib.of_batch_workspace_bytes(1, hs, ws, 3, 4, 4, f) == 0
        assert lib.of_session_bytes(H, W, 3, 4, 4, f) == 0
    assert lib.of_plan_create(0, 5, 1, 1, 1) is None
    assert b"H and W" in lib.of_last_error()
    assert lib.of_compute(None, None, None, None, None, None) == 1
    assert b"NULL plan" in lib.of_last_error()
    lib.of_plan_destroy(None)
