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
                (64, 64, 2, 99, 1, 0), (64, 64, 2, 2, -1, 0), (64, 64, 2, 2, 1, 64),
                (1, 1 << 24, 1, 1, 1, 0), (1 << 24, 1, 1, 1, 1, 0), (1 << 15, 1 << 15, 1, 1, 1, 0)]:
        assert lib.of_plan_workspace_bytes(*bad) == 0
    # widths and heights up to 2^24 - 1 (24-bit row offsets) with H * W below 2^30
    assert lib.of_plan_workspace_bytes(1, (1 << 24) - 1, 1, 1, 1, 0) > 0
    # OF_FLAG_NORMALIZE adds two level-0 float32 planes; the Gaussian window needs nothing more
    assert lib.of_plan_workspace_bytes(H, W, 3, 4, 4, 8) == expect + 2 * a(H * W * 4)
    assert lib.of_plan_workspace_bytes(H, W, 3, 4, 4, 16) == expect
    # OF_FLAG_GRAPH changes the launch mode only
    assert lib.of_plan_workspace_bytes(H, W, 3, 4, 4, 32) == expect
    # the plan-only flags (equalisation, graph capture) are refused by batches and servers; the
    # Gaussian window is accepted by every form
    import ctypes
    hs, ws = (ctypes.c_int * 1)(H), (ctypes.c_int * 1)(W)
    assert lib.of_batch_workspace_bytes(1, hs, ws, 3, 4, 4, 0) > 0
    for f in (8, 32):
        assert lib.of_batch_workspace_bytes(1, hs, ws, 3, 4, 4, f) == 0
        assert lib.of_session_bytes(H, W, 3, 4, 4, f) == 0
    assert lib.of_batch_workspace_bytes(1, hs, ws, 3, 4, 4, 16) == lib.of_batch_workspace_bytes(1, hs, ws, 3, 4, 4, 0)
    assert lib.of_session_bytes(H, W, 3, 4, 4, 16) == lib.of_session_bytes(H, W, 3, 4, 4, 0)
    assert lib.of_plan_create(0, 5, 1, 1, 1) is None
    assert b"H and W" in lib.of_last_error()
    assert lib.of_compute(None, None, None, None, None, None) == 1
    assert b"NULL plan" in lib.of_last_error()
    lib.of_plan_destroy(None)


def test_host_side_rejections_of_the_newer_entry_points(lib):
    """Argument checks that reject before any HIP call."""
    import ctypes
    from paper_1306_2461_amd import _binding as B
    assert lib.of_session_create(0, 5, 3, 4, 4, 0, None, 0) is None
    assert lib.of_session_create(64, 64, 3, 4, 4, B.OF_FLAG_NORMALIZE, None, 0) is None
    assert b"plans only" in lib.of_last_error()
    assert lib.of_session_push_many(None, 0, None, None, None, None, None) == B.OF_EINVAL
    lib.of_session_destroy(None)
    assert lib.of_server_open_ex(None, 64, 64, None, 0) is None
    assert lib.of_plan_set_bubble(None, None, None) == B.OF_EINVAL
    assert lib.of_batch_set_masks(None, None, None) == B.OF_EINVAL
    assert lib.of_session_set_mask(None, None, None) == B.OF_EINVAL
    assert lib.of_bubble_step(None, None, 1, 0, None, None, None, None, None) == B.OF_EINVAL
    assert lib.of_plan_set_timing(None, 1) == B.OF_EINVAL
    assert lib.of_compute_noalloc(64, 64, 3, 4, 2, B.OF_FLAG_GRAPH, None, None, None, None, None) == B.OF_EINVAL
    assert lib.of_compute_noalloc(64, 64, 9, 4, 2, 0, None, None, None, None, None) == B.OF_EINVAL
    # the allocation-free form holds a 1024 x 1024 FP32 pair at 4 levels, not a 2048 x 2048 one
    cap = lib.of_noalloc_scratch_bytes()
    assert lib.of_plan_workspace_bytes(1024, 1024, 4, 8, 4, 0) <= cap < lib.of_plan_workspace_bytes(2048, 2048, 4, 8, 4, 0)
    # batch workspace grows by the argument blocks of the graph slots and the eager ring
    hs, ws = (ctypes.c_int * 2)(64, 96), (ctypes.c_int * 2)(80, 33)
    assert lib.of_batch_workspace_bytes(2, hs, ws, 2, 3, 2, 0) > lib.of_plan_workspace_bytes(64, 80, 2, 3, 2, 0) + \
        lib.of_plan_workspace_bytes(96, 33, 2, 3, 2, 0)
