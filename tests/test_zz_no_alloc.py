"""of_compute_noalloc: the allocation-free entry point (a fixed device scratch array inside the
library instead of a plan workspace) gives the same bits as of_compute with a plan in the
default launch configuration, on two calls in a row, the second with a smaller frame."""
import ctypes

import numpy as np
import pytest

import synth
from gpu_util import announce, dev, to_dev

pytestmark = pytest.mark.gpu


def _noalloc(lib, I1, I2, L, r, K, flags=0):
    import torch
    H, W = I1.shape
    u = torch.full((H, W), float("nan"), dtype=torch.float32, device=dev())
    v = torch.full((H, W), float("nan"), dtype=torch.float32, device=dev())
    st = lib.of_compute_noalloc(H, W, L, r, K, flags, I1.data_ptr(), I2.data_ptr(), u.data_ptr(),
                                v.data_ptr(), torch.cuda.current_stream().cuda_stream)
    return st, u, v


def test_noalloc_matches_plan_twice_then_smaller(gpu_lib):
    import torch
    ofmi = gpu_lib
    from paper_1306_2461_amd import _binding as B
    lib = B.load()
    assert lib.of_noalloc_scratch_bytes() >= (16 << 20)
    big1, big2, _, _ = synth.make_pair("c2", 3)
    small1, small2 = big1[:200, :333].copy(), big2[:200, :333].copy()
    cases = [(big1, big2, 4, 8, 4, 0), (small1, small2, 3, 5, 3, 0),
             (small1, small2, 3, 4, 2, B.OF_FLAG_FP16_STORAGE)]
    for I1, I2, L, r, K, flags in cases:
        H, W = I1.shape
        announce(f"noalloc {H}x{W} L={L} r={r} K={K} flags={flags}")
        d1, d2 = to_dev(I1), to_dev(I2)
        st, u, v = _noalloc(lib, d1, d2, L, r, K, flags)
        assert st == 0, B.last_error()
        plan = ofmi.Plan(H, W, L, r, K, fp16=bool(flags & B.OF_FLAG_FP16_STORAGE), device=dev())
        pu, pv = plan.compute(d1, d2)
        torch.cuda.synchronize()
        assert np.array_equal(u.cpu().numpy(), pu.cpu().numpy())
        assert np.array_equal(v.cpu().numpy(), pv.cpu().numpy())
        plan.close()


def test_noalloc_rejects_oversize_and_bad_arguments(gpu_lib):
    import torch
    from paper_1306_2461_amd import _binding as B
    lib = B.load()
    cap = lib.of_noalloc_scratch_bytes()
    need = lib.of_plan_workspace_bytes(2048, 2048, 4, 8, 4, 0)
    assert need > cap
    d = torch.zeros((2048, 2048), dtype=torch.uint8, device=dev())
    st, _, _ = _noalloc(lib, d, d, 4, 8, 4)
    assert st == B.OF_ENOMEM and b"scratch" in lib.of_last_error()
    small = torch.zeros((64, 64), dtype=torch.uint8, device=dev())
    st, _, _ = _noalloc(lib, small, small, 3, 4, 2, B.OF_FLAG_GRAPH)
    assert st == B.OF_EINVAL
    st = lib.of_compute_noalloc(64, 64, 3, 4, 2, 0, None, small.data_ptr(), small.data_ptr(),
                                small.data_ptr(), None)
    assert st == B.OF_EINVAL
    torch.cuda.synchronize()
