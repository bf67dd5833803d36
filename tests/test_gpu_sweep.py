"""Table-1 style sweep at the paper's region of interest: the shape of Table 1 (error falls
with n_iter toward the (4, 7) reference; time per field is affine in n_iter), checked against
the paper's printed values in tests/golden/table1.json."""
import json
import os

import numpy as np
import pytest

import synth
from gpu_util import announce, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1.json")


def test_table1_shape(gpu_lib):
    from paper_1306_2461_amd.sweep import table1_sweep
    paper = json.load(open(GOLDEN))
    I1, I2, _, _ = synth.make_pair("t1", 0)
    announce("table-1 sweep 1792x384 r=10")
    res = table1_sweep(to_dev(I1), to_dev(I2), reps=20)
    for L in (3, 4):
        e = np.array(res[L]["error_percent"])
        fps = np.array(res[L]["fields_per_s"])
        pe = np.array(paper[f"n_lev_{L}"]["error_percent"])
        # like the paper: the error shrinks from n_iter = 1 to n_iter = 6 and is smallest last
        assert e[0] > e[5] and e[-1] <= e[:-1].min() + 1e-9 and pe[0] > pe[5]
        # time per field affine in n_iter (the paper's rows fit t = a + b n_iter)
        t = 1.0 / fps
        k = np.arange(1, 8)
        b, a = np.polyfit(k, t, 1)
        assert b > 0 and np.max(np.abs(a + b * k - t)) < 0.25 * t.max()
    assert res[4]["error_percent"][-1] == 0.0
