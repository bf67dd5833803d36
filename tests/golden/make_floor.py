"""Writes tests/golden/floor/<case>.npz: the per-pixel FP32 rounding floor of the oracle's
operation order for every case of tests/floor_util.py (the oracle and the seeded input
generators only; no GPU).  Run from the repository root:

    python tests/golden/make_floor.py [case ...]
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))                    # tests/
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))   # repository root

import floor_util  # noqa: E402


def main(names):
    for name in names or sorted(floor_util.CASES):
        t = time.perf_counter()
        f = floor_util.case_floor(name)
        floor_util.save_floor(name, f)
        tol = floor_util.CASES[name][6]
        print(f"{name}: shape {f.shape}, max floor {f.max():.3e} px, {(f > tol).sum()} px over "
              f"{tol:g}, {time.perf_counter() - t:.1f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
