"""Writes the oracle's end states of the 512^2 four-quadrant Riemann problem
(seeded +-5 % quadrant states, transmissive, CFL 0.5) at t = 0.25, for the
full-size trajectory tests: one run from the FP64 initial state and one from
that state rounded to FP32 (what FP32 storage holds).  Only the oracle runs
here.  Stored per run: the step count and end time, every 8th cell in x and
y (offset 3), the full middle row and column, and the per-field minimum and
maximum over the grid; compressed (numpy savez_compressed).

    python tests/golden/make_fullsize_golden.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2601_04400_amd import inputs  # noqa: E402

N, T_END, STRIDE, OFFSET = 512, 0.25, 8, 3


def sample(U):
    return {"cells": U[:, OFFSET::STRIDE, OFFSET::STRIDE].copy(),
            "row": U[:, N // 2, :].copy(), "col": U[:, :, N // 2].copy(),
            "fmin": U.reshape(4, -1).min(axis=1), "fmax": U.reshape(4, -1).max(axis=1)}


def main():
    c = oracle.config(nx=N, ny=N)
    U0 = oracle.prim_to_cons(c, inputs.riemann2d_prim(N, N))
    for name, U in (("f64", U0), ("f32ic", U0.astype(np.float32).astype(np.float64))):
        t0 = time.perf_counter()
        Ue, te, steps, fb = oracle.run(c, U, T_END)
        s = sample(Ue)
        path = os.path.join(HERE, f"riemann2d_512_t025_{name}.npz")
        np.savez_compressed(path, steps=steps, t=te, fallbacks=fb, stride=STRIDE, offset=OFFSET, **s)
        print(f"{path}: {steps} steps to t = {te}, {fb} fallback faces, {time.perf_counter() - t0:.1f} s "
              f"({oracle.threads()} threads)", flush=True)


if __name__ == "__main__":
    main()
