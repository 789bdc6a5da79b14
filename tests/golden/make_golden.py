"""Write the stored oracle outputs under tests/golden/.

Calls only the CPU oracle (oracle/) and the seeded input generator; nothing
here comes from the GPU path.  Run from the repository root:

    python tests/golden/make_golden.py
"""
from __future__ import annotations

import hashlib
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2306_16731_amd import workloads as wl  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def c1_case(seed: int = 0):
    """16 patches of 3x3 interior volumes, 2D Euler, N = 5, one step, CFL 0.4."""
    b = wl.make_uniform(16, 3, dim=2, nq=5, seed=seed)
    lam0 = oracle.batch_lambda(b.data, b.sizes, b.offsets, 2, 5)
    dt = wl.CFL * wl.H_DEFAULT / (2 * float(np.max(lam0)))
    out, lam = oracle.batch_update(b.data, b.sizes, b.offsets, 2, 5, dt, wl.H_DEFAULT, wl.GAMMA, False)
    return b, dt, out, lam


def input_digest(data: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(data, dtype="<f8").tobytes()).hexdigest()


def main():
    b, dt, out, lam = c1_case(0)
    path = os.path.join(HERE, "c1_2d_p3_T16_seed0.txt")
    with open(path, "w") as f:
        f.write("# One explicit Euler step of the Rusanov FV scheme (paper Sec. 2.2 update, Eq. 2 flux,\n")
        f.write("# Euler user terms of Sec. 5) over 16 patches of 3x3 interior volumes, 2D, N = 5,\n")
        f.write("# gamma = 1.4, h = 1/48, dt = CFL h / (d max lambda0) with CFL = 0.4; per-patch eigenvalue\n")
        f.write("# of the new state (end of Sec. 2.2).  Written by tests/golden/make_golden.py from the oracle.\n")
        f.write(f"input_sha256 {input_digest(b.data)}\n")
        f.write(f"dt {dt!r}\n")
        for t in range(16):
            f.write(f"lambda {t} {float(lam[t])!r}\n")
        for t in range(16):
            v = out[b.offsets[t]:b.offsets[t] + 25 * 5].reshape(5, 5, 5)
            for j in range(1, 4):
                for i in range(1, 4):
                    f.write(f"q {t} {j} {i} " + " ".join(repr(float(x)) for x in v[j, i]) + "\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
