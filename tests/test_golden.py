"""The oracle still produces the stored config-1 result (guards against silent drift of
the oracle or the input generator)."""
import numpy as np

import oracle
from tests.golden import make_golden as mg


def _read(path):
    lam, q, meta = {}, {}, {}
    for line in open(path):
        if line.startswith("#"):
            continue
        parts = line.split()
        if parts[0] == "lambda":
            lam[int(parts[1])] = float(parts[2])
        elif parts[0] == "q":
            q[tuple(int(x) for x in parts[1:4])] = np.array([float(x) for x in parts[4:]])
        else:
            meta[parts[0]] = parts[1]
    return meta, lam, q


def test_c1_golden():
    import os
    meta, lam, q = _read(os.path.join(os.path.dirname(mg.__file__), "c1_2d_p3_T16_seed0.txt"))
    b, dt, out, got_lam = mg.c1_case(0)
    assert mg.input_digest(b.data) == meta["input_sha256"]
    assert float(meta["dt"]) == dt
    for t in range(16):
        assert got_lam[t] == lam[t]
        v = out[b.offsets[t]:b.offsets[t] + 125].reshape(5, 5, 5)
        for j in range(1, 4):
            for i in range(1, 4):
                assert np.array_equal(v[j, i], q[(t, j, i)])
