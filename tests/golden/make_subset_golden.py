"""Writes the oracle's solutions of the 2000-sphere standalone subsets used by the GPU parity tests.

The subsets are the 2000 spheres nearest the trap centre of the N = 10^4 time-stepping workload
(with the rank-3 trace slip) and of the N = 10^5 benchmark workload, each solved as its own system
by the oracle (dense assembly from the symbolic pair blocks, LAPACK solve, output pass). Only
`oracle/` and the seeded input generator are used; a hash of the centres ties each file to its
inputs.

    python tests/golden/make_subset_golden.py
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import galerkin  # noqa: E402
from paper_1411_0278_amd import inputs  # noqa: E402

SUBSET = 2000


def subsets():
    return {"cfg1_subset2000": inputs.nearest_to_origin(inputs.config1(), SUBSET),
            "cfg2_subset2000": inputs.nearest_to_origin(inputs.config2(), SUBSET)}


def centres_hash(R):
    return hashlib.sha256(np.ascontiguousarray(R, dtype=np.float64).tobytes()).hexdigest()[:16]


def main():
    for name, w in subsets().items():
        t = time.perf_counter()
        ref = galerkin.solve(w)
        np.savez_compressed(os.path.join(HERE, name + ".npz"), V=ref["V"], W=ref["W"], S=ref["S"],
                            Sigma=ref["Sigma"], centres_sha=centres_hash(w.R))
        print(f"{name}: n = {w.n}, oracle solve {time.perf_counter() - t:.1f} s", flush=True)


if __name__ == "__main__":
    main()
