"""Write the oracle's eigenvalues for k-point 0 of the two large LCAO
configurations, which the GPU parity tests compare with (the oracle takes
minutes there, too long to run inside a test):

  oracle_eig_lcao_n3000_k0.txt : n = 3000, seed 2002, the first 4x4x4 point
  oracle_eig_lcao_n4096_k0.txt : n = 4096, seed 4004, the first 2x2x2 point

Every value comes from ``oracle`` (plain FP64 CPU oracle) on inputs from
``paper_1402_4247_amd.inputs``; nothing here touches the GPU library.
Run from the repository root: ``python tests/golden/make_oracle_fixtures.py``.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1402_4247_amd import inputs as G  # noqa: E402

CASES = [
    ("oracle_eig_lcao_n3000_k0.txt", lambda: G.config2(3000, 1, 2002), "n = 3000, seed 2002, k = (-3/8, -3/8, -3/8)"),
    ("oracle_eig_lcao_n4096_k0.txt", lambda: G.config4(4096, 1, 4004), "n = 4096, seed 4004, k = (-1/4, -1/4, -1/4)"),
]


def main():
    for fname, gen, what in CASES:
        path = os.path.join(HERE, fname)
        Hs, Ss = gen()
        t = time.time()
        st, w, _ = O.solve_k(Hs[0], Ss[0], vectors=False)
        el = time.time() - t
        if st != 0:
            raise RuntimeError(f"oracle status {st} for {what}")
        header = (f"oracle eigenvalues (ascending) of the LCAO pencil {what}; "
                  f"written by tests/golden/make_oracle_fixtures.py ({O.max_threads()} threads, {el:.0f} s)")
        np.savetxt(path, w, fmt="%.17e", header=header)
        print(f"{fname}: {len(w)} values, {el:.0f} s", flush=True)


if __name__ == "__main__":
    main()
