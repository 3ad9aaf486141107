"""Writes box_chain_256_lowest64.txt: the lowest 64 eigenvalues of the
256-site open-boundary chain (N_b = 2048) from the oracle's full H and S,
with the data the GPU test needs for its per-eigenvalue bound.  Calls only
the oracle and the seeded input generator.  Runs about a minute on 8 cores.

    python tests/golden/make_box_chain_eigs.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1408_3839_amd import workloads as wl  # noqa: E402


def main():
    s = wl.config(3)
    H, S = oracle.full_matrices(s)
    w, v = oracle.lowest_generalized_eigs(H, S, 64)
    un = np.sum(v * v, axis=0)
    nh = np.linalg.norm(H, 2)
    ns = np.linalg.norm(S, 2)
    out = os.path.join(HERE, "box_chain_256_lowest64.txt")
    with open(out, "w") as f:
        f.write("# lowest 64 eigenvalues of (H, S), 256-site open chain, N_b = 2048\n")
        f.write("# oracle.full_matrices + oracle.lowest_generalized_eigs (FP64)\n")
        f.write(f"# norm2_H {nh:.17e}\n# norm2_S {ns:.17e}\n")
        f.write("# index eigenvalue |u|^2 (u^T S u = 1)\n")
        for i in range(64):
            f.write(f"{i} {w[i]:.17e} {un[i]:.17e}\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
