"""Writes the stored K-block iterates used by tests/test_gpu_blocks.py at the block size of the
paper's experiments (blocks of 100 points; Section 4).

Every value comes from the FP64 block oracle (``oracle/blocks.py``: exact block projections by NNLS)
on the seeded generator of ``paper_1608_02227_amd/workloads.py``; nothing is taken from the GPU
path.  The oracle needs several minutes (each projection of a 100-point block solves a 9,900-column
NNLS: about 10 s at n = 2 and 90 s at n = 20).  Re-run with ``python tests/golden/make_block_golden.py
[--force]`` (existing files are kept unless forced).
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import blocks as B  # noqa: E402
from paper_1608_02227_amd import workloads as W  # noqa: E402

# Blocks of 100 points: one full block (q = 100, partners past the 64th lane, several 16-row
# tiles of the Schur complement) and a ragged one; n = 2 and the paper's n = 20
CASES = [
    # N, n, p, gamma, seed, noise, iterations stored
    (150, 2, 100, 0.05, 7, 0.1, [1, 2, 3, 5]),
    (120, 20, 100, 0.05, 8, 0.1, [1, 2, 3]),
]


def write(N, n, p, g, seed, noise, ks):
    out = os.path.join(HERE, f"blocks_N{N}_n{n}_p{p}_seed{seed}.npz")
    if os.path.exists(out) and "--force" not in sys.argv:
        print("kept", out)
        return
    x, ybar = W.sq_norm(N, n, noise, seed)
    L = B.lipschitz_inter(x, g, p)[0]
    its = []
    B.papg_blocks(x, ybar, g, p, 0.0, L=L, max_iters=max(ks), check_every=10 ** 6, iterates=its)
    th = {k: t for k, t in its if k in ks}
    meta = {"N": N, "n": n, "p": p, "gamma": g, "seed": seed, "noise": noise, "L": L, "ks": ks,
            "generator": "workloads.sq_norm", "oracle": "oracle.blocks.papg_blocks (constant step 1/L)"}
    np.savez_compressed(out, meta=json.dumps(meta), **{f"theta_{k}": th[k] for k in ks})
    print("wrote", out)


def main():
    for case in CASES:
        write(*case)


if __name__ == "__main__":
    main()
