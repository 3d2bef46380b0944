"""Writes the stored K-block iterates used by tests/test_gpu_blocks.py at the block size of the
paper's experiments (blocks of 100 points; Section 4).

Every value comes from the FP64 block oracle (``oracle/blocks.py``: exact block projections by NNLS)
on the seeded generator of ``paper_1608_02227_amd/workloads.py``; nothing is taken from the GPU
path.  The oracle needs about a minute (each projection of a 100-point block solves a 9,900-column
NNLS).  Re-run with ``python tests/golden/make_block_golden.py``.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import blocks as B  # noqa: E402
from paper_1608_02227_amd import workloads as W  # noqa: E402

# N = 150 with blocks of 100: one full block (q = 100, partners past the 64th lane, several
# 16-row tiles of the Schur complement) and a ragged block of 50
N, n, p, g, seed, noise = 150, 2, 100, 0.05, 7, 0.1
KS = [1, 2, 3, 5]


def main():
    x, ybar = W.sq_norm(N, n, noise, seed)
    L = B.lipschitz_inter(x, g, p)[0]
    its = []
    B.papg_blocks(x, ybar, g, p, 0.0, L=L, max_iters=max(KS), check_every=10 ** 6, iterates=its)
    th = {k: t for k, t in its if k in KS}
    meta = {"N": N, "n": n, "p": p, "gamma": g, "seed": seed, "noise": noise, "L": L, "ks": KS,
            "generator": "workloads.sq_norm", "oracle": "oracle.blocks.papg_blocks (constant step 1/L)"}
    out = os.path.join(HERE, f"blocks_N{N}_n{n}_p{p}_seed{seed}.npz")
    np.savez_compressed(out, meta=json.dumps(meta), **{f"theta_{k}": th[k] for k in KS})
    print("wrote", out)


if __name__ == "__main__":
    main()
