"""Writes ot_amr_grid.txt: the static 3-level block list of the Orszag-Tang AMR
problem (base 256^2 as 16 x 16 blocks of 16^2 cells).

Blocks are flagged with the oracle's regrid error estimator (paper Sec. 4.5:
filter F = 0.05, bias B = 0.6, eps = 1e-12 for rho and 0.1 for |B|, R = 2,
xi = 0) evaluated on the analytic t = 0 data sampled at each level, with
the threshold TAU below; the flagged leaves are refined and the tree is closed
under 2:1 balance (faces, edges and corners).  Calls only the oracle, the
shared input generator and the test helpers.

    python tests/golden/make_ot_amr_grid.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as orc  # noqa: E402
from paper_1204_5849_amd import workloads as W  # noqa: E402
from tests.helpers import balance  # noqa: E402

TAU = 0.01
LEVELS = 3


def block_errors(w, level_blocks):
    p = orc.params_from_workload(w)
    A = orc.load_workload(w)
    errs = {}
    for b in level_blocks:
        lv = int(w.keys[b, 1])
        t = np.ascontiguousarray(A.state[b])
        e1 = orc.estimate(p, t, (16, 16, 1), 0, 0, eps=1e-12, filt=0.05, bias=0.6, ratio=2.0,
                          xi=0.0, level=lv)
        # the estimator works on conserved data; |B| is taken from B directly
        e2 = orc.estimate(p, t, (16, 16, 1), 1, 0, eps=0.1, filt=0.05, bias=0.6, ratio=2.0,
                          xi=0.0, level=lv)
        errs[b] = max(e1, e2)
    return errs


def build(tau=TAU):
    w = W.orszag_tang(nbase=16)
    keys = w.keys
    for lv in range(1, LEVELS):
        w = W.ot_amr(keys)
        leaves = np.nonzero(W.leaf_mask(keys) & (keys[:, 1] == lv))[0]
        errs = block_errors(w, leaves)
        flag = [b for b in leaves if errs[b] > tau]
        if not flag:
            break
        kids = W.children_of(keys[flag], 2)
        keys = balance(np.concatenate([keys, kids]), 2, w.sims)
    return keys


if __name__ == "__main__":
    keys = build()
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ot_amr_grid.txt")
    with open(out, "w") as f:
        f.write("# Orszag-Tang static AMR block list: sim level ix iy iz (written by make_ot_amr_grid.py)\n")
        for k in keys:
            f.write(" ".join(str(int(v)) for v in k) + "\n")
    print(len(keys), np.bincount(keys[:, 1]), int(W.leaf_mask(keys).sum()))
