"""Pins of the oracle's regrid decision (paper Sec. 4.5): hand-checked small
cases, 2:1 balance of the result by brute force, order independence."""
import itertools

import numpy as np
import pytest

from oracle.regrid import regrid
from paper_1204_5849_amd import workloads as W
from tests.helpers import random_tree


def _sims(nbase, bc):
    return [W.SimDesc(nbase=nbase, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), bc=bc)]


def _leaves(keys):
    ks = {tuple(k) for k in keys}
    par = {(s, l - 1, x >> 1, y >> 1, z >> 1) for (s, l, x, y, z) in ks if l > 1}
    return ks - par


def _touch(a, b, sim, ndim):
    """Blocks a and b (any levels) share a face, edge or corner (periodic wrap)."""
    lf = max(a[1], b[1])
    lo, hi = [], []
    for k in (a, b):
        sh = lf - k[1]
        c = (k[2], k[3], k[4])
        lo.append([c[d] << sh for d in range(3)])
        hi.append([(c[d] + 1) << sh for d in range(3)])
    for d in range(ndim):
        n = sim.nbase[d] << (lf - 1)
        ok = False
        for off in ((0,) if sim.bc[d][0] != "periodic" else (0, n, -n)):
            if lo[0][d] <= hi[1][d] + off and lo[1][d] + off <= hi[0][d]:
                ok = True
        if not ok:
            return False
    return True


def _balanced(keys, sims, ndim):
    lv = sorted(_leaves(keys))
    for a, b in itertools.combinations(lv, 2):
        if a[0] == b[0] and abs(a[1] - b[1]) > 1 and _touch(a, b, sims[a[0]], ndim):
            return False
    return True


def _err(keys, value):
    return {tuple(int(v) for v in k): value for k in keys}


def test_nothing_flagged_keeps_tree():
    sims = _sims((4, 4, 1), (("periodic",) * 2,) * 3)
    keys = W.base_keys(0, sims[0].nbase, 2)
    out = regrid(keys, sims, 2, _err(keys, 0.5), 1.0, 0.0, 4)
    assert out == sorted(tuple(int(v) for v in k) for k in keys)


def test_single_flag_refines_one_block():
    sims = _sims((4, 4, 1), (("periodic",) * 2,) * 3)
    keys = W.base_keys(0, sims[0].nbase, 2)
    err = _err(keys, 0.0)
    err[(0, 1, 1, 2, 0)] = 5.0
    out = set(regrid(keys, sims, 2, err, 1.0, -1.0, 4))
    want = {tuple(int(v) for v in k) for k in keys} | {(0, 2, 2 + i, 4 + j, 0) for i in (0, 1) for j in (0, 1)}
    assert out == want


def test_closure_refines_coarser_neighbours_including_corners():
    """Refining a level-2 leaf at the corner of its parent forces the three
    level-1 leaves touching that corner (face, face, diagonal) to refine."""
    sims = _sims((4, 4, 1), (("outflow",) * 2,) * 3)
    base = W.base_keys(0, sims[0].nbase, 2)
    keys = np.concatenate([base, W.children_of(base[[5]], 2)])  # block (1,1) refined
    keys_t = [tuple(int(v) for v in k) for k in keys]
    err = _err(keys, 0.0)
    err[(0, 2, 2, 2, 0)] = 5.0   # lower-left child of (1,1)
    out = set(regrid(keys, sims, 2, err, 1.0, -1.0, 4))
    kids = {(0, 3, 4 + i, 4 + j, 0) for i in (0, 1) for j in (0, 1)}
    forced = set()
    for (x, y) in ((0, 1), (1, 0), (0, 0)):
        forced |= {(0, 2, 2 * x + i, 2 * y + j, 0) for i in (0, 1) for j in (0, 1)}
    assert out == set(keys_t) | kids | forced
    assert _balanced(out, sims, 2)


def test_coarsening_and_its_cancellation():
    sims = _sims((4, 4, 1), (("periodic",) * 2,) * 3)
    base = W.base_keys(0, sims[0].nbase, 2)
    keys = np.concatenate([base, W.children_of(base[[5, 6]], 2)])  # (1,1) and (2,1) refined
    err = _err(keys, 0.5)
    # (1,1) is smooth: its children are destroyed
    err[(0, 1, 1, 1, 0)] = 0.01
    out = set(regrid(keys, sims, 2, err, 1.0, 0.1, 4))
    assert not any(k[1] == 2 and (k[2] >> 1, k[3] >> 1) == (1, 1) for k in out)
    assert any(k[1] == 2 and (k[2] >> 1, k[3] >> 1) == (2, 1) for k in out)
    # a flagged level-2 leaf of (2,1) next to (1,1) refines to level 3, which
    # would touch the coarsened (1,1): the destruction is cancelled
    err[(0, 2, 4, 2, 0)] = 5.0
    out = set(regrid(keys, sims, 2, err, 1.0, 0.1, 4))
    assert (0, 2, 2, 2, 0) in out and (0, 3, 8, 4, 0) in out
    assert _balanced(out, sims, 2)


def test_max_level_is_respected():
    sims = _sims((2, 2, 1), (("periodic",) * 2,) * 3)
    keys = W.base_keys(0, sims[0].nbase, 2)
    out = regrid(keys, sims, 2, _err(keys, 9.0), 1.0, -1.0, 1)
    assert out == sorted(tuple(int(v) for v in k) for k in keys)


@pytest.mark.parametrize("ndim,bc", [(2, "periodic"), (2, "outflow"), (3, "periodic"), (3, "mixed")])
def test_random_trees_balanced_and_order_independent(ndim, bc):
    rng = np.random.default_rng(11 + ndim)
    if bc == "mixed":
        bcs = (("periodic", "periodic"), ("outflow", "outflow"), ("periodic", "periodic"))
    else:
        bcs = ((bc, bc),) * 3
    nb = (3, 2, 2) if ndim == 3 else (4, 3, 1)
    sims = _sims(nb, bcs)
    keys = random_tree(sims, ndim, 3, 0.35, rng)
    ks = [tuple(int(v) for v in k) for k in keys]
    err = {k: float(rng.random()) for k in ks}
    out = regrid(ks, sims, ndim, err, 0.8, 0.15, 4)
    assert _balanced(out, sims, ndim)
    # every flagged leaf below the finest level is refined
    lv = _leaves(ks)
    outset = set(out)
    for k in lv:
        if err[k] > 0.8 and k[1] < 4:
            assert (0, k[1] + 1, 2 * k[2], 2 * k[3], 2 * k[4] if ndim == 3 else 0) in outset
    # the parent of every new block exists
    for k in out:
        if k[1] > 1:
            assert (k[0], k[1] - 1, k[2] >> 1, k[3] >> 1, k[4] >> 1) in outset
    rev = list(reversed(ks))
    assert regrid(rev, sims, ndim, err, 0.8, 0.15, 4) == out
