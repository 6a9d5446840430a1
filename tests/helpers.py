"""Test-side helpers: tree construction with 2:1 closure, random states,
error norms.  Nothing here is shared with the HIP library."""
from __future__ import annotations

import numpy as np

from paper_1204_5849_amd import workloads as W


def neighbours_exist_coarse(keyset, key, ndim, sims):
    """2:1 check for one block: every neighbour region of its parent exists at the
    parent's level (faces, edges and corners), with periodic wrap."""
    s, lv, ix, iy, iz = key
    if lv <= 1:
        return True
    pc = [ix >> 1, iy >> 1, iz >> 1]
    sim = sims[s]
    nb = [sim.nbase[d] << (lv - 2) for d in range(3)]
    rng = [(-1, 0, 1) if d < ndim else (0,) for d in range(3)]
    for dz in rng[2]:
        for dy in rng[1]:
            for dx in rng[0]:
                c = [pc[0] + dx, pc[1] + dy, pc[2] + dz]
                skip = False
                for d in range(ndim):
                    if c[d] < 0 or c[d] >= nb[d]:
                        side = 0 if c[d] < 0 else 1
                        if sim.bc[d][side] == "periodic":
                            c[d] %= nb[d]
                        else:
                            skip = True
                if skip:
                    continue
                if (s, lv - 1, c[0], c[1], c[2]) not in keyset:
                    return False
    return True


def balance(keys, ndim, sims):
    """Refine leaves until every block satisfies 2:1 (with diagonals): the
    neighbour regions of every block's parent exist at the parent's level."""
    keyset = set(tuple(int(v) for v in k) for k in keys)

    def ensure(key):
        if key in keyset:
            return
        s, lv, ix, iy, iz = key
        par = (s, lv - 1, ix >> 1, iy >> 1, iz >> 1)
        ensure(par)
        for kid in W.children_of(np.array([par]), ndim):
            keyset.add(tuple(int(v) for v in kid))

    changed = True
    while changed:
        changed = False
        for key in sorted(keyset, key=lambda k: -k[1]):
            s, lv, ix, iy, iz = key
            if lv <= 2:
                continue
            pc = [ix >> 1, iy >> 1, iz >> 1]
            sim = sims[s]
            nb = [sim.nbase[d] << (lv - 2) for d in range(3)]
            rng = [(-1, 0, 1) if d < ndim else (0,) for d in range(3)]
            for dz in rng[2]:
                for dy in rng[1]:
                    for dx in rng[0]:
                        c = [pc[0] + dx, pc[1] + dy, pc[2] + dz]
                        skip = False
                        for d in range(ndim):
                            if c[d] < 0 or c[d] >= nb[d]:
                                side = 0 if c[d] < 0 else 1
                                if sim.bc[d][side] == "periodic":
                                    c[d] %= nb[d]
                                else:
                                    skip = True
                        if skip:
                            continue
                        want = (s, lv - 1, c[0], c[1], c[2])
                        if want not in keyset:
                            ensure(want)
                            changed = True
    return np.array(sorted(keyset), dtype=np.int32)


def refine(keys, which, ndim):
    """Add the children of the selected leaves."""
    keys = np.asarray(keys, dtype=np.int32)
    kids = W.children_of(keys[which], ndim)
    return np.concatenate([keys, kids])


def random_tree(sims, ndim, levels, frac, rng):
    keys = np.concatenate([W.base_keys(i, s.nbase, ndim) for i, s in enumerate(sims)])
    for lv in range(1, levels):
        leaves = W.leaf_mask(keys)
        cand = np.nonzero(leaves & (keys[:, 1] == lv))[0]
        if len(cand) == 0:
            break
        pick = rng.random(len(cand)) < frac
        if not pick.any():
            pick[rng.integers(len(cand))] = True
        keys = refine(keys, cand[pick], ndim)
        keys = balance(keys, ndim, sims)
    return keys


def rel_linf(a, b, axis_var=1):
    """Per-variable relative L-infinity: max|a-b| / max|b| over all but the variable axis."""
    a = np.moveaxis(np.asarray(a, dtype=np.float64), axis_var, 0).reshape(a.shape[axis_var], -1)
    b = np.moveaxis(np.asarray(b, dtype=np.float64), axis_var, 0).reshape(b.shape[axis_var], -1)
    num = np.abs(a - b).max(axis=1)
    den = np.abs(b).max(axis=1)
    den = np.where(den == 0, 1.0, den)
    return num / den


def l1(a, b):
    return float(np.mean(np.abs(np.asarray(a) - np.asarray(b))))


def order(e_coarse, e_fine, ratio=2.0):
    return float(np.log(e_coarse / e_fine) / np.log(ratio))
