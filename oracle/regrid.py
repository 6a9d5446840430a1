"""Regrid decision of the MAP paper, Sec. 4.5 -- TEST INFRASTRUCTURE ONLY.

Plain Python over sets of block keys (sim, level, ix, iy, iz); the reference
the library's host tree edit is checked against.  Nothing here is used by the
product path.

Rules (the paper's wording, with the reading noted):
  * a leaf whose error estimate exceeds the refinement threshold is refined
    (its 2^d children are created), unless it is already at the finest
    allowed level;
  * the children of a block are destroyed when the estimate on the block
    itself (which holds the restriction of its children) is below the
    coarsening threshold; the printed text says "larger", which would
    destroy exactly the blocks that need resolution, so it is read as
    "smaller".  Only blocks whose children are all leaves, none of them
    being refined, are candidates;
  * the new tree must stay 2:1 balanced across faces, edges and corners
    (with periodic wrap): where a new leaf would touch a leaf two or more
    levels coarser, the coarser leaf is refined, or, if it exists only
    because its children were destroyed, the destruction is cancelled;
    repeated until nothing changes (refinements only grow, destructions
    only shrink, so the result does not depend on the order of the checks).
"""
from __future__ import annotations


def _children(key, ndim):
    s, l, x, y, z = key
    out = []
    for c in range(1 << ndim):
        cz = (c >> 2) & 1 if ndim == 3 else 0
        out.append((s, l + 1, 2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + cz))
    return out


def _parent(key):
    s, l, x, y, z = key
    return (s, l - 1, x >> 1, y >> 1, z >> 1)


def regrid(keys, sims, ndim, err, tau_refine, tau_coarsen, max_level):
    """New block list after one regrid.

    keys: iterable of (sim, level, ix, iy, iz), leaves and parents.
    sims: per simulation, an object with .nbase (3 ints, base blocks per
          dimension) and .bc (3 pairs of 'periodic' / 'outflow').
    err:  dict key -> largest estimate over the block's cells, for every leaf
          and every block whose children are all leaves.
    Returns the sorted list of keys of the new tree."""
    keys = {tuple(int(v) for v in k) for k in keys}
    parents = {_parent(k) for k in keys if k[1] > 1}
    leaves = keys - parents

    refine = {k for k in leaves if err[k] > tau_refine and k[1] < max_level}
    coarsen = set()
    for p in parents:
        kids = _children(p, ndim)
        if all(c in leaves and c not in refine for c in kids) and err[p] < tau_coarsen:
            coarsen.add(p)

    def new_leaves():
        out = set(leaves)
        for p in coarsen:
            out -= set(_children(p, ndim))
            out.add(p)
        for k in refine:
            out.discard(k)
            out |= set(_children(k, ndim))
        return out

    def neighbours(key):
        s, l, x, y, z = key
        sim = sims[s]
        c = (x, y, z)
        rng = [(-1, 0, 1)] * ndim + [(0,)] * (3 - ndim)
        for dz in rng[2]:
            for dy in rng[1]:
                for dx in rng[0]:
                    if dx == dy == dz == 0:
                        continue
                    n = []
                    ok = True
                    for d, dd in enumerate((dx, dy, dz)):
                        if d >= ndim:
                            n.append(0)
                            continue
                        nb = sim.nbase[d] << (l - 1)
                        v = c[d] + dd
                        if v < 0 or v >= nb:
                            if sim.bc[d][0 if v < 0 else 1] != "periodic":
                                ok = False
                                break
                            v %= nb
                        n.append(v)
                    if ok:
                        yield (s, l, n[0], n[1], n[2])

    while True:
        nl = new_leaves()
        changed = False
        for a in sorted(nl):
            for nb in neighbours(a):
                # the new leaf covering the neighbour region, if it is coarser
                s, l, x, y, z = nb
                for b_l in range(l - 1, 0, -1):
                    sh = l - b_l
                    b = (s, b_l, x >> sh, y >> sh, z >> sh)
                    if b in nl:
                        if b_l <= a[1] - 2:
                            if b in coarsen:
                                coarsen.discard(b)
                            else:
                                refine.add(b)
                                if b[1] > 1 and _parent(b) in coarsen:
                                    coarsen.discard(_parent(b))
                            changed = True
                        break
        if not changed:
            break

    nl = new_leaves()
    out = set(nl)
    for k in nl:
        while k[1] > 1:
            k = _parent(k)
            out.add(k)
    return sorted(out)
