"""The library's host tree edit (map_regrid, no GPU needed) against the
oracle's regrid decision, key set for key set, on random 2:1 trees with
random estimates; and its error paths."""
import numpy as np
import pytest

from oracle.regrid import regrid as oracle_regrid
from paper_1204_5849_amd import native as N
from paper_1204_5849_amd import workloads as W
from tests.helpers import random_tree


def _ctx(ndim, sims, keys):
    p = N.make_params(ndim)
    return N.map_init_blocks(p, sims, keys)


@pytest.mark.parametrize("ndim,bc,seed", [(2, "periodic", 1), (2, "outflow", 2), (2, "mixed", 3),
                                          (3, "periodic", 4), (3, "mixed", 5)])
def test_map_regrid_equals_oracle(ndim, bc, seed):
    rng = np.random.default_rng(100 + seed)
    if bc == "mixed":
        bcs = (("periodic", "periodic"), ("outflow", "outflow"), ("periodic", "periodic"))
    else:
        bcs = ((bc, bc),) * 3
    nb = (3, 2, 2) if ndim == 3 else (5, 4, 1)
    sims = [W.SimDesc(nbase=nb, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), bc=bcs),
            W.SimDesc(nbase=(2, 2, 2 if ndim == 3 else 1), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                      bc=((("periodic", "periodic"),) * 3))]
    keys = np.concatenate([random_tree([s], ndim, 3, 0.4, rng) + np.array([i, 0, 0, 0, 0], np.int32)
                           for i, s in enumerate(sims)])
    ctx = _ctx(ndim, sims, keys)
    try:
        _, slot = N.map_query(ctx)
        for trial in range(4):
            err_key = rng.random(len(keys))
            err_slot = np.zeros(len(keys))
            err_slot[slot] = err_key
            tr, tc, ml = (0.85, 0.2, 4) if trial < 3 else (0.5, 0.5, 3)
            got = N.map_regrid(ctx, err_slot, tr, tc, ml)
            want = oracle_regrid([tuple(k) for k in keys], sims, ndim,
                                 {tuple(int(v) for v in k): e for k, e in zip(keys, err_key)},
                                 tr, tc, ml)
            assert [tuple(int(v) for v in k) for k in got] == want
            # the result is a valid tree for the planner (2:1 balanced, complete)
            N.map_destroy(_ctx(ndim, sims, got))
    finally:
        N.map_destroy(ctx)


def test_map_regrid_capacity_and_arguments():
    sims = [W.SimDesc(nbase=(2, 2, 1), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                      bc=((("periodic", "periodic"),) * 3))]
    keys = W.base_keys(0, sims[0].nbase, 2)
    ctx = _ctx(2, sims, keys)
    try:
        L = N.lib()
        import ctypes as C
        err = np.full(len(keys), 5.0)
        rp = N.map_regrid_params(1.0, 0.0, 3)
        n = C.c_int(-1)
        st = L.map_regrid(ctx, err.ctypes.data_as(C.POINTER(C.c_double)), C.byref(rp), None, 0,
                          C.byref(n))
        assert st == N.MAP_ENOMEM and n.value == 4 + 16
        rp.max_level = 0
        assert L.map_regrid(ctx, err.ctypes.data_as(C.POINTER(C.c_double)), C.byref(rp), None, 0,
                            C.byref(n)) == N.MAP_EINVAL
        assert L.map_regrid(ctx, None, C.byref(rp), None, 0, C.byref(n)) == N.MAP_EINVAL
    finally:
        N.map_destroy(ctx)
