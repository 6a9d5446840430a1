"""Host-side tests of libmap.so (no GPU): exported symbols, block-tree
validation errors, Morton slot order, the neighbour tables against a
brute-force geometric search and the cycle's fill selection against the
cells the prolongation reads."""
import os
import re

import numpy as np
import pytest

from paper_1204_5849_amd import native as N
from paper_1204_5849_amd import workloads as W
from tests.helpers import random_tree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(N.LIB_PATH):
        from paper_1204_5849_amd import build
        build.build()
    return N.lib()


def test_every_declared_symbol_is_exported(L):
    hdr = open(os.path.join(ROOT, "include", "map.h")).read()
    names = set(re.findall(r"^\s*(?:map_status|const char\s*\*|void)\s*(map_\w+)\s*\(", hdr, re.M))
    assert {"map_init_blocks", "map_step", "map_fill_ghosts", "map_cfl_dt", "map_restrict",
            "map_prolong", "map_last_error", "map_destroy"} <= names
    for n in names:
        assert hasattr(L, n), n
    assert names == set(N.EXPORTS)


def _status(params, sims, keys):
    ctx = N.C.c_void_p()
    st = N.lib().map_init_blocks(N.C.byref(ctx), N.C.byref(params), len(sims), N.make_sims(sims),
                                 len(keys), N.make_keys(keys))
    if st == N.MAP_OK:
        N.map_destroy(ctx)
    return st


def _sims2d(nb=(2, 2, 1), bc="periodic"):
    return [W.SimDesc(lo=(0, 0, 0), hi=(1, 1, 1), nbase=nb, bc=((bc, bc),) * 3)]


def test_every_export_has_declared_argument_types():
    """Without declared argument types ctypes passes Python ints as 32-bit C
    ints, which would truncate device and stream pointers."""
    L = N.lib()
    for name in N.EXPORTS:
        assert getattr(L, name).argtypes is not None, name


def test_tree_errors():
    p = N.make_params(2)
    sims = _sims2d()
    base = W.base_keys(0, (2, 2, 1), 2)
    assert _status(p, sims, base) == N.MAP_OK
    assert _status(p, sims, np.concatenate([base, base[:1]])) == N.MAP_ETREE      # duplicate
    assert _status(p, sims, base[1:]) == N.MAP_ETREE                              # base incomplete
    kids = W.children_of(base[:1], 2)
    assert _status(p, sims, np.concatenate([base, kids])) == N.MAP_OK
    assert _status(p, sims, np.concatenate([base, kids[:3]])) == N.MAP_ETREE      # siblings
    orphan = np.array([[0, 3, 0, 0, 0]], dtype=np.int32)
    assert _status(p, sims, np.concatenate([base, orphan])) == N.MAP_ETREE        # no parent
    bad = np.array([[0, 1, 5, 0, 0]], dtype=np.int32)
    assert _status(p, sims, np.concatenate([base, bad])) == N.MAP_ETREE           # out of range
    # 2:1 violation: level 3 next to a level-1 leaf
    sims4 = _sims2d((4, 4, 1))
    b4 = W.base_keys(0, (4, 4, 1), 2)
    l2 = W.children_of(b4[:1], 2)
    l3 = W.children_of(l2[3:4], 2)  # refine the child touching (1,1) corner
    assert _status(p, sims4, np.concatenate([b4, l2, l3])) == N.MAP_ETREE
    l2b = W.children_of(b4[[0, 1, 4, 5]], 2)
    assert _status(p, sims4, np.concatenate([b4, l2b, l3])) == N.MAP_OK


def test_param_errors():
    sims = _sims2d()
    base = W.base_keys(0, (2, 2, 1), 2)
    assert _status(N.make_params(4), sims, base) == N.MAP_EINVAL
    assert _status(N.make_params(2, limiter=7), sims, base) == N.MAP_EINVAL
    assert _status(N.make_params(2, gamma=1.0), sims, base) == N.MAP_EINVAL
    assert _status(N.make_params(2, riemann=5), sims, base) == N.MAP_EINVAL
    # MMC splits fluxes (Sec. 3.1); it has no Riemann solver to replace
    assert _status(N.make_params(2, scheme="mmc", riemann="hllc"), sims, base) == N.MAP_EINVAL
    assert _status(N.make_params(2, scheme="weno", riemann="hllc"), sims, base) == N.MAP_OK
    sims3 = [W.SimDesc(lo=(0, 0, 0), hi=(1, 1, 1), nbase=(2, 2, 2), bc=(("periodic",) * 2,) * 3)]
    assert _status(N.make_params(3, scheme="mmc"), sims3, W.base_keys(0, (2, 2, 2), 3)) == N.MAP_OK
    assert _status(N.make_params(3, scheme="mmc", riemann="hllc"), sims3,
                   W.base_keys(0, (2, 2, 2), 3)) == N.MAP_EINVAL
    mixed = [W.SimDesc(lo=(0, 0, 0), hi=(1, 1, 1), nbase=(2, 2, 1),
                       bc=(("periodic", "outflow"),) * 3)]
    assert _status(N.make_params(2), mixed, base) == N.MAP_EINVAL


def test_call_order_and_workspace_errors():
    w = W.orszag_tang(2)
    ctx = N.map_init_blocks(N.make_params(2), w.sims, w.keys)
    sz, _ = N.map_query(ctx)
    L = N.lib()
    assert L.map_step(ctx, 256, 256, 256, None) == N.MAP_ESTATE
    assert L.map_fill_ghosts(ctx, 256, None) == N.MAP_ESTATE
    assert L.map_bind_workspace(ctx, None, 10 ** 9, None) == N.MAP_EINVAL
    assert L.map_bind_workspace(ctx, 256, sz.workspace_bytes - 1, None) == N.MAP_ENOMEM
    assert b"need" in L.map_last_error()
    N.map_destroy(ctx)


def _morton(x, y, z):
    out = 0
    for b in range(21):
        out |= ((x >> b) & 1) << (3 * b) | ((y >> b) & 1) << (3 * b + 1) | ((z >> b) & 1) << (3 * b + 2)
    return out


@pytest.mark.parametrize("ndim", [2, 3])
def test_morton_slot_order(ndim):
    rng = np.random.default_rng(ndim)
    nb = (3, 2, 1) if ndim == 2 else (2, 2, 2)
    sims = [W.SimDesc(lo=(0, 0, 0), hi=(1, 1, 1), nbase=nb, bc=(("periodic",) * 2,) * 3)] * 2
    keys = random_tree(sims, ndim, 3, 0.3, rng)
    p = N.make_params(ndim)
    ctx = N.map_init_blocks(p, sims, keys)
    sz, slot = N.map_query(ctx)
    lmax = int(keys[:, 1].max())
    order = sorted(range(len(keys)), key=lambda i: (keys[i, 0], _morton(
        int(keys[i, 2]) << (lmax - keys[i, 1]), int(keys[i, 3]) << (lmax - keys[i, 1]),
        int(keys[i, 4]) << (lmax - keys[i, 1])), keys[i, 1]))
    assert [int(slot[i]) for i in order] == list(range(len(keys)))
    index = {tuple(k): i for i, k in enumerate(keys.tolist())}
    for i, (s, lv, x, y, z) in enumerate(keys.tolist()):
        if lv > 1:
            assert slot[index[(s, lv - 1, x >> 1, y >> 1, z >> 1)]] < slot[i]
    assert sz.nleaves == int(W.leaf_mask(keys).sum())
    N.map_destroy(ctx)


@pytest.mark.parametrize("ndim,bc", [(2, "periodic"), (2, "outflow"), (3, "periodic"), (3, "mixed")])
def test_neighbours_match_brute_force(ndim, bc):
    rng = np.random.default_rng(11 + ndim)
    nb = (3, 4, 1) if ndim == 2 else (2, 3, 2)
    if bc == "mixed":
        bcs = (("periodic", "periodic"), ("outflow", "outflow"), ("periodic", "periodic"))
    else:
        bcs = ((bc, bc),) * 3
    sims = [W.SimDesc(lo=(0, 0, 0), hi=(1, 1, 1), nbase=nb, bc=bcs)]
    keys = random_tree(sims, ndim, 3, 0.35, rng)
    ctx = N.map_init_blocks(N.make_params(ndim), sims, keys)
    got = N.map_neighbors(ctx, len(keys))
    N.map_destroy(ctx)
    n = 16
    index = {tuple(k): i for i, k in enumerate(keys.tolist())}
    for i, (s, lv, kx, ky, kz) in enumerate(keys.tolist()):
        kc = (kx, ky, kz)
        for dz in ((-1, 0, 1) if ndim == 3 else (0,)):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    di = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
                    if (dx, dy, dz) == (0, 0, 0):
                        assert got[i, di] == -2
                        continue
                    # one ghost cell of that direction, mapped through the boundary
                    src = []
                    for d, dd in enumerate((dx, dy, dz)):
                        if d >= ndim:
                            src.append(0)
                            continue
                        loc = -1 if dd < 0 else (n if dd > 0 else 0)
                        G = kc[d] * n + loc
                        Nl = nb[d] * n << (lv - 1)
                        if G < 0 or G >= Nl:
                            G = G % Nl if bcs[d][0] == "periodic" else min(max(G, 0), Nl - 1)
                        src.append(G // n)
                    want = index.get((s, lv, *src), -1)
                    assert got[i, di] == want, (i, (dx, dy, dz))


@pytest.mark.parametrize("ndim,bc,seed", [(2, "periodic", 3), (2, "outflow", 4), (3, "periodic", 5),
                                          (3, "mixed", 6)])
def test_fill_selection_is_what_the_prolongation_reads(ndim, bc, seed):
    """The parent ghost cells a cycle's fill refreshes: every parent cell that
    the limited-linear prolongation (Sec. 4.3 step 6) reads for the ghost
    regions without a same-level source, found by enumerating those fine
    ghost cells, is inside the selection, whose directions and box are
    exactly those of the cells read."""
    rng = np.random.default_rng(seed)
    nb = (3, 2, 1) if ndim == 2 else (2, 2, 2)
    if bc == "mixed":
        bcs = (("periodic", "periodic"), ("outflow", "outflow"), ("periodic", "periodic"))
    else:
        bcs = ((bc, bc),) * 3
    sims = [W.SimDesc(lo=(0, 0, 0), hi=(1, 1, 1), nbase=nb, bc=bcs)]
    keys = random_tree(sims, ndim, 3, 0.4, rng)
    ctx = N.map_init_blocks(N.make_params(ndim), sims, keys)
    neigh = N.map_neighbors(ctx, len(keys))
    par, dirs, box = N.map_fill_selection(ctx)
    N.map_destroy(ctx)
    n, ng = 16, 2
    index = {tuple(k): i for i, k in enumerate(keys.tolist())}
    want = {}  # parent -> list of arrays of read parent cells [m, 3]
    for i, (s, lv, kx, ky, kz) in enumerate(keys.tolist()):
        pro = [d for d in range(27) if d != 13 and neigh[i, d] == -1]
        if not pro:
            continue
        p = index[(s, lv - 1, kx >> 1, ky >> 1, kz >> 1)]
        cpos = (kx & 1, ky & 1, kz & 1)
        for d in pro:
            dd = (d % 3 - 1, (d // 3) % 3 - 1, d // 9 - 1)
            axes = []
            for a in range(3):
                if a >= ndim:
                    axes.append(np.array([0]))
                else:
                    axes.append({-1: np.arange(-ng, 0), 0: np.arange(0, n), 1: np.arange(n, n + ng)}[dd[a]])
            f = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, 3)
            c = f.copy()
            for a in range(ndim):
                c[:, a] = np.floor_divide(cpos[a] * n + f[:, a], 2)
            reads = [c]
            for a in range(ndim):
                for sgn in (-1, 1):
                    e = c.copy()
                    e[:, a] += sgn
                    reads.append(e)
            want.setdefault(p, []).extend(reads)
    assert sorted(par.tolist()) == sorted(want)
    assert len(set(par.tolist())) == len(par)
    for p, m, b in zip(par.tolist(), dirs.tolist(), box.tolist()):
        cells = np.unique(np.concatenate(want[p]), axis=0)
        assert cells.min() >= -ng and cells.max() <= n + ng - 1
        side = np.where(cells < 0, 0, np.where(cells >= n, 2, 1))
        side[:, ndim:] = 1
        di = side[:, 2] * 9 + side[:, 1] * 3 + side[:, 0]
        got_dirs = {k for k in range(27) if (m >> k) & 1}
        assert got_dirs == set(di[di != 13].tolist()), p
        lo, hi = cells.min(axis=0), cells.max(axis=0)
        assert b[:ndim] == lo[:ndim].tolist() and b[3:3 + ndim] == hi[:ndim].tolist(), p


def test_each_step_instance_is_compiled_once():
    """The 3-D step kernel template is instantiated from two translation units
    compiled with different instruction schedulers; an instance defined in
    both would leave the linker to pick one of the two copies, so the sets of
    instances must be disjoint (and together hold all 60)."""
    import shutil
    import subprocess
    from paper_1204_5849_amd import build as B
    objs = [os.path.join(B.PKG, "_build", f) for f in ("k_step3_hip.o", "k_step3_ilp_hip.o")]
    if not all(os.path.exists(o) for o in objs) or not shutil.which("nm"):
        pytest.skip("step objects not built here")
    sets = []
    for o in objs:
        out = subprocess.run(["nm", "-C", o], capture_output=True, text=True, check=True).stdout
        sets.append(set(re.findall(r"k_step3<([^>]*)>", out)))
    assert not (sets[0] & sets[1]), sorted(sets[0] & sets[1])
    # 2 precisions x 2 (resistivity) x (3 LF limiters + 2 WENO stages) x 2 fluxes,
    # the FP32 ones for two workgroups per CU and for one
    assert len(sets[0] | sets[1]) == 60


def test_totals_static_rejects_too_many_leaves():
    """map_totals_static checks, before touching the device, that the leaves'
    partial sums fit its fixed scratch (MAP_STATIC_SCRATCH_DOUBLES / 9 =
    58254 leaves)."""
    from paper_1204_5849_amd import native as N
    from paper_1204_5849_amd import workloads as W
    w = W.orszag_tang(256)  # 65536 leaves
    ctx = N.map_init_blocks(N.make_params(2), w.sims, w.keys)
    try:
        st = N.lib().map_totals_static(ctx, None, None, None)
        assert st == N.MAP_EINVAL
        msg = N.lib().map_last_error().decode()
        assert "static scratch" in msg and "58254" in msg, msg
    finally:
        N.map_destroy(ctx)


def test_launch_config_checks():
    """map_get_launch / map_set_launch_config on the host: defaults, and the
    workgroup shapes a scheme and precision do not have are rejected."""
    from paper_1204_5849_amd import native as N
    from paper_1204_5849_amd import workloads as W
    w2 = W.orszag_tang(2)
    w3 = W.harris3d(nbase=2, levels=1)
    cases = [(N.make_params(2), w2, True), (N.make_params(2, scheme="mmc"), w2, False),
             (N.make_params(3, precision="fp32"), w3, True), (N.make_params(3), w3, False),
             (N.make_params(3, precision="fp32", scheme="mmc"), w3, False)]
    for p, w, shape1 in cases:
        ctx = N.map_init_blocks(p, w.sims, w.keys)
        try:
            cfg = N.map_get_launch(ctx)
            assert cfg["mode"] == N.MAP_LAUNCH_BATCHED and cfg["grid_step"] == 0
            assert cfg["step_shape"] == 0
            if shape1:
                N.map_set_launch_config(ctx, {"step_shape": 1})
                assert N.map_get_launch(ctx)["step_shape"] == 1
            else:
                with pytest.raises(N.MapError):
                    N.map_set_launch_config(ctx, {"step_shape": 1})
            with pytest.raises(N.MapError):
                N.map_set_launch_config(ctx, {"restrict_split": -2})
            with pytest.raises(N.MapError):
                N.map_set_launch_config(ctx, {"cfl_in_update": 2})
            # the update forms CFL maxima only in 2-D LF, and by default only
            # on trees of at least 4 leaves per CU
            assert cfg["cfl_in_update"] == -1 and cfg["cfl_in_update_on"] == 0
            N.map_set_launch_config(ctx, {"cfl_in_update": 1, "cfl_in_update_on": 0})
            got = N.map_get_launch(ctx)
            assert got["cfl_in_update"] == 1
            assert got["cfl_in_update_on"] == int(p.ndim == 2 and p.scheme == N.MAP_LF)
        finally:
            N.map_destroy(ctx)
    ctx = N.map_init_blocks(N.make_params(2), w2.sims, w2.keys)
    try:
        N.map_set_launch_config(ctx, {"step_shape": 1})
        assert N.map_get_launch(ctx)["step_blocks_per_group"] == 7
    finally:
        N.map_destroy(ctx)
    # batched 2-D LF launches over at least 4 leaves per CU take the CFL maxima in the
    # update by default; 0 turns it off, and -1 restores the rule
    wk = W.kh_ensemble(nsims=64)
    ctx = N.map_init_blocks(N.make_params(2), wk.sims, wk.keys)
    try:
        assert N.map_get_launch(ctx)["cfl_in_update_on"] == 1
        N.map_set_launch_config(ctx, {"cfl_in_update": 0})
        assert N.map_get_launch(ctx)["cfl_in_update_on"] == 0
        N.map_set_launch_config(ctx, {"cfl_in_update": -1})
        assert N.map_get_launch(ctx)["cfl_in_update_on"] == 1
        # a launch per block leaves it to the CFL pass unless forced
        N.map_set_launch_config(ctx, {"mode": N.MAP_LAUNCH_PER_BLOCK})
        assert N.map_get_launch(ctx)["cfl_in_update_on"] == 0
        N.map_set_launch_config(ctx, {"cfl_in_update": 1})
        assert N.map_get_launch(ctx)["cfl_in_update_on"] == 1
    finally:
        N.map_destroy(ctx)


def test_regrid_interval_formula():
    """map_regrid_interval (Sec. 4.5): dtr = c_r 2 n_g dx_min / alpha_g per
    simulation and the whole steps of dt in it; with the CFL dt this is
    c_r 2 n_g n_dim dt / c_cfl."""
    from paper_1204_5849_amd import native as N
    from paper_1204_5849_amd import workloads as W
    w = W.orszag_tang(2)  # 32 x 32 cells on the unit square: dx_min = 1/32
    ctx = N.map_init_blocks(N.make_params(2), w.sims, w.keys)
    try:
        rec = np.zeros((1, N.DT_WORDS))
        rec[0, 0], rec[0, 3] = 1e-3, 2.0
        dtr, steps = N.map_regrid_interval(ctx, rec, 1.0)
        assert dtr[0] == pytest.approx(2 * 2 * (1 / 32) / 2.0, rel=1e-15)
        assert steps[0] == 62
        cfl, alpha, dx = 0.4, 1.7, 1 / 32
        rec[0, 0], rec[0, 3] = cfl * dx / (2 * alpha), alpha
        dtr, steps = N.map_regrid_interval(ctx, rec, 0.5)
        assert dtr[0] == pytest.approx(0.5 * 2 * 2 * 2 * rec[0, 0] / cfl, rel=1e-14)
        assert steps[0] in (9, 10)  # 0.5 * 2 n_g n_dim / c_cfl = 10, up to rounding
        for bad_cr, bad_dt in ((0.0, 1e-3), (1.0, 0.0)):
            rec[0, 0] = bad_dt
            with pytest.raises(N.MapError):
                N.map_regrid_interval(ctx, rec, bad_cr)
    finally:
        N.map_destroy(ctx)
