"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bar (FP64): relative L-infinity per variable, max|gpu - oracle| / max|oracle|,
<= 1e-11 after N steps; stages whose arithmetic is a copy or a fixed-order
average (ghost fill, prolongation, restriction, the initial conversion) must
match bit for bit.  psi is held to that bar against its natural scale
c_h max|B| (the GLM pair psi +- c_h B_n travels together; in divergence-free
problems psi itself is a cancellation residue many orders below that scale),
and to 1e-8 against its own max|psi|.
FP32 results are compared in relative L1 (stated per test).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1204_5849_amd import native as N  # noqa: E402
from paper_1204_5849_amd import workloads as W  # noqa: E402
from tests.helpers import random_tree, rel_linf  # noqa: E402

TOL64 = 1e-11


def _say(msg):
    print(f"[gpu-parity] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    N.lib()  # fails loudly if libmap.so is missing
    return "cuda:0"


def _sim(w, **kw):
    from paper_1204_5849_amd.sim import Simulation
    s = Simulation(w, **kw)
    s.load_initial()
    return s


def _leaf_interiors(w, U):
    leaves = w.leaf_mask()
    if w.ndim == 3:
        return U[leaves][:, :, 2:-2, 2:-2, 2:-2]
    return U[leaves][:, :, :, 2:-2, 2:-2]


PSI_PLAIN_TOL = 1e-8


def _check(w, gpu, ora, tol, what, ch=None):
    """Per-variable relative L-infinity <= tol.  With ch given, psi is held
    to tol against its scale c_h max|B| and, in addition, to PSI_PLAIN_TOL
    against its own max|psi|."""
    g, o = _leaf_interiors(w, gpu), _leaf_interiors(w, ora)
    err = rel_linf(g, o)
    psi_plain = err[8]
    if ch is not None:
        scale = max(np.abs(o[:, 8]).max(), float(np.max(ch)) * np.abs(o[:, 4:7]).max())
        err[8] = np.abs(g[:, 8] - o[:, 8]).max() / scale
    _say(f"{what}: rel Linf per var {np.array2string(err, precision=2)}, psi plain "
         f"{psi_plain:.2e}")
    assert np.all(err <= tol), (what, err)
    if ch is not None:
        assert psi_plain <= PSI_PLAIN_TOL, (what, psi_plain)


def test_init_fill_bitwise_ot(dev, orc):
    _say("orszag_tang 128^2 init + fill")
    w = W.orszag_tang(8)
    s = _sim(w)
    A = orc.load_workload(w)
    assert np.array_equal(s.state_by_key(), A.state)


def _tree(ndim, seed, bc="periodic", levels=3):
    rng = np.random.default_rng(seed)
    nb = (3, 2, 1) if ndim == 2 else (2, 2, 2)
    if bc == "mixed":
        bcs = (("periodic", "periodic"), ("outflow", "outflow"), ("periodic", "periodic"))
    else:
        bcs = ((bc, bc),) * 3
    sims = [W.SimDesc(lo=(0, 0, 0), hi=(1, 1, 1), nbase=nb, bc=bcs)]
    return sims, random_tree(sims, ndim, levels, 0.35, rng)


def _tree_ic(wl, sim, lv, x, y, z, g):
    tp = 2 * np.pi
    return [1.0 + 0.3 * np.sin(tp * x) * np.cos(tp * y), 0.4 * np.sin(tp * y),
            0.3 * np.sin(tp * (x + z)), 0.1 * np.cos(tp * z), 0.5 + 0.2 * np.cos(tp * y),
            0.3 * np.sin(tp * x), 0.2 + 0.1 * np.sin(tp * z), 1.0 + 0.2 * np.cos(tp * x),
            0.05 * np.sin(tp * y)]


@pytest.mark.parametrize("ndim,bc", [(2, "periodic"), (2, "outflow"), (3, "periodic"), (3, "mixed")])
def test_init_fill_bitwise_amr(dev, orc, ndim, bc):
    """Restriction, same-level copies, outflow clamping and prolongated ghosts."""
    _say(f"amr tree init+fill ndim={ndim} bc={bc}")
    sims, keys = _tree(ndim, 31 + ndim, bc)
    w = W.Workload(name="tree", ndim=ndim, sims=sims, keys=keys, ic=_tree_ic)
    s = _sim(w)
    A = orc.load_workload(w)
    assert (keys[:, 1] == 3).any()
    assert np.array_equal(s.state_by_key(), A.state)


def test_cfl_record_matches(dev, orc):
    _say("cfl record orszag_tang")
    w = W.orszag_tang(8)
    s = _sim(w)
    A = orc.load_workload(w)
    s.cfl()
    s.sync()
    rec = s.dt.cpu().numpy()[0][:4]
    r = A.cfl()[0]
    np.testing.assert_allclose(rec, [r.dt, r.ch, r.damp, r.alpha], rtol=1e-14)


def _run_both(w, nsteps, **kw):
    import oracle as orc
    s = _sim(w, **kw)
    A = orc.load_workload(w)
    tr = A.run(nsteps, trace=True)
    dts = []
    for _ in range(nsteps):
        s.advance(1)
        s.sync()  # the dt record is written on the simulation's stream
        dts.append(s.dt.cpu().numpy().copy())
    return s, A, tr, np.array(dts)


@pytest.mark.parametrize("nsteps", [1, 100])
def test_orszag_tang_lf_fp64(dev, nsteps):
    """Configuration 1: OT 128^2, 8x8 blocks, LF + minmod, FP64, 100 steps."""
    _say(f"orszag_tang LF fp64 {nsteps} steps")
    w = W.orszag_tang(8)
    s, A, tr, dts = _run_both(w, nsteps)
    np.testing.assert_allclose(dts[:, 0, 0], tr[:, 0, 0], rtol=1e-11)
    _check(w, s.state_by_key(), A.state, TOL64 if nsteps > 1 else 1e-13, f"OT {nsteps} steps",
           ch=tr[-1, :, 1])


@pytest.mark.parametrize("ndim,scheme,limiter,bc", [
    (2, "lf", "minmod", "periodic"), (2, "mmc", "vanleer", "periodic"), (2, "lf", "vanleer", "outflow"),
    (2, "mmc", "minmod", "outflow"), (3, "lf", "minmod", "periodic"), (3, "lf", "minmod", "mixed")])
def test_amr_tree_steps_fp64(dev, ndim, scheme, limiter, bc):
    """Random 2:1 trees: step, reflux, restriction and fill over 8 cycles."""
    _say(f"amr tree steps ndim={ndim} {scheme}/{limiter} bc={bc}")
    sims, keys = _tree(ndim, 7 + ndim + len(bc), bc)
    w = W.Workload(name="tree", ndim=ndim, sims=sims, keys=keys, ic=_tree_ic, scheme=scheme,
                   limiter=limiter)
    s, A, tr, dts = _run_both(w, 8)
    np.testing.assert_allclose(dts[:, 0, 0], tr[:, 0, 0], rtol=1e-12)
    _check(w, s.state_by_key(), A.state, TOL64, "tree 8 cycles", ch=tr[-1, :, 1])
    # parents hold the restriction of the final leaves; after a full ghost
    # fill every padded tile matches the oracle's
    s.fill()
    full = s.state_by_key()
    for k in range(8):
        assert np.abs(full[:, k] - A.state[:, k]).max() <= TOL64 * np.abs(A.state[:, k]).max() + 1e-300


def test_amr_resistive_3d_fp64(dev):
    _say("harris 3d small, eta, fastspeed GLM, 4 steps")
    w = W.harris3d(nbase=2, levels=3, precision="fp64")
    s, A, tr, dts = _run_both(w, 4)
    np.testing.assert_allclose(dts[:, 0, :4], tr[:, 0], rtol=1e-12)
    _check(w, s.state_by_key(), A.state, TOL64, "harris small 4 steps", ch=tr[-1, :, 1])


def test_blast3d_small_fp64(dev):
    _say("blast 3d small fp64 5 steps")
    w = W.blast3d(nbase=2, levels=2, precision="fp64")
    s, A, tr, dts = _run_both(w, 5)
    _check(w, s.state_by_key(), A.state, TOL64, "blast small 5 steps", ch=tr[-1, :, 1])


def test_kh_ensemble_small_fp64(dev):
    """Uneven simulations in one launch: per-simulation dt and fill."""
    _say("kh ensemble 5 sims fp64 10 steps")
    w = W.kh_ensemble(nsims=5, kmin=2, kmax=5, precision="fp64")
    s, A, tr, dts = _run_both(w, 10)
    np.testing.assert_allclose(dts[:, :, 0], tr[:, :, 0], rtol=1e-12)
    _check(w, s.state_by_key(), A.state, TOL64, "kh 10 steps", ch=tr[-1, :, 1])


def test_ot_amr_config_mmc_fp64(dev):
    """Configuration 2 block list (3840 blocks, MMC + van Leer), 3 cycles."""
    import os
    _say("ot amr 3840 blocks mmc 3 steps")
    path = os.path.join(os.path.dirname(__file__), "golden", "ot_amr_grid.txt")
    keys = np.loadtxt(path, dtype=np.int32, comments="#")
    w = W.ot_amr(keys)
    s, A, tr, dts = _run_both(w, 3)
    _check(w, s.state_by_key(), A.state, TOL64, "ot amr 3 steps", ch=tr[-1, :, 1])


def test_totals_match(dev, orc):
    _say("totals kh small")
    w = W.kh_ensemble(nsims=3, kmin=2, kmax=4, precision="fp64")
    s = _sim(w)
    A = orc.load_workload(w)
    np.testing.assert_allclose(s.totals(), A.totals(), rtol=1e-13, atol=1e-15)


def test_graph_equals_eager_and_per_block_equals_batched(dev):
    _say("graph vs eager vs per-block")
    sims, keys = _tree(2, 5, "outflow")
    w = W.Workload(name="tree", ndim=2, sims=sims, keys=keys, ic=_tree_ic)
    a = _sim(w)
    b = _sim(w)
    c = _sim(w, launch="per_block")
    a.advance(5)
    b.graph_run(5)
    c.advance(5)
    # the cycle leaves same-level ghosts of leaves unspecified: compare full
    # tiles after a full fill
    for x in (a, b, c):
        x.fill()
    ua, ub, uc = a.state_by_key(), b.state_by_key(), c.state_by_key()
    assert np.array_equal(ua, ub)
    assert np.array_equal(ua, uc)
    a.advance(4)
    a.fill()
    a2 = a.state_by_key()
    b.graph_run(4)  # replays of the captured cycle pair keep matching
    b.fill()
    assert np.array_equal(a2, b.state_by_key())


@pytest.mark.parametrize("case", ["tree2d", "tree3d", "harris3d"])
def test_cycle_fill_writes_what_a_full_fill_writes(dev, case):
    """The fill inside a cycle copies only the parent ghost cells that the
    prolongation stencil reads (map_fill_selection) and then prolongates:
    a full ghost fill afterwards leaves those parent cells and every
    prolongated ghost cell of every block unchanged, bit for bit.  On the
    random trees the selection is mostly whole frames; on the Harris sheet
    (refined slabs) it is the planes next to the coarse side."""
    _say(f"cycle fill against a full fill: {case}")
    if case == "harris3d":
        w = W.harris3d(nbase=2, levels=3, precision="fp64")
    else:
        ndim = 2 if case == "tree2d" else 3
        sims, keys = _tree(ndim, 21 + ndim, "mixed")
        w = W.Workload(name="tree", ndim=ndim, sims=sims, keys=keys, ic=_tree_ic)
    ndim, keys = w.ndim, w.keys
    s = _sim(w)
    s.advance(3)
    a = s.state_by_key()
    par, dirs, box = N.map_fill_selection(s.ctx)
    neigh = N.map_neighbors(s.ctx, len(keys))
    s.fill()
    b = s.state_by_key()
    assert len(par) > 0
    n, ng = 16, 2
    c = np.arange(-ng, n + ng)
    if ndim == 3:
        z, y, x = np.meshgrid(c, c, c, indexing="ij")
    else:
        y, x = np.meshgrid(c, c, indexing="ij")
        y, x = y[None], x[None]
        z = np.zeros_like(x)
    assert x.shape == a.shape[2:]

    def side(v):
        return np.where(v < 0, 0, np.where(v >= n, 2, 1))

    di = side(z) * 9 + side(y) * 3 + side(x)
    partial = 0
    for p, m, bx in zip(par.tolist(), dirs.tolist(), box.tolist()):
        sel = (np.right_shift(m, di) & 1).astype(bool) & (di != 13)
        sel &= (x >= bx[0]) & (x <= bx[3]) & (y >= bx[1]) & (y <= bx[4])
        if ndim == 3:
            sel &= (z >= bx[2]) & (z <= bx[5])
        assert sel.any()
        partial += int(sel.sum() < (di != 13).sum())
        assert np.array_equal(a[p][:, sel], b[p][:, sel]), p
    if case == "harris3d":
        assert partial == len(par)  # every frame is filled in part
    nprol = 0
    for i in range(len(keys)):
        pro = [d for d in range(27) if d != 13 and neigh[i, d] == -1]
        if pro:
            nprol += 1
            sel = np.isin(di, pro)
            assert np.array_equal(a[i][:, sel], b[i][:, sel]), i
    assert nprol > 0
    _say(f"{len(par)} parents, {partial} with partial frames, {nprol} blocks with prolongated ghosts")


@pytest.mark.parametrize("ndim,scheme,precision", [(2, "lf", "fp64"), (3, "lf", "fp64"),
                                                    (3, "weno", "fp64"), (3, "lf", "fp32")])
def test_cycles_in_one_call_equal_cycle_by_cycle(dev, ndim, scheme, precision):
    """n cycles in one call (alternating U and the shadow, or in place for
    WENO; eager or as replays of the captured pair) leave the state and the
    last cycle's dt records of n calls of one cycle, bit for bit, for odd and
    even counts and repeated calls."""
    import dataclasses
    _say(f"n cycles per call vs one per call ndim={ndim} {scheme} {precision}")
    sims, keys = _tree(ndim, 7 + ndim, "mixed")
    w = W.Workload(name="tree", ndim=ndim, sims=sims, keys=keys, ic=_tree_ic)
    w = dataclasses.replace(w, scheme=scheme, precision=precision)
    ref, a, b = _sim(w), _sim(w), _sim(w)
    for n in (5, 4, 1, 2):
        for _ in range(n):
            ref.advance(1)
        a.advance(n)
        b.graph_run(n)
        # the cycle leaves same-level ghosts of leaves unspecified: compare
        # full tiles after a full fill
        for x in (ref, a, b):
            x.fill()
            x.sync()
        rdt, ru = ref.dt.cpu().numpy(), ref.state_by_key()
        for x in (a, b):
            assert np.array_equal(x.dt.cpu().numpy(), rdt), n
            assert np.array_equal(x.state_by_key(), ru), n


@pytest.mark.parametrize("case", ["ot_amr", "harris64_L4"])
def test_chained_dt_on_levels_with_many_parents(dev, orc, case):
    """Levels with at least as many parents as compute units restrict one
    parent per workgroup and form the next cycle's CFL maxima of their
    children there.  On the 3840-block Orszag-Tang grid (256 and 640 parents
    per level, MMC + van Leer) and on a 3-D Harris tree with 512 parents on
    level 3: n cycles in one call (eager and graph) equal n one-cycle calls
    bit for bit, and the dt trace and state follow the oracle."""
    import dataclasses
    import os
    if case == "ot_amr":
        path = os.path.join(os.path.dirname(__file__), "golden", "ot_amr_grid.txt")
        w = W.ot_amr(np.loadtxt(path, dtype=np.int32, comments="#"))
        nsteps = 4
    else:
        w = W.harris3d(nbase=4, levels=4, precision="fp64")
        nsteps = 3
    w = dataclasses.replace(w, precision="fp64")
    lv = w.keys[:, 1]
    leaf = w.leaf_mask()
    nparents = max(int(((~leaf) & (lv == v)).sum()) for v in set(lv.tolist()))
    _say(f"chained dt {case}: {len(w.keys)} blocks, largest parent level {nparents}")
    assert nparents >= 256
    ref, a, b = _sim(w), _sim(w), _sim(w)
    dts = []
    for _ in range(nsteps):
        ref.advance(1)
        ref.sync()
        dts.append(ref.dt.cpu().numpy()[:, :4].copy())
    a.advance(nsteps)
    b.graph_run(nsteps)
    for x in (ref, a, b):
        x.fill()
        x.sync()
    ru = ref.state_by_key()
    for x in (a, b):
        assert np.array_equal(x.dt.cpu().numpy(), ref.dt.cpu().numpy())
        assert np.array_equal(x.state_by_key(), ru)
    A = orc.load_workload(w)
    tr = A.run(nsteps, trace=True)
    np.testing.assert_allclose(np.array(dts)[:, :, :4], tr, rtol=1e-13)
    _check(w, ru, A.state, TOL64, f"chained dt {case} {nsteps} cycles", ch=tr[-1, :, 1])


@pytest.mark.parametrize("ndim", [2, 3])
def test_chained_dt_two_simulations(dev, orc, ndim):
    """Two simulations of different sizes and edges, each a random 2:1 tree
    with parents and leaves without one: the dt records of each, formed in a
    cycle's restriction and the pass over the leaves without a parent, equal
    those of one cycle per call bit for bit, and the state matches the
    oracle."""
    _say(f"chained dt, two simulations, ndim={ndim}")
    # seeds for which both simulations have parents and level-1 leaves
    rng = np.random.default_rng(42 if ndim == 2 else 39)
    nb = ((3, 2, 1), (2, 2, 1)) if ndim == 2 else ((3, 2, 2), (2, 2, 3))
    per = (("periodic", "periodic"),) * 3
    mixed = (("periodic", "periodic"), ("outflow", "outflow"), ("periodic", "periodic"))
    sims = [W.SimDesc(lo=(0, 0, 0), hi=(1, 1, 1), nbase=nb[0], bc=per),
            W.SimDesc(lo=(0, 0, 0), hi=(2, 1, 2), nbase=nb[1], bc=mixed)]
    keys = random_tree(sims, ndim, 3, 0.35 if ndim == 2 else 0.15, rng)
    w = W.Workload(name="tree2", ndim=ndim, sims=sims, keys=keys, ic=_tree_ic)
    leaves = W.leaf_mask(keys)
    for sim in (0, 1):
        mine = keys[:, 0] == sim
        assert (mine & (keys[:, 1] > 1)).any() and (mine & (keys[:, 1] == 1) & leaves).any()
    ref, a = _sim(w), _sim(w)
    for _ in range(4):
        ref.advance(1)
    a.advance(4)
    A = orc.load_workload(w)
    A.run(4)
    for x in (ref, a):
        x.fill()
        x.sync()
    assert np.array_equal(a.dt.cpu().numpy(), ref.dt.cpu().numpy())
    assert np.array_equal(a.state_by_key(), ref.state_by_key())
    _check(w, a.state_by_key(), A.state, TOL64, f"two simulations ndim={ndim}")


def test_determinism_3d(dev):
    _say("determinism blast small fp32")
    w = W.blast3d(nbase=2, levels=2, precision="fp32")
    a = _sim(w)
    b = _sim(w)
    a.graph_run(4)
    b.graph_run(4)
    a.fill()
    b.fill()
    assert np.array_equal(a.state_by_key(), b.state_by_key())


@pytest.mark.parametrize("name", ["ot", "blast", "ot_amr", "tree2d"])
def test_fp32_mixed_l1_vs_fp64_oracle(dev, name):
    """FP32 state with FP64 pressure recovery and CFL against the FP64 oracle:
    relative L1 of rho, e and |B| <= 1e-4 (OT 100 steps, blast 10 steps, the
    3840-block OT AMR grid with MMC + van Leer 20 steps, a random 2-D 2:1 tree
    with outflow sides 20 steps; the last three cross coarse-fine faces, so
    reflux, restriction and ghost prolongation enter the error)."""
    import os
    import oracle as orc
    if name == "ot":
        w, n = W.orszag_tang(8, precision="fp32"), 100
    elif name == "blast":
        w, n = W.blast3d(nbase=2, levels=2, precision="fp32"), 10
    elif name == "ot_amr":
        path = os.path.join(os.path.dirname(__file__), "golden", "ot_amr_grid.txt")
        w, n = W.ot_amr(np.loadtxt(path, dtype=np.int32, comments="#"), precision="fp32"), 20
    else:
        sims, keys = _tree(2, 23, "outflow")
        w = W.Workload(name="tree", ndim=2, sims=sims, keys=keys, ic=_tree_ic, precision="fp32")
        n = 20
    if name != "ot":
        assert not w.leaf_mask().all()  # the tree has parents: coarse-fine faces
    _say(f"fp32 vs fp64 oracle {name} {n} steps")
    s = _sim(w)
    A = orc.load_workload(w)
    s.advance(n)
    A.run(n)
    g = _leaf_interiors(w, s.state_by_key())
    o = _leaf_interiors(w, A.state)
    for k, nm in ((0, "rho"), (7, "e")):
        e = np.abs(g[:, k] - o[:, k]).mean() / np.abs(o[:, k]).mean()
        _say(f"  {nm} rel L1 {e:.2e}")
        assert e <= 1e-4
    bg = np.sqrt((g[:, 4:7] ** 2).sum(axis=1))
    bo = np.sqrt((o[:, 4:7] ** 2).sum(axis=1))
    e = np.abs(bg - bo).mean() / np.abs(bo).mean()
    _say(f"  |B| rel L1 {e:.2e}")
    assert e <= 1e-4


def test_status_flags(dev):
    _say("status flags")
    w = W.orszag_tang(2)
    s = _sim(w)
    s.advance(2)
    st, cnt = s.flags()
    assert st == N.MAP_OK and cnt[2] == 0 and cnt[3] == 0
    slot = int(s.slot_of_key[0])
    s.U[slot, 7, 0, 5, 5] = 0.0  # e = 0 -> negative pressure, forced from the host
    s.cfl()
    st, cnt = s.flags()
    assert st == N.MAP_ENEGPRESSURE and cnt[2] >= 1
    s.U[slot, 0, 0, 6, 6] = float("nan")
    s.cfl()
    st, cnt = s.flags()
    assert st == N.MAP_ENONFINITE and cnt[3] >= 1


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_uniform_state_bitwise_amr(dev, ndim, precision):
    """A uniform state stays exactly uniform over whole cycles (fill,
    prolongation, step with EGLM sources and resistivity, reflux,
    restriction) on a 3-level tree, in both precisions."""
    _say(f"uniform state amr ndim={ndim} {precision}")
    sims, keys = _tree(ndim, 13 + ndim, "mixed" if ndim == 3 else "outflow")
    w = W.Workload(name="uni", ndim=ndim, sims=sims, keys=keys, precision=precision,
                   eta=1e-3 if ndim == 3 else 0.0, glm_mode="fastspeed" if ndim == 3 else "paper",
                   ic=lambda wl, s, lv, x, y, z, g: [1.2, 0.3, -0.2, 0.1, 0.4, 0.5, -0.6, 0.9, 0.0])
    s = _sim(w)
    u0 = s.U.clone()
    s.graph_run(4)
    s.advance(1)
    s.fill()
    s.sync()
    assert torch.equal(s.U, u0)


def test_step_rejects_aliased_output(dev):
    """The update reads neighbour interiors of U_in while other blocks are
    written, so an output overlapping the input is refused."""
    w = W.orszag_tang(2)
    s = _sim(w)
    s.cfl()
    with pytest.raises(N.MapError) as e:
        N.map_step(s.ctx, s.U, s.U, s.dt, s.sp)
    assert e.value.status == N.MAP_EINVAL
    out = torch.zeros_like(s.U)
    torch.cuda.synchronize()  # out is cleared on torch's stream
    N.map_step(s.ctx, s.U, out, s.dt, s.sp)
    s.sync()
    assert torch.isfinite(out).all()


@pytest.mark.parametrize("name", ["harris", "blast"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_cycle_leaves_parents_restricted(dev, name, precision):
    """After whole cycles (step, reflux, restriction) every parent equals,
    bit for bit, what the restriction pass computes from the final leaves."""
    if name == "harris":
        w = W.harris3d(nbase=2, levels=3, precision=precision)
    else:
        w = W.blast3d(nbase=2, levels=2, precision=precision)
    _say(f"parents restricted after cycles {name} {precision}")
    s = _sim(w)
    s.advance(3)
    s.sync()
    before = s.U.clone()
    s.restrict()
    s.sync()
    assert torch.equal(s.U, before)
