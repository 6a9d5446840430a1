"""Pins of the oracle's block-tree operations (Sec. 4.3 of the paper):
blocked == monolithic, uniform states on AMR grids, conservation with
reflux, exactness of prolongation and restriction on linear fields."""
import numpy as np
import pytest

from paper_1204_5849_amd import workloads as W
from tests.helpers import random_tree


def _assemble(orc, p, w, A, N):
    """Monolithic copy of a single-level blocked state."""
    big = np.zeros(orc.tile_shape(p, (N, N, N if p.ndim == 3 else 1)))
    n = w.n
    for b, (s, lv, ix, iy, iz) in enumerate(w.keys):
        if p.ndim == 2:
            big[:, 0, 2 + iy * n:2 + (iy + 1) * n, 2 + ix * n:2 + (ix + 1) * n] = A.state[b, :, 0, 2:-2, 2:-2]
        else:
            big[:, 2 + iz * n:2 + (iz + 1) * n, 2 + iy * n:2 + (iy + 1) * n,
                2 + ix * n:2 + (ix + 1) * n] = A.state[b, :, 2:-2, 2:-2, 2:-2]
    return big


@pytest.mark.parametrize("scheme,limiter", [("lf", "minmod"), ("mmc", "vanleer"), ("weno", "minmod")])
def test_blocked_equals_monolithic_bitwise_2d(orc, scheme, limiter):
    w = W.orszag_tang(nbase=4, scheme=scheme, limiter=limiter)
    A = orc.load_workload(w)
    p = A.p
    big = _assemble(orc, p, w, A, 64)
    A.run(12)
    orc.grid_run(p, (1 / 64, 1 / 64), big, (64, 64, 1), [("periodic", "periodic")] * 3, 12)
    assert np.array_equal(_assemble(orc, p, w, A, 64)[:, :, 2:-2, 2:-2], big[:, :, 2:-2, 2:-2])


def test_blocked_equals_monolithic_bitwise_3d(orc):
    w = W.harris3d(nbase=2, levels=1, precision="fp64")
    w.sims[0].bc = (("periodic", "periodic"),) * 3  # monolithic mode wraps y too
    A = orc.load_workload(w)
    p = A.p
    N = 32
    big = _assemble(orc, p, w, A, N)
    dx = 4.0 / N
    A.run(3)
    orc.grid_run(p, (dx, dx, dx), big, (N, N, N), [("periodic", "periodic")] * 3, 3)
    assert np.array_equal(_assemble(orc, p, w, A, N)[:, 2:-2, 2:-2, 2:-2], big[:, 2:-2, 2:-2, 2:-2])


def _exact_totals(A, w):
    """Volume-weighted leaf totals per variable, summed exactly (fsum)."""
    import math
    inter = A.interior()
    out = []
    for k in range(inter.shape[1]):
        terms = []
        for b in np.nonzero(A.leaf)[0]:
            dx = w.dx(int(A.keys[b, 0]), int(A.keys[b, 1]))
            vol = dx[0] * dx[1] * (dx[2] if w.ndim == 3 else 1.0)
            terms.extend((inter[b, k].ravel() * vol).tolist())
        out.append(math.fsum(terms))
    return np.array(out)


def _tree_workload(ndim, scheme, limiter, seed, levels=3, eglm=True):
    rng = np.random.default_rng(seed)
    if ndim == 2:
        sims = [W.SimDesc(lo=(0, 0, 0), hi=(1, 1, 1), nbase=(3, 2, 1),
                          bc=(("periodic", "periodic"),) * 3)]
    else:
        sims = [W.SimDesc(lo=(0, 0, 0), hi=(1, 1, 1), nbase=(2, 2, 2),
                          bc=(("periodic", "periodic"),) * 3)]
    keys = random_tree(sims, ndim, levels, 0.3, rng)

    def ic(wl, sim, lv, x, y, z, gidx):
        tp = 2 * np.pi
        return [1.0 + 0.3 * np.sin(tp * x) * np.cos(tp * y), 0.4 * np.sin(tp * y),
                0.3 * np.sin(tp * (x + z)), 0.1, 0.5 + 0.2 * np.cos(tp * y),
                0.3 * np.sin(tp * x), 0.2, 1.0 + 0.2 * np.cos(tp * x), 0.05 * np.sin(tp * y)]

    return W.Workload(name="tree", ndim=ndim, sims=sims, keys=keys, ic=ic, n=8 if ndim == 3 else 16,
                      scheme=scheme, limiter=limiter, eglm_sources=eglm)


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("scheme,limiter", [("lf", "minmod"), ("mmc", "vanleer"), ("weno", "minmod")])
def test_glm_conserves_on_amr_tree(orc, ndim, scheme, limiter):
    """GLM mode on a random 2:1-balanced periodic tree: with reflux, the
    volume-weighted totals of mass, momentum, energy and B are conserved."""
    w = _tree_workload(ndim, scheme, limiter, seed=ndim * 10 + ["lf", "mmc", "weno"].index(scheme),
                       eglm=False)
    A = orc.load_workload(w)
    assert (A.keys[:, 1] == 3).any()
    t0 = _exact_totals(A, w)
    # the domain volume is 1, so max|u| bounds each total
    scale = np.abs(A.interior()[A.leaf]).max(axis=(0, 2, 3, 4))
    A.run(4)
    t1 = _exact_totals(A, w)
    assert np.all(np.abs(t1[:8] - t0[:8]) <= 1e-13 * scale[:8]), (t1 - t0)


@pytest.mark.parametrize("ndim", [2, 3])
def test_uniform_state_bitwise_on_amr_tree(orc, ndim):
    w = _tree_workload(ndim, "lf", "minmod", seed=7 + ndim)
    w.ic = lambda wl, sim, lv, x, y, z, g: [1.2, 0.3, -0.2, 0.1, 0.4, 0.5, -0.6, 0.9, 0.0]
    for scheme in ("lf", "mmc", "weno"):
        w.scheme = scheme
        A = orc.load_workload(w)
        s0 = A.state.copy()
        A.run(2)
        assert np.array_equal(A.state, s0)


def _linear(x, y, z):
    return 0.7 + 1.3 * x - 0.4 * y + 0.25 * z


@pytest.mark.parametrize("ndim", [2, 3])
def test_fill_is_exact_for_linear_fields(orc, ndim):
    """Copies, restriction and minmod prolongation reproduce a linear field
    exactly at every ghost cell whose stencils stay inside the domain."""
    rng = np.random.default_rng(21 + ndim)
    nb = (4, 4, 1) if ndim == 2 else (2, 2, 2)
    sims = [W.SimDesc(lo=(0, 0, 0), hi=(1, 1, 1), nbase=nb, bc=(("outflow", "outflow"),) * 3)]
    keys = random_tree(sims, ndim, 3, 0.35, rng)
    n = 16 if ndim == 2 else 8
    w = W.Workload(name="lin", ndim=ndim, sims=sims, keys=keys, n=n,
                   ic=lambda wl, s, lv, x, y, z, g: [_linear(x, y, z)] * 9)
    p = orc.make_params(ndim=ndim)
    A = orc.Amr(p, n, sims, keys)
    leaves = np.nonzero(A.leaf)[0]
    orc.interior(p, A.state)[leaves] = w.primitive_blocks(leaves)
    A.restrict()
    A.fill()
    checked = 0
    for b in range(len(keys)):
        s, lv, ix, iy, iz = keys[b]
        dx = w.dx(0, lv)
        N = [w.cells_at_level(0, d, lv) for d in range(3)]
        g = [np.arange(-2, n + 2) for _ in range(ndim)] + ([np.zeros(1, int)] if ndim == 2 else [])
        G = np.meshgrid(*(g[d] + [ix, iy, iz][d] * n for d in range(3)), indexing="ij")
        # safe: the cell and a 4-cell margin inside the domain (coarse stencil)
        safe = np.ones(G[0].shape, bool)
        for d in range(ndim):
            safe &= (G[d] >= 4) & (G[d] < N[d] - 4)
        X = (G[0] + 0.5) * dx[0]
        Y = (G[1] + 0.5) * dx[1]
        Z = (G[2] + 0.5) * dx[2] if ndim == 3 else np.zeros_like(X, dtype=float)
        want = _linear(X, Y, Z).transpose(2, 1, 0)  # -> [z][y][x]
        got = A.state[b, 0]
        safe = safe.transpose(2, 1, 0)
        assert np.allclose(got[safe], want[safe], rtol=0, atol=1e-13)
        checked += safe.sum()
    assert checked > 0


def test_prolong_block_mean_equals_parent(orc, rng):
    """The 2^d children prolonged from one parent average back to it, and the
    interpolation is exact for a linear field."""
    sims = [W.SimDesc(lo=(0, 0, 0), hi=(1, 1, 1), nbase=(2, 2, 1), bc=(("periodic", "periodic"),) * 3)]
    keys = np.concatenate([W.base_keys(0, (2, 2, 1), 2),
                           W.children_of(np.array([[0, 1, 1, 0, 0]]), 2)])
    p = orc.make_params(ndim=2)
    A = orc.Amr(p, 16, sims, keys)
    A.state[:] = rng.normal(size=A.state.shape)
    A.fill()
    for b in range(4, 8):
        A.prolong_block(b)
    par = A.state[1, :, 0, 2:-2, 2:-2]
    kids = np.zeros((9, 32, 32))
    for b in range(4, 8):
        s, lv, ix, iy, iz = keys[b]
        cx, cy = ix - 2, iy
        kids[:, cy * 16:(cy + 1) * 16, cx * 16:(cx + 1) * 16] = A.state[b, :, 0, 2:-2, 2:-2]
    mean = 0.25 * (kids[:, 0::2, 0::2] + kids[:, 1::2, 0::2] + kids[:, 0::2, 1::2] + kids[:, 1::2, 1::2])
    np.testing.assert_allclose(mean, par, rtol=0, atol=4e-15 * np.abs(par).max())


def test_restrict_preserves_volume_integral(orc, rng):
    sims = [W.SimDesc(lo=(0, 0, 0), hi=(1, 1, 1), nbase=(2, 2, 2), bc=(("periodic", "periodic"),) * 3)]
    keys = random_tree(sims, 3, 3, 0.4, rng)
    p = orc.make_params(ndim=3)
    A = orc.Amr(p, 8, sims, keys)
    A.state[:] = rng.normal(size=A.state.shape)
    t_leaves = A.totals()[0]
    A.restrict()
    base = keys[:, 1] == 1
    vol = (1 / 16) ** 3
    t_base = orc.interior(p, A.state)[base].sum(axis=(0, 2, 3, 4)) * vol
    np.testing.assert_allclose(t_base, t_leaves, rtol=1e-12, atol=1e-12)
    uni = np.ones_like(A.state) * 0.3
    A.state[:] = uni
    A.restrict()
    assert np.array_equal(A.state, uni)


def _threaded_run(orc, w, threads, nsteps):
    before = orc.get_threads()
    orc.set_threads(threads)
    try:
        A = orc.load_workload(w)
        tr = A.run(nsteps, trace=True)
        return A.state.copy(), tr, A.counters()
    finally:
        orc.set_threads(before)


@pytest.mark.parametrize("ndim,scheme,cond", [(2, "lf", "off"), (2, "mmc", "off"),
                                             (3, "lf", "off"), (3, "weno", "off"),
                                             (3, "lf", "field")])
def test_threads_give_the_one_thread_result_bitwise(orc, ndim, scheme, cond):
    """The block loops of the tree (fill, restriction, CFL, step, reflux,
    conduction) run on several threads; state, dt records and counters
    equal the one-thread run bit for bit."""
    rng = np.random.default_rng(77 + ndim)
    nb = (3, 2, 1) if ndim == 2 else (2, 2, 2)
    bcs = (("periodic", "periodic"), ("outflow", "outflow"), ("periodic", "periodic"))
    sims = [W.SimDesc(lo=(0, 0, 0), hi=(1, 1, 1), nbase=nb, bc=bcs)]
    keys = random_tree(sims, ndim, 3, 0.35, rng)

    def ic(wl, sim, lv, x, y, z, g):
        tp = 2 * np.pi
        return [1.0 + 0.3 * np.sin(tp * x) * np.cos(tp * y), 0.4 * np.sin(tp * y),
                0.3 * np.sin(tp * (x + z)), 0.1 * np.cos(tp * z), 0.5 + 0.2 * np.cos(tp * y),
                0.3 * np.sin(tp * x), 0.2 + 0.1 * np.sin(tp * z), 1.0 + 0.2 * np.cos(tp * x),
                0.05 * np.sin(tp * y)]

    w = W.Workload(name="tree", ndim=ndim, sims=sims, keys=keys, ic=ic, scheme=scheme,
                   limiter="vanleer" if scheme == "mmc" else "minmod", eta=1e-3 if ndim == 3 else 0.0,
                   cond=cond, kappa0=0.05 if cond != "off" else 0.0)
    s1, t1, c1 = _threaded_run(orc, w, 1, 3)
    s8, t8, c8 = _threaded_run(orc, w, 8, 3)
    assert np.array_equal(t1, t8)
    assert np.array_equal(c1, c8)
    assert np.array_equal(s1, s8)
