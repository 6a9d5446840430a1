"""Full-size checks at the benchmark's shapes and launch configuration.

* The whole 128^3 Harris sheet with 4 levels (22016 blocks, 79.2 M leaf
  cells), two whole cycles in the benchmark's launch configuration
  (autotuned, graph-captured) against the oracle run on the host's cores over
  every leaf: FP64 to 1e-11 relative L-infinity, dt records to 1e-12; FP32
  (the headline state) in volume-weighted relative L1 per variable.
* Sampled outputs: one batched step launch (persistent grid picked by the
  autotuner, as in bench.py) on the 128^3 Harris sheet with 4 levels, for
  leaves whose 26 same-level neighbours exist; the oracle steps the same blocks
  on padded tiles it assembles itself from the seeded generator, with the same
  caller-chosen dt record.
* Properties at any size: a uniform state is preserved bit for bit over whole
  cycles on the full 4-level grid; plain GLM conserves mass, momentum, energy
  and B on the full periodic blast grid (FP64).
* The full 64-run KH ensemble against the oracle for two cycles (FP64).
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1204_5849_amd import native as N  # noqa: E402
from paper_1204_5849_amd import workloads as W  # noqa: E402
from tests.helpers import rel_linf  # noqa: E402


def _say(msg):
    print(f"[gpu-full] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    N.lib()
    return "cuda:0"


# FP32 state against the FP64 oracle after two whole cycles of the full
# Harris sheet: volume-weighted relative L1 of rho, e and |B| (each FP32
# rounding of a state of size 1 is 6e-8; two cycles of arithmetic stay
# within a few of those).
FP32_L1_TOL = 1e-6


@pytest.fixture(scope="module")
def harris_oracle(orc):
    """The oracle's two cycles of the full Harris sheet (FP64, all host cores
    up to 16), with the dt records; the generator's primitive data is formed
    once and handed to both sides."""
    import os
    w = W.harris3d(precision="fp64")
    leaves = np.nonzero(w.leaf_mask())[0]
    pos = np.full(len(w.keys), -1, dtype=np.int64)
    pos[leaves] = np.arange(len(leaves))
    _say(f"harris 128^3 L4: generator data for {len(leaves)} leaves")
    prim = w.primitive_blocks(leaves)

    def cached(blocks):
        return prim[pos[np.asarray(blocks, dtype=np.int64)]]

    before = orc.get_threads()
    threads = min(16, os.cpu_count() or 1)
    orc.set_threads(threads)
    try:
        w.primitive_blocks = cached
        _say(f"  oracle load and 2 cycles on {threads} threads")
        A = orc.load_workload(w)
        tr = A.run(2, trace=True)
    finally:
        orc.set_threads(before)
    _say("  oracle done")
    return w, A, tr, cached


def _leaf_norms(w, sim, A, chunk=1024):
    """Over every leaf interior, per variable (9) and |B| (index 9): max |g - o|,
    max |o|, volume-weighted sum |g - o| and sum |o|."""
    leaves = np.nonzero(w.leaf_mask())[0]
    out = np.zeros((4, 10))
    for s in range(0, len(leaves), chunk):
        idx = leaves[s:s + chunk]
        g = sim.state_by_key(idx)[:, :, 2:-2, 2:-2, 2:-2]
        o = A.state[idx][:, :, 2:-2, 2:-2, 2:-2]
        vol = np.array([np.prod(w.dx(int(k[0]), int(k[1]))) for k in w.keys[idx]])
        gb = np.sqrt((g[:, 4:7] ** 2).sum(axis=1))[:, None]
        ob = np.sqrt((o[:, 4:7] ** 2).sum(axis=1))[:, None]
        g = np.concatenate([g, gb], axis=1)
        o = np.concatenate([o, ob], axis=1)
        d = np.abs(g - o)
        out[0] = np.maximum(out[0], d.max(axis=(0, 2, 3, 4)))
        out[1] = np.maximum(out[1], np.abs(o).max(axis=(0, 2, 3, 4)))
        out[2] += (d.sum(axis=(2, 3, 4)) * vol[:, None]).sum(axis=0)
        out[3] += (np.abs(o).sum(axis=(2, 3, 4)) * vol[:, None]).sum(axis=0)
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_harris_full_size_cycles_vs_oracle(dev, harris_oracle, precision):
    from paper_1204_5849_amd.sim import Simulation
    w64, A, tr, cached = harris_oracle
    w = W.harris3d(precision=precision)
    w.primitive_blocks = cached
    _say(f"harris 128^3 L4 {precision}: load, autotune, 2 graph cycles")
    sim = Simulation(w, precision=precision)
    sim.load_initial()
    sim.autotune()
    sim.graph_run(2)
    sim.sync()
    rec = sim.dt.cpu().numpy()[0]
    st, cnt = sim.flags()
    assert st == 0 and cnt[2] == 0 and cnt[3] == 0
    nrm = _leaf_norms(w, sim, A)
    linf = nrm[0] / np.where(nrm[1] > 0, nrm[1], 1.0)
    l1 = nrm[2] / np.where(nrm[3] > 0, nrm[3], 1.0)
    names = ["rho", "mx", "my", "mz", "Bx", "By", "Bz", "e", "psi", "|B|"]
    _say("  rel Linf " + " ".join(f"{n} {v:.2e}" for n, v in zip(names, linf)))
    _say("  rel L1   " + " ".join(f"{n} {v:.2e}" for n, v in zip(names, l1)))
    if precision == "fp64":
        np.testing.assert_allclose(rec[:4], tr[-1, 0, :4], rtol=1e-12)
        psi_scale = max(nrm[1][8], tr[-1, 0, 1] * nrm[1][4:7].max())
        assert np.all(linf[:8] <= 1e-11), linf
        assert nrm[0][8] / psi_scale <= 1e-11
    else:
        np.testing.assert_allclose(rec[:4], tr[-1, 0, :4], rtol=1e-5)
        assert l1[0] <= FP32_L1_TOL and l1[7] <= FP32_L1_TOL and l1[9] <= FP32_L1_TOL, l1
    del sim
    torch.cuda.empty_cache()


def _pick_interior_leaves(w, ctx, per_level=3, seed=3):
    """Leaves whose 26 neighbours are leaves of their own level (so every
    ghost is a copy of point-sampled initial data, not a restriction or a
    prolongation), away from outflow edges."""
    nb = N.map_neighbors(ctx, len(w.keys))
    leaves = w.leaf_mask()
    rng = np.random.default_rng(seed)
    out = []
    for lv in sorted(set(w.keys[:, 1].tolist())):
        cand = []
        for b in np.nonzero(leaves & (w.keys[:, 1] == lv))[0]:
            row = np.delete(nb[b], 13)
            if (row < 0).any() or not leaves[row].all():
                continue
            s, _, ix, iy, iz = w.keys[b]
            sim = w.sims[s]
            ok = True
            for d, i in enumerate((ix, iy, iz)):
                nmax = sim.nbase[d] << (lv - 1)
                if sim.bc[d][0] == "outflow" and (i == 0 or i == nmax - 1):
                    ok = False
            if ok:
                cand.append(b)
        if cand:
            out.extend(rng.choice(cand, size=min(per_level, len(cand)), replace=False).tolist())
    return out


def _oracle_tile(orc, w, p, b):
    """Padded tile of block b from the generator: the 3x3x3 same-level
    neighbourhood (periodic wrap), converted to conserved variables."""
    s, lv, ix, iy, iz = (int(v) for v in w.keys[b])
    n = w.n
    sim = w.sims[s]
    index = {tuple(k): i for i, k in enumerate(w.keys.tolist())}
    big = np.zeros((9, 3 * n, 3 * n, 3 * n))
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                c = [ix + dx, iy + dy, iz + dz]
                for d in range(3):
                    c[d] %= sim.nbase[d] << (lv - 1)
                j = index[(s, lv, c[0], c[1], c[2])]
                prim = w.primitive_blocks([j])[0]
                big[:, (dz + 1) * n:(dz + 2) * n, (dy + 1) * n:(dy + 2) * n,
                    (dx + 1) * n:(dx + 2) * n] = prim
    tile = np.ascontiguousarray(big[:, n - 2:2 * n + 2, n - 2:2 * n + 2, n - 2:2 * n + 2])
    return orc.prim_to_cons(p, tile)


@pytest.mark.parametrize("precision,tol", [("fp32", 2e-5), ("fp64", 1e-12)])
def test_harris_full_size_sampled_step(dev, orc, precision, tol):
    from paper_1204_5849_amd.sim import Simulation
    w = W.harris3d(precision=precision)  # 128^3 base, 4 levels, 22016 blocks
    _say(f"harris 128^3 L4 {precision}: load, autotune, one step launch")
    sim = Simulation(w, precision=precision)
    sim.load_initial()
    sim.autotune()  # trial steps write the shadow state; U's interiors are kept
    sim.sync()
    rec = torch.tensor([[2.0e-4, 1.3, math.exp(-2.0e-4 * 1.3 / 0.18), 1.3]], dtype=torch.float64,
                       device=sim.device)
    out = torch.zeros_like(sim.U)
    torch.cuda.synchronize()  # rec and out are written on torch's stream
    N.map_step(sim.ctx, sim.U, out, rec, sim.sp)
    sim.sync()
    sim.U = out
    p = orc.params_from_workload(w)
    orec = orc.make_dtrec(*rec.cpu().numpy()[0].tolist())
    picks = _pick_interior_leaves(w, sim.ctx)
    assert len(picks) >= 6
    got = sim.state_by_key(picks)
    for i, b in enumerate(picks):
        tile = _oracle_tile(orc, w, p, b)
        lv = int(w.keys[b, 1])
        unew, _, _ = orc.step_tile(p, w.dx(0, lv), tile, (16, 16, 16), orec)
        g = got[i][:, 2:-2, 2:-2, 2:-2]
        err = rel_linf(g[None], unew[None])
        scale = max(np.abs(unew[8]).max(), 1.3 * np.abs(unew[4:7]).max())
        err[8] = np.abs(g[8] - unew[8]).max() / scale
        _say(f"  block {b} level {lv}: max rel Linf {err.max():.2e}")
        assert np.all(err <= tol), (b, err)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_uniform_state_full_grid(dev, precision):
    from paper_1204_5849_amd.sim import Simulation
    w = W.harris3d(precision=precision)
    w.ic = lambda wl, sim, lv, x, y, z, g: [1.1, 0.2, -0.1, 0.05, 0.6, -0.3, 0.2, 1.4, 0.0]
    _say(f"uniform state, harris grid 22016 blocks, {precision}, 3 graph cycles")
    sim = Simulation(w, precision=precision)
    sim.load_initial()
    u0 = sim.U.clone()
    sim.graph_run(3)
    sim.fill()
    sim.sync()
    assert torch.equal(sim.U, u0)


def test_glm_conservation_full_blast_fp64(dev):
    from paper_1204_5849_amd.sim import Simulation
    w = W.blast3d(precision="fp64")
    w.eglm_sources = False
    _say("blast 128^3 L2 fp64 GLM: totals over 4 cycles")
    sim = Simulation(w, precision="fp64")
    sim.load_initial()
    t0 = sim.totals()[0]
    sim.advance(4)
    t1 = sim.totals()[0]
    scale = np.abs(t0) + 1e-300
    rel = np.abs(t1[:8] - t0[:8]) / np.maximum(scale[:8], 1e-3)
    _say(f"  relative change of totals {np.array2string(rel, precision=2)}")
    assert np.all(rel <= 1e-12)


def test_kh_full_ensemble_fp64(dev, orc):
    from paper_1204_5849_amd.sim import Simulation
    w = W.kh_ensemble(precision="fp64")
    _say(f"kh ensemble 64 runs, {len(w.keys)} blocks, fp64, 2 cycles")
    sim = Simulation(w, precision="fp64")
    sim.load_initial()
    A = orc.load_workload(w)
    assert np.array_equal(sim.state_by_key(), A.state)
    tr = A.run(2, trace=True)
    sim.advance(2)
    sim.sync()
    np.testing.assert_allclose(sim.dt.cpu().numpy()[:, 0], tr[-1, :, 0], rtol=1e-13)
    g = sim.state_by_key()
    leaves = w.leaf_mask()
    err = rel_linf(g[leaves][:, :, :, 2:-2, 2:-2], A.state[leaves][:, :, :, 2:-2, 2:-2])
    _say(f"  rel Linf per var {np.array2string(err[:8], precision=2)}")
    assert np.all(err[:8] <= 1e-11)
