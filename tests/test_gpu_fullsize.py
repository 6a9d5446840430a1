"""Full-size checks at the benchmark's shapes and launch configuration.

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
