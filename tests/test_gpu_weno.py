"""GPU parity of the WENO scheme with TVD Runge-Kutta 2 (Sec. 3.3 of the
paper) through the C ABI against the FP64 oracle: the same bar as the LF
path (FP64 relative L-infinity per variable <= 1e-11; psi against c_h max|B|;
FP32 in relative L1), on uniform grids, random 2:1 trees with both boundary
kinds, the resistive 3-D Harris sheet and the 3-D blast, plus the cycle
forms (in place, graph replay, per-block launches) and exact invariants."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1204_5849_amd import native as N  # noqa: E402
from paper_1204_5849_amd import workloads as W  # noqa: E402
from tests.test_gpu_parity import (TOL64, _check, _leaf_interiors, _run_both, _say, _sim,  # noqa: E402
                                   _tree, _tree_ic)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    N.lib()  # fails loudly if libmap.so is missing
    return "cuda:0"


def _weno(w):
    w.scheme = "weno"
    return w


def test_weno_single_step_ot_fp64(dev):
    _say("weno orszag_tang 64^2 fp64 1 step")
    w = _weno(W.orszag_tang(4))
    s, A, tr, dts = _run_both(w, 1)
    np.testing.assert_allclose(dts[:, 0, 0], tr[:, 0, 0], rtol=1e-13)
    _check(w, s.state_by_key(), A.state, 1e-13, "weno OT 1 step", ch=tr[-1, :, 1])


def test_weno_orszag_tang_fp64(dev):
    _say("weno orszag_tang 128^2 fp64 40 steps")
    w = _weno(W.orszag_tang(8))
    s, A, tr, dts = _run_both(w, 40)
    np.testing.assert_allclose(dts[:, 0, 0], tr[:, 0, 0], rtol=1e-11)
    _check(w, s.state_by_key(), A.state, TOL64, "weno OT 40 steps", ch=tr[-1, :, 1])


@pytest.mark.parametrize("ndim,bc", [(2, "periodic"), (2, "outflow"), (3, "periodic"), (3, "mixed")])
def test_weno_amr_tree_steps_fp64(dev, ndim, bc):
    """Random 2:1 trees: both stages, the boundary procedure on the stage
    state, reflux with the stage-averaged fluxes, restriction, fill."""
    _say(f"weno amr tree ndim={ndim} bc={bc} 6 cycles")
    sims, keys = _tree(ndim, 17 + ndim + len(bc), bc)
    w = W.Workload(name="tree", ndim=ndim, sims=sims, keys=keys, ic=_tree_ic, scheme="weno")
    s, A, tr, dts = _run_both(w, 6)
    np.testing.assert_allclose(dts[:, 0, 0], tr[:, 0, 0], rtol=1e-12)
    _check(w, s.state_by_key(), A.state, TOL64, "weno tree 6 cycles", ch=tr[-1, :, 1])
    s.fill()
    full = s.state_by_key()
    for k in range(8):
        assert np.abs(full[:, k] - A.state[:, k]).max() <= TOL64 * np.abs(A.state[:, k]).max() + 1e-300


def test_weno_harris_resistive_3d_fp64(dev):
    _say("weno harris 3d small, eta, fastspeed GLM, 4 steps")
    w = _weno(W.harris3d(nbase=2, levels=3, precision="fp64"))
    s, A, tr, dts = _run_both(w, 4)
    np.testing.assert_allclose(dts[:, 0, :4], tr[:, 0], rtol=1e-12)
    _check(w, s.state_by_key(), A.state, TOL64, "weno harris 4 steps", ch=tr[-1, :, 1])


def test_weno_blast3d_fp64(dev):
    _say("weno blast 3d small fp64 5 steps")
    w = _weno(W.blast3d(nbase=2, levels=2, precision="fp64"))
    s, A, tr, dts = _run_both(w, 5)
    _check(w, s.state_by_key(), A.state, TOL64, "weno blast 5 steps", ch=tr[-1, :, 1])


def _lowp_ic(wl, sim, lv, x, y, z, g):
    """Fast flow over a density step at nearly zero pressure: reconstructed
    energies undershoot the kinetic energy and the fall-backs fire."""
    tp = 2 * np.pi
    return [1.0 + 0.8 * (np.sin(tp * x) > 0.3), 3.0 * np.sin(tp * x), 0.5 * np.cos(tp * y), 0.0 * x,
            0.05 + 0 * x, 0.0 * x, 0.0 * x, 1e-4 + 0 * x, 0.0 * x]


@pytest.mark.parametrize("scheme", ["weno", "lf"])
def test_fallback_counters_and_state_match_oracle(dev, scheme):
    """Face states replaced by the cell value: the same count on both sides
    (counter [1]), and the states still agree."""
    import oracle as orc
    _say(f"{scheme} low-pressure fall-back counters, 2-D tree, 2 steps")
    sims, keys = _tree(2, 41, "periodic")
    w = W.Workload(name="lowp", ndim=2, sims=sims, keys=keys, ic=_lowp_ic, scheme=scheme)
    s = _sim(w)
    A = orc.load_workload(w)
    s.flags()
    s.advance(2)
    A.run(2)
    _, cnt = s.flags()
    want = A.counters()
    _say(f"  counters gpu {list(cnt[:2])} oracle {list(want[:2])}")
    assert want[1] > 0
    assert cnt[1] == want[1]
    _check(w, s.state_by_key(), A.state, TOL64, f"{scheme} low-pressure 2 steps")


@pytest.mark.parametrize("name", ["ot", "blast"])
def test_weno_fp32_l1_vs_fp64_oracle(dev, name):
    """FP32 WENO against the FP64 oracle: relative L1 of rho, e and |B|
    <= 1e-4 (OT 40 steps, blast 10 steps)."""
    import oracle as orc
    if name == "ot":
        w, n = _weno(W.orszag_tang(8, precision="fp32")), 40
    else:
        w, n = _weno(W.blast3d(nbase=2, levels=2, precision="fp32")), 10
    _say(f"weno fp32 vs fp64 oracle {name} {n} steps")
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


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_weno_uniform_state_bitwise_amr(dev, ndim, precision):
    _say(f"weno uniform state amr ndim={ndim} {precision}")
    sims, keys = _tree(ndim, 13 + ndim, "mixed" if ndim == 3 else "outflow")
    w = W.Workload(name="uni", ndim=ndim, sims=sims, keys=keys, precision=precision, scheme="weno",
                   eta=1e-3 if ndim == 3 else 0.0, glm_mode="fastspeed" if ndim == 3 else "paper",
                   ic=lambda wl, s, lv, x, y, z, g: [1.2, 0.3, -0.2, 0.1, 0.4, 0.5, -0.6, 0.9, 0.0])
    s = _sim(w)
    u0 = s.U.clone()
    s.graph_run(3)
    s.advance(1)
    s.fill()
    s.sync()
    assert torch.equal(s.U, u0)


def test_weno_step_in_place_equals_separate_output(dev):
    """Stage 2 reads u^n only at the cell it writes: map_step(U, U) gives the
    same leaves, bit for bit, as map_step(U, V)."""
    _say("weno step in place vs separate output")
    sims, keys = _tree(2, 3, "periodic")
    w = W.Workload(name="tree", ndim=2, sims=sims, keys=keys, ic=_tree_ic, scheme="weno")
    s = _sim(w)
    s.cfl()
    out = torch.zeros_like(s.U)
    torch.cuda.synchronize()  # out is cleared on torch's stream
    N.map_step(s.ctx, s.U, out, s.dt, s.sp)
    N.map_step(s.ctx, s.U, s.U, s.dt, s.sp)
    s.sync()
    leaves = torch.as_tensor(np.asarray(s.slot_of_key)[w.leaf_mask()], device=s.U.device).long()
    a = s.U[leaves][:, :, :, 2:-2, 2:-2]
    b = out[leaves][:, :, :, 2:-2, 2:-2]
    assert torch.equal(a, b)


def test_weno_graph_equals_eager_and_per_block(dev):
    _say("weno graph vs eager vs per-block")
    sims, keys = _tree(3, 5, "mixed")
    w = W.Workload(name="tree", ndim=3, sims=sims, keys=keys, ic=_tree_ic, scheme="weno")
    a = _sim(w)
    b = _sim(w)
    c = _sim(w, launch="per_block")
    a.advance(5)
    b.graph_run(5)
    c.advance(5)
    for x in (a, b, c):
        x.fill()
    ua = a.state_by_key()
    assert np.array_equal(ua, b.state_by_key())
    assert np.array_equal(ua, c.state_by_key())


def test_weno_conserves_with_reflux_fp64(dev):
    """Plain GLM on a periodic 3-level tree: volume-weighted totals of mass,
    momentum, energy and B stay constant over whole WENO cycles."""
    _say("weno conservation amr 2d fp64")
    sims, keys = _tree(2, 29, "periodic")
    w = W.Workload(name="tree", ndim=2, sims=sims, keys=keys, ic=_tree_ic, scheme="weno",
                   eglm_sources=False)
    s = _sim(w)
    t0 = s.totals()
    s.advance(6)
    t1 = s.totals()
    scale = np.abs(_leaf_interiors(w, s.state_by_key())).max(axis=(0, 2, 3, 4))
    assert np.all(np.abs(t1[0, :8] - t0[0, :8]) <= 1e-13 * scale[:8]), t1 - t0
