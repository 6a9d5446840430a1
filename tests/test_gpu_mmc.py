"""GPU parity of the modified MacCormack update (paper Sec. 3.1) on 3-D
blocks, and of the resistive terms with MMC in 2-D and 3-D, against the
FP64 oracle through the C ABI (same bars as tests/test_gpu_parity.py)."""
import dataclasses

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1204_5849_amd import native as N  # noqa: E402
from paper_1204_5849_amd import workloads as W  # noqa: E402
from tests.test_gpu_parity import TOL64, _check, _run_both, _sim, _tree, _tree_ic  # noqa: E402


def _say(msg):
    print(f"[gpu-mmc] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    N.lib()
    return "cuda:0"


@pytest.mark.parametrize("limiter,bc,eta", [("minmod", "periodic", 0.0), ("vanleer", "mixed", 0.0),
                                            ("paper", "periodic", 0.0), ("vanleer", "mixed", 2e-3)])
def test_mmc3_tree_fp64(dev, limiter, bc, eta):
    """Random 3-D 2:1 trees with reflux, restriction and prolongation: 6
    cycles of MMC against the oracle (FP64, relative L-infinity 1e-11)."""
    _say(f"mmc 3-D tree {limiter} bc={bc} eta={eta}")
    sims, keys = _tree(3, 41 + len(bc) + int(eta > 0), bc)
    w = W.Workload(name="tree", ndim=3, sims=sims, keys=keys, ic=_tree_ic, scheme="mmc",
                   limiter=limiter, eta=eta)
    assert (keys[:, 1] == 3).any()
    s, A, tr, dts = _run_both(w, 6)
    np.testing.assert_allclose(dts[:, 0, 0], tr[:, 0, 0], rtol=1e-12)
    _check(w, s.state_by_key(), A.state, TOL64, f"mmc3 tree {limiter} 6 cycles", ch=tr[-1, :, 1])


def test_mmc3_harris_resistive_fp64(dev):
    """The resistive Harris sheet (base 32^3, 3 levels) with MMC + van Leer
    and fast-speed GLM, 4 cycles."""
    w = dataclasses.replace(W.harris3d(nbase=2, levels=3, precision="fp64"), scheme="mmc",
                            limiter="vanleer")
    _say(f"mmc harris {len(w.keys)} blocks, 4 cycles")
    s, A, tr, dts = _run_both(w, 4)
    _check(w, s.state_by_key(), A.state, TOL64, "mmc3 harris 4 cycles", ch=tr[-1, :, 1])


def test_mmc2_resistive_fp64(dev):
    """2-D MMC with resistivity on a random tree, 8 cycles."""
    sims, keys = _tree(2, 19, "outflow")
    w = W.Workload(name="tree", ndim=2, sims=sims, keys=keys, ic=_tree_ic, scheme="mmc",
                   limiter="vanleer", eta=3e-3)
    _say("mmc 2-D resistive tree, 8 cycles")
    s, A, tr, dts = _run_both(w, 8)
    _check(w, s.state_by_key(), A.state, TOL64, "mmc2 resistive 8 cycles", ch=tr[-1, :, 1])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_mmc3_uniform_state_bitwise(dev, precision):
    sims, keys = _tree(3, 23, "mixed")
    w = W.Workload(name="uni", ndim=3, sims=sims, keys=keys, precision=precision, scheme="mmc",
                   limiter="vanleer", eta=1e-3, glm_mode="fastspeed",
                   ic=lambda wl, s, lv, x, y, z, g: [1.2, 0.3, -0.2, 0.1, 0.4, 0.5, -0.6, 0.9, 0.0])
    _say(f"mmc3 uniform state {precision}")
    s = _sim(w)
    u0 = s.U.clone()
    s.graph_run(4)
    s.advance(1)
    s.fill()
    s.sync()
    assert torch.equal(s.U, u0)


def test_mmc3_glm_conservation_fp64(dev):
    """Plain GLM on a periodic 3-level tree: the eight MHD totals are kept to
    1e-13 over 4 cycles (reflux closes the coarse-fine faces)."""
    sims, keys = _tree(3, 29, "periodic")
    w = W.Workload(name="tree", ndim=3, sims=sims, keys=keys, ic=_tree_ic, scheme="mmc",
                   limiter="minmod", eglm_sources=False)
    s = _sim(w)
    t0 = s.totals()[0]
    s.advance(4)
    t1 = s.totals()[0]
    scale = np.abs(s.state_by_key()[w.leaf_mask()]).max(axis=(0, 2, 3, 4))
    rel = np.abs(t1[:8] - t0[:8]) / scale[:8]
    _say(f"mmc3 glm totals change / max|u| {np.array2string(rel, precision=2)}")
    assert np.all(rel <= 1e-13)


def test_mmc3_graph_eager_per_block_bitwise(dev):
    sims, keys = _tree(3, 31, "mixed")
    w = W.Workload(name="tree", ndim=3, sims=sims, keys=keys, ic=_tree_ic, scheme="mmc",
                   limiter="minmod", eta=1e-3)
    a, b = _sim(w), _sim(w)
    c = _sim(w, launch="per_block")
    a.graph_run(3)
    b.advance(3)
    c.advance(3)
    for x in (a, b, c):
        x.fill()
        x.sync()
    ua = a.state_by_key()
    assert np.array_equal(b.state_by_key(), ua)
    assert np.array_equal(c.state_by_key(), ua)


def test_mmc3_fp32_l1(dev, orc):
    """FP32 state against the FP64 oracle: volume-weighted relative L1 of rho,
    e and |B| <= 1e-6 after 4 cycles of the small resistive Harris sheet."""
    w64 = dataclasses.replace(W.harris3d(nbase=2, levels=3, precision="fp64"), scheme="mmc",
                              limiter="vanleer")
    w32 = dataclasses.replace(w64, precision="fp32")
    s = _sim(w32)
    s.advance(4)
    A = orc.load_workload(w64)
    A.run(4)
    leaves = w64.leaf_mask()
    g = s.state_by_key()[leaves][:, :, 2:-2, 2:-2, 2:-2]
    o = A.state[leaves][:, :, 2:-2, 2:-2, 2:-2]
    vol = np.array([np.prod(w64.dx(int(k[0]), int(k[1]))) for k in w64.keys[leaves]])[:, None, None, None]

    def rl1(x, y):
        return float((np.abs(x - y) * vol).sum() / (np.abs(y) * vol).sum())

    bg, bo = np.sqrt((g[:, 4:7] ** 2).sum(axis=1)), np.sqrt((o[:, 4:7] ** 2).sum(axis=1))
    l1 = [rl1(g[:, 0], o[:, 0]), rl1(g[:, 7], o[:, 7]), rl1(bg, bo)]
    _say(f"mmc3 fp32 rel L1 rho {l1[0]:.2e} e {l1[1]:.2e} |B| {l1[2]:.2e}")
    assert max(l1) <= 1e-6
