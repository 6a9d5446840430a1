"""GPU parity of the HLLC face flux (the solver the paper names for its LF
and WENO schemes) through the C ABI against the FP64 oracle: FP64 relative
L-infinity per variable <= 1e-11 (psi against c_h max|B|), FP32 in relative
L1, on grids and random 2:1 trees with both schemes, plus the invariants
HLLC adds (a stationary contact stays in place)."""
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


def _hllc(w, scheme=None):
    w.riemann = "hllc"
    if scheme:
        w.scheme = scheme
    return w


@pytest.mark.parametrize("scheme", ["lf", "weno"])
def test_hllc_orszag_tang_fp64(dev, scheme):
    _say(f"{scheme}+hllc orszag_tang 128^2 fp64 30 steps")
    w = _hllc(W.orszag_tang(8), scheme)
    s, A, tr, dts = _run_both(w, 30)
    np.testing.assert_allclose(dts[:, 0, 0], tr[:, 0, 0], rtol=1e-11)
    _check(w, s.state_by_key(), A.state, TOL64, f"{scheme}+hllc OT 30 steps", ch=tr[-1, :, 1])


@pytest.mark.parametrize("ndim,bc,scheme", [(2, "periodic", "lf"), (2, "outflow", "weno"),
                                            (3, "mixed", "lf"), (3, "periodic", "weno")])
def test_hllc_amr_tree_steps_fp64(dev, ndim, bc, scheme):
    _say(f"hllc amr tree ndim={ndim} bc={bc} {scheme} 5 cycles")
    sims, keys = _tree(ndim, 61 + ndim + len(bc), bc)
    w = W.Workload(name="tree", ndim=ndim, sims=sims, keys=keys, ic=_tree_ic, scheme=scheme,
                   riemann="hllc")
    s, A, tr, dts = _run_both(w, 5)
    np.testing.assert_allclose(dts[:, 0, 0], tr[:, 0, 0], rtol=1e-12)
    _check(w, s.state_by_key(), A.state, TOL64, f"hllc tree {scheme} 5 cycles", ch=tr[-1, :, 1])


def test_hllc_harris_resistive_3d_fp64(dev):
    _say("lf+hllc harris 3d small, eta, fastspeed GLM, 4 steps")
    w = _hllc(W.harris3d(nbase=2, levels=3, precision="fp64"))
    s, A, tr, dts = _run_both(w, 4)
    np.testing.assert_allclose(dts[:, 0, :4], tr[:, 0], rtol=1e-12)
    _check(w, s.state_by_key(), A.state, TOL64, "hllc harris 4 steps", ch=tr[-1, :, 1])


def test_hllc_blast3d_weno_fp64(dev):
    _say("weno+hllc blast 3d small fp64 5 steps")
    w = _hllc(W.blast3d(nbase=2, levels=2, precision="fp64"), "weno")
    s, A, tr, dts = _run_both(w, 5)
    _check(w, s.state_by_key(), A.state, TOL64, "weno+hllc blast 5 steps", ch=tr[-1, :, 1])


def _contact_ic(wl, sim, lv, x, y, z, g):
    rho = np.where((x > 0.25) & (x < 0.75), 2.0, 0.5)
    zero = 0.0 * x
    return [rho, zero, zero, zero, 0.7 + zero, -0.3 + zero, 0.2 + zero, 1.0 + zero, zero]


@pytest.mark.parametrize("scheme", ["lf", "weno"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_hllc_stationary_contact_stays(dev, scheme, precision):
    """A density jump at rest with equal pressure and field on a 2-level tree
    stays in place over whole cycles (prolongation, reflux and restriction
    included)."""
    _say(f"hllc stationary contact {scheme} {precision}")
    sims, keys = _tree(2, 71, "periodic", levels=2)
    w = W.Workload(name="contact", ndim=2, sims=sims, keys=keys, ic=_contact_ic, scheme=scheme,
                   riemann="hllc", precision=precision)
    s = _sim(w)
    u0 = _leaf_interiors(w, s.state_by_key())
    s.graph_run(6)
    u1 = _leaf_interiors(w, s.state_by_key())
    tol = 1e-12 if precision == "fp64" else 1e-5
    # momentum is zero: its change is measured against 1
    scale = np.maximum(np.abs(u0[:, :8]).max(axis=(0, 2, 3, 4)), 1.0)
    err = np.abs(u1[:, :8] - u0[:, :8]).max(axis=(0, 2, 3, 4)) / scale
    _say(f"  max change per variable (relative, momentum absolute) {np.array2string(err, precision=2)}")
    assert np.all(err <= tol)


def test_hllc_fp32_l1_vs_fp64_oracle(dev):
    """WENO + HLLC in FP32 against the FP64 oracle on OT: relative L1 of rho,
    e and |B| <= 1e-4 after 30 steps."""
    import oracle as orc
    _say("weno+hllc fp32 vs fp64 oracle OT 30 steps")
    w = _hllc(W.orszag_tang(8, precision="fp32"), "weno")
    s = _sim(w)
    A = orc.load_workload(w)
    s.advance(30)
    A.run(30)
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


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_hllc_uniform_state_bitwise_3d(dev, precision):
    _say(f"hllc uniform state 3d {precision}")
    sims, keys = _tree(3, 16, "mixed")
    w = W.Workload(name="uni", ndim=3, sims=sims, keys=keys, precision=precision, scheme="weno",
                   riemann="hllc", eta=1e-3, glm_mode="fastspeed",
                   ic=lambda wl, s, lv, x, y, z, g: [1.2, 0.3, -0.2, 0.1, 0.4, 0.5, -0.6, 0.9, 0.0])
    s = _sim(w)
    u0 = s.U.clone()
    s.graph_run(2)
    s.advance(1)
    s.fill()
    s.sync()
    assert torch.equal(s.U, u0)
