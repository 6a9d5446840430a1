"""Launch shapes (the autotuner's search space) change nothing in the
results: every workgroup shape, persistent grid and restriction split gives
the state of the default launch bit for bit."""
import dataclasses

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1204_5849_amd import native as N  # noqa: E402
from paper_1204_5849_amd import workloads as W  # noqa: E402
from tests.test_gpu_parity import _sim, _tree, _tree_ic  # noqa: E402


def _say(msg):
    print(f"[gpu-launch] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    N.lib()
    return "cuda:0"


CONFIGS = [dict(step_shape=1), dict(grid_step=256, grid_fill=256), dict(restrict_split=0),
           dict(restrict_split=1 << 30), dict(step_shape=1, grid_step=512, restrict_split=64),
           dict(cfl_in_update=1), dict(cfl_in_update=1, step_shape=1, grid_step=256),
           dict(cfl_in_update=0)]


@pytest.mark.parametrize("ndim,scheme,precision", [(2, "lf", "fp64"), (2, "weno", "fp32"),
                                                   (3, "lf", "fp32"), (3, "weno", "fp32")])
def test_launch_shapes_give_the_same_state(dev, ndim, scheme, precision):
    sims, keys = _tree(ndim, 61 + ndim, "mixed")
    w = W.Workload(name="tree", ndim=ndim, sims=sims, keys=keys, ic=_tree_ic, scheme=scheme,
                   precision=precision, eta=1e-3 if ndim == 3 else 0.0)
    ref = _sim(w)
    ref.graph_run(3)
    ref.fill()
    want = ref.state_by_key()
    for cfg in CONFIGS:
        s = _sim(w)
        s.set_launch_config(**cfg)
        got_cfg = s.launch_config()
        s.graph_run(3)
        s.fill()
        _say(f"ndim={ndim} {scheme} {precision} {got_cfg}")
        assert np.array_equal(s.state_by_key(), want), cfg


def test_autotune_picks_from_its_search_space(dev):
    w = dataclasses.replace(W.harris3d(nbase=4, levels=3, precision="fp32"))
    s = _sim(w)
    u0 = s.state_by_key()
    cfg = s.autotune()
    _say(f"harris 64^3 L3 fp32 autotuned: {cfg}")
    assert cfg["step_shape"] in (0, 1) and cfg["grid_step"] % 256 == 0
    assert cfg["restrict_split"] >= 0
    # the trials leave U's interiors and parent frames as they were
    leaves = w.leaf_mask()
    got = s.state_by_key()
    assert np.array_equal(got[leaves][:, :, 2:-2, 2:-2, 2:-2], u0[leaves][:, :, 2:-2, 2:-2, 2:-2])


@pytest.mark.parametrize("poke", ["e0", "nan"])
def test_cfl_in_update_counts_like_the_cfl_pass(dev, poke):
    """The 2-D LF update's CFL maxima (map_launch.cfl_in_update) count the
    cells with p <= 0 and the non-finite cells exactly as the CFL pass does:
    a cell poked from the host, then cycles whose dt chain through the
    update, give the same counters, status and state with it on and off."""
    w = W.orszag_tang(2)
    got = []
    for on in (0, 1):
        s = _sim(w)
        s.set_launch_config(cfl_in_update=on)
        assert s.launch_config()["cfl_in_update_on"] == on
        s.advance(1)
        s.flags()
        slot = int(s.slot_of_key[0])
        if poke == "e0":
            s.U[slot, 7, 0, 5, 5] = 0.0  # e = 0 -> negative pressure
        else:
            s.U[slot, 0, 0, 6, 6] = float("nan")
        s.advance(3)
        st, cnt = s.flags()
        _say(f"poke {poke} cfl_in_update={on}: status {st} counters {list(cnt)}")
        got.append((st, list(cnt), s.state_by_key()))
    assert got[0][0] == got[1][0] and got[0][1] == got[1][1]
    assert got[0][1][2] + got[0][1][3] >= 1
    assert np.array_equal(got[0][2], got[1][2], equal_nan=True)
