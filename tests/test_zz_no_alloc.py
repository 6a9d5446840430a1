"""The allocation-free totals entry point (map_totals_static, fixed device
scratch) against map_totals (workspace scratch), through the C ABI: two
calls in a row, the second on a smaller block list, each bit for bit equal
to map_totals on the same state."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1204_5849_amd import native as N  # noqa: E402
from paper_1204_5849_amd import workloads as W  # noqa: E402


def _say(msg):
    print(f"[gpu-static] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    N.lib()
    return "cuda:0"


def _totals_both(sim):
    ns = len(sim.wl.sims)
    a = torch.full((ns, 9), -1.0, dtype=torch.float64, device=sim.device)
    b = torch.full((ns, 9), -2.0, dtype=torch.float64, device=sim.device)
    torch.cuda.synchronize()
    N.map_totals(sim.ctx, sim.U, a, sim.sp)
    N.map_totals_static(sim.ctx, sim.U, b, sim.sp)
    sim.sync()
    return a.cpu().numpy(), b.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_totals_static_equals_totals(dev, precision):
    from paper_1204_5849_amd.sim import Simulation
    big = W.harris3d(nbase=2, levels=4, precision=precision)
    small = W.kh_ensemble(nsims=3, precision=precision)
    nb, ns = int(big.leaf_mask().sum()), int(small.leaf_mask().sum())
    assert ns < nb
    for w in (big, small):
        sim = Simulation(w, precision=precision)
        sim.load_initial()
        sim.advance(2)
        want, got = _totals_both(sim)
        _say(f"{w.name} {precision}: {int(w.leaf_mask().sum())} leaves, "
             f"{len(w.sims)} simulation(s), totals[0][:3] {want[0][:3]}")
        assert np.array_equal(got, want)
        assert np.all(np.isfinite(got))
        del sim
