"""Pins of the oracle's WENO scheme with TVD Runge-Kutta 2 (Sec. 3.3 of the
paper): the face reconstruction against textbook exactness and symmetry
properties, the scheme against the paper's accuracy tables (Sec. 5.1, 5.3)
and against conservation and uniform-state invariants."""
import numpy as np
import pytest

from tests.test_oracle_convergence import _adv1d_l1, _adv2d_l1, _table
from tests.helpers import order


# ---------------------------------------------------------------- face states
def test_weno_face_exact_for_parabola_cell_averages(orc):
    """Cell averages of c + k x^2 about the cell centre (u_{i-1} = u_{i+1}):
    both smoothness weights are equal, the reconstruction is the third-order
    one, and the point value of the parabola at the face is recovered."""
    for c, k in [(0.0, 1.0), (0.3, -2.5), (1.7, 0.01)]:
        avg = lambda j: c + k * (j * j + 1.0 / 12.0)  # mean of c + k x^2 over [j-1/2, j+1/2]
        face = c + k * 0.25
        assert orc.weno_face(avg(-1), avg(0), avg(1), 0) == pytest.approx(face, rel=1e-14, abs=1e-15)
        assert orc.weno_face(avg(-1), avg(0), avg(1), 1) == pytest.approx(face, rel=1e-14, abs=1e-15)


def test_weno_face_exact_for_linear_data(orc):
    """Both candidate stencils are exact on linear data, so is their blend."""
    for a, b in [(0.2, 1.0), (-3.0, 0.125), (5.0, -7.5)]:
        u = [a + b * j for j in (-1, 0, 1)]
        assert orc.weno_face(*u, 0) == pytest.approx(a + 0.5 * b, rel=1e-14, abs=1e-14)
        assert orc.weno_face(*u, 1) == pytest.approx(a - 0.5 * b, rel=1e-14, abs=1e-14)


def test_weno_face_mirror_symmetry(orc):
    """The right state of the left face is the left state of the right face of
    the mirrored data; this fixes the reading of the garbled denominator."""
    rng = np.random.default_rng(11)
    for um, u0, up in rng.normal(size=(200, 3)):
        assert orc.weno_face(um, u0, up, 1) == orc.weno_face(up, u0, um, 0)


def test_weno_face_blends_the_two_candidates(orc):
    """The face value is a convex blend of the two second-order candidates
    (the centred average with the downwind cell and the upwind extrapolation)."""
    rng = np.random.default_rng(12)
    for um, u0, up in rng.normal(size=(200, 3)):
        c1, c2 = 0.5 * (u0 + up), 0.5 * (3 * u0 - um)
        f = orc.weno_face(um, u0, up, 0)
        assert min(c1, c2) - 1e-14 <= f <= max(c1, c2) + 1e-14


def test_weno_face_is_essentially_non_oscillatory_at_a_step(orc):
    """Across a jump the weight of the stencil crossing it vanishes: no new
    extremum is created at the face next to the jump."""
    assert abs(orc.weno_face(0.0, 0.0, 1.0, 0)) < 1e-20
    assert orc.weno_face(0.0, 1.0, 1.0, 0) == pytest.approx(1.0, abs=1e-20)
    assert orc.weno_face(1.0, 1.0, 0.0, 1) == pytest.approx(1.0, abs=1e-20)


# ---------------------------------------------------------------- one stage
def test_weno_scalar_stage_mirror_symmetry(orc):
    """Linear advection, a > 0 on a profile and a < 0 on its mirror image give
    mirrored results: the left and right states are taken from the right cells."""
    rng = np.random.default_rng(4)
    N = 40
    u0 = np.sin(2 * np.pi * np.arange(N) / N) + np.where(np.arange(N) % 9 == 0, 0.7, 0.0)
    u0 += 0.1 * rng.normal(size=N)
    out = []
    for a, prof in [(1.3, u0), (-1.3, u0[::-1].copy())]:
        p = orc.make_params(ndim=2, physics=orc.SCALAR, scheme="weno", adv=(a, 0.0, 0.0))
        tile = np.zeros(orc.tile_shape(p, (N, 1, 1)))
        tile[0, 0, :, 2:-2] = prof
        orc.grid_fill(p, tile, (N, 1, 1), [("periodic", "periodic")] * 3)
        rec = orc.make_dtrec(0.3 / N / 1.3, alpha=1.3)
        u1, _, _ = orc.step_tile(p, (1 / N, 1 / N), tile, (N, 1, 1), rec)
        out.append(u1[0, 0, 0])
    np.testing.assert_allclose(out[0], out[1][::-1], rtol=0, atol=1e-14)


# ---------------------------------------------------------------- accuracy tables
def test_table2_advection1d_weno(orc):
    """Table 2's WENO rows: magnitudes within 15 %, order within 0.1 (one
    period at CFL 0.4; the paper does not state its final time or CFL)."""
    ref = _table("table2_advection1d.txt")
    e128 = _adv1d_l1(orc, 128, "weno", "minmod")
    e256 = _adv1d_l1(orc, 256, "weno", "minmod")
    assert e128 == pytest.approx(ref[("WENO", 128)], rel=0.15)
    assert e256 == pytest.approx(ref[("WENO", 256)], rel=0.15)
    assert abs(order(e128, e256) - order(ref[("WENO", 128)], ref[("WENO", 256)])) < 0.1


def test_table3_advection2d_weno_order(orc):
    """Table 3's WENO order between N = 64 and 128 (2.05) within 0.1."""
    ref = _table("table3_advection2d.txt")
    e64 = _adv2d_l1(orc, 64, "weno")
    e128 = _adv2d_l1(orc, 128, "weno")
    assert abs(order(e64, e128) - order(ref[("WENO", 64)], ref[("WENO", 128)])) < 0.1
