"""Pins of the oracle's LF and MMC schemes (Sec. 3 of the paper) against
textbook reductions, closed forms and exact invariants."""
import math

import numpy as np
import pytest

from paper_1204_5849_amd import workloads as W


# ---------------------------------------------------------------- scalar reductions
def _scalar_1d(orc, scheme, limiter, a, N=48, seed=3):
    """One step of the oracle on a 1-D periodic scalar profile (a 2-D tile one
    cell high, uniform in y) -> (u0, u1, nu)."""
    rng = np.random.default_rng(seed)
    p = orc.make_params(ndim=2, physics=orc.SCALAR, scheme=scheme, limiter=limiter,
                        adv=(a, 0.0, 0.0))
    x = np.arange(N)
    u0 = np.sin(2 * np.pi * x / N) + 0.3 * rng.normal(size=N) * (x % 7 == 0)
    u0 += np.where((x > N // 3) & (x < N // 2), 1.0, 0.0)
    tile = np.zeros(orc.tile_shape(p, (N, 1, 1)))
    tile[0, 0, :, 2:-2] = u0
    orc.grid_fill(p, tile, (N, 1, 1), [("periodic", "periodic")] * 3)
    dx = 1.0 / N
    nu = 0.37 * np.sign(a)
    dt = abs(nu) * dx / abs(a)
    rec = orc.make_dtrec(dt, ch=0.0, damp=1.0, alpha=abs(a))
    u1, _, _ = orc.step_tile(p, (dx, dx), tile, (N, 1, 1), rec)
    return u0, u1[0, 0, 0], nu


def _mm(a, b):
    return np.where(a * b > 0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)), 0.0)


@pytest.mark.parametrize("a", [1.3, -0.8])
def test_lf_scalar_is_muscl_hancock(orc, a):
    """Linear advection: the LF scheme is the MUSCL-Hancock upwind scheme,
    f_{i+1/2} = a (u_i + (1 - nu) D_i / 2) for a > 0 (mirror for a < 0)."""
    u0, u1, nu = _scalar_1d(orc, "lf", "minmod", a)
    up, um = np.roll(u0, -1), np.roll(u0, 1)
    D = _mm(u0 - um, up - u0)
    if a > 0:
        f = a * (u0 + 0.5 * (1 - nu) * D)               # face i+1/2
    else:
        f = a * (up - 0.5 * (1 + nu) * np.roll(D, -1))  # face i+1/2 from the right cell
    want = u0 - nu / a * (f - np.roll(f, 1))
    np.testing.assert_allclose(u1, want, rtol=0, atol=1e-13)


def _phi(r, kind):
    if kind == "minmod":
        return np.maximum(0.0, np.minimum(1.0, r))
    return (r + np.abs(r)) / (1.0 + np.abs(r))


@pytest.mark.parametrize("limiter", ["minmod", "vanleer"])
def test_mmc_scalar_is_sweby_lax_wendroff(orc, limiter):
    """Linear advection with alpha = a: MMC is Sweby's flux-limited
    Lax-Wendroff scheme f = a u_i + phi(r_i) a (1 - nu)(u_{i+1} - u_i)/2."""
    a = 1.1
    u0, u1, nu = _scalar_1d(orc, "mmc", limiter, a)
    up, um = np.roll(u0, -1), np.roll(u0, 1)
    dplus, dminus = up - u0, u0 - um
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(dplus != 0, dminus / np.where(dplus == 0, 1, dplus), 0.0)
    f = a * u0 + 0.5 * _phi(r, limiter) * a * (1 - nu) * dplus
    want = u0 - nu / a * (f - np.roll(f, 1))
    np.testing.assert_allclose(u1, want, rtol=0, atol=1e-13)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("scheme", ["mmc", "lf"])
def test_3d_scalar_along_each_axis(orc, scheme, axis):
    """A 3-D tile whose data varies along one axis only, advected along that
    axis: every line is the 1-D textbook scheme (Sweby's limited
    Lax-Wendroff for MMC, MUSCL-Hancock upwind for LF), so a stride or sign
    slip in any one dimension of the 3-D code shows."""
    a, N = 1.1, 24
    adv = [0.0, 0.0, 0.0]
    adv[axis] = a
    p = orc.make_params(ndim=3, physics=orc.SCALAR, scheme=scheme, limiter="minmod", adv=adv)
    n = [4, 4, 4]
    n[axis] = N
    x = np.arange(N)
    u0 = np.sin(2 * np.pi * x / N) + np.where((x > N // 3) & (x < N // 2), 1.0, 0.0)
    tile = np.zeros(orc.tile_shape(p, n))
    shape = [1, 1, 1]
    shape[2 - axis] = N
    sl = [slice(2, -2)] * 3
    tile[(0, *sl)] = np.broadcast_to(u0.reshape(shape), tile[(0, *sl)].shape)
    orc.grid_fill(p, tile, n, [("periodic", "periodic")] * 3)
    nu = 0.37
    dt = nu / (a * N)
    rec = orc.make_dtrec(dt, ch=0.0, damp=1.0, alpha=a)
    u1, _, _ = orc.step_tile(p, (1 / N, 1 / N, 1 / N), tile, n, rec)
    line = np.moveaxis(u1[0], 2 - axis, 0)[:, 0, 0]
    up, um = np.roll(u0, -1), np.roll(u0, 1)
    dplus, dminus = up - u0, u0 - um
    if scheme == "mmc":
        with np.errstate(divide="ignore", invalid="ignore"):
            r = np.where(dplus != 0, dminus / np.where(dplus == 0, 1, dplus), 0.0)
        f = a * u0 + 0.5 * _phi(r, "minmod") * a * (1 - nu) * dplus
    else:
        f = a * (u0 + 0.5 * (1 - nu) * _mm(dminus, dplus))
    want = u0 - nu / a * (f - np.roll(f, 1))
    np.testing.assert_allclose(line, want, rtol=0, atol=1e-13)
    # and the tile is still uniform across the other two axes
    assert np.all(np.moveaxis(u1[0], 2 - axis, 0) == line[:, None, None])


def test_mmc_without_limiter_is_first_order_rusanov(orc):
    """With the flux limiter switched to zero correction (constant data on one
    side), MMC's base flux h is the Lax-Friedrichs-split upwind flux."""
    p = orc.make_params(ndim=2, physics=orc.SCALAR, scheme="mmc", adv=(0.9, 0, 0))
    N = 16
    tile = np.zeros(orc.tile_shape(p, (N, 1, 1)))
    tile[0, 0, :, 2:-2] = np.where(np.arange(N) < 8, 1.0, 0.0)  # a step: g+ ratios give phi = 0
    orc.grid_fill(p, tile, (N, 1, 1), [("periodic", "periodic")] * 3)
    rec = orc.make_dtrec(0.01, alpha=0.9)
    u1, _, _ = orc.step_tile(p, (1 / N, 1 / N), tile, (N, 1, 1), rec)
    u0 = tile[0, 0, 2, 2:-2]
    nu = 0.9 * 0.01 * N
    # at the two discontinuities the limited correction vanishes: upwind update
    assert u1[0, 0, 0, 8] == pytest.approx(u0[8] - nu * (u0[8] - u0[7]), abs=1e-15)


# ---------------------------------------------------------------- MHD invariants
def _uniform_tile(orc, p, n, w):
    tile = np.zeros(orc.tile_shape(p, n))
    u = orc.prim_to_cons(p, np.array(w, dtype=float).reshape(9, 1)).ravel()
    for k in range(9):
        tile[k] = u[k]
    return tile


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("scheme,limiter", [("lf", "minmod"), ("lf", "vanleer"), ("mmc", "vanleer"),
                                            ("mmc", "minmod"), ("weno", "minmod")])
def test_uniform_state_is_preserved_bitwise(orc, ndim, scheme, limiter):
    p = orc.make_params(ndim=ndim, scheme=scheme, limiter=limiter, eta=1e-3 if ndim == 3 else 0.0)
    n = (8, 8, 8) if ndim == 3 else (12, 12, 1)
    w = [1.3, 0.2, -0.4, 0.7, 0.5, -0.3, 0.9, 0.8, 0.0]
    tile = _uniform_tile(orc, p, n, w)
    u0 = tile.copy()
    dx = (1 / n[0],) * 3
    orc.grid_run(p, dx, tile, n, [("periodic", "periodic")] * 3, 3)
    assert np.array_equal(tile, u0)


@pytest.mark.parametrize("scheme", ["lf", "mmc", "weno"])
def test_psi_of_uniform_field_decays_by_cd_per_step(orc, scheme):
    """Uniform state with psi0 != 0: only the damping term acts, psi_k = psi0 c_d^k
    (once per step also with the two Runge-Kutta stages of WENO)."""
    p = orc.make_params(ndim=2, cd=0.18, scheme=scheme)
    n = (8, 8, 1)
    tile = _uniform_tile(orc, p, n, [1.0, 0.1, 0.2, 0.0, 0.3, 0.4, 0.0, 1.0, 0.5])
    u0 = tile.copy()
    k = 5
    orc.grid_run(p, (1 / 8, 1 / 8), tile, n, [("periodic", "periodic")] * 3, k)
    assert np.array_equal(tile[:8], u0[:8])
    np.testing.assert_allclose(tile[8], 0.5 * 0.18 ** k, rtol=2 * k * 2.3e-16)


def _ot_grid(orc, p, N):
    w = W.orszag_tang(nbase=N // 16)
    prim = w.primitive_blocks(np.arange(len(w.keys)))  # [nb,9,1,16,16]
    nb = N // 16
    big = np.zeros(orc.tile_shape(p, (N, N, 1)))
    for b, (s, lv, ix, iy, iz) in enumerate(w.keys):
        big[:, 0, 2 + iy * 16:2 + (iy + 1) * 16, 2 + ix * 16:2 + (ix + 1) * 16] = prim[b][:, 0]
    big[:] = orc.prim_to_cons(p, big)
    return big, w


@pytest.mark.parametrize("scheme,limiter", [("lf", "minmod"), ("mmc", "vanleer"), ("weno", "minmod")])
def test_glm_conserves_on_periodic_grid(orc, scheme, limiter):
    """Plain GLM (EGLM sources off): mass, momentum, energy and B totals are
    conserved to rounding on a periodic grid; mean psi decays by c_d per step."""
    p = orc.make_params(ndim=2, scheme=scheme, limiter=limiter, eglm_sources=False)
    N = 64
    big, _ = _ot_grid(orc, p, N)
    rng = np.random.default_rng(5)
    big[8, 0, 2:-2, 2:-2] = 0.01 * rng.normal(size=(N, N))  # nonzero psi
    t0 = big[:, 0, 2:-2, 2:-2].sum(axis=(1, 2))
    k = 20
    orc.grid_run(p, (1 / N, 1 / N), big, (N, N, 1), [("periodic", "periodic")] * 3, k)
    t1 = big[:, 0, 2:-2, 2:-2].sum(axis=(1, 2))
    scale = np.abs(big[:8, 0, 2:-2, 2:-2]).sum(axis=(1, 2))
    assert np.all(np.abs(t1[:8] - t0[:8]) <= 1e-13 * scale)
    assert t1[8] == pytest.approx(t0[8] * 0.18 ** k, rel=1e-9, abs=1e-12 * abs(t0[8]))


def test_eglm_sources_closed_form(orc):
    """Linear B and psi: central differences are exact, so the sources are
    -(div B) B and -B.grad(psi) with div B = c_x + c_y and grad psi = (0, q)."""
    p = orc.make_params(ndim=2)
    n = (8, 8, 1)
    dx = (0.1, 0.05)
    tile = np.zeros(orc.tile_shape(p, n))
    ys, xs = np.meshgrid(np.arange(-2, 10) + 0.5, np.arange(-2, 10) + 0.5, indexing="ij")
    X, Y = xs * dx[0], ys * dx[1]
    cx, cy, q = 0.7, -0.3, 1.9
    tile[0] = 1.0
    tile[4, 0] = 0.2 + cx * X
    tile[5, 0] = -0.1 + cy * Y
    tile[6, 0] = 0.4
    tile[8, 0] = q * Y
    S = orc.eglm_source(p, dx, tile, n)
    B = tile[4:7, 0, 2:-2, 2:-2]
    div = cx + cy
    for j in range(3):
        np.testing.assert_allclose(S[1 + j, 0], -div * B[j], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(S[7, 0], -B[1] * q, rtol=1e-12, atol=1e-14)
    assert np.all(S[[0, 4, 5, 6, 8]] == 0)


@pytest.mark.parametrize("ndim", [2, 3])
def test_resistive_sine_mode_closed_form(orc, ndim):
    """B_z = A sin(kx): R_z = -eta A sin(kx) sin^2(k dx)/dx^2 and
    R_e = eta A^2 sin(k dx) sin(2k dx) cos(2kx) / (2 dx^2)."""
    eta, A = 0.01, 0.7
    p = orc.make_params(ndim=ndim, eta=eta)
    N = 16
    n = (N, 4, 4) if ndim == 3 else (N, 4, 1)
    dx = 1.0 / N
    k = 2 * np.pi
    tile = np.zeros(orc.tile_shape(p, n))
    xc = (np.arange(-2, N + 2) + 0.5) * dx
    tile[0] = 1.0
    tile[6] = A * np.sin(k * xc)[None, None, :]
    R = orc.resistive(p, (dx, dx, dx), tile, n)
    x = (np.arange(N) + 0.5) * dx
    Rz = -eta * A * np.sin(k * x) * np.sin(k * dx) ** 2 / dx ** 2
    Re = eta * A * A * np.sin(k * dx) * np.sin(2 * k * dx) * np.cos(2 * k * x) / (2 * dx ** 2)
    np.testing.assert_allclose(R[6], np.broadcast_to(Rz, R[6].shape), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(R[7], np.broadcast_to(Re, R[7].shape), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(R[4], 0, atol=1e-14)
    np.testing.assert_allclose(R[5], 0, atol=1e-14)


def test_resistive_rotated_mode(orc):
    """B_x = A sin(k z) in 3-D: R_x = -eta A sin(kz) sin^2(k dz)/dz^2."""
    eta, A = 0.02, 0.3
    p = orc.make_params(ndim=3, eta=eta)
    N = 16
    n = (4, 4, N)
    dz = 1.0 / N
    k = 2 * np.pi
    tile = np.zeros(orc.tile_shape(p, n))
    zc = (np.arange(-2, N + 2) + 0.5) * dz
    tile[0] = 1.0
    tile[4] = A * np.sin(k * zc)[:, None, None]
    R = orc.resistive(p, (0.25, 0.25, dz), tile, n)
    z = (np.arange(N) + 0.5) * dz
    want = -eta * A * np.sin(k * z) * np.sin(k * dz) ** 2 / dz ** 2
    np.testing.assert_allclose(R[4], np.broadcast_to(want[:, None, None], R[4].shape), rtol=1e-11,
                               atol=1e-13)


def test_dt_record_modes(orc):
    """dt = c_cfl dx/(n_dim alpha); PAPER: c_h = c_cfl dx/dt and factor c_d;
    FASTSPEED: c_h = alpha and factor exp(-dt c_h / c_r); eta caps dt."""
    p = orc.make_params(ndim=3, glm_mode="paper")
    r = orc.dtrec(p, 2.0, 0.01)
    assert r.dt == pytest.approx(0.4 * 0.01 / 6.0, rel=1e-15)
    assert r.ch == pytest.approx(0.4 * 0.01 / r.dt, rel=1e-15)
    assert r.damp == 0.18
    p = orc.make_params(ndim=3, glm_mode="fastspeed", cr=0.18)
    r = orc.dtrec(p, 2.0, 0.01)
    assert r.ch == 2.0 and r.damp == pytest.approx(math.exp(-r.dt * 2.0 / 0.18), rel=1e-15)
    p = orc.make_params(ndim=2, eta=10.0)
    r = orc.dtrec(p, 1.0, 0.01)
    assert r.dt == pytest.approx(0.4 * 1e-4 / (2 * 10.0), rel=1e-15)


def test_lf_positivity_fallback_keeps_state_admissible(orc):
    """Fast flow at nearly zero pressure: limited face states of the energy
    undershoot the kinetic energy, the fall-back zeroes those slopes, and the
    result stays finite."""
    p = orc.make_params(ndim=2)
    N = 16
    n = (N, N, 1)
    tile = np.zeros(orc.tile_shape(p, n))
    w = np.zeros((9, 1, N + 4, N + 4))
    w[0] = 1.0
    w[7] = 1e-6
    w[1] = 3.0 * np.sin(2 * np.pi * (np.arange(N + 4) - 2 + 0.5) / N)[None, None, :]
    w[4] = 0.5
    tile[:] = orc.prim_to_cons(p, w)
    orc.grid_fill(p, tile, n, [("periodic", "periodic")] * 3)
    rec = orc.dtrec(p, orc.tile_maxspeed(p, tile, n), 1 / N)
    u1, _, cnt = orc.step_tile(p, (1 / N, 1 / N), tile, n, rec)
    assert np.all(np.isfinite(u1))
    assert cnt[0] + cnt[1] > 0


# ---------------------------------------------------------------- positivity fall-back
# Hand-computed pins of the reading of Sec. 3.2 (the slopes of limiter1 and the
# face states of limiter2): a cell any of whose 2d limited face states has
# rho <= 0 or p <= 0 takes zero slopes in EVERY dimension for the step; a
# corrector face state with rho <= 0 or p <= 0 is replaced by the predicted
# state u~ of its own cell (not by u^n).  Every number below is worked out by
# hand in the comments and is exact in binary.

def _cons_tile(orc, p, n):
    """Padded tile of rho = 1, m = 0, B = 0, psi = 0 (conserved variables)."""
    t = np.zeros(orc.tile_shape(p, n))
    t[0] = 1.0
    return t


def test_lf_fallback_zeroes_every_slope_of_the_cell(orc):
    """2-D tile of 5 x 5 cells, gamma = 5/3.  Background rho = 1, m = 0,
    e = 1/4.  Row y = 2: m_x = 0 | 1 | 2 and e = 1/4 | 3/4 | 9/4 left of,
    at and right of the cell c = (2, 2) (e = m^2/2 + 1/4, so p = 1/6 in each
    cell), and rho = 1/2 below c, 3/2 above it.

    Limited slopes of c (minmod): x: dm = min(1, 1) = 1, de = min(1/2, 3/2)
    = 1/2; y: drho = min(1/2, 1/2) = 1/2, every other slope 0.  Its right
    x face state (rho 1, m 3/2, e 1) has e - m^2/(2 rho) = -1/8 < 0, so the
    cell falls back.  Every other cell's slopes are 0 (each sits next to a
    flat side).  With all slopes 0 the predictor moves nothing: u~ = u
    exactly.  Resetting only the x slopes would leave drho_y = 1/2, whose
    pressure difference moves m_y; not resetting at all moves rho, m_x, e."""
    p = orc.make_params(ndim=2, gamma=5.0 / 3.0, eglm_sources=False)
    n = (5, 5, 1)
    u = _cons_tile(orc, p, n)
    u[7] = 0.25
    Y, X = 2 + 2, 2 + 2                       # padded indices of c
    u[1, 0, Y, :X] = 0.0
    u[1, 0, Y, X] = 1.0
    u[1, 0, Y, X + 1:] = 2.0
    u[7, 0, Y, :X] = 0.25
    u[7, 0, Y, X] = 0.75
    u[7, 0, Y, X + 1:] = 2.25
    u[0, 0, Y - 1, X] = 0.5
    u[0, 0, Y + 1, X] = 1.5
    assert all(orc.pressure(p, u[:, 0, j, i]) > 0 for j in range(9) for i in range(9))
    rec = orc.make_dtrec(0.01, ch=0.0, damp=1.0, alpha=3.0)
    ut, sl, lr, cnt = orc.lf_states(p, (0.1, 0.1), u, n, rec)
    assert cnt[0] == 1 and cnt[1] == 0
    assert np.all(sl[:, :, 0, Y, X] == 0.0)
    assert np.all(sl == 0.0)
    # u~ = u on the predictor's region (the interior and one ring)
    np.testing.assert_array_equal(ut[:, :, 1:-1, 1:-1], u[:, :, 1:-1, 1:-1])
    # so every face flux receives the cells' own states
    np.testing.assert_array_equal(lr[0, 0, :, 0, Y, X], u[:, 0, Y, X])
    np.testing.assert_array_equal(lr[0, 1, :, 0, Y, X - 1], u[:, 0, Y, X])
    np.testing.assert_array_equal(lr[1, 0, :, 0, Y, X], u[:, 0, Y, X])


def test_lf_fallback_face_state_is_the_predicted_state(orc):
    """A row of 5 cells (2-D tile one cell high), gamma = 3/2, dt/dx = 1/4.
    rho = 1; m_x = -2 | 0 | 2 and e = 3 | 3/4 | 3 left of, at and right of
    the cell c = 2 (p = 1/2, 3/8, 1/2).

    Slopes of c: dm = min(2, 2) = 2, de = minmod(-9/4, 9/4) = 0; the
    neighbours' slopes are 0.  Predictor face states of c: m = +-1, e = 3/4,
    p = (3/4 - 1/2)/2 = 1/8 > 0, so no slope fall-back.  Their fluxes:
    rho: +-1; m: 1 + 1/8 on both sides; e: +-(3/4 + 1/8) = +-7/8.  So
    u~_c = (1 - (1/8)(2), 0, ..., 3/4 - (1/8)(7/4), 0) = (3/4, 0, ..., 17/32, 0).
    Corrector states of c: u~_c +- (0, 1, 0...) have e - m^2/(2 rho) =
    17/32 - 2/3 < 0, so both the left state of face c+1/2 and the right state
    of face c-1/2 become u~_c = (3/4, 0, 0, 0, 0, 0, 0, 17/32, 0); u^n_c
    would be (1, 0, ..., 3/4, 0).  The other states are the neighbours' u^n."""
    p = orc.make_params(ndim=2, gamma=1.5, eglm_sources=False)
    n = (5, 1, 1)
    u = _cons_tile(orc, p, n)
    X = 2 + 2
    u[1, 0, :, :X] = -2.0
    u[1, 0, :, X + 1:] = 2.0
    u[7] = 3.0
    u[7, 0, :, X] = 0.75
    rec = orc.make_dtrec(0.25, ch=0.0, damp=1.0, alpha=4.0)
    ut, sl, lr, cnt = orc.lf_states(p, (1.0, 1.0), u, n, rec)
    assert cnt[0] == 0 and cnt[1] == 2
    assert sl[0, 1, 0, 2, X] == 2.0 and np.count_nonzero(sl) == 3  # rows y = -1, 0, 1
    want_ut = np.array([0.75, 0, 0, 0, 0, 0, 0, 17.0 / 32.0, 0])
    np.testing.assert_array_equal(ut[:, 0, 2, X], want_ut)
    np.testing.assert_array_equal(lr[0, 0, :, 0, 2, X], want_ut)       # left state of c+1/2
    np.testing.assert_array_equal(lr[0, 1, :, 0, 2, X], u[:, 0, 2, X + 1])
    np.testing.assert_array_equal(lr[0, 1, :, 0, 2, X - 1], want_ut)   # right state of c-1/2
    np.testing.assert_array_equal(lr[0, 0, :, 0, 2, X - 1], u[:, 0, 2, X - 1])
