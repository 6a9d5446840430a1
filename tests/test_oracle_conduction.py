"""Pins of the oracle's thermal-conduction subcycle (Sec. 3.4 of the paper;
the field-aligned form of its conduction test): closed forms of the
isotropic scheme and of the operator along the field, the sub-step time
step, conservation with reflux, and the paper's comparison of the subcycle
against conduction at every step."""
import math

import numpy as np
import pytest

from paper_1204_5849_amd import workloads as W
from tests.helpers import random_tree

G = 5.0 / 3.0


def _tile(orc, p, n, prim_fn):
    """Padded tile with primitives prim_fn(X, Y, Z) -> 9 arrays at every padded
    cell centre (unit cell size, centres at index + 0.5)."""
    shape = orc.tile_shape(p, n)
    nz, ny, nx = shape[1:]
    g = 2
    zs = np.arange(nz) - (g if p.ndim == 3 else 0) + 0.5
    ys, xs = np.arange(ny) - g + 0.5, np.arange(nx) - g + 0.5
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    w = np.array([np.broadcast_to(v, X.shape) for v in prim_fn(X, Y, Z)], dtype=float)
    return orc.prim_to_cons(p, w)


def _interior(p, a):
    return a[:, 2:-2, 2:-2, 2:-2] if p.ndim == 3 else a[:, :, 2:-2, 2:-2]


def test_isotropic_constant_kappa_is_the_three_point_heat_step(orc):
    """rho = 1, v = B = 0, constant kappa: T = p and
    e_new = e + kappa dt/dx^2 (T_{i+1} - 2 T_i + T_{i-1}) along each axis."""
    p = orc.make_params(ndim=2, cond="iso", kappa0=0.7, kappa_exp=0.0)
    n = (16, 12, 1)
    rng = np.random.default_rng(2)
    pr = 1.0 + 0.3 * rng.random((n[1] + 4, n[0] + 4))
    u = _tile(orc, p, n, lambda X, Y, Z: [1, 0, 0, 0, 0, 0, 0, pr[None], 0])
    dx = (0.1, 0.2)
    enew, _ = orc.conduct_tile(p, dx, u, n, 0.003)
    T = pr
    lap = (T[2:-2, 3:-1] - 2 * T[2:-2, 2:-2] + T[2:-2, 1:-3]) / dx[0] ** 2 + \
          (T[3:-1, 2:-2] - 2 * T[2:-2, 2:-2] + T[1:-3, 2:-2]) / dx[1] ** 2
    want = u[7, 0, 2:-2, 2:-2] + 0.003 * 0.7 * lap
    np.testing.assert_allclose(enew[0], want, rtol=1e-13)


def test_sine_mode_decays_by_the_discrete_factor(orc):
    """Linear case: a temperature mode sin(kx) decays per sub-step by
    1 - 4 (gamma - 1) kappa dt/dx^2 sin^2(k dx/2), on a periodic grid over
    several sub-steps of the grid driver."""
    N, kappa = 32, 0.05
    p = orc.make_params(ndim=2, cond="iso", kappa0=kappa, kappa_exp=0.0, cond_max_sub=4)
    dx = 1.0 / N
    x = (np.arange(N) + 0.5) * dx
    w = np.zeros((9, 1, 5, N + 4))
    w[0] = 1.0
    w[7, 0, :, 2:-2] = 1.0 + 1e-3 * np.sin(2 * np.pi * x)
    w[7, 0, :, :2], w[7, 0, :, -2:] = w[7, 0, :, -4:-2], w[7, 0, :, 2:4]
    u = orc.prim_to_cons(p, w)
    bc = [("periodic", "periodic")] * 3
    orc.grid_fill(p, u, (N, 1, 1), bc)
    tr, _ = orc.grid_run(p, (dx, dx), u, (N, 1, 1), bc, 1)
    rec = orc.dtrec(p, orc.tile_maxspeed(p, orc.prim_to_cons(p, w), (N, 1, 1)), dx,
                    orc.tile_cond_rate(p, orc.prim_to_cons(p, w), (N, 1, 1)))
    assert rec.nsub >= 2
    # the MHD step leaves a uniform-in-velocity pressure mode nearly
    # unchanged; compare the conduction part through a pure conduction run
    q = orc.make_params(ndim=2, cond="iso", kappa0=kappa, kappa_exp=0.0)
    v = orc.prim_to_cons(q, w)
    dt = 1e-4
    for _ in range(5):
        orc.grid_fill(q, v, (N, 1, 1), bc)
        e, _ = orc.conduct_tile(q, (dx, dx), v, (N, 1, 1), dt)
        v[7, 0, 2, 2:-2] = e[0, 0]
    g = 1 - 4 * (G - 1) * kappa * dt / dx ** 2 * math.sin(math.pi * dx) ** 2
    amp = (v[7, 0, 2, 2:-2] * (G - 1) - 1.0)
    np.testing.assert_allclose(amp, 1e-3 * g ** 5 * np.sin(2 * np.pi * x), rtol=0, atol=1e-15)


def test_face_kappa_is_the_geometric_mean(orc):
    """kappa = kappa0 T^(5/2): across one face between T = 1 and T = 4 the
    flux is sqrt(kappa(1) kappa(4)) (T_R - T_L)/dx = kappa0 4^(5/4) 3/dx."""
    p = orc.make_params(ndim=2, cond="iso", kappa0=0.01, kappa_exp=2.5)
    n = (4, 1, 1)
    Tcell = np.array([1, 1, 1, 1, 4, 4, 4, 4], dtype=float)  # padded x: cells -2..5
    u = _tile(orc, p, n, lambda X, Y, Z: [1, 0, 0, 0, 0, 0, 0, Tcell[None, None, :], 0])
    dt, dx = 1e-3, 0.5
    enew, _ = orc.conduct_tile(p, (dx, dx), u, n, dt)
    q = 0.01 * 4 ** 1.25 * 3 / dx
    # the face between cells 1 and 2 is inside the tile: cell 1 gains, cell 2 loses
    assert enew[0, 0, 1] - u[7, 0, 2, 3] == pytest.approx(dt * q / dx, rel=1e-13)
    assert enew[0, 0, 2] - u[7, 0, 2, 4] == pytest.approx(-dt * q / dx, rel=1e-13)


@pytest.mark.parametrize("ndim", [2, 3])
def test_field_aligned_no_flux_across_the_field(orc, ndim):
    """B along x, T varying only across it: nothing moves (bitwise)."""
    p = orc.make_params(ndim=ndim, cond="field", kappa0=0.3, kappa_exp=2.5)
    n = (8, 8, 8 if ndim == 3 else 1)
    u = _tile(orc, p, n, lambda X, Y, Z: [1, 0, 0, 0, 0.8, 0, 0,
                                         1 + 0.2 * np.sin(Y) + 0.1 * np.cos(0.7 * Z), 0])
    enew, _ = orc.conduct_tile(p, (0.1,) * 3, u, n, 0.01)
    assert np.array_equal(enew, _interior(p, u)[7])


def test_field_aligned_linear_profile_across_an_oblique_field(orc):
    """B at 45 degrees, T linear in the direction across it: b . grad T = 0 at
    every face (the face gradients are exact for linear T)."""
    p = orc.make_params(ndim=2, cond="field", kappa0=0.3, kappa_exp=0.0)
    n = (8, 8, 1)
    u = _tile(orc, p, n, lambda X, Y, Z: [1, 0, 0, 0, 0.6, 0.6, 0, 1 + 0.05 * (X - Y), 0])
    enew, _ = orc.conduct_tile(p, (1.0, 1.0), u, n, 0.01)
    np.testing.assert_allclose(enew, _interior(p, u)[7], rtol=0, atol=1e-15)


def test_field_aligned_quadratic_along_an_oblique_field(orc):
    """B along (1, 1), T = c (x + y)^2 = 2 c s^2 with s along the field:
    div(kappa b (b.grad T)) = 4 c kappa, reproduced exactly by the face
    gradients (exact for quadratics) with constant kappa."""
    c, kappa, dt = 0.01, 0.3, 0.002
    p = orc.make_params(ndim=2, cond="field", kappa0=kappa, kappa_exp=0.0)
    n = (8, 8, 1)
    u = _tile(orc, p, n, lambda X, Y, Z: [1, 0, 0, 0, 0.6, 0.6, 0, 1 + c * (X + Y) ** 2, 0])
    enew, _ = orc.conduct_tile(p, (1.0, 1.0), u, n, dt)
    np.testing.assert_allclose(enew - _interior(p, u)[7], dt * 4 * c * kappa, rtol=1e-9)


def test_sub_step_time_step(orc):
    """dt_c = c_cfl dx^2/(n_dim kmax); the step is capped at max_sub dt_c and
    split into ceil(dt/dt_c) equal sub-steps."""
    p = orc.make_params(ndim=3, cond="iso", kappa0=1.0, cond_max_sub=6, cfl=0.4)
    alpha, dx = 2.0, 0.01
    dt_mhd = 0.4 * dx / (3 * alpha)
    kmax = 0.4 * dx * dx / (3 * (dt_mhd / 2.5))  # dt_c = dt_mhd / 2.5
    r = orc.dtrec(p, alpha, dx, kmax)
    assert r.dt == pytest.approx(dt_mhd, rel=1e-15) and r.nsub == 3
    assert r.dt_sub == pytest.approx(dt_mhd / 3, rel=1e-15)
    r = orc.dtrec(p, alpha, dx, kmax * 100)  # dt_c = dt_mhd / 250: capped at 6 dt_c
    assert r.nsub == 6 and r.dt == pytest.approx(6 * dt_mhd / 250, rel=1e-13)
    assert r.ch == pytest.approx(0.4 * dx / r.dt, rel=1e-15)
    r = orc.dtrec(orc.make_params(ndim=3), alpha, dx, kmax)
    assert r.nsub == 0 and r.dt == pytest.approx(dt_mhd, rel=1e-15)


def _hot_spot_ic(wl, sim, lv, x, y, z, g):
    zero = 0.0 * x
    rho = np.where((np.abs(x - 0.5) < 0.12) & (np.abs(y - 0.5) < 0.12), 0.05, 0.1) + zero
    return [rho, zero, zero, zero, 1.0 + zero, 1.0 + zero, zero, 0.1 + zero, zero]


@pytest.mark.parametrize("ndim,cond", [(2, "iso"), (2, "field"), (3, "field")])
def test_conduction_conserves_energy_on_amr_tree(orc, ndim, cond):
    """Periodic 2:1 tree: the subcycle with reflux keeps the total energy."""
    rng = np.random.default_rng(70 + ndim)
    nb = (2, 2, 1) if ndim == 2 else (2, 2, 2)
    sims = [W.SimDesc(lo=(0, 0, 0), hi=(1, 1, 1), nbase=nb, bc=(("periodic", "periodic"),) * 3)]
    keys = random_tree(sims, ndim, 3, 0.4, rng)
    w = W.Workload(name="cond", ndim=ndim, sims=sims, keys=keys, ic=_hot_spot_ic,
                   n=16 if ndim == 2 else 8, cond=cond, kappa0=0.01, kappa_exp=2.5,
                   cond_max_sub=5)
    A = orc.load_workload(w)
    from tests.test_oracle_amr import _exact_totals
    t0 = _exact_totals(A, w)
    r = A.cfl()
    assert r[0].nsub >= 2
    orc.lib().orc_amr_conduct(A.h, (orc.DtRec * 1)(r[0]))
    t1 = _exact_totals(A, w)
    assert abs(t1[7] - t0[7]) <= 1e-13 * abs(t0[7])
    assert np.array_equal(t1[:7], t0[:7])


def test_blocked_equals_monolithic_with_conduction(orc):
    """The subcycle on a single-level tree equals the subcycle of the
    monolithic grid bit for bit (LF and WENO, field-aligned Spitzer kappa)."""
    from tests.test_oracle_amr import _assemble
    for scheme in ("lf", "weno"):
        w = W.orszag_tang(nbase=2, scheme=scheme)
        w.cond, w.kappa0, w.kappa_exp, w.cond_max_sub = "field", 2e-4, 2.5, 4
        A = orc.load_workload(w)
        p = A.p
        big = _assemble(orc, p, w, A, 32)
        tr = A.run(3, trace=True)
        orc.grid_run(p, (1 / 32, 1 / 32), big, (32, 32, 1), [("periodic", "periodic")] * 3, 3)
        assert np.array_equal(_assemble(orc, p, w, A, 32)[:, :, 2:-2, 2:-2], big[:, :, 2:-2, 2:-2])


def _strip(orc, N, max_sub, t_end):
    """A hot strip of low density at the bottom of the unit square under an
    oblique field, with conduction along the field (the set-up of the paper's
    conduction test, periodic in x and open in y); temperature at t_end by
    linear interpolation between the two steps around it."""
    p = orc.make_params(ndim=2, scheme="weno", cond="field", kappa0=0.001, kappa_exp=2.5,
                        cond_max_sub=max_sub)
    dx = 1.0 / N
    x = -0.5 + (np.arange(-2, N + 2) + 0.5) * dx
    X, Y = np.meshgrid(x, x)
    w = np.zeros((9, 1, N + 4, N + 4))
    w[0, 0] = np.where((np.abs(X) < 0.1) & (Y < -0.4), 0.01, 0.1)
    w[4], w[5], w[7] = 1.0, 1.0, 0.1
    u = orc.prim_to_cons(p, w)
    bc = [("periodic", "periodic"), ("outflow", "outflow"), ("periodic", "periodic")]

    def temp():
        i = orc.interior(p, u)[:, 0]
        ke = 0.5 * (i[1] ** 2 + i[2] ** 2 + i[3] ** 2) / i[0]
        me = 0.5 * (i[4] ** 2 + i[5] ** 2 + i[6] ** 2)
        return (p.gamma - 1) * (i[7] - ke - me) / i[0]

    t, T0 = 0.0, temp()
    while True:
        tr, _ = orc.grid_run(p, (dx, dx), u, (N, N, 1), bc, 1)
        T1 = temp()
        if t + tr[0] >= t_end:
            return T0 + (t_end - t) / tr[0] * (T1 - T0)
        t, T0 = t + tr[0], T1


def test_subcycle_approaches_conduction_at_every_step(orc):
    """The paper compares its subcycle with conduction at every step (a time
    step limited by conduction): fewer, shorter MHD steps per sub-step bring
    the two closer, and with up to 20 sub-steps per step the temperatures
    differ by a few per cent at most in the hot region."""
    ref = _strip(orc, 32, 1, 0.004)
    diffs = [np.abs(_strip(orc, 32, m, 0.004) - ref).max() / ref.max() for m in (20, 5, 2)]
    assert diffs[0] > diffs[1] > diffs[2] > 0
    assert diffs[0] < 0.05


@pytest.mark.parametrize("d", [0, 1, 2])
def test_field_aligned_mirror_symmetry(orc, d):
    """Reflecting a tile along d (B_d and v_d change sign) reflects the
    conduction update: the face field is the mean of the two cells', so
    neither side is preferred."""
    p = orc.make_params(ndim=3, cond="field", kappa0=0.05, kappa_exp=2.5)
    n = (6, 6, 6)
    rng = np.random.default_rng(90 + d)
    shape = orc.tile_shape(p, n)[1:]
    B = [0.5 + 0.3 * rng.random(shape), 0.4 * rng.random(shape) - 0.2, 0.3 * rng.random(shape)]
    pr = 1.0 + 0.5 * rng.random(shape)
    rho = 1.0 + 0.2 * rng.random(shape)
    w = np.array([rho, 0 * rho, 0 * rho, 0 * rho, B[0], B[1], B[2], pr, 0 * rho])
    u = orc.prim_to_cons(p, w)
    axis = 3 - d  # array axes are [var, z, y, x]
    m = np.flip(u, axis=axis).copy()
    m[1 + d] *= -1
    m[4 + d] *= -1
    a, _ = orc.conduct_tile(p, (0.1, 0.2, 0.15), u, n, 1e-3)
    b, _ = orc.conduct_tile(p, (0.1, 0.2, 0.15), m, n, 1e-3)
    np.testing.assert_allclose(np.flip(b, axis=2 - d), a, rtol=1e-13)
