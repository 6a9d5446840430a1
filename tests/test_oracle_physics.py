"""Pins of the oracle's pointwise physics against the mathematics:
flux Jacobian spectrum, rotation covariance, Euler and textbook special
cases, limiter truth tables, EOS round trip.  (Sec. 2 and Sec. 3 of the paper.)"""
import math

import numpy as np
import pytest


def _state(rng, psi=0.0):
    rho = 0.5 + rng.random()
    v = rng.normal(size=3) * 0.7
    B = rng.normal(size=3)
    p = 0.3 + rng.random()
    return np.array([rho, *v, *B, p, psi])


def _cons(orc, p, w):
    return orc.prim_to_cons(p, w.reshape(9, 1)).ravel()


def _jacobian(orc, p, u, d, ch):
    J = np.zeros((9, 9))
    for j in range(9):
        h = 1e-6 * max(1.0, abs(u[j]))
        up, um = u.copy(), u.copy()
        up[j] += h
        um[j] -= h
        J[:, j] = (orc.flux(p, up, d, ch) - orc.flux(p, um, d, ch)) / (2 * h)
    return J


@pytest.mark.parametrize("d", [0, 1, 2])
def test_flux_jacobian_spectrum(orc, rng, d):
    """Eigenvalues of dF_d/du are v_d +- c_f, v_d +- c_a, v_d +- c_s, v_d (MHD,
    textbook) and +-c_h (the GLM pair); orc_speed is |v_d| + c_f."""
    p = orc.make_params(ndim=3, gamma=1.4)
    ch = 2.7
    for _ in range(5):
        w = _state(rng, psi=0.3)
        u = _cons(orc, p, w)
        lam = np.sort(np.linalg.eigvals(_jacobian(orc, p, u, d, ch)).real)
        rho, v, B, pr = w[0], w[1:4], w[4:7], w[7]
        a2 = 1.4 * pr / rho
        b2 = B @ B / rho
        bn2 = B[d] ** 2 / rho
        disc = math.sqrt((a2 + b2) ** 2 - 4 * a2 * bn2)
        cf = math.sqrt(0.5 * (a2 + b2 + disc))
        cs = math.sqrt(0.5 * (a2 + b2 - disc))
        ca = math.sqrt(bn2)
        want = np.sort([v[d] - cf, v[d] - ca, v[d] - cs, v[d], v[d] + cs, v[d] + ca,
                        v[d] + cf, -ch, ch])
        np.testing.assert_allclose(lam, want, rtol=0, atol=2e-6)
        assert orc.speed(p, u, d) == pytest.approx(abs(v[d]) + cf, rel=1e-13)


def test_flux_rotation_covariance(orc, rng):
    """Relabelling the axes cyclically maps F_d onto F_{d+1}."""
    p = orc.make_params(ndim=3)

    def cyc(u):
        out = u.copy()
        out[1:4] = u[[3, 1, 2]]
        out[4:7] = u[[6, 4, 5]]
        return out

    for _ in range(5):
        u = _cons(orc, p, _state(rng, psi=0.2))
        for d in range(3):
            a = orc.flux(p, cyc(u), (d + 1) % 3, 1.3)
            b = cyc(orc.flux(p, u, d, 1.3))
            np.testing.assert_allclose(a, b, rtol=1e-14, atol=1e-14)
            assert orc.speed(p, cyc(u), (d + 1) % 3) == pytest.approx(orc.speed(p, u, d), rel=1e-14)


def test_flux_reduces_to_euler(orc, rng):
    """B = 0, psi = 0: the Euler flux and the sound speed."""
    p = orc.make_params(ndim=3, gamma=1.4)
    w = _state(rng)
    w[4:7] = 0.0
    u = _cons(orc, p, w)
    rho, v, pr = w[0], w[1:4], w[7]
    E = pr / 0.4 + 0.5 * rho * v @ v
    for d in range(3):
        f = orc.flux(p, u, d, 5.0)
        want = np.zeros(9)
        want[0] = rho * v[d]
        want[1:4] = rho * v[d] * v
        want[1 + d] += pr
        want[7] = (E + pr) * v[d]
        np.testing.assert_allclose(f, want, rtol=1e-13, atol=1e-14)
        assert orc.speed(p, u, d) == pytest.approx(abs(v[d]) + math.sqrt(1.4 * pr / rho), rel=1e-13)


def test_fast_speed_special_cases(orc):
    """B parallel to d: max(a, b); B normal to d: sqrt(a^2 + b^2) (textbook)."""
    p = orc.make_params(ndim=3, gamma=5.0 / 3.0)
    rho, pr = 2.0, 0.5
    a = math.sqrt(5.0 / 3.0 * pr / rho)
    for Bmag in (0.3, 2.0):
        b = Bmag / math.sqrt(rho)
        par = _cons(orc, p, np.array([rho, 0, 0, 0, Bmag, 0, 0, pr, 0.0]))
        assert orc.speed(p, par, 0) == pytest.approx(max(a, b), rel=1e-14)
        assert orc.speed(p, par, 1) == pytest.approx(math.sqrt(a * a + b * b), rel=1e-14)


def test_eos_round_trip(orc, rng):
    p = orc.make_params(ndim=3, gamma=5.0 / 3.0)
    for _ in range(10):
        w = _state(rng)
        u = _cons(orc, p, w)
        assert orc.pressure(p, u) == pytest.approx(w[7], rel=1e-13)
        e = w[7] / (2.0 / 3.0) + 0.5 * w[0] * w[1:4] @ w[1:4] + 0.5 * w[4:7] @ w[4:7]
        assert u[7] == pytest.approx(e, rel=1e-14)
        np.testing.assert_allclose(u[1:4], w[0] * w[1:4], rtol=1e-15)


@pytest.mark.parametrize("a,b,mm,vl", [
    (1.0, 2.0, 1.0, 4.0 / 3.0),
    (2.0, 1.0, 1.0, 4.0 / 3.0),
    (-1.0, -3.0, -1.0, -1.5),
    (1.0, -1.0, 0.0, 0.0),
    (-2.0, 5.0, 0.0, 0.0),
    (0.0, 3.0, 0.0, 0.0),
    (3.0, 0.0, 0.0, 0.0),
    (0.0, 0.0, 0.0, 0.0),
])
def test_limiter_tables(orc, a, b, mm, vl):
    assert orc.limiter("minmod", a, b) == mm
    assert orc.limiter("minmod", b, a) == mm
    assert orc.limiter("vanleer", a, b) == pytest.approx(vl, rel=1e-15)
    assert orc.limiter("vanleer", b, a) == pytest.approx(vl, rel=1e-15)


def test_paper_phi_is_ratio_form(orc, rng):
    """phi(r) = r for |r| <= 1, else 1, applied as phi(a/b) b."""
    for _ in range(50):
        a, b = rng.normal(size=2)
        r = a / b
        want = (r if abs(r) <= 1 else 1.0) * b
        assert orc.limiter("paper", a, b) == pytest.approx(want, rel=1e-14)
        # minmod as a flux limiter phi(r) = max(0, min(1, r))
        assert orc.limiter("minmod", a, b) == pytest.approx(max(0.0, min(1.0, r)) * b, rel=1e-14, abs=0)
