"""Pins of the reference's Carnahan-Starling EOS, coexistence and psi (Eq. 10), independent of its own code."""
import numpy as np
import pytest
from scipy import integrate

A, B, RG = 1.0, 4.0, 1.0


def test_critical_point_textbook_constants(ora):
    # Carnahan-Starling van der Waals-type EOS, textbook critical constants to four digits:
    # b rho_c = 0.5218, b R T_c / a = 0.3773, Z_c = p_c / (rho_c R T_c) = 0.3590.
    rc, tc, pc = ora.cs_critical(A, B, RG)
    assert abs(B * rc - 0.5218) < 1e-4
    assert abs(B * RG * tc / A - 0.3773) < 1e-4
    assert abs(pc / (rc * RG * tc) - 0.3590) < 1e-4
    # eta_c is the root of 1 - 5 eta - 20 eta^2 - 4 eta^3 + 5 eta^4 - eta^5 = 0 (eliminating T from
    # p' = p'' = 0 by hand); the reference finds rho_c by bisection on a different function.
    eta = B * rc / 4
    assert abs(1 - 5 * eta - 20 * eta**2 - 4 * eta**3 + 5 * eta**4 - eta**5) < 1e-12
    # scale invariance: rho_c ~ 1/b, T_c ~ a/(b R)
    rc2, tc2, _ = ora.cs_critical(2.0, 3.0, 0.5)
    assert abs(rc2 * 3.0 - rc * B) < 1e-12
    assert abs(tc2 * 3.0 * 0.5 / 2.0 - tc * B * RG / A) < 1e-12


@pytest.mark.parametrize("eta", [1e-3, 0.01, 0.03])
def test_pressure_matches_virial_series(ora, eta):
    # Carnahan-Starling compressibility: Z = 1 + sum_{n>=1} (n^2 + 3 n) eta^n.
    T = 0.07
    rho = 4 * eta / B
    Z = 1.0 + sum((n * n + 3 * n) * eta**n for n in range(1, 80))
    p_series = rho * RG * T * Z - A * rho * rho
    assert ora.cs_pressure(rho, T) == pytest.approx(p_series, rel=1e-13)


@pytest.mark.parametrize("rho", [0.01, 0.1, 0.3, 0.45])
def test_derivatives_and_gibbs_duhem(ora, rho):
    T = 0.0943287 * 0.7
    h = 1e-5 * rho
    p = lambda r: ora.cs_pressure(r, T)
    d1 = (p(rho + h) - p(rho - h)) / (2 * h)
    d2 = (p(rho + h) - 2 * p(rho) + p(rho - h)) / (h * h)
    assert ora.cs_dpdrho(rho, T) == pytest.approx(d1, rel=1e-7, abs=1e-9)
    assert ora.cs_d2pdrho2(rho, T) == pytest.approx(d2, rel=1e-4, abs=1e-6)
    mu = lambda r: ora.cs_mu(r, T)
    dmu = (mu(rho + h) - mu(rho - h)) / (2 * h)
    assert dmu == pytest.approx(ora.cs_dpdrho(rho, T) / rho, rel=1e-7, abs=1e-9)


@pytest.mark.parametrize("t", [0.5, 0.6, 0.7, 0.85, 0.9])
def test_maxwell_equal_pressure_and_equal_area(ora, t):
    _, tc, _ = ora.cs_critical()
    T = t * tc
    rv, rl = ora.cs_maxwell(T)
    assert 0 < rv < rl
    pv, pl = ora.cs_pressure(rv, T), ora.cs_pressure(rl, T)
    assert pl == pytest.approx(pv, rel=1e-9, abs=1e-15)
    # Equal-area rule in the specific volume: integral_{rho_v}^{rho_l} (p(rho) - p_b) / rho^2 d rho = 0,
    # by adaptive quadrature (independent of the closed-form chemical potential used by the solver).
    f = lambda r: (ora.cs_pressure(r, T) - pv) / (r * r)
    pts = np.geomspace(rv, rl, 40)
    tot, mag = 0.0, 0.0
    for lo, hi in zip(pts[:-1], pts[1:]):
        v, _ = integrate.quad(f, lo, hi, epsabs=0, epsrel=1e-12, limit=200)
        tot += v
        m, _ = integrate.quad(lambda r: abs(f(r)), lo, hi, epsabs=0, epsrel=1e-10, limit=200)
        mag += m
    assert abs(tot) < 1e-8 * mag
    # both densities sit outside the spinodal region (dp/drho > 0)
    assert ora.cs_dpdrho(rv, T) > 0 and ora.cs_dpdrho(rl, T) > 0


@pytest.mark.parametrize("t", [0.5, 0.7, 0.85])
def test_psi_eq10_and_cap(ora, t):
    _, tc, _ = ora.cs_critical()
    sim = ora.Sim(8, 8, t)
    cap = ora.cs_rho_cap(sim.T)
    # psi is real up to the cap and p(cap) = cap / 3 there
    assert ora.cs_pressure(cap, sim.T) == pytest.approx(cap / 3, rel=1e-10)
    rv, rl = sim.coexistence()
    assert rl < cap
    for rho in [rv, 0.5 * (rv + rl), rl]:
        s = ora.psi(sim, rho)
        # Eq. (10) with c = 1 and G = -1: p = rho/3 + G psi^2 / 2, so psi^2 = 2 (rho/3 - p)
        assert s * s == pytest.approx(2 * (rho / 3 - ora.cs_pressure(rho, sim.T)), rel=1e-12)
        assert s > 0
    assert ora.psi(sim, cap * 1.01) == 0.0  # clamped
