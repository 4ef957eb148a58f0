"""Pins of the reference's Carnahan-Starling EOS, coexistence and psi (Eq. 10), independent of its own code."""
import os

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


# ------------------------------------------------------------------------------------------------ Eq. (11)-(13)
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "pw_eos_table1.txt")


def table1():
    rows = []
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            ratio, r1, r2, tv, tm, tl = (float(v) for v in line.split())
            rows.append(dict(ratio=ratio, rho1=r1, rho2=r2, tv=tv, tm=tm, tl=tl))
    return rows


@pytest.mark.parametrize("row", table1(), ids=lambda r: f"ratio{r['ratio']:g}")
def test_pw_breakpoints_reproduce_table1(ora, row):
    r1, r2 = ora.pw_breakpoints(row["tv"], row["tm"], row["tl"], 1.0, row["ratio"])
    # the printed rho_1 carry 4 significant digits and rho_2 4 to 7; the paper's own rounding reaches 4.2e-4
    assert abs(r1 - row["rho1"]) <= 1e-3 * row["rho1"]
    assert abs(r2 - row["rho2"]) <= 1e-4 * row["rho2"]


@pytest.mark.parametrize("row", table1(), ids=lambda r: f"ratio{r['ratio']:g}")
def test_pw_printed_breakpoints_nearly_solve_eq12_13(row):
    # independent of the solver: the printed values must be near-roots of the two balances as written in the paper
    rv, rl, r1, r2, tv, tm, tl = 1.0, row["ratio"], row["rho1"], row["rho2"], row["tv"], row["tm"], row["tl"]
    t12 = [(r1 - rv) * tv, (r2 - r1) * tm, (rl - r2) * tl]
    t13 = [np.log(r1 / rv) * tv, np.log(r2 / r1) * tm, np.log(rl / r2) * tl]
    assert abs(sum(t12)) <= 2e-3 * sum(abs(t) for t in t12)
    assert abs(sum(t13)) <= 2e-3 * sum(abs(t) for t in t13)


@pytest.mark.parametrize("row", table1(), ids=lambda r: f"ratio{r['ratio']:g}")
def test_pw_coexistence_by_quadrature(ora, row):
    """Equal pressure at rho_v and rho_l, and equal chemical potential: the integral of dp / rho from rho_v to rho_l
    vanishes, evaluated here by quadrature of the reference's p(rho) (not by the closed form of Eq. 13)."""
    tv, tm, tl, rv, rl = row["tv"], row["tm"], row["tl"], 1.0, row["ratio"]
    r1, r2 = ora.pw_breakpoints(tv, tm, tl, rv, rl)
    p = lambda r: ora.pw_pressure(tv, tm, tl, r1, r2, r)
    assert p(rl) == pytest.approx(p(rv), rel=1e-12, abs=1e-12)
    dp = lambda r, h=1e-6: (p(r + h) - p(r - h)) / (2 * h)
    pts = [rv, r1, r2, rl]
    total = sum(integrate.quad(lambda r: dp(r) / r, a, b, epsabs=1e-13, epsrel=1e-12)[0]
                for a, b in zip(pts[:-1], pts[1:]))
    scale = tv * np.log(r1 / rv) + abs(tm) * np.log(r2 / r1) + tl * np.log(rl / r2)
    assert abs(total) <= 1e-9 * scale
    # continuity and slopes of Eq. (11)
    for r, t_left, t_right in ((r1, tv, tm), (r2, tm, tl)):
        assert p(r * (1 - 1e-9)) == pytest.approx(p(r), abs=1e-6)
        assert (p(r) - p(r * (1 - 1e-6))) / (r * 1e-6) == pytest.approx(t_left, rel=1e-5)
        assert (p(r * (1 + 1e-6)) - p(r)) / (r * 1e-6) == pytest.approx(t_right, rel=1e-5)


def test_pw_rho_cap(ora):
    # liquid slope below c_s^2 = 1/3: psi stays real above rho_2 (no cap)
    r1, r2 = ora.pw_breakpoints(0.25, -0.02, 0.3, 1.0, 10.0)
    assert ora.pw_rho_cap(0.25, -0.02, 0.3, r1, r2) > 1e100
    # liquid slope above 1/3: p(rho) = rho/3 at the cap
    cap = ora.pw_rho_cap(0.25, -0.02, 0.4, r1, r2)
    assert cap > r2
    assert ora.pw_pressure(0.25, -0.02, 0.4, r1, r2, cap) == pytest.approx(cap / 3.0, rel=1e-12)


def test_pw_flat_interface_settles_at_eq12_13_densities(ora):
    """A liquid slab in a periodic 4 x 120 box under the piecewise EOS (ratio 10 of Table 1) settles with bulk
    densities within 1 % of the coexistence pair the break points were solved for: the step really uses Eq. (11)
    (a Carnahan-Starling or mis-segmented pressure settles elsewhere). A = -0.3 brings the pseudo-potential's own
    coexistence rule close to the equal-area one for this EOS."""
    s = ora.Sim(4, 120, 1.0, periodic_y=True, piecewise=(0.25, -0.02, 0.3, 1.0, 10.0), A=-0.3)
    rv, rl = s.coexistence()
    y = np.arange(120)[:, None]
    rho = np.where((y >= 30) & (y < 90), rl, rv) * np.ones((1, 4))
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    s.f[:] = rho[:, :, None] * w
    s.run(6000)
    r, _ = s.density()
    assert abs(r[60, 0] - rl) <= 0.01 * rl
    assert abs(r[0, 0] - rv) <= 0.01 * rv
    assert s.mass() == pytest.approx(rho.sum(), rel=1e-12)


def test_pw_breakpoints_found_wherever_a_root_exists(ora):
    """Brute force over a grid of slopes and ratios: scan rho_1 across (rho_v, rho_l) with rho_2 from Eq. (12);
    where Eq. (13) changes sign between feasible points (rho_1 < rho_2 < rho_l), the reference must return break
    points in segment order satisfying both equations; whatever it returns must satisfy them."""
    import itertools
    found = 0
    for tv, tm, tl, rl in itertools.product([0.05, 0.25, 0.33], [-0.001, -0.02, -0.5, -5.0], [0.01, 0.3, 1.0, 10.0],
                                            [1.01, 2.0, 10.0, 1000.0]):
        rv = 1.0
        x = np.linspace(rv, rl, 20001)[1:-1]
        y = (tv * (rv - x) + tm * x - tl * rl) / (tm - tl)                    # Eq. (12) solved for rho_2
        ok = (x < y) & (y < rl)
        h = tv * np.log(x / rv) + tm * np.log(np.where(ok, y, 1.0) / x) + tl * np.log(rl / np.where(ok, y, 1.0))
        sign_change = bool(np.any(ok[:-1] & ok[1:] & (np.sign(h[:-1]) != np.sign(h[1:]))))
        try:
            r1, r2 = ora.pw_breakpoints(tv, tm, tl, rv, rl)
        except ValueError:
            assert not sign_change, (tv, tm, tl, rl)
            continue
        found += 1
        assert rv < r1 < r2 < rl
        e12 = (r1 - rv) * tv + (r2 - r1) * tm + (rl - r2) * tl
        e13 = np.log(r1 / rv) * tv + np.log(r2 / r1) * tm + np.log(rl / r2) * tl
        assert abs(e12) <= 1e-12 * rl * max(tv, abs(tm), tl)
        assert abs(e13) <= 1e-12 * max(tv, abs(tm), tl) * np.log(rl / rv) + 1e-15
    assert found > 100
