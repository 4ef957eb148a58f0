"""Whole-scheme pins of the reference: conservation, symmetry, mechanical equilibrium, Laplace law, Poiseuille
flow, contact angles on flat walls, and the contact-angle measurement itself on analytic caps."""
import numpy as np
import pytest
from scipy import integrate, optimize

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


@pytest.fixture(scope="module")
def c1_run(ora):
    """200 x 100, T = 0.85 T_c, theta = 90 deg, semicircle R = 30 on the bottom wall, 2000 steps."""
    sim = ora.Sim(200, 100, 0.85)
    sim.init_droplets(100.0, 0.5, 30.0)
    m0 = sim.mass()
    sim.run(2000)
    return sim, m0


def test_mass_conserved(c1_run):
    sim, m0 = c1_run
    assert abs(sim.mass() - m0) <= 1e-12 * m0
    assert sim.counters.tolist() == [0, 0]


def test_neutral_wetting_mirror_symmetry_and_angle(ora, c1_run):
    sim, _ = c1_run
    rho, _ = sim.density()
    a = rho[1:-1, 101:200]
    b = rho[1:-1, 99:0:-1]
    assert np.abs(a - b).max() <= 1e-12 * rho.max()
    th, R, xc, yc, n = ora.measure_contact_angle(rho, (40, 161, 1, 70), wall=0)
    assert abs(np.rad2deg(th) - 90.0) < 1.0
    assert abs(xc - 100.0) < 1e-9


def test_uniform_state_stays_at_rest(ora):
    sim = ora.Sim(12, 10, 0.85)
    sim.f[1:-1] = 0.3 * W
    f0 = sim.f.copy()
    sim.run(200)
    assert np.abs(sim.f - f0).max() < 1e-16


@pytest.mark.parametrize("deg", [60, 120])
def test_flat_wall_contact_angle(ora, deg):
    """Measured vs prescribed angle on the bottom wall (the paper reports agreement within about 2 deg for its
    EOS, Sec. 4.2); accepted here within 3 deg."""
    sim = ora.Sim(200, 100, 0.85, theta_bottom=np.deg2rad(deg), theta_top=np.pi / 2)
    sim.init_droplets(100.0, 0.5, 30.0)
    sim.run(7500)
    rho, _ = sim.density()
    th = np.rad2deg(ora.measure_contact_angle(rho, (0, 200, 1, 90), wall=0)[0])
    assert abs(th - deg) < 3.0, th


def _eps0_coexistence(ora, T):
    """Flat-interface densities predicted for the pseudo-potential force by mechanical stability:
    p(rho_v) = p(rho_l) = p_b and integral (p_b - p) psi'/psi d rho = 0 (psi from Eq. 10 with G = -1)."""
    p = lambda r: ora.cs_pressure(r, T)
    dp = lambda r: ora.cs_dpdrho(r, T)
    rc, _, _ = ora.cs_critical()
    s1 = optimize.brentq(dp, 1e-6, rc)
    s2 = optimize.brentq(dp, rc, 0.9)
    dlnpsi = lambda r: (1 / 3 - dp(r)) / (2 * (r / 3 - p(r)))

    def resid(pb):
        rv = optimize.brentq(lambda r: p(r) - pb, 1e-12, s1, xtol=1e-15)
        rl = optimize.brentq(lambda r: p(r) - pb, s2, 0.9, xtol=1e-15)
        v, _ = integrate.quad(lambda r: (pb - p(r)) * dlnpsi(r), rv, rl, epsabs=0, epsrel=1e-11, limit=400)
        return v, rv, rl

    pb = optimize.brentq(lambda q: resid(q)[0], max(p(s2), 1e-12), p(s1) * (1 - 1e-9), xtol=1e-16)
    _, rv, rl = resid(pb)
    return rv, rl


def _slab(ora, A, steps=30000):
    ny = 200
    sim = ora.Sim(4, ny, 0.85, A=A, periodic_y=True)
    rv, rl = sim.coexistence()
    y = np.arange(ny)
    rho = rv + (rl - rv) * 0.5 * (np.tanh((y - 50) / 2.5) - np.tanh((y - 150) / 2.5))
    sim.f[:] = rho[:, None, None] * W
    sim.run(steps)
    r, _ = sim.density()
    return sim, r[0, 0], r[100, 0]


def test_flat_interface_follows_mechanical_stability_rule(ora):
    """Plain Shan-Chen force (A = 0): the bulk densities of a flat interface satisfy the mechanical-stability
    integral with psi'/psi (not Maxwell's rule); bulk EOS pressures are equal (mechanical equilibrium)."""
    sim, rv_lb, rl_lb = _slab(ora, 0.0)
    rv, rl = _eps0_coexistence(ora, sim.T)
    assert rv_lb == pytest.approx(rv, rel=2e-4)
    assert rl_lb == pytest.approx(rl, rel=2e-5)
    pv, pl = ora.cs_pressure(rv_lb, sim.T), ora.cs_pressure(rl_lb, sim.T)
    assert abs(pl - pv) < 1e-4 * pv


def test_hybrid_force_mechanical_equilibrium(ora):
    """A = -0.6 (the paper's choice, Sec. 3.1): equal bulk EOS pressures; coexistence between the A = 0 rule and
    Maxwell (reported, not pinned: no closed form for the hybrid force)."""
    sim, rv_lb, rl_lb = _slab(ora, -0.6)
    pv, pl = ora.cs_pressure(rv_lb, sim.T), ora.cs_pressure(rl_lb, sim.T)
    assert abs(pl - pv) < 1e-4 * pv
    rv_m, rl_m = sim.coexistence()
    rv0, rl0 = _eps0_coexistence(ora, sim.T)
    assert rv0 < rv_lb < rv_m and rl0 < rl_lb < rl_m


def test_laplace_law(ora):
    """Free droplets in a periodic box: p_in - p_out = sigma / R through the origin (R = equimolar radius)."""
    res = []
    for R in [12, 15, 18, 21, 24]:
        sim = ora.Sim(128, 128, 0.85, periodic_y=True)
        sim.init_droplets(64.0, 64.0, float(R))
        sim.run(4000)
        r, _ = sim.density()
        rin, rout = r[64, 64], r[0, 0]
        Reff = np.sqrt((r - rout).sum() / (np.pi * (rin - rout)))
        res.append((Reff, ora.cs_pressure(rin, sim.T) - ora.cs_pressure(rout, sim.T)))
    res = np.array(res)
    x, y = 1 / res[:, 0], res[:, 1]
    Amat = np.stack([x, np.ones_like(x)], 1)
    (k, b), *_ = np.linalg.lstsq(Amat, y, rcond=None)
    fit = Amat @ [k, b]
    r2 = 1 - ((y - fit) ** 2).sum() / ((y - y.mean()) ** 2).sum()
    assert k > 0
    assert r2 > 0.999
    assert abs(b) < 0.05 * y.min()


def test_poiseuille_channel(ora):
    """Uniform density (no interaction force), body force g along x, walls at y = 0.5 and ny - 1.5 (halfway
    bounce-back): u(y) = g / (2 rho nu) (y - y_b)(y_t - y), nu = (tau - 1/2)/3."""
    ny, g, rho0 = 34, 1e-6, 0.3
    sim = ora.Sim(4, ny, 0.85, body_force=(g, 0.0))
    sim.f[1:-1] = rho0 * W
    sim.run(40000)
    rho = sim.f[1:-1, 0].sum(-1)
    u = (sim.f[1:-1, 0] @ EX + g / 2) / rho
    y = np.arange(1, ny - 1)
    ua = g / (2 * rho0 * (1 / 6)) * (y - 0.5) * (ny - 1.5 - y)
    assert np.abs(u - ua).max() < 2e-3 * ua.max()


def _cap_field(nx, ny, xc, yc, R, wall, rl=0.3, rv=0.03, W_=5.0):
    x = np.arange(nx)[None, :]
    y = np.arange(ny)[:, None]
    r = np.sqrt((x - xc) ** 2 + (y - yc) ** 2)
    rho = rv + (rl - rv) * 0.5 * (1 - np.tanh(2 * (r - R) / W_))
    return rho


@pytest.mark.parametrize("deg", [30, 45, 70, 90, 110, 135, 160])
@pytest.mark.parametrize("wall", [0, 1])
def test_measurement_on_analytic_caps(ora, deg, wall):
    nx, ny, R = 300, 160, 60.0
    th = np.deg2rad(deg)
    if wall == 0:
        yw = 0.5
        yc = yw - R * np.cos(th)
        box = (0, nx, 1, ny - 1)
    else:
        yw = ny - 1.5
        yc = yw + R * np.cos(th)
        box = (0, nx, 1, ny - 1)
    rho = _cap_field(nx, ny, 150.3, yc, R, wall)
    got, Rf, xf, yf, n = ora.measure_contact_angle(rho, box, wall=wall)
    assert abs(np.rad2deg(got) - deg) < 0.1
    assert abs(Rf - R) < 0.1
