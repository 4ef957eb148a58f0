"""Pins of the reference's MRT collision (Eq. 1-6 and 15 with a general Lambda of Eq. 2) and of the surface-tension
source of Eq. (16)-(17), independent of its own code: moments built here from the velocities, hand-derived lattice
sums on polynomial fields, and the physics the paper states (surface tension proportional to 1 - kappa, with the
coexistence densities unchanged)."""
import numpy as np
import pytest

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
E2 = EX**2 + EY**2
# moment basis in the order of Eq. (4), from the velocities (Lallemand and Luo)
M = np.stack([np.ones(9), -4 + 3 * E2, 4 - 21 / 2 * E2 + 9 / 2 * E2**2, EX, (-5 + 3 * E2) * EX, EY,
              (-5 + 3 * E2) * EY, EX**2 - EY**2, EX * EY])


def random_node(rng, scale=0.3):
    rho = rng.uniform(0.05, 0.5)
    return W * rho * (1 + scale * rng.standard_normal(9))


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_mrt_with_equal_rates_is_bgk(ora, tau):
    """Lambda = (1/tau) I on the non-conserved moments: the MRT form reduces to BGK with Guo forcing."""
    rng = np.random.default_rng(int(tau * 10))
    bgk = ora.Sim(4, 4, 0.7, tau=tau)
    mrt = ora.Sim(4, 4, 0.7, tau=tau, mrt=(1 / tau,) * 3)
    for _ in range(8):
        f = random_node(rng)
        F = rng.standard_normal(2) * 1e-3
        a = ora.collide_node(bgk, f, *F)
        b = ora.collide_mrt_node(mrt, f, *F)
        np.testing.assert_allclose(b, a, rtol=0, atol=2e-16 * 20 * f.sum())


@pytest.mark.parametrize("rates", [(1.1, 1.3, 1.2), (0.7, 1.9, 1.5), (1.64, 1.54, 1.9)])
def test_mrt_relaxes_each_moment_at_its_rate(ora, rates):
    """F = 0, Q = 0: every non-conserved moment m_k relaxes as m*_k - m_eq,k = (1 - s_k)(m_k - m_eq,k), with
    s = (s_e, s_eps, s_q, s_q) on e, eps, q_x, q_y and 1/tau on p_xx, p_xy; rho and j are unchanged."""
    tau = 0.8
    sim = ora.Sim(4, 4, 0.7, tau=tau, mrt=rates)
    rng = np.random.default_rng(3)
    s_e, s_eps, s_q = rates
    for _ in range(6):
        f = random_node(rng)
        fs = ora.collide_mrt_node(sim, f, 0.0, 0.0)
        m, ms = M @ f, M @ fs
        rho, vx, vy = m[0], m[3] / m[0], m[5] / m[0]
        v2 = vx * vx + vy * vy
        meq = rho * np.array([1, -2 + 3 * v2, 1 - 3 * v2, vx, -vx, vy, -vy, vx * vx - vy * vy, vx * vy])
        for k, s in [(1, s_e), (2, s_eps), (4, s_q), (6, s_q), (7, 1 / tau), (8, 1 / tau)]:
            assert ms[k] - meq[k] == pytest.approx((1 - s) * (m[k] - meq[k]), abs=1e-15 * rho * 10), k
        for k in (0, 3, 5):
            assert ms[k] == pytest.approx(m[k], abs=1e-15 * rho * 10)


def test_mrt_conserves_mass_and_adds_force(ora):
    rng = np.random.default_rng(8)
    sim = ora.Sim(4, 4, 0.7, tau=0.9, mrt=(1.2, 1.5, 1.7), kappa=0.5)
    for _ in range(8):
        f = random_node(rng)
        F = rng.standard_normal(2) * 1e-3
        Q = rng.standard_normal(3) * 1e-3
        fs = ora.collide_mrt_node(sim, f, *F, Q)
        assert fs.sum() == pytest.approx(f.sum(), rel=1e-14)
        assert fs @ EX == pytest.approx(f @ EX + F[0], abs=1e-15)
        assert fs @ EY == pytest.approx(f @ EY + F[1], abs=1e-15)


def test_source_shifts_the_stress_as_a_pressure_tensor(ora):
    """The source of Eq. (16) enters the post-collision moments as C: the trace of the momentum flux moves by
    C_e / 3 = s_e (Q_xx + Q_yy) / 2, its deviatoric part by -(1/tau)(Q - tr Q / 2), and nothing else moves."""
    rng = np.random.default_rng(9)
    tau, s_e = 0.9, 1.3
    sim = ora.Sim(4, 4, 0.7, tau=tau, mrt=(s_e, 1.5, 1.7), kappa=0.5)
    f = random_node(rng)
    F = rng.standard_normal(2) * 1e-3
    Q = np.array([2e-3, -1e-3, 5e-4])
    d = ora.collide_mrt_node(sim, f, *F, Q) - ora.collide_mrt_node(sim, f, *F)
    pxx, pyy, pxy = (d * EX * EX).sum(), (d * EY * EY).sum(), (d * EX * EY).sum()
    tol = 2e-16  # round-off of O(0.3) populations
    assert pxx + pyy == pytest.approx(s_e * (Q[0] + Q[1]) / 2, abs=tol)
    assert pxx - pyy == pytest.approx(-(Q[0] - Q[1]) / tau, abs=tol)
    assert pxy == pytest.approx(-Q[2] / tau, abs=tol)
    assert abs(d.sum()) < tol and abs(d @ EX) < tol and abs(d @ EY) < tol


@pytest.mark.parametrize("A", [0.0, -0.6])
def test_q_tensor_on_a_polynomial_field(ora, A):
    """psi = c + a y^2 (walls, x-uniform): the lattice sums of Eq. (17) are exact polynomials, derived by hand with
    sum w e_x^4 = 1, sum w e_x^2 e_y^2 = 1/3, sum w e_x^6 = 1, sum w e_x^4 e_y^2 = 1/3."""
    nx, ny, c, a, kappa, G = 3, 9, 0.4, 0.003, 0.7, -1.0
    sim = ora.Sim(nx, ny, 0.7, A=A, kappa=kappa)
    y = np.arange(ny, dtype=float)
    psi = np.repeat((c + a * y**2)[:, None], nx, axis=1)
    q = ora.qtensor(sim, psi)
    yy = y[1:-1]
    p = c + a * yy**2
    k = kappa * G / 2
    qyy = k * ((1 - A) * p * a + A / 2 * (2 * a * c + a * a * (6 * yy**2 + 1)))
    qxx = k * ((1 - A) * p * a / 3 + A / 2 * (2 * a * c / 3 + a * a * (2 * yy**2 + 1 / 3)))
    np.testing.assert_allclose(q[1, 1:-1, 0], qyy, rtol=1e-12, atol=1e-17)
    np.testing.assert_allclose(q[0, 1:-1, 0], qxx, rtol=1e-12, atol=1e-17)
    np.testing.assert_allclose(q[2, 1:-1, 0], 0.0, atol=1e-17)


def slab(ora, T, kappa, steps=6000):
    s = ora.Sim(4, 160, T, periodic_y=True, kappa=kappa)
    rv, rl = s.coexistence()
    y = np.arange(160)[:, None]
    rho = (rv + (rl - rv) * 0.5 * (np.tanh((y - 40) / 2.5) - np.tanh((y - 120) / 2.5))) * np.ones((1, 4))
    s.f[:] = rho[:, :, None] * W
    s.run(steps)
    return s.density()[0]


def test_flat_interface_is_independent_of_kappa(ora):
    """For a profile varying in y only Q_yy = 3 Q_xx on the D2Q9 weights, and the source leaves the normal stress
    unchanged: the whole flat profile is the same for every kappa (to round-off accumulated over the run), so the
    coexistence densities are (as the source's purpose requires). A different factor on either diagonal entry of
    Eq. (16) breaks this."""
    r0 = slab(ora, 0.85, 0.0)
    for kappa in (0.5, 0.9):
        r = slab(ora, 0.85, kappa)
        assert np.abs(r - r0).max() <= 1e-10 * r0.max()
    s = ora.Sim(4, 160, 0.85)
    rv, rl = s.coexistence()
    assert r0[0, 0] < rv < rl and abs(r0[80, 0] - rl) < 0.01 * rl   # a settled slab, not the initial state


def laplace_sigma(ora, kappa, radii=(14, 18, 22, 26), T=0.85, steps=4000):
    res = []
    for R in radii:
        s = ora.Sim(96, 96, T, periodic_y=True, kappa=kappa)
        s.init_droplets([48.0], [48.0], [float(R)])
        s.run(steps)
        r, _ = s.density()
        rin, rout = r[48, 48], r[0, 0]
        Reff = np.sqrt((r - rout).sum() / (np.pi * (rin - rout)))
        res.append((1 / Reff, ora.cs_pressure(rin, s.T) - ora.cs_pressure(rout, s.T)))
    x, y = np.array(res).T
    (k, b), *_ = np.linalg.lstsq(np.stack([x, np.ones_like(x)], 1), y, rcond=None)
    return k, b, y.min()


def test_surface_tension_scales_as_one_minus_kappa(ora):
    """Free droplets (R = 14..26 in a periodic 96 x 96 box, 0.85 T_c): the Laplace-law slope at kappa = 0.5 and
    -0.5 is (1 - kappa) times the slope at kappa = 0, within 6 % (finite interface width); Eq. (17) without the
    factor G/2 would give 1 + 2 kappa (2.0 and 0.0)."""
    s0, b0, m0 = laplace_sigma(ora, 0.0)
    assert s0 > 0 and abs(b0) < 0.05 * m0
    for kappa in (0.5, -0.5):
        s, b, m = laplace_sigma(ora, kappa)
        assert s / s0 == pytest.approx(1 - kappa, rel=0.06), (kappa, s / s0)
        assert abs(b) < 0.05 * m
