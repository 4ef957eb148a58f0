"""Pins of the reference's collision with forcing (Eq. 1-6) and interaction force (Eq. 7-10)."""
import numpy as np
import pytest

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)

# Orthogonal D2Q9 moment matrix in the moment order of Eq. (4): (rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy),
# textbook form (Lallemand and Luo), built here from the velocities.
M = np.stack([
    np.ones(9),
    -4 + 3 * (EX**2 + EY**2),
    4 - 21 / 2 * (EX**2 + EY**2) + 9 / 2 * (EX**2 + EY**2) ** 2,
    EX,
    (-5 + 3 * (EX**2 + EY**2)) * EX,
    EY,
    (-5 + 3 * (EX**2 + EY**2)) * EY,
    EX**2 - EY**2,
    EX * EY,
])


def mrt_step(f, F, last_row_printed=False):
    """Eq. (15) without C: m* = m - Lam (m - m_eq) + (I - Lam/2) S, Lam = diag(0,1,...,1) (Sec. 3.1), m_eq from
    Eq. (4), S from Eq. (6). The last entry of S is v_x F_y + v_y F_x (the second moment of the forcing); the text
    prints v_x F_x + v_y F_y there, which `last_row_printed` selects to show it does not match."""
    m = M @ f
    rho = m[0]
    vx = (m[3] + F[0] / 2) / rho
    vy = (m[5] + F[1] / 2) / rho
    v2 = vx * vx + vy * vy
    meq = rho * np.array([1, -2 + 3 * v2, 1 - 3 * v2, vx, -vx, vy, -vy, vx * vx - vy * vy, vx * vy])
    vf = vx * F[0] + vy * F[1]
    last = vf if last_row_printed else vx * F[1] + vy * F[0]
    S = np.array([0, 6 * vf, -6 * vf, F[0], -F[0], F[1], -F[1], 2 * (vx * F[0] - vy * F[1]), last])
    lam = np.diag([0, 1, 1, 1, 1, 1, 1, 1, 1.0])
    mstar = m - lam @ (m - meq) + (np.eye(9) - lam / 2) @ S
    return np.linalg.solve(M, mstar)


def test_moment_matrix_is_orthogonal():
    G = M @ M.T
    assert np.allclose(G - np.diag(np.diag(G)), 0)


@pytest.mark.parametrize("seed", range(6))
def test_bgk_tau1_equals_mrt_of_the_paper(ora, seed):
    rng = np.random.default_rng(seed)
    sim = ora.Sim(4, 4, 0.7, tau=1.0)
    rho = rng.uniform(0.01, 0.5)
    f = W * rho * (1 + 0.2 * rng.standard_normal(9))
    F = rng.standard_normal(2) * 1e-3
    got = ora.collide_node(sim, f, F[0], F[1])
    want = mrt_step(f, F)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-15 * rho * 50)
    # the printed last entry of Eq. (6) is not the forcing's second moment: it does not reproduce the scheme
    bad = mrt_step(f, F, last_row_printed=True)
    assert np.abs(bad - got).max() > 1e-9 * np.abs(F).max()


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_collision_conserves_mass_and_adds_force(ora, tau):
    rng = np.random.default_rng(11)
    sim = ora.Sim(4, 4, 0.7, tau=tau)
    for _ in range(10):
        rho = rng.uniform(0.01, 0.5)
        f = W * rho * (1 + 0.3 * rng.standard_normal(9))
        F = rng.standard_normal(2) * 1e-3
        fs = ora.collide_node(sim, f, F[0], F[1])
        assert fs.sum() == pytest.approx(f.sum(), rel=1e-14)
        # momentum after collision: j + F (half from v, half from the source term)
        assert fs @ EX == pytest.approx(f @ EX + F[0], abs=1e-15)
        assert fs @ EY == pytest.approx(f @ EY + F[1], abs=1e-15)


def test_equilibrium_second_moment(ora):
    # tau = 1, F = 0: f* = f_eq with sum f_eq e_a e_b = rho/3 delta_ab + rho v_a v_b
    rng = np.random.default_rng(5)
    sim = ora.Sim(4, 4, 0.7, tau=1.0)
    rho = 0.3
    f = W * rho * (1 + 0.1 * rng.standard_normal(9))
    f *= rho / f.sum()
    fs = ora.collide_node(sim, f, 0.0, 0.0)
    vx, vy = f @ EX / rho, f @ EY / rho
    assert fs @ (EX * EX) == pytest.approx(rho / 3 + rho * vx * vx, rel=1e-13)
    assert fs @ (EY * EY) == pytest.approx(rho / 3 + rho * vy * vy, rel=1e-13)
    assert fs @ (EX * EY) == pytest.approx(rho * vx * vy, rel=1e-12, abs=1e-17)


def _set_density(sim, rho):
    sim.f[:] = rho[:, :, None] * W
    if not sim.p.periodic_y:
        sim.f[0] = 0
        sim.f[-1] = 0


@pytest.mark.parametrize("A", [0.0, -0.6, 0.5])
def test_total_force_vanishes_on_periodic_lattice(ora, A):
    # Pairwise interactions (Eq. 7) and a discrete gradient (Eq. 8) both sum to zero over a periodic domain:
    # momentum conservation of Eq. (9).
    rng = np.random.default_rng(2)
    sim = ora.Sim(24, 20, 0.7, A=A, periodic_y=True)
    _set_density(sim, rng.uniform(0.01, 0.4, (20, 24)))
    Fx, Fy = sim.force()
    scale = np.abs(Fx).max()
    assert abs(Fx.sum()) < 1e-13 * scale * Fx.size
    assert abs(Fy.sum()) < 1e-13 * scale * Fy.size


@pytest.mark.parametrize("A", [0.0, -0.6, 0.4])
def test_force_is_minus_gradient_of_nonideal_pressure(ora, A):
    """For a smooth field every A gives F = -grad(G psi^2/2) = -grad(p_EOS - rho/3) to second order in the
    wavenumber (Eq. 9-10 with c = 1 and sum_a w_a e_a e_a = identity for the weights of Eq. 7)."""
    n = 128
    sim = ora.Sim(n, n, 0.7, A=A, periodic_y=True)
    x = np.arange(n)
    k = 2 * np.pi / n
    rho = 0.2 + 0.01 * np.sin(k * x)[None, :] + 0.008 * np.cos(k * x)[:, None]
    _set_density(sim, rho)
    Fx, Fy = sim.force()
    T = sim.T
    dU = np.vectorize(lambda r: ora.cs_dpdrho(r, T) - 1 / 3)(rho)
    gx = 0.01 * k * np.cos(k * x)[None, :] * np.ones((n, 1))
    gy = -0.008 * k * np.sin(k * x)[:, None] * np.ones((1, n))
    ex, ey = -dU * gx, -dU * gy
    err = max(np.abs(Fx - ex).max(), np.abs(Fy - ey).max())
    assert err < 0.01 * max(np.abs(ex).max(), np.abs(ey).max())


def test_uniform_density_gives_zero_force(ora):
    sim = ora.Sim(10, 10, 0.7, theta_bottom=np.pi / 2, theta_top=np.pi / 2)
    _set_density(sim, np.full((10, 10), 0.3))
    Fx, Fy = sim.force()
    assert np.abs(Fx).max() == 0.0 and np.abs(Fy).max() < 1e-17
