"""Pins of the reference's Martys-Chen walls (Eq. 14), the fluid-solid force the paper compares against, with the
wall rows as solid nodes that take no part in the fluid-fluid force.

Hand-derived fixed point: for a uniform fluid at rest next to a flat wall, the fluid-fluid force of Eq. 9 misses
the wall neighbours, F_i = G psi^2 (1 - A/2) sum_wall w e (the potential part contributes A U with U = G psi^2/2,
the Shan-Chen part (1 - A) G psi^2), and Eq. 14 adds F_s = -G_w psi sum_wall w e. The rest state is exact iff
G_w = G psi (1 - A/2); a more negative G_w attracts the fluid to the wall (density rises in the boundary row), a
less negative one repels it."""
import numpy as np
import pytest

W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def uniform_run(ora, rho, A, G_w, steps=40, nx=6, ny=10, T=0.85):
    s = ora.Sim(nx, ny, T, A=A, G_w=G_w)
    s.f[:] = rho * W
    s.run(steps)
    return s


@pytest.mark.parametrize("A", [0.0, -0.6, 0.4])
@pytest.mark.parametrize("rho", [0.05, 0.25])
def test_uniform_rest_state_is_a_fixed_point_at_the_matching_G_w(ora, A, rho):
    probe = ora.Sim(4, 4, 0.85, A=A)
    psi = ora.psi(probe, rho)
    gw = -1.0 * psi * (1 - A / 2)
    s = uniform_run(ora, rho, A, (gw, gw))
    assert np.abs(s.f[1:-1] - rho * W).max() <= 1e-14 * rho


@pytest.mark.parametrize("A", [0.0, -0.6])
def test_more_negative_G_w_attracts_the_fluid(ora, A):
    rho = 0.05
    psi = ora.psi(ora.Sim(4, 4, 0.85, A=A), rho)
    gw0 = -psi * (1 - A / 2)
    for dg, sign in ((-0.05, 1), (0.05, -1)):
        s = uniform_run(ora, rho, A, (gw0 + dg, gw0 + dg), steps=200)
        r, _ = s.density()
        bottom, top, middle = r[1, 0], r[-2, 0], r[5, 0]
        assert sign * (bottom - middle) > 1e-4 * rho
        assert bottom == pytest.approx(top, rel=1e-12)          # both walls alike
        assert np.all(r[0] == 0) and np.all(r[-1] == 0)          # solid rows carry no fluid
    assert s.mass() == pytest.approx(rho * 6 * 8, rel=1e-13)


def test_walls_act_independently(ora):
    """Different G_w on the two walls: each boundary row follows its own wall (the bottom attracts, the top is at
    the fixed point and stays at the bulk density until the disturbance from the bottom arrives)."""
    rho, A = 0.05, -0.6
    psi = ora.psi(ora.Sim(4, 4, 0.85, A=A), rho)
    gw0 = -psi * (1 - A / 2)
    s = uniform_run(ora, rho, A, (gw0 - 0.05, gw0), steps=3, ny=40)
    r, _ = s.density()
    assert r[1, 0] > rho * (1 + 1e-5)
    assert r[-2, 0] == pytest.approx(rho, rel=1e-14)
