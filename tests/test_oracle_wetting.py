"""Pins of the reference's geometric ghost-density rule (Sec. 4, Eq. 19-21).

The rule extrapolates the density to the ghost layer so that the density gradient meets the wall at the prescribed
contact angle. The pins below do not retype the formula; they check what the geometry fixes:
  * a linear density field whose level lines meet the wall at angle theta (through the liquid, the dense side) is
    extrapolated exactly, by Eq. 19 and by every iterate of Eq. 21;
  * the exact root of Eq. 20 (with its square root) is Eq. 19 itself, so the iteration converges to it;
  * theta -> pi - theta flips the sign of the correction; theta = 90 deg copies rho_2 into the ghost.
"""
import numpy as np
import pytest


def linear_field_at_angle(theta, g=0.03, base=0.2):
    """rho(x, y) of a linear field whose iso-lines make angle theta with the bottom wall, measured through the
    dense side. The dense side lies at -x along the wall, so grad rho = g (-sin theta, -cos theta)."""
    gx, gy = -g * np.sin(theta), -g * np.cos(theta)
    return lambda x, y: base + gx * x + gy * y


@pytest.mark.parametrize("deg", [10, 30, 45, 60, 89, 90, 100, 135, 150, 170])
@pytest.mark.parametrize("iters", [0, 1, 2, 4, 7])
def test_linear_field_extrapolated_exactly(ora, deg, iters):
    th = np.deg2rad(deg)
    rho = linear_field_at_angle(th)
    i = 5.0
    # row 0 = ghost, row 1 = boundary node, row 2 = second fluid node (indices of Sec. 4)
    got = ora.ghost_density(rho(i - 1, 1), rho(i + 1, 1), rho(i, 1), rho(i, 2), th, iters)
    assert got == pytest.approx(rho(i, 0), rel=1e-13, abs=1e-15)


@pytest.mark.parametrize("deg", [40, 60, 80, 100, 120, 140])
def test_iteration_converges_to_eq19(ora, deg):
    th = np.deg2rad(deg)
    rng = np.random.default_rng(7)
    for _ in range(20):
        r1, r2, rm, rp = rng.uniform(0.01, 0.5, 4)
        T = rp - rm
        eq19 = ora.ghost_density(rm, rp, r1, r2, th, 0)
        assert eq19 - r2 == pytest.approx(abs(T) / np.tan(th), rel=1e-12, abs=1e-15)
        # contraction factor ~ cos^2 theta: 3000 iterates are converged to machine precision here
        conv = ora.ghost_density(rm, rp, r1, r2, th, 3000)
        assert conv == pytest.approx(eq19, rel=1e-11, abs=1e-14)


def test_iterates_monotone_towards_root(ora):
    # theta < 90 deg, start below the root: iterates increase to cot(theta) |T| (Sec. 4: "more iterations change
    # the angle little" because the contraction factor is cos^2 theta)
    th = np.deg2rad(15)
    rm, rp, r1, r2 = 0.10, 0.20, 0.30, 0.32
    vals = [ora.ghost_density(rm, rp, r1, r2, th, k) for k in range(1, 12)]
    assert all(b > a for a, b in zip(vals, vals[1:]))
    root = r2 + abs(rp - rm) / np.tan(th)
    assert all(v < root for v in vals)


@pytest.mark.parametrize("iters", [0, 1, 3, 4, 6])
def test_supplementary_angle_antisymmetry(ora, iters):
    rng = np.random.default_rng(3)
    for _ in range(20):
        r1, r2, rm, rp = rng.uniform(0.01, 0.5, 4)
        th = rng.uniform(0.1, np.pi / 2)
        d1 = ora.ghost_density(rm, rp, r1, r2, th, iters) - r2
        d2 = ora.ghost_density(rm, rp, r1, r2, np.pi - th, iters) - r2
        assert d2 == pytest.approx(-d1, rel=1e-12, abs=1e-15)


def test_neutral_wetting_copies_second_row(ora):
    for iters in [0, 1, 4]:
        got = ora.ghost_density(0.1, 0.4, 0.3, 0.25, np.pi / 2, iters)
        assert abs(got - 0.25) < 1e-16 * 10


def test_lattice_row_mapping(ora):
    """On a lattice the ghost rows are rows 0 and ny-1; they use boundary rows 1 / ny-2 and second rows
    2 / ny-3, and the tangential difference wraps periodically in x."""
    nx, ny = 16, 9
    sim = ora.Sim(nx, ny, 0.8, theta_bottom=np.deg2rad(50), theta_top=np.deg2rad(120), wet_iters=4)
    x = np.arange(nx)
    y = np.arange(ny)
    rho = 0.2 + 0.05 * np.sin(2 * np.pi * x[None, :] / nx) * (1 + 0.1 * y[:, None]) + 0.004 * y[:, None] ** 2
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    sim.f[:] = rho[:, :, None] * w
    sim.f[0] = 0
    sim.f[-1] = 0
    got, _ = sim.density()
    np.testing.assert_allclose(got[1:-1], rho[1:-1], rtol=1e-14)
    for xi in range(nx):
        xm, xp = (xi - 1) % nx, (xi + 1) % nx
        b = ora.ghost_density(rho[1, xm], rho[1, xp], rho[1, xi], rho[2, xi], np.deg2rad(50), 4)
        t = ora.ghost_density(rho[ny - 2, xm], rho[ny - 2, xp], rho[ny - 2, xi], rho[ny - 3, xi], np.deg2rad(120), 4)
        assert got[0, xi] == pytest.approx(b, rel=1e-15)
        assert got[ny - 1, xi] == pytest.approx(t, rel=1e-15)
