"""Pins of two reference parts by hand-derived closed forms: the split of the hybrid force of Eq. (9) between its
potential part (weight A) and its pairwise part (weight 1 - A), and the initial droplet profile.

Force. On a quadratic field psi(x, y) = c + b x^2 + a y^2 the lattice sums of Eq. (7)-(9) are exact. With the
weights w(1) = 1/3, w(2) = 1/12, a central difference of psi across one link is 4 b x (x-links) or 4 a y (y-links)
whatever the other coordinate, so
    sum_a w_a psi(x + e_a) e_a = (2 b x, 2 a y),
and for U = G psi^2 / 2 (Eq. 8), using psi(+)^2 - psi(-)^2 = (psi(+) - psi(-)) (psi(+) + psi(-)) and summing the
three rows (or columns) the difference crosses with weights 1/3, 1/12, 1/12,
    sum_a w_a U(x + e_a) e_a = (2 G b x (psi + b + a/3), 2 G a y (psi + a + b/3)).
Eq. (9) then gives
    F_x = -2 G b x (psi + A (b + a/3)),   F_y = -2 G a y (psi + A (a + b/3)),
so A enters only through the curvature terms: swapping A and 1 - A, or dropping either part, moves F by
2 G b x (1 - 2A)(b + a/3) or more.

Initial state. rho = rho_v + (rho_l - rho_v) (1 - tanh(2 (r - R)/W)) / 2 (the workloads' profile): at r = R the
mean of the two densities, at r = R -+ W/2 the values rho_v + (rho_l - rho_v)(1 +- tanh 1)/2; distances to the
nearest periodic image in x; several droplets combine by the maximum; populations at rest, f_i = w_i rho.
"""
import math

import numpy as np
import pytest

W_LB = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def _quadratic(nx, ny, c, b, a, x0, y0):
    x = np.arange(nx, dtype=float) - x0
    y = np.arange(ny, dtype=float) - y0
    X, Y = np.meshgrid(x, y)
    return X, Y, c + b * X * X + a * Y * Y


@pytest.mark.parametrize("A", [0.0, -0.6, 0.4, 1.0])
@pytest.mark.parametrize("G", [-1.0, -0.37])
def test_hybrid_force_on_a_quadratic_psi_field(ora, A, G):
    nx, ny = 40, 30
    c, b, a = 0.3, 2e-4, -3e-4
    X, Y, psi = _quadratic(nx, ny, c, b, a, 19.0, 14.0)
    sim = ora.Sim(nx, ny, 0.7, A=A, G=G)  # walls: rows 0 and ny-1 are read as given (the ghost rows)
    Fx, Fy = ora.force_psi(sim, psi)
    ex = -2 * G * b * X * (psi + A * (b + a / 3))
    ey = -2 * G * a * Y * (psi + A * (a + b / 3))
    # x wraps at the seam, where the field is not quadratic: compare the interior columns of the fluid rows
    inner = (slice(1, ny - 1), slice(1, nx - 1))
    scale = max(np.abs(ex[inner]).max(), np.abs(ey[inner]).max())
    assert np.abs(Fx[inner] - ex[inner]).max() < 1e-13 * scale
    assert np.abs(Fy[inner] - ey[inner]).max() < 1e-13 * scale
    # the curvature (A) terms are resolved: they are far above the tolerance
    assert 2 * abs(G * b) * 19 * abs(b + a / 3) > 1e-9 * scale


def test_force_split_is_not_symmetric_in_A(ora):
    """The A part and the (1 - A) part of Eq. (9) differ on a curved field: A = 0.3 and A = 0.7 give different
    forces, by the closed form above."""
    nx, ny = 24, 20
    X, Y, psi = _quadratic(nx, ny, 0.25, 0.0, 5e-4, 0.0, 9.0)
    f3 = ora.force_psi(ora.Sim(nx, ny, 0.7, A=0.3), psi)[1]
    f7 = ora.force_psi(ora.Sim(nx, ny, 0.7, A=0.7), psi)[1]
    a, G = 5e-4, -1.0
    # F_y(0.7) - F_y(0.3) = -2 G a y * 0.4 a
    want = -2 * G * a * Y * 0.4 * a
    rows = slice(1, ny - 1)
    np.testing.assert_allclose((f7 - f3)[rows], want[rows], rtol=0, atol=1e-15)
    assert np.abs(want[rows]).max() > 1e-7


def test_martys_chen_wall_term_on_a_uniform_field(ora):
    """Eq. (14) beside a flat solid row: sum_a w_a S(x + e_a) e_a = (0, -1/2) on the bottom boundary row, (0, 1/2)
    on the top one, so F_s = (0, G_w psi / 2) and (0, -G_w psi / 2); the uniform fluid field adds a known Eq. (9)
    part from the solid rows' psi = 0."""
    nx, ny = 12, 10
    psi = np.full((ny, nx), 0.4)
    psi[0] = psi[-1] = 0.0
    G, A, gw = -1.0, -0.6, (-0.7, -1.3)
    sim = ora.Sim(nx, ny, 0.7, A=A, G=G, G_w=gw)
    Fx, Fy = ora.force_psi(sim, psi)
    p = 0.4
    # beside the bottom solid row (psi = 0 there) only the upper neighbours count: sum w psi e_y = p/2 and
    # sum w U e_y = (G/4) p^2, so Eq. (9) gives -(G p^2 / 4)(2 - A); mirrored at the top
    fluid_part = -A * (G / 4) * p * p - (1 - A) * G * p * (0.5 * p)
    assert np.abs(Fx).max() == 0.0
    np.testing.assert_allclose(Fy[1], fluid_part + 0.5 * gw[0] * p, rtol=1e-14)
    np.testing.assert_allclose(Fy[ny - 2], -fluid_part - 0.5 * gw[1] * p, rtol=1e-14)
    np.testing.assert_allclose(Fy[2:ny - 2], 0.0, atol=1e-17)
    # the wall strength that cancels the fluid part: G_w = G psi (1 - A/2)
    gw0 = G * p * (1 - A / 2)
    Fy0 = ora.force_psi(ora.Sim(nx, ny, 0.7, A=A, G=G, G_w=(gw0, gw0)), psi)[1]
    assert np.abs(Fy0).max() < 1e-16


def _init(ora, nx, ny, drops, W=5.0, rho_l=0.4, rho_v=0.02, periodic_y=False):
    sim = ora.Sim(nx, ny, 0.7, periodic_y=periodic_y)
    xc, yc, R = zip(*drops)
    sim.init_droplets(list(xc), list(yc), list(R), width=W, rho_l=rho_l, rho_v=rho_v)
    return sim


def _rho(sim):
    return sim.f.sum(axis=2)


def test_initial_profile_closed_form_values(ora):
    rho_l, rho_v, W, R = 0.4, 0.02, 5.0, 10.0
    sim = _init(ora, 60, 50, [(30.0, 25.0, R)], W=W, rho_l=rho_l, rho_v=rho_v)
    rho = _rho(sim)
    # populations at rest: f_i = w_i rho exactly
    np.testing.assert_allclose(sim.f[1:-1], rho[1:-1, :, None] * W_LB, rtol=1e-15, atol=0)
    # r = R (nodes (40, 25), (20, 25), (30, 35)): the mean of the two densities
    mid = 0.5 * (rho_l + rho_v)
    assert rho[25, 40] == pytest.approx(mid, rel=1e-15)
    assert rho[25, 20] == pytest.approx(mid, rel=1e-15)
    assert rho[35, 30] == pytest.approx(mid, rel=1e-15)
    # r = R -+ W/2 at nodes: centre at a half-integer x
    t1 = math.tanh(1.0)
    sim2 = _init(ora, 60, 50, [(30.5, 25.0, R)], W=W, rho_l=rho_l, rho_v=rho_v)
    rho2 = _rho(sim2)
    # node (38, 25) is at r = 7.5 = R - W/2, node (43, 25) at r = 12.5 = R + W/2
    assert rho2[25, 38] == pytest.approx(rho_v + (rho_l - rho_v) * (1 + t1) / 2, rel=1e-14)
    assert rho2[25, 43] == pytest.approx(rho_v + (rho_l - rho_v) * (1 - t1) / 2, rel=1e-14)
    # far inside / outside
    assert rho[25, 30] == pytest.approx(rho_v + (rho_l - rho_v) * (1 + math.tanh(4.0)) / 2, rel=1e-14)
    assert rho[2, 2] == pytest.approx(rho_v, rel=1e-6)


def test_initial_profile_nearest_image_in_x(ora):
    """A droplet centred at x = 1 on a 40-column lattice: column 39 is at distance 2 (through the seam), not 38."""
    rho_l, rho_v, W, R = 0.4, 0.02, 5.0, 6.0
    sim = _init(ora, 40, 30, [(1.0, 15.0, R)], W=W, rho_l=rho_l, rho_v=rho_v)
    rho = _rho(sim)
    prof = lambda r: rho_v + (rho_l - rho_v) * 0.5 * (1.0 - math.tanh(2.0 * (r - R) / W))
    assert rho[15, 39] == pytest.approx(prof(2.0), rel=1e-15)
    assert rho[15, 3] == pytest.approx(prof(2.0), rel=1e-15)
    assert rho[15, 35] == pytest.approx(prof(6.0), rel=1e-15)
    # mirror symmetry about the centre through the seam
    for d in range(1, 15):
        assert rho[15, (1 + d) % 40] == rho[15, (1 - d) % 40]


def test_initial_profile_overlapping_droplets_take_the_maximum(ora):
    rho_l, rho_v, W = 0.4, 0.02, 5.0
    d1, d2 = (20.0, 20.0, 8.0), (31.0, 20.0, 6.0)
    both = _rho(_init(ora, 60, 40, [d1, d2], W=W, rho_l=rho_l, rho_v=rho_v))
    one = _rho(_init(ora, 60, 40, [d1], W=W, rho_l=rho_l, rho_v=rho_v))
    two = _rho(_init(ora, 60, 40, [d2], W=W, rho_l=rho_l, rho_v=rho_v))
    rows = slice(1, 39)
    np.testing.assert_array_equal(both[rows], np.maximum(one, two)[rows])
    # between the two centres both profiles matter, and the sum would differ from the maximum
    assert both[20, 27] < one[20, 27] + two[20, 27] - rho_v * 0.5


def test_initial_profile_has_no_populations_in_wall_rows(ora):
    sim = _init(ora, 20, 12, [(10.0, 0.5, 5.0)])
    assert np.abs(sim.f[0]).max() == 0.0 and np.abs(sim.f[-1]).max() == 0.0
