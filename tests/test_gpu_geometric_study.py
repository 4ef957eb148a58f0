"""Sec. 4's studies of the geometric wall on the GPU (density ratio 100 of Table 1, kappa = 0.5, A = -0.6,
Lambda = diag(0,1,...,1), Sec. 3.1's semicircle R = 30): the iteration count of Eq. 21 at a prescribed 15 deg
(Fig. 5), and the instability of the tan form (Eq. 19) near 0 deg that motivates Eq. 20."""
import math

import pytest

pytestmark = pytest.mark.gpu

PW100 = (0.1633, -0.02, 0.33333, 1.0, 100.0)


def settle(deg, iters, nx=800, ny=100, steps=100000, ratio_eos=PW100):
    """(stable, measured angle in deg or None, ghost clamps)."""
    import paper_1501_05430_amd as P
    sim = P.LBM(P.make_params(nx, ny, 1.0, piecewise=ratio_eos, kappa=0.5, wet_iters=iters, check_every=500))
    sim.apply_wetting(math.radians(deg), math.pi / 2)
    sim.init_droplet(nx / 2, 0.5, 30.0)
    try:
        sim.step(steps)
    except P.LbmError as e:
        assert e.code == 4
        d = sim.diag()
        sim.close()
        return False, None, d["ghost_clamps"]
    th = math.degrees(sim.measure_contact_angle((0, nx, 1, ny - 20), 0)[0])
    d = sim.diag()
    sim.close()
    return True, th, d["ghost_clamps"]


def test_iteration_count_at_15_degrees():
    """Fig. 5: the first line of Eq. 21 alone (wet_iters = 1) leaves a prescribed 15 deg at about 30 deg (measured
    29.1; the paper's no-iteration case, about 30), four iterates bring it to 16.7 (the paper: 15.2), and more
    iterates change it little (16.5 at 6, 16.2 at 8). Eq. 19 itself measures 16.5 deg."""
    th = {}
    for k in (0, 1, 4, 6, 8):
        ok, t, _ = settle(15, k)
        assert ok, k
        th[k] = t
    print("\n  " + ", ".join(f"wet_iters={k}: {v:.2f}" for k, v in th.items()))
    assert 25.0 <= th[1] <= 33.0, th
    assert abs(th[4] - 15.0) <= 3.0, th
    assert abs(th[6] - th[4]) <= 1.0 and abs(th[8] - th[4]) <= 1.0, th
    assert abs(th[0] - 15.0) <= 3.0, th


def test_tan_form_fails_near_zero_degrees():
    """Sec. 4: cot(theta) in Eq. 19 grows without bound as theta -> 0, and at 5 deg the tan form drives the ghost
    densities out of range (clamped) until the run diverges, while four iterates of Eq. 21 stay stable."""
    ok, _, clamps = settle(5, 0, nx=1200, steps=20000)
    assert not ok and clamps > 0
    ok, t, clamps = settle(5, 4, nx=1200, steps=20000)
    assert ok and clamps == 0


PW1000 = (0.2, -0.01, 0.33333, 1.0, 1000.0)


def run_cap(deg, R, nx, ny, steps, eos=PW100, start="cap", box_top=10, iters=4):
    """The paper's setting (Table 1 EOS, kappa = 0.5, A = -0.6) with a droplet started as the cap at the prescribed
    angle (start='cap') or as Sec. 3.1's semicircle; returns (stable, attached, measured angle or None, ghost
    clamps). Attached: liquid (rho above the mean of the coexistence pair) in the boundary row."""
    import paper_1501_05430_amd as P
    sim = P.LBM(P.make_params(nx, ny, 1.0, piecewise=eos, kappa=0.5, wet_iters=iters, check_every=500))
    t = math.radians(deg)
    sim.apply_wetting(t, math.pi / 2)
    sim.init_droplet(nx / 2, 0.5 - R * math.cos(t) if start == "cap" else 0.5, R)
    try:
        sim.step(steps)
    except P.LbmError as e:
        assert e.code == 4
        sim.close()
        return False, None, None, None
    rho = sim.rho()
    attached = bool((rho[1] > 0.5 * (eos[3] + eos[4])).any())
    th = None
    if attached:
        th = math.degrees(sim.measure_contact_angle((0, nx, 1, ny - box_top), 0)[0])
    d = sim.diag()
    sim.close()
    return d["nonfinite"] == 0, attached, th, d["ghost_clamps"]


def equal_area_radius(deg, R0=30.0):
    """Radius of the cap at angle deg with the area of Sec. 3.1's semicircle of radius R0: R^2 (t - sin t cos t) =
    pi R0^2 / 2."""
    t = math.radians(deg)
    return math.sqrt(math.pi * R0 * R0 / 2 / (t - math.sin(t) * math.cos(t)))


@pytest.mark.parametrize("ratio,angles", [(100, (15, 30, 45, 90)), (1000, (45, 90))])
def test_angle_range_at_large_density_ratios(ratio, angles):
    """Figs. 6-8: with four iterates the geometric wall holds a range of angles at density ratios of 100 and 1000
    without losing stability (400 x 100, semicircle R = 30, 150 000 steps). Measured: 16.9 / 29.6 / 44.9 / 92.6 deg
    at ratio 100 and 44.6 / 91.6 deg at ratio 1000 for the prescribed values, each within 3 deg (the
    acceptance bound of this test). Fig. 8: the density next to the wall equals the bulk density (no near-wall layer). Obtuse angles
    and the acute ones at ratio 1000 are in the tests below."""
    import paper_1501_05430_amd as P
    eos = PW100 if ratio == 100 else PW1000
    for deg in angles:
        nx, ny = 400, 100
        sim = P.LBM(P.make_params(nx, ny, 1.0, piecewise=eos, kappa=0.5, check_every=500))
        sim.apply_wetting(math.radians(deg), math.pi / 2)
        sim.init_droplet(nx / 2, 0.5, 30.0)
        sim.step(150000)
        th = math.degrees(sim.measure_contact_angle((0, nx, 1, ny - 10), 0)[0])
        r = sim.rho()
        d = sim.diag()
        sim.close()
        assert d["nonfinite"] == 0 and d["ghost_clamps"] == 0, deg
        assert abs(th - deg) <= 3.0, (deg, th)
        assert abs(r[1, 0] - r[30, 0]) <= 1e-3 * r[30, 0], (deg, r[1, 0], r[30, 0])


def test_acute_angles_at_ratio_1000_come_from_the_start_not_the_scheme():
    """At a density ratio of 1000, 15 and 30 deg diverge when the droplet starts as Sec. 3.1's semicircle (the
    spreading from 90 deg), at R = 30 and at R = 60 alike; started as the cap at the prescribed angle with the
    semicircle's area they are stable and hold the angle (measured 12.1 and 29.2 deg; 14.6 and 28.7 at ratio
    100). Sec. 5's claim of a nearly 0-180 deg range at ratio 1000 holds for the scheme; the start decides."""
    for deg, lo, hi in ((15, 10.0, 18.0), (30, 27.0, 33.0)):
        ok, _, _, _ = run_cap(deg, 30.0, 800, 100, 150000, eos=PW1000, start="semi")
        assert not ok, deg
        R = equal_area_radius(deg)
        ok, attached, th, clamps = run_cap(deg, R, 1200, 100, 150000, eos=PW1000)
        print(f"\n  ratio 1000, {deg} deg from the cap of R = {R:.1f}: {th:.2f} deg")
        assert ok and attached and clamps == 0, deg
        assert lo <= th <= hi, (deg, th)


def test_obtuse_overshoot_shrinks_with_resolution():
    """Obtuse caps read high at Sec. 3.1's radius and converge as the droplet is refined (cap start, ratio 100,
    150 000 (R/30)^1.5 steps): 135 deg measures 141.2 / 138.0 / 136.2 deg at R = 30 / 60 / 90, so the overshoot is
    a resolution error (roughly 1/R), within 3 deg at R = 90; 150 deg measures 163.8 / 160.7 (/ 157.2 at R = 120)
    at R = 60 / 90, converging more slowly."""
    th = {}
    for deg, radii in ((135, (30.0, 60.0, 90.0)), (150, (60.0, 90.0))):
        for R in radii:
            nx, ny = int(400 * R / 30), int(100 * R / 30)
            ok, attached, t, clamps = run_cap(deg, R, nx, ny, int(150000 * (R / 30.0) ** 1.5))
            assert ok and attached and clamps == 0, (deg, R)
            th[(deg, R)] = t
    print("\n  " + ", ".join(f"{d} deg R={R:g}: {v:.2f}" for (d, R), v in th.items()))
    assert th[(135, 30.0)] > th[(135, 60.0)] > th[(135, 90.0)] > 135.0, th
    assert abs(th[(135, 90.0)] - 135.0) <= 3.0, th
    assert th[(150, 60.0)] > th[(150, 90.0)] > 150.0, th


def test_iteration_count_at_165_degrees():
    """The 165 deg leg of the iteration study (ratio 100, R = 30): for every iteration count, from the semicircle
    and from the cap, the droplet leaves the wall (it ends on the neutral top wall or floats), and stays there up to
    R = 120 with four iterates (the paper's range figures stop at 150 deg). The run stays finite; Eq. 19 alone
    (wet_iters = 0, cot 165 deg = -3.73) clamps ghost densities below zero from the cap start, the iterates of
    Eq. 21 never do."""
    for start in ("semi", "cap"):
        for k in (0, 1, 4, 8):
            ok, attached, _, clamps = run_cap(165, 30.0, 800, 140, 100000, start=start, iters=k)
            assert ok and not attached, (start, k)
            if k > 0:
                assert clamps == 0, (start, k)
            elif start == "cap":
                assert clamps > 0
