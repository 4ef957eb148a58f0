"""The MRT collision (Eq. 15 with a general relaxation matrix, Eq. 2) and the surface-tension source of Eq. 16-17
through the C-ABI: FP64 steps against the CPU reference (Carnahan-Starling and the piecewise-linear EOS of Table 1,
the paper's Lambda = diag(0,1,...,1) with kappa, and general rates), periodic rows, an FP32 slice, the BGK limit,
bitwise mirror symmetry, and the Laplace law's slope against kappa."""
import math

import numpy as np
import pytest

from gpu_helpers import oracle_pops

pytestmark = pytest.mark.gpu

PW = {10: (0.25, -0.02, 0.3, 1.0, 10.0), 100: (0.1633, -0.02, 0.33333, 1.0, 100.0),
      1000: (0.2, -0.01, 0.33333, 1.0, 1000.0)}
ROCKY = (1.64, 1.54, 1.9)   # s_e, s_eps, s_q far from the stress rate

CASES = {
    "cs085_mrt_k05": (0.85, None, dict(tau=0.8, mrt=ROCKY, kappa=0.5)),
    "cs07_k05": (0.7, None, dict(kappa=0.5)),                        # Sec. 3.1's Lambda with the source
    "cs07_mrt_k05": (0.7, None, dict(tau=0.8, mrt=(1.1, 1.2, 1.3), kappa=0.5)),
    "cs07_mrt": (0.7, None, dict(tau=0.8, mrt=ROCKY)),
    "cs085_k05_eq19_sc": (0.85, None, dict(kappa=0.5, wet_iters=0, A=0.0)),
    "pw10_k05": (1.0, 10, dict(kappa=0.5)),
    "pw100_k09": (1.0, 100, dict(kappa=0.9)),
    "pw1000_k05": (1.0, 1000, dict(kappa=0.5)),
    "pw100_mrt_k05_gravity": (1.0, 100, dict(tau=0.9, mrt=(1.2, 1.4, 1.1), kappa=0.5, body_force=(0.0, -1e-5))),
}


def pair(ora, T, ratio, kw, nx=200, ny=100, precision="f64", R=30.0, th_b=None, th_t=None, drop=True):
    import paper_1501_05430_amd as P
    pw = PW[ratio] if ratio else None
    th_b = np.radians(np.linspace(30.0, 150.0, nx)) if th_b is None else th_b
    th_t = np.radians(np.linspace(120.0, 60.0, nx)) if th_t is None else th_t
    ref = ora.Sim(nx, ny, T, theta_bottom=th_b, theta_top=th_t, piecewise=pw, **kw)
    ref.init_droplets([nx / 2], [0.5], [R])
    lib_kw = {k: v for k, v in kw.items()}
    sim = P.LBM(P.make_params(nx, ny, T, precision=precision, piecewise=pw,
                              **P.fp32_options(T, precision, piecewise=pw), **lib_kw))
    sim.apply_wetting(th_b, th_t)
    sim.init_droplet(nx / 2, 0.5, R)
    return ref, sim


@pytest.mark.parametrize("name", list(CASES))
def test_wall_droplet_fp64_matches_reference(ora, name):
    """200 x 100 (ragged last tile), a different contact angle in every wall column, 300 steps."""
    T, ratio, kw = CASES[name]
    ref, sim = pair(ora, T, ratio, kw)
    for n in (1, 299):
        ref.run(n)
        sim.step(n)
        f_ref = oracle_pops(ref)
        err = np.abs(sim.populations() - f_ref).max() / np.abs(f_ref).max()
        assert err <= 1e-12, (n, err)
    assert sim.mass() == pytest.approx(ref.mass(), rel=1e-12)
    sim.close()


def test_periodic_free_droplet_matches_reference(ora):
    import paper_1501_05430_amd as P
    kw = dict(tau=0.8, mrt=(1.1, 1.2, 1.3), kappa=0.5)
    ref = ora.Sim(96, 80, 0.85, periodic_y=True, **kw)
    ref.init_droplets([48.0, 10.0], [40.0, 3.0], [20.0, 8.0])     # the second droplet crosses the wrap in y
    sim = P.LBM(P.make_params(96, 82, 0.85, boundary="periodic", **kw))
    sim.init_droplet([48.0, 10.0], [41.0, 4.0], [20.0, 8.0])
    ref.run(200)
    sim.step(200)
    r_ref, _ = ref.density()
    err = np.abs(sim.rho()[1:-1] - r_ref).max() / np.abs(r_ref).max()
    sim.close()
    assert err <= 1e-12, err


@pytest.mark.parametrize("name", ["cs07_k05", "pw100_k09"])
def test_fp32_shifted_slice(ora, name):
    T, ratio, kw = CASES[name]
    ref, sim = pair(ora, T, ratio, kw, precision="f32_shifted")
    ref.run(100)
    sim.step(100)
    r_ref, _ = ref.density()
    rl = ref.coexistence()[1]
    err = np.abs(sim.rho()[1:-1] - r_ref[1:-1]).max() / rl
    sim.close()
    assert err <= 1e-5, err


@pytest.mark.parametrize("tau", [0.8, 1.0])
def test_mrt_with_equal_rates_matches_bgk(tau):
    """Rates all 1/tau and kappa = 0 (the MRT kernel path) against the BGK path: the same scheme, so the two agree
    to round-off after 500 steps."""
    import paper_1501_05430_amd as P
    from paper_1501_05430_amd import workloads as W
    case = W.c1_neutral()
    out = []
    for mrt in (None, (1 / tau,) * 3):
        sim = P.LBM(P.make_params(case.nx, case.ny, 0.85, tau=tau, mrt=mrt))
        sim.apply_wetting(math.radians(60.0), math.radians(90.0))
        sim.init_droplet(case.xc, case.yc, case.R)
        sim.step(500)
        out.append(sim.populations())
        sim.close()
    err = np.abs(out[1] - out[0]).max() / np.abs(out[0]).max()
    assert 0 < err <= 1e-13 or err == 0, err


@pytest.mark.parametrize("kw", [dict(tau=0.8, mrt=(1.1, 1.2, 1.3), kappa=0.5), dict(kappa=0.5)],
                         ids=["mrt_kappa", "tau1_kappa"])
@pytest.mark.parametrize("precision", ["f64", "f32", "f32_shifted"])
def test_mirror_symmetry_bitwise(precision, kw):
    """A wall droplet symmetric about x = nx/2 and a free droplet symmetric about both mid-lines stay exactly
    symmetric through the MRT collision and the source term, with general rates and with the paper's relaxation
    matrix diag(0,1,...,1)."""
    import paper_1501_05430_amd as P
    extra = P.fp32_options(0.85, precision)
    sim = P.LBM(P.make_params(200, 100, 0.85, precision=precision, **extra, **kw))
    sim.apply_wetting(math.radians(60.0), math.radians(60.0))
    sim.init_droplet(100.0, 0.5, 30.0)
    sim.step(1500)
    r = sim.rho()[1:-1]
    sim.close()
    assert np.array_equal(r, r[:, (-np.arange(200)) % 200])
    sim = P.LBM(P.make_params(128, 130, 0.85, precision=precision, boundary="periodic", **extra, **kw))
    sim.init_droplet(64.0, 65.0, 24.0)
    sim.step(1500)
    r = sim.rho()[1:-1]
    sim.close()
    assert np.array_equal(r, r[:, (-np.arange(128)) % 128])
    assert np.array_equal(r, np.roll(r[::-1], 1, axis=0))


def laplace_slope(kappa, radii=(16, 20, 24, 28, 32), T=0.85, n=128, steps=8000):
    import paper_1501_05430_amd as P
    import oracle
    res = []
    for R in radii:
        sim = P.LBM(P.make_params(n, n + 2, T, boundary="periodic", kappa=kappa))
        sim.init_droplet(n / 2, n / 2 + 1, float(R))
        sim.step(steps)
        Tabs = sim.eos_info()["T"]
        r = sim.rho()[1:-1]
        sim.close()
        rin, rout = r[n // 2, n // 2], r[0, 0]
        Reff = np.sqrt((r - rout).sum() / (np.pi * (rin - rout)))
        res.append((1 / Reff, oracle.cs_pressure(rin, Tabs) - oracle.cs_pressure(rout, Tabs)))
    x, y = np.array(res).T
    (k, b), *_ = np.linalg.lstsq(np.stack([x, np.ones_like(x)], 1), y, rcond=None)
    return k, b, y.min()


def test_surface_tension_scales_as_one_minus_kappa():
    """Free droplets R = 16..32 in a periodic 128 x 128 box at 0.85 T_c: the Laplace-law slope at kappa = 0.5 is
    half the slope at kappa = 0 (within 6 %: finite interface width; measured 0.483), as the paper states for the
    source."""
    k0, b0, m0 = laplace_slope(0.0)
    k5, b5, m5 = laplace_slope(0.5)
    print(f"\n  sigma(kappa=0) = {k0:.4e}, sigma(kappa=0.5) = {k5:.4e}, ratio {k5 / k0:.4f}")
    # a small finite-size intercept (about 4e-6 either way) is a larger share of the halved pressure jumps
    assert abs(b0) < 0.1 * m0 and abs(b5) < 0.1 * m5
    assert k5 / k0 == pytest.approx(0.5, rel=0.06)


def test_geometric_angles_hold_across_surface_tension():
    """Sec. 5's surface-tension study (Fig. 9): the geometric wall at a density ratio of 100 (Table 1), R = 30 on a
    200 x 100 lattice, prescribed 45 / 90 / 135 deg with kappa = 0, 0.9, 0.98 (surface tension down to 2 %),
    60 000 steps (settled: unchanged to 200 000). Measured here 45.9 / 90.0 / 143.2, 41.9 / 93.1 / 144.8 and
    41.3 / 91.5 / 140.3 deg (the paper reports 46 / 90 / 134 and 45 / 90 / 137 for kappa = 0.9 / 0.98 on a lattice
    it does not state). Checked: stable, within 5 deg of the prescribed angle for 45 and 90 deg and 10 deg for 135
    deg (obtuse caps read high at this resolution), and within 5 deg of each other across kappa."""
    import paper_1501_05430_amd as P
    pw = PW[100]
    got = {}
    for kappa in (0.0, 0.9, 0.98):
        for deg in (45, 90, 135):
            sim = P.LBM(P.make_params(200, 100, 1.0, piecewise=pw, kappa=kappa, check_every=1000))
            sim.apply_wetting(math.radians(deg), math.pi / 2)
            sim.init_droplet(100.0, 0.5, 30.0)
            sim.step(60000)
            got[kappa, deg] = math.degrees(sim.measure_contact_angle((0, 200, 1, 80), 0)[0])
            d = sim.diag()
            sim.close()
            assert d["nonfinite"] == 0 and d["ghost_clamps"] == 0
    print("\n  " + ", ".join(f"kappa={k} set={a}: {v:.2f}" for (k, a), v in got.items()))
    for deg, tol in ((45, 5.0), (90, 5.0), (135, 10.0)):
        vals = [got[k, deg] for k in (0.0, 0.9, 0.98)]
        assert max(abs(v - deg) for v in vals) <= tol, (deg, vals)
        assert max(vals) - min(vals) <= 5.0, (deg, vals)
