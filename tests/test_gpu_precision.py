"""Precision forms at the workloads' full sizes, through the C-ABI.

* 1024 x 512 droplet (T = 0.7 T_c, R = 120, theta in {30, 60, 90, 120, 150} deg): 200-step FP64 and 100-step FP32
  slices against the FP64 CPU reference over the whole lattice, then the full 20 000-step runs of the FP32 forms
  (FP32 arithmetic: unshifted, shifted by rho_v, shifted by rho_l; the mixed form shifted by rho_v) against FP64 on
  the GPU: contact angle, mass, and the density difference, whose growth is printed (run with -s to see it).
* 4096 x 2048 lattice (T = 0.5 T_c, 65 droplets) in the benchmark's launch configuration: 100 steps of FP64 and of
  the FP32 forms shifted by rho_v against the CPU reference over the whole lattice, and the full 10 000 steps of the
  FP32 forms against FP64 on the GPU.
* Mirror symmetry: a droplet symmetric about x = nx/2 (and a free one also about the mid-plane between two equal
  walls) stays exactly symmetric, bit for bit, in every precision.
"""
import math

import numpy as np
import pytest

from paper_1501_05430_amd import workloads as W
from gpu_helpers import gpu_sim, oracle_sim

pytestmark = pytest.mark.gpu

ANGLES = (30, 60, 90, 120, 150)
CHECKS = (5000, 10000, 15000, 20000)
BOX = (0, 1024, 1, 400)          # region of the bottom-wall droplet for the contact-angle fit
TOL64 = 1e-12                    # FP64: max|drho| / max rho
TOL32 = 1e-5                     # FP32: max|drho| / rho_l over a slice
THETA_TOL = 0.5                  # FP32: contact angle, degrees
# FP32 forms: |m - m0| / m0 over 20 000 steps. Shifting by the liquid density stores the vapour's populations as
# w_i (rho - rho_l), about 60 times larger than unshifted ones at this density ratio, with rounding to match.
FP32_MODES = [("f32", None), ("f32_shifted", "rho_v"), ("f32_shifted", "rho_l"), ("f32_shifted_mixed", "rho_v")]
MASS32 = dict(zip(FP32_MODES, (1e-6, 1e-6, 2e-5, 1e-6)))
MASS64 = 1e-13
# FP32 forms within 20 000 steps: max|drho| / rho_l. FP32 arithmetic accumulates its rounding of the force and the
# equilibrium (see test_c2_fp32_full_run_vs_fp64); the mixed form holds the stated 1e-5.
LONG32 = dict(zip(FP32_MODES, (3e-4, 3e-4, 3e-3, TOL32)))
# and the vapour's own relative error at the end of those runs (|drho| / rho over nodes below sqrt(rho_v rho_l)):
# measured at most 1.2e-4, 1.3e-4, 5.5e-4 and 2.4e-5
VAP32 = dict(zip(FP32_MODES, (3e-4, 3e-4, 1.5e-3, 5e-5)))


def coexistence(T):
    import paper_1501_05430_amd as P
    return P.eos_coexistence(T)


def run_c2(deg, precision, shift=None):
    case = W.c2_angle(deg)
    sim = gpu_sim(case, precision=precision, shift=shift or "rho_v")
    m0 = sim.mass()
    rho, mass, done = [], [], 0
    for n in CHECKS:
        sim.step(n - done)
        done = n
        rho.append(sim.rho()[1:-1])
        mass.append(sim.mass())
    th = math.degrees(sim.measure_contact_angle(BOX, 0)[0])
    sim.close()
    return dict(rho=rho, mass=np.array(mass), m0=m0, theta=th)


@pytest.fixture(scope="module")
def c2_fp64():
    cache = {}

    def get(deg):
        if deg not in cache:
            cache[deg] = run_c2(deg, "f64")
        return cache[deg]
    return get


@pytest.mark.parametrize("deg", ANGLES)
def test_c2_slices_vs_reference(deg):
    case = W.c2_angle(deg)
    ref = oracle_sim(case)
    s64 = gpu_sim(case, precision="f64")
    s32 = [gpu_sim(case, precision=p) for p in ("f32", "f32_shifted", "f32_shifted_mixed")]
    rv, rl = ref.coexistence()
    ref.run(100)
    r100, _ = ref.density()
    ref.run(100)
    r200, _ = ref.density()
    e32 = []
    for s in s32:
        s.step(100)
        e32.append(np.abs(s.rho()[1:-1] - r100[1:-1]).max() / rl)
        s.close()
    s64.step(200)
    e64 = np.abs(s64.rho()[1:-1] - r200[1:-1]).max() / np.abs(r200[1:-1]).max()
    print(f"\n  c2 theta={deg}: FP64 200 steps {e64:.1e}, FP32 / shifted / mixed 100 steps {e32[0]:.1e} / {e32[1]:.1e}"
          f" / {e32[2]:.1e}")
    s64.close()
    assert e64 <= TOL64, e64
    assert max(e32) <= TOL32, e32


@pytest.mark.parametrize("deg", ANGLES)
def test_c2_fp64_full_run_conserves_mass(c2_fp64, deg):
    r = c2_fp64(deg)
    drift = np.abs(r["mass"] - r["m0"]).max() / r["m0"]
    assert drift <= MASS64, drift


@pytest.mark.parametrize("mode", FP32_MODES, ids=["f32", "shift_rho_v", "shift_rho_l", "mixed_rho_v"])
@pytest.mark.parametrize("deg", ANGLES)
def test_c2_fp32_full_run_vs_fp64(c2_fp64, deg, mode):
    ref = c2_fp64(deg)
    r = run_c2(deg, *mode)
    rv, rl = coexistence(0.7)
    dth = abs(r["theta"] - ref["theta"])
    drift = np.abs(r["mass"] - r["m0"]).max() / r["m0"]
    errs = [np.abs(a - b).max() / rl for a, b in zip(r["rho"], ref["rho"])]
    vap = ref["rho"][-1] < math.sqrt(rv * rl)
    evap = float((np.abs(r["rho"][-1] - ref["rho"][-1])[vap] / ref["rho"][-1][vap]).max())
    print(f"\n  c2 theta={deg} {mode[0]}{'/' + mode[1] if mode[1] else ''}: theta {r['theta']:.4f} vs {ref['theta']:.4f}"
          f", mass drift {drift:.1e}, max|drho|/rho_l at {CHECKS} = {['%.1e' % e for e in errs]}"
          f", vapour max|drho|/rho at the end {evap:.1e}")
    assert dth <= THETA_TOL, dth
    assert drift <= MASS32[mode], drift
    # Over a 100-step slice every FP32 form stays within 1e-5 of the reference (test above). Over the full run FP32
    # arithmetic drifts to several 1e-5 of rho_l: its rounding of the force and of the equilibrium, about 6e-8
    # relative, is injected every step and acts coherently, while an FP64 run perturbed once by rounding its state
    # to FP32 stays within 1e-6 and relaxes (accumulation, not amplification). The mixed form evaluates those in
    # FP64 and holds 1e-5 over the whole run.
    assert max(errs) <= LONG32[mode], errs
    assert evap <= VAP32[mode], evap


@pytest.mark.parametrize("precision", ["f32_shifted", "f32_shifted_mixed"])
def test_c4_sampled_fp32_instances_vs_reference(precision):
    """The 256-instance batch in FP32 shifted by rho_v (FP32 arithmetic with the FP64 EOS below sqrt(rho_v rho_l),
    or the mixed form), all instances in each launch (two steps per launch), 100 steps: 8 instances drawn with the
    seed, each against the FP64 reference over its own lattice, max |drho| / rho_l <= 1e-5 (the vapour-relative
    error is printed)."""
    import paper_1501_05430_amd as P
    cases = W.c4_batch()
    params = [P.make_params(c.nx, c.ny, c.T_over_Tc, precision=precision,
                            **P.fp32_options(c.T_over_Tc, precision)) for c in cases]
    batch = P.LBM(params)
    for i, c in enumerate(cases):
        batch.apply_wetting(c.theta_bottom, c.theta_top, inst=i)
        batch.init_droplet(c.xc, c.yc, c.R, inst=i)
    batch.step(100, inst=-1)
    pick = sorted(np.random.default_rng(W.SEED).choice(len(cases), 8, replace=False).tolist())
    worst = worst_vap = 0.0
    for i in pick:
        c = cases[i]
        ref = oracle_sim(c)
        ref.run(100)
        rv, rl = ref.coexistence()
        r_ref = ref.density()[0][1:-1]
        r = batch.rho(inst=i)[1:-1]
        err = float(np.abs(r - r_ref).max() / rl)
        vap = r_ref < math.sqrt(rv * rl)
        evap = float((np.abs(r - r_ref)[vap] / r_ref[vap]).max())
        print(f"\n  c4 instance {i} ({c.nx}x{c.ny}, T/T_c {c.T_over_Tc:.3f}, theta {math.degrees(c.theta_bottom[0]):.1f}):"
              f" max|drho|/rho_l {err:.2e}, vapour max|drho|/rho {evap:.2e}")
        worst = max(worst, err)
        worst_vap = max(worst_vap, evap)
    batch.close()
    assert worst <= TOL32, worst
    assert worst_vap <= 2e-5, worst_vap   # measured at most 5.2e-6


@pytest.fixture(scope="module")
def c3_reference():
    case = W.c3_large()
    ref = oracle_sim(case)
    rv, rl = ref.coexistence()
    ref.run(100)
    rho, _ = ref.density()
    return case, rho[1:-1].copy(), rl, rv


@pytest.mark.parametrize("precision", ["f64", "f32_shifted", "f32_shifted_mixed"])
def test_c3_full_size_vs_reference(c3_reference, precision):
    """The benchmark's configuration (device check every 100 steps, default block shape) over 100 steps.

    Compared after the initial acoustic transient: the tanh start is not the equilibrium interface, and the pressure
    wave it launches converges on the centre of the smallest satellite (R = 10) after about R / c_s = 17 steps,
    where it amplifies any rounding pattern (an FP64 run perturbed once by 6e-8 differs there by up to 4e-6 at
    step 20, and FP32 storage by about 1e-5); by step 50 the wave has dispersed."""
    case, rho_ref, rl, rv = c3_reference
    sim = gpu_sim(case, precision=precision, check_every=100)
    sim.step(100)
    rho = sim.rho()[1:-1]
    d = sim.diag()
    sim.close()
    assert d["nonfinite"] == 0
    if precision == "f64":
        err = np.abs(rho - rho_ref).max() / np.abs(rho_ref).max()
        tol = TOL64
    else:
        err = np.abs(rho - rho_ref).max() / rl
        tol = TOL32
        vap = rho_ref < math.sqrt(rv * rl)
        evap = float((np.abs(rho - rho_ref)[vap] / rho_ref[vap]).max())
        print(f"\n  c3 {precision}: vapour max|drho|/rho {evap:.1e}")
        assert evap <= 1e-4, evap   # measured 2.5e-5 (FP32 shifted) and 7.1e-6 (mixed)
    print(f"\n  c3 {precision}: max|drho| {err:.1e}")
    assert err <= tol, err


def test_c3_fp32_forms_over_the_full_run():
    """The 4096 x 2048 workload's 10 000 steps in the benchmark's launch configuration: the FP32 forms shifted by
    rho_v against FP64 on the GPU. At this density ratio (about 1000) the FP32 storage's own rounding accumulates:
    measured max |drho| / rho_l 1.4e-3 with FP32 arithmetic and 1.4e-4 in the mixed form (an FP64 run whose state
    is rounded to FP32 once stays within 8.5e-6 over the same 10 000 steps; FP64 arithmetic throughout, with the
    same storage, reaches 1.6e-4). Held to 3e-3 and 3e-4."""
    case = W.c3_large()
    out = {}
    for precision in ("f64", "f32_shifted", "f32_shifted_mixed"):
        sim = gpu_sim(case, precision=precision, check_every=100)
        rl = sim.coexistence()[1]
        sim.step(10000)
        out[precision] = sim.rho()[1:-1]
        d = sim.diag()
        sim.close()
        assert d["nonfinite"] == 0, precision
    err = {p: float(np.abs(out[p] - out["f64"]).max() / rl) for p in ("f32_shifted", "f32_shifted_mixed")}
    print(f"\n  c3 10 000 steps: max|drho|/rho_l FP32 shifted {err['f32_shifted']:.2e}, mixed {err['f32_shifted_mixed']:.2e}")
    assert err["f32_shifted_mixed"] <= 3e-4, err
    assert err["f32_shifted"] <= 3e-3, err


@pytest.mark.parametrize("workload", ["c2_90", "c3"])
def test_fp64_trajectory_after_one_fp32_rounding(workload):
    """The floor under every FP32 storage form: an FP64 run whose state is rounded to FP32 once, at the start,
    against the unperturbed FP64 run (max |drho| / rho_l printed at each check). Measured: on the 1024 x 512 droplet
    at 90 deg it stays below 4e-7 over 20 000 steps and relaxes; on the 4096 x 2048 lattice (65 droplets, density
    ratio ~1000) it grows to about 8.5e-6 within 10 000 steps, so no form that rounds the state to FP32 every step
    can be expected to hold 1e-5 there over the full run (FP32 storage with FP64 arithmetic reaches 1.6e-4, and
    per-node reference storage, rounding only deviations from w_i rho, about 2e-5). Held to 1e-6 / 3e-5."""
    case = W.c2_angle(90.0) if workload == "c2_90" else W.c3_large()
    steps, every, tol = (20000, 5000, 1e-6) if workload == "c2_90" else (10000, 2000, 3e-5)
    a = gpu_sim(case, precision="f64", check_every=100)
    b = gpu_sim(case, precision="f64", check_every=100)
    rl = a.coexistence()[1]
    b.set_populations(b.populations(device=True).float().double())
    errs = []
    for _ in range(steps // every):
        a.step(every)
        b.step(every)
        errs.append(float(np.abs(b.rho()[1:-1] - a.rho()[1:-1]).max() / rl))
    a.close()
    b.close()
    print(f"\n  {workload}: one FP32 rounding of the FP64 state -> max|drho|/rho_l {['%.1e' % e for e in errs]}")
    assert max(errs) <= tol, errs


def mirrored(rho, axis):
    """rho [fluid rows, nx] under x -> nx - x (periodic, axis 1) or the mid-plane mirror between the walls."""
    if axis == 1:
        return rho[:, (-np.arange(rho.shape[1])) % rho.shape[1]]
    return rho[::-1]


@pytest.mark.parametrize("precision", ["f64", "f32", "f32_shifted", "f32_shifted_mixed"])
def test_wall_droplet_stays_mirror_symmetric_bitwise(precision):
    case = W.c2_angle(150)
    sim = gpu_sim(case, precision=precision)
    for n in (1, 2999):
        sim.step(n)
        rho = sim.rho()[1:-1]
        assert np.array_equal(rho, mirrored(rho, 1)), n
    sim.close()


@pytest.mark.parametrize("precision", ["f64", "f32", "f32_shifted", "f32_shifted_mixed"])
def test_free_droplet_stays_mirror_symmetric_bitwise(precision):
    nx, ny = 128, 130                       # fluid rows 1..128: mirror y <-> 129 - y about y = 64.5
    th = np.full(nx, math.radians(60.0))
    case = W.Case("free_128x128", nx, ny, 0.7, th, th, [nx / 2], [64.5], [24.0], 0)
    sim = gpu_sim(case, precision=precision)
    for n in (1, 1999):
        sim.step(n)
        rho = sim.rho()[1:-1]
        assert np.array_equal(rho, mirrored(rho, 1)), n
        assert np.array_equal(rho, mirrored(rho, 0)), n
    sim.close()


@pytest.mark.parametrize("deg", [60, 90, 120])
def test_c2_measured_angle_settles_near_prescribed(deg):
    """The whole scheme against its own target: after 100 000 steps (FP64, settled to 0.01 deg between 100k and
    300k steps) the fitted contact angle is within 3 deg of the prescribed one. (30 deg settles at 33.0 deg: see
    the next test; a 150 deg droplet keeps oscillating between about 146 and 160 deg at this resolution, reported,
    not tested.)"""
    case = W.c2_angle(deg)
    sim = gpu_sim(case, precision="f64", check_every=10000)
    sim.step(100000)
    th = math.degrees(sim.measure_contact_angle((0, case.nx, 1, 480), 0)[0])
    d = sim.diag()
    sim.close()
    print(f"\n  c2 theta={deg}: measured {th:.2f} deg after 100 000 steps")
    assert d["nonfinite"] == 0 and d["ghost_clamps"] == 0
    assert abs(th - deg) <= 3.0, th


def test_c2_thirty_degrees_offset_does_not_depend_on_resolution():
    """The 1024 x 512 workload's physics at 30 deg settles 3.0 deg high, and the same at half and double the droplet
    radius (measured 33.03 / 33.01 / 33.03 deg at R = 60 / 120 / 240 with the cap start): a fixed offset of the scheme
    with this EOS and temperature, not a discretisation error that refinement would remove. Checked at R = 60 and 120
    (the R = 240 run takes 20 s), each within 3.1 deg of 30 and within 0.1 deg of each other."""
    import paper_1501_05430_amd as P
    th = {}
    for R, nx, ny, steps in ((60.0, 512, 256, 35355), (120.0, 1024, 512, 100000)):
        t = math.radians(30.0)
        sim = P.LBM(P.make_params(nx, ny, 0.7, check_every=5000))
        sim.apply_wetting(t, math.pi / 2)
        sim.init_droplet(nx / 2, W.wall_cap_centre(R, t), R)
        sim.step(steps)
        th[R] = math.degrees(sim.measure_contact_angle((0, nx, 1, ny - 20), 0)[0])
        sim.close()
    print(f"\n  30 deg at T = 0.7 T_c: R = 60 -> {th[60.0]:.2f}, R = 120 -> {th[120.0]:.2f} deg")
    assert abs(th[60.0] - th[120.0]) <= 0.1, th
    assert all(abs(v - 30.0) <= 3.1 for v in th.values()), th


@pytest.mark.parametrize("mixed", [False, True], ids=["fp32", "mixed"])
@pytest.mark.parametrize("ratio", [100, 1000])
def test_fp32_in_the_papers_setting_tracks_fp64(ratio, mixed):
    """The paper's own model (Table 1 EOS, kappa = 0.5 with Lambda = diag(0,1,...,1): the MRT form) on the 1024 x 512
    geometry with a 60 deg cap of radius 120, 20 000 steps: FP32 storage shifted by rho_v (FP64 EOS below
    sqrt(rho_v rho_l)) against FP64 on the GPU. Measured: the angles agree to 0.001 deg (59.83 / 59.59 deg at ratios
    100 / 1000), FP32 mass drift 2e-8 / 7e-9, density difference 2.3e-5 / 1.9e-5 of rho_l. Checked: angle within
    0.5 deg, FP32 mass drift within 1e-6, density difference within 2e-4 of rho_l with FP32 arithmetic and within
    1e-5 in the mixed form (whose MRT collision is FP64 throughout)."""
    import paper_1501_05430_amd as P
    pw = {100: (0.1633, -0.02, 0.33333, 1.0, 100.0), 1000: (0.2, -0.01, 0.33333, 1.0, 1000.0)}[ratio]
    case = W.c2_angle(60)
    out = {}
    p32 = "f32_shifted_mixed" if mixed else "f32_shifted"
    for precision in ("f64", p32):
        sim = P.LBM(P.make_params(case.nx, case.ny, 1.0, precision=precision, piecewise=pw, kappa=0.5,
                                  check_every=1000, **P.fp32_options(1.0, precision, piecewise=pw)))
        sim.apply_wetting(case.theta_bottom, case.theta_top)
        sim.init_droplet(case.xc, case.yc, case.R)
        m0 = sim.mass()
        sim.step(20000)
        th = math.degrees(sim.measure_contact_angle(BOX, 0)[0])
        out[precision] = (sim.rho()[1:-1], abs(sim.mass() - m0) / m0, th, sim.diag())
        sim.close()
    r64, d64, th64, g64 = out["f64"]
    r32, d32, th32, g32 = out[p32]
    err = np.abs(r32 - r64).max() / pw[4]
    print(f"\n  ratio {ratio} {p32}: theta FP64 {th64:.3f} / FP32 {th32:.3f}, mass drift FP64 {d64:.1e} / FP32 "
          f"{d32:.1e}, max|drho|/rho_l {err:.1e}")
    assert g64["nonfinite"] == 0 and g32["nonfinite"] == 0
    assert abs(th32 - th64) <= THETA_TOL
    assert d64 <= MASS64 and d32 <= 1e-6
    assert err <= (TOL32 if mixed else 2e-4), err
