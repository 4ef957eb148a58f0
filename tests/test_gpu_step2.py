"""The two-step kernel (two time steps per launch, lbm_step2.hip) against one-step launches, bit for bit in every
precision, and against the FP64 reference, through the C-ABI. It runs the same per-node arithmetic, so every population must
match exactly: across lattice shapes (ragged tiles, lattices narrower than a tile, the fewest rows), block shapes,
strip heights, odd and even step counts, both EOS, the force and wetting options, the general collisions (MRT with
the surface-tension source, BGK at any tau), checked steps in between and the batched form."""
import math

import numpy as np
import pytest

from paper_1501_05430_amd import workloads as W
from gpu_helpers import gpu_sim, oracle_sim, oracle_pops

pytestmark = pytest.mark.gpu

PW100 = (0.25, -0.03, 0.35, 1.0, 100.0)  # a ratio-100 piecewise EOS (slopes of the Table 1 kind)


def case_of(nx, ny, T, th_b, th_t, drops):
    return W.Case(f"s2_{nx}x{ny}", nx, ny, T, np.full(nx, math.radians(th_b)) if np.isscalar(th_b) else th_b,
                  np.full(nx, math.radians(th_t)), [d[0] for d in drops], [d[1] for d in drops],
                  [d[2] for d in drops], 0)


def pair(case, steps, variant2, precision="f32_shifted", strip_rows=0, check_every=0, **kw):
    one = gpu_sim(case, precision=precision, step_variant=5, check_every=check_every, **kw)
    two = gpu_sim(case, precision=precision, step_variant=variant2, strip_rows=strip_rows, check_every=check_every,
                  **kw)
    one.step(steps)
    two.step(steps)
    a, b = one.populations(), two.populations()
    d1, d2 = one.diag(), two.diag()
    one.close()
    two.close()
    return a, b, d1, d2


@pytest.mark.parametrize("precision", ["f32_shifted", "f32_shifted_mixed", "f64"])
@pytest.mark.parametrize("nx,ny,steps,variant,rows", [
    (300, 80, 40, 11, 0),     # two tiles of 4 wavefronts, default strips
    (300, 80, 41, 11, 7),     # odd step count: the last step is a one-step launch
    (257, 37, 30, 12, 5),     # eight wavefronts, ragged rows
    (130, 24, 30, 9, 3),      # one wavefront: three tiles of 58 or fewer columns
    (61, 20, 24, 10, 1),      # one-row strips
    (40, 12, 20, 11, 64),     # narrower than a tile; one strip holds every row
    (7, 10, 16, 9, 2),        # fewer columns than the tile's halo (columns repeat across lanes)
    (96, 4, 18, 10, 1),       # two fluid rows: every row is a boundary row
    (96, 5, 18, 11, 2),       # three fluid rows
    (64, 6, 22, 9, 1),        # four fluid rows, one-row strips
])
def test_two_step_equals_one_step_bitwise(nx, ny, steps, variant, rows, precision):
    drops = [(nx * 0.5, 0.5, max(2.0, min(nx, 2 * ny) * 0.3)), (nx * 0.2, ny * 0.6, max(1.5, min(nx, ny) * 0.08))]
    th_b = np.radians(np.linspace(35.0, 145.0, nx))
    case = case_of(nx, ny, 0.8, th_b, 110.0, drops)
    a, b, _, _ = pair(case, steps, variant, precision=precision, strip_rows=rows)
    assert np.isfinite(a).all()
    assert np.array_equal(a, b), np.abs(a - b).max()


@pytest.mark.parametrize("precision", ["f32", "f32_shifted", "f32_shifted_mixed", "f64"])
@pytest.mark.parametrize("kw", [dict(A=0.0, wet_iters=0), dict(wet_iters=7, A=-0.3), dict(body_force=(1e-6, -2e-6)),
                                dict(piecewise=PW100), dict(wet_iters=1)])
def test_two_step_options_bitwise(precision, kw):
    # T = 0.8: the plain Shan-Chen force (A = 0) diverges within 30 steps on this lattice at 0.7 T_c
    case = case_of(200, 60, 0.8 if "piecewise" not in kw else 0.5, 50.0, 125.0, [(100, 0.5, 22.0), (40, 35, 7.0)])
    extra = dict(kw)
    pw = extra.pop("piecewise", None)
    if pw is not None:
        import paper_1501_05430_amd as P
        extra.update(piecewise=pw)
        one = P.LBM(P.make_params(case.nx, case.ny, 0.5, precision=precision, step_variant=5,
                                  **P.fp32_options(0.5, precision, piecewise=pw), **extra))
        two = P.LBM(P.make_params(case.nx, case.ny, 0.5, precision=precision, step_variant=11, strip_rows=9,
                                  **P.fp32_options(0.5, precision, piecewise=pw), **extra))
        for s in (one, two):
            s.apply_wetting(case.theta_bottom, case.theta_top)
            s.init_droplet(case.xc, case.yc, case.R)
            s.step(36)
        a, b = one.populations(), two.populations()
        one.close()
        two.close()
    else:
        a, b, _, _ = pair(case, 36, 11, precision=precision, strip_rows=9, **extra)
    assert np.isfinite(a).all()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("check_every", [1, 3, 8, 100])
def test_checked_steps_between_two_step_launches(check_every):
    """A check reads its step's input state: a checked step paired with the unchecked step before it is the second
    step of a checked two-step launch, any other checked step a checked one-step launch. The state, the checks and
    the mass they report match a run of one-step launches only (the mass up to the order of its sums)."""
    case = case_of(150, 40, 0.8, 60.0, 90.0, [(75, 0.5, 15.0)])
    a, b, d1, d2 = pair(case, 57, 11, check_every=check_every)
    assert np.array_equal(a, b)
    assert d1["checks"] == d2["checks"] > 0
    assert d2["mass"] == pytest.approx(d1["mass"], rel=1e-12)
    assert d2["nonfinite"] == d1["nonfinite"] == 0


@pytest.mark.parametrize("precision", ["f32_shifted", "f64"])
@pytest.mark.parametrize("check_every,steps", [(2, 20), (5, 23)])
def test_checked_two_step_launches_count_the_clamps(precision, check_every, steps):
    """Checked two-step launches count what checked one-step launches count. A droplet started above the largest
    density with real psi (0.5 against 0.458 at 0.85 T_c) makes psi clamp in the fluid and the ghost densities clamp
    at the walls for the first steps; checks every 2 steps (each the second step of a two-step launch) and every 5
    (an odd period: checked one-step launches, the final check inside a two-step launch) give the same checks, psi
    clamps, ghost-row clamps and non-finite counts as one-step launches, the mass up to the order of its sums, the
    state bit for bit."""
    nx, ny = 96, 40
    th = np.radians(np.linspace(40.0, 140.0, nx))
    case = W.Case("s2_clamp", nx, ny, 0.85, th, th[::-1].copy(), [48.0], [0.5], [14.0], 0)
    out = []
    for variant in (5, 11):
        sim = gpu_sim(case, precision=precision, step_variant=variant, check_every=check_every, init=False)
        sim.init_droplet(case.xc, case.yc, case.R, rho_l=0.5)
        sim.step(steps)
        out.append((sim.populations(), sim.diag()))
        sim.close()
    (a, d1), (b, d2) = out
    assert d1["psi_clamps"] > 0 and d1["ghost_clamps"] > 0, d1
    assert np.array_equal(a, b)
    for k in ("checks", "psi_clamps", "ghost_clamps", "nonfinite"):
        assert d2[k] == d1[k], (k, d1, d2)
    assert d2["mass"] == pytest.approx(d1["mass"], rel=1e-12)


def test_graph_chunks_and_remainders_bitwise():
    case = case_of(180, 50, 0.75, 70.0, 95.0, [(90, 0.5, 18.0)])
    one = gpu_sim(case, precision="f32_shifted", step_variant=5, check_every=10)
    two = gpu_sim(case, precision="f32_shifted", check_every=10, step_variant=11)
    for n in (1, 7, 20, 33, 64, 2):
        one.step(n)
        two.step(n)
        assert np.array_equal(one.populations(), two.populations()), n
    assert one.diag()["checks"] == two.diag()["checks"]
    one.close()
    two.close()


def test_batched_two_step_equals_single_contexts():
    import paper_1501_05430_amd as P
    rng = np.random.default_rng(7)
    cases = []
    for k in range(6):
        nx, ny = [(64, 32), (128, 64), (97, 21), (256, 40), (33, 9), (200, 70)][k]
        th = math.radians(rng.uniform(30, 150))
        cases.append(W.Case(f"b{k}", nx, ny, rng.uniform(0.6, 0.9), np.full(nx, th), np.full(nx, math.pi / 2),
                            [nx / 2], [W.wall_cap_centre(0.3 * ny, th)], [0.3 * ny], 0))
    params = [P.make_params(c.nx, c.ny, c.T_over_Tc, precision="f32_shifted", step_variant=10, strip_rows=6,
                            **P.fp32_options(c.T_over_Tc, "f32_shifted")) for c in cases]
    batch = P.LBM(params)
    for i, c in enumerate(cases):
        batch.apply_wetting(c.theta_bottom, c.theta_top, inst=i)
        batch.init_droplet(c.xc, c.yc, c.R, inst=i)
    batch.step(31, inst=-1)
    for i, c in enumerate(cases):
        single = gpu_sim(c, precision="f32_shifted", step_variant=5)
        single.step(31)
        assert np.array_equal(batch.populations(inst=i), single.populations()), i
        single.close()
    batch.close()


@pytest.mark.parametrize("check_every", [2, 5])
def test_batched_checked_two_step_launches_per_instance(check_every):
    """Checks inside two-step launches of a batch: the k_finalize_diag fold over each instance's range of the
    two-step task table gives every instance the checks, clamp counts and mass (up to the order of its sums) of the
    same instance stepped alone with one-step launches (with a period of 2 every check is inside a two-step launch;
    with 5, only the final one). Two of the five instances start above the largest density with real psi, so
    their psi and ghost-row clamp counts are not zero."""
    import paper_1501_05430_amd as P
    rng = np.random.default_rng(11)
    cases, rho_l = [], []
    for k, (nx, ny) in enumerate([(64, 32), (97, 21), (150, 40), (33, 9), (128, 64)]):
        th = np.radians(np.linspace(rng.uniform(30, 60), rng.uniform(120, 150), nx))
        T = 0.85 if k in (1, 2) else rng.uniform(0.6, 0.9)
        cases.append(W.Case(f"bc{k}", nx, ny, T, th, th[::-1].copy(), [nx / 2], [0.5], [0.35 * ny], 0))
        rho_l.append(0.5 if k in (1, 2) else 0.0)
    params = [P.make_params(c.nx, c.ny, c.T_over_Tc, precision="f32_shifted", step_variant=9, strip_rows=5,
                            check_every=check_every, **P.fp32_options(c.T_over_Tc, "f32_shifted")) for c in cases]
    batch = P.LBM(params)
    for i, c in enumerate(cases):
        batch.apply_wetting(c.theta_bottom, c.theta_top, inst=i)
        batch.init_droplet(c.xc, c.yc, c.R, inst=i, rho_l=rho_l[i])
    batch.step(23, inst=-1)
    clamps = [0, 0]
    for i, c in enumerate(cases):
        single = gpu_sim(c, precision="f32_shifted", step_variant=5, check_every=check_every, init=False)
        single.init_droplet(c.xc, c.yc, c.R, rho_l=rho_l[i])
        single.step(23)
        d1, d2 = single.diag(), batch.diag(inst=i)
        assert np.array_equal(batch.populations(inst=i), single.populations()), i
        for k in ("checks", "psi_clamps", "ghost_clamps", "nonfinite"):
            assert d2[k] == d1[k], (i, k, d1, d2)
        assert d2["mass"] == pytest.approx(d1["mass"], rel=1e-12), i
        if rho_l[i] > 0:
            clamps[0] += d1["psi_clamps"]
            clamps[1] += d1["ghost_clamps"]
        single.close()
    batch.close()
    assert clamps[0] > 0 and clamps[1] > 0, clamps


def test_selection_outside_the_two_step_form_steps_one_at_a_time():
    """Periodic rows are one-step only: a context asking for the two-step kernel runs them with one-step launches
    (same results as asking for one-step launches)."""
    case = case_of(120, 40, 0.8, 60.0, 90.0, [(60, 0.5, 12.0)])
    a, b, _, _ = pair(case, 15, 11, boundary="periodic")
    assert np.array_equal(a, b)


GENERAL = [dict(kappa=0.5), dict(mrt=(1.2, 0.8, 1.1), kappa=-0.4), dict(mrt=(0.9, 1.3, 1.0), tau=0.8),
           dict(tau=0.8), dict(tau=1.3, A=-0.3, body_force=(1e-6, -2e-6)), dict(kappa=0.5, piecewise=PW100),
           dict(boundary="martys_chen", G_w=(-0.3, -0.25)),
           dict(boundary="martys_chen", G_w=(-0.35, -0.2), tau=0.8, kappa=0.4)]


@pytest.mark.parametrize("precision", ["f32_shifted", "f32_shifted_mixed", "f64"])
@pytest.mark.parametrize("kw", GENERAL)
@pytest.mark.parametrize("variant,rows", [(11, 9), (9, 4)])
def test_two_step_general_collision_bitwise(precision, kw, variant, rows):
    """The general instance of the two-step kernel (MRT of Eq. 15 with the source of Eq. 16-17, BGK at any tau,
    Martys-Chen walls of Eq. 14) against one-step launches of the general one-step kernel, bit for bit, over 36
    steps."""
    import paper_1501_05430_amd as P
    T = 0.5 if "piecewise" in kw else 0.8
    case = case_of(200, 60, T, 50.0, 125.0, [(100, 0.5, 22.0), (40, 35, 7.0)])
    extra = dict(kw)
    pw = extra.pop("piecewise", None)
    sims = []
    for v, h in ((5, 0), (variant, rows)):
        s = P.LBM(P.make_params(case.nx, case.ny, T, precision=precision, step_variant=v, strip_rows=h,
                                piecewise=pw, **P.fp32_options(T, precision, piecewise=pw), **extra))
        s.apply_wetting(case.theta_bottom, case.theta_top)
        s.init_droplet(case.xc, case.yc, case.R)
        s.step(36)
        sims.append(s)
    a, b = sims[0].populations(), sims[1].populations()
    for s in sims:
        s.close()
    assert np.isfinite(a).all()
    assert np.array_equal(a, b), np.abs(a - b).max()


@pytest.mark.parametrize("kw", [dict(kappa=0.5), dict(mrt=(1.2, 0.8, 1.1), tau=0.9),
                                dict(boundary="martys_chen", G_w=(-0.3, -0.2))])
def test_two_step_general_collision_vs_reference(kw):
    """FP64 through two-step launches of the general kernel against the FP64 reference, element by element
    (1e-12 of the largest population) after 60 steps."""
    case = case_of(160, 48, 0.75, 55.0, 100.0, [(80, W.wall_cap_centre(16.0, math.radians(55)), 16.0), (30, 30, 6)])
    sim = gpu_sim(case, precision="f64", step_variant=11, strip_rows=7, **kw)
    ref = oracle_sim(case, **{k: v for k, v in kw.items() if k != "boundary"})  # G_w selects the reference's walls
    sim.step(60)
    ref.run(60)
    f_ref = oracle_pops(ref)
    err = np.abs(sim.populations() - f_ref).max() / np.abs(f_ref).max()
    sim.close()
    assert err <= 1e-12, err


def test_batched_two_step_mixes_collisions():
    """One two-step launch over instances with different collisions (MRT with the source, BGK at tau = 0.8 and 0.9)
    equals each instance stepped alone with one-step launches, bit for bit. (A tau = 1 BGK instance in such a batch
    takes the general BGK form, whose rounding differs from the tau = 1 specialisation's, so none is included.)"""
    import paper_1501_05430_amd as P
    opts = [dict(tau=0.9), dict(kappa=0.5), dict(tau=0.8), dict(mrt=(1.2, 0.8, 1.1), kappa=0.3)]
    cases = [case_of(nx, ny, 0.8, th, 90.0, [(nx / 2, 0.5, 0.3 * ny)])
             for nx, ny, th in ((128, 48, 60.0), (97, 33, 120.0), (200, 40, 80.0), (64, 64, 45.0))]
    params = [P.make_params(c.nx, c.ny, 0.8, precision="f32_shifted", step_variant=11, strip_rows=6,
                            **P.fp32_options(0.8, "f32_shifted"), **o) for c, o in zip(cases, opts)]
    batch = P.LBM(params)
    for i, c in enumerate(cases):
        batch.apply_wetting(c.theta_bottom, c.theta_top, inst=i)
        batch.init_droplet(c.xc, c.yc, c.R, inst=i)
    batch.step(24, inst=-1)
    for i, (c, o) in enumerate(zip(cases, opts)):
        single = gpu_sim(c, precision="f32_shifted", step_variant=5, **o)
        single.step(24)
        assert np.array_equal(batch.populations(inst=i), single.populations()), (i, o)
        single.close()
    batch.close()


@pytest.mark.parametrize("steps", [100, 101])
def test_two_step_fp32_vs_reference(steps):
    """FP32 shifted storage through two-step launches against the FP64 reference: max |drho| / rho_l <= 1e-5."""
    case = case_of(256, 96, 0.7, 60.0, 90.0, [(128, W.wall_cap_centre(30.0, math.radians(60)), 30.0), (50, 60, 9)])
    sim = gpu_sim(case, precision="f32_shifted", step_variant=11, strip_rows=16)
    ref = oracle_sim(case)
    sim.step(steps)
    ref.run(steps)
    rho_l = ref.coexistence()[1]
    err = np.abs(sim.populations() - oracle_pops(ref)).sum(axis=0).max() / rho_l
    drho = np.abs(sim.rho()[1:-1] - ref.density()[0][1:-1]).max() / rho_l
    print(f"\n  two-step FP32 vs reference after {steps} steps: max|drho|/rho_l = {drho:.2e}")
    assert drho <= 1e-5 and err <= 1e-4
    sim.close()


@pytest.mark.parametrize("precision", ["f32_shifted", "f32_shifted_mixed", "f64"])
def test_two_step_equals_one_step_over_a_long_run(precision):
    """The 1024 x 512 droplet at 90 deg (T = 0.7 T_c, R = 120) over 4000 steps: two-step and one-step launches agree
    bit for bit at every 1000 steps (each kernel inlines the same node arithmetic, whose rounding is spelled out)."""
    case = W.c2_angle(90.0)
    one = gpu_sim(case, precision=precision, step_variant=5)
    two = gpu_sim(case, precision=precision, step_variant=11)  # forced: the comparison must not rest on the default
    for _ in range(4):
        one.step(1000)
        two.step(1000)
        assert np.array_equal(one.populations(), two.populations())
    one.close()
    two.close()
