"""GPU parity: the HIP path against the FP64 CPU reference, element by element, through the C-ABI."""
import math

import numpy as np
import pytest

from paper_1501_05430_amd import workloads as W
from gpu_helpers import gpu_sim, oracle_sim, oracle_pops, rel_max

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def small_case(nx, ny, T, th_b_deg, th_t_deg, drops):
    return W.Case(f"small_{nx}x{ny}", nx, ny, T, np.full(nx, math.radians(th_b_deg)),
                  np.full(nx, math.radians(th_t_deg)), [d[0] for d in drops], [d[1] for d in drops],
                  [d[2] for d in drops], 0)


def test_eos_info_matches_reference(ora):
    import paper_1501_05430_amd as P
    for t in [0.5, 0.6, 0.7, 0.85, 0.9]:
        with P.LBM(P.make_params(16, 8, t)) as sim:
            info = sim.eos_info()
        rc, tc, _ = ora.cs_critical()
        rv, rl = ora.cs_maxwell(t * tc)
        assert info["T_c"] == pytest.approx(tc, rel=1e-13)
        assert info["rho_c"] == pytest.approx(rc, rel=1e-12)
        assert info["rho_v"] == pytest.approx(rv, rel=1e-11)
        assert info["rho_l"] == pytest.approx(rl, rel=1e-12)
        assert info["rho_cap"] == pytest.approx(ora.cs_rho_cap(t * tc), rel=1e-12)


@pytest.mark.parametrize("nx,ny,steps,thb,tht,A,iters", [
    (157, 37, 40, 60, 120, -0.6, 4),    # 3 ragged strips in x, ragged rows
    (130, 24, 40, 45, 150, 0.0, 0),     # plain Shan-Chen force, Eq. 19 ghost
    (64, 20, 30, 70, 100, -0.6, 1),     # exactly one wavefront wide (wrap mode)
    (40, 12, 30, 120, 60, -0.6, 4),     # narrower than a wavefront
    (65, 9, 30, 80, 80, -0.3, 7),       # one column past a wavefront: 2 strips, 7 fluid rows
    (200, 5, 20, 50, 130, -0.6, 4),     # 3 fluid rows: every strip touches both walls
    (300, 4, 20, 90, 90, -0.6, 4),      # 2 fluid rows (the minimum)
])
def test_fp64_small_lattices(nx, ny, steps, thb, tht, A, iters):
    drops = [(nx * 0.5, 0.5, min(nx, 2 * ny) * 0.3), (nx * 0.15, ny * 0.6, 3.0)]
    case = small_case(nx, ny, 0.8, thb, tht, drops)
    sim = gpu_sim(case, wet_iters=iters, A=A)
    ref = oracle_sim(case, wet_iters=iters, A=A)
    assert rel_max(sim.populations(), oracle_pops(ref)) < TOL64
    for n in (1, steps - 1):
        sim.step(n)
        ref.run(n)
        assert rel_max(sim.populations(), oracle_pops(ref)) < TOL64, f"after {ref.steps} steps"
    rho_ref, _ = ref.density()
    assert rel_max(sim.rho(), rho_ref) < TOL64  # ghost rows included
    sim.close()


@pytest.mark.parametrize("tau", [0.8, 1.3])
def test_fp64_general_tau(tau):
    case = small_case(140, 30, 0.8, 70, 110, [(70, 0.5, 14.0)])
    sim = gpu_sim(case, tau=tau)
    ref = oracle_sim(case, tau=tau)
    sim.step(30)
    ref.run(30)
    assert rel_max(sim.populations(), oracle_pops(ref)) < TOL64
    sim.close()


def test_fp64_body_force_channel():
    case = small_case(70, 20, 0.8, 90, 90, [])
    sim = gpu_sim(case, body_force=(1e-5, -2e-6))
    ref = oracle_sim(case, body_force=(1e-5, -2e-6))
    sim.step(50)
    ref.run(50)
    assert rel_max(sim.populations(), oracle_pops(ref)) < TOL64
    sim.close()


@pytest.fixture(scope="module")
def c1_pair():
    case = W.c1_neutral()
    sim = gpu_sim(case, check_every=100)
    ref = oracle_sim(case)
    m0 = ref.mass()
    sim.step(case.steps)
    ref.run(case.steps)
    yield case, sim, ref, m0
    sim.close()


def test_c1_full_run_fp64(c1_pair):
    case, sim, ref, m0 = c1_pair
    rho_ref, _ = ref.density()
    assert rel_max(sim.rho(), rho_ref) < TOL64
    assert rel_max(sim.populations(), oracle_pops(ref)) < TOL64


def test_c1_mass_symmetry_angle(c1_pair):
    case, sim, ref, m0 = c1_pair
    m = sim.mass()
    assert abs(m - m0) <= 1e-12 * m0
    d = sim.diag()
    assert d["checks"] == case.steps // 100 and d["nonfinite"] == 0 and d["psi_clamps"] == 0
    assert d["mass"] == pytest.approx(m, rel=1e-13)
    rho = sim.rho()
    assert np.abs(rho[1:-1, 101:200] - rho[1:-1, 99:0:-1]).max() <= 1e-12 * rho.max()
    th, R, xc, yc, n = sim.measure_contact_angle((40, 161, 1, 70), wall=0)
    import oracle
    th_ref, R_ref, xc_ref, yc_ref, n_ref = oracle.measure_contact_angle(ref.density()[0], (40, 161, 1, 70), 0)
    assert n == n_ref
    assert th == pytest.approx(th_ref, abs=1e-9)
    assert R == pytest.approx(R_ref, rel=1e-9)
    assert abs(math.degrees(th) - 90.0) < 1.0


@pytest.mark.parametrize("rows", [1, 3, 8, 16, 64])
def test_strip_rows_bitwise_invariant(rows):
    case = small_case(190, 50, 0.75, 55, 125, [(95, 0.5, 20.0), (30, 30, 6.0)])
    base = gpu_sim(case, strip_rows=16)
    base.step(25)
    other = gpu_sim(case, strip_rows=rows)
    other.step(25)
    assert np.array_equal(base.populations(), other.populations())
    base.close()
    other.close()


@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5, 6, 7, 8])
def test_step_variants_bitwise_invariant(variant):
    case = small_case(190, 50, 0.75, 55, 125, [(95, 0.5, 20.0), (30, 30, 6.0)])
    for prec in ["f64", "f32"]:
        base = gpu_sim(case, precision=prec, step_variant=1)
        base.step(25)
        other = gpu_sim(case, precision=prec, step_variant=variant, strip_rows=5)
        other.step(25)
        assert np.array_equal(base.populations(), other.populations())
        base.close()
        other.close()


def test_graph_replay_matches_plain_launches():
    import paper_1501_05430_amd as P
    case = small_case(150, 40, 0.8, 60, 90, [(75, 0.5, 15.0)])
    a = gpu_sim(case, check_every=8)      # 64-step graphs replayed (16-step chunks), remainder plain
    a.step(100)
    b = gpu_sim(case, check_every=0)
    for _ in range(100):
        b.step(1)                          # plain single launches
    assert np.array_equal(a.populations(), b.populations())
    assert a.diag()["checks"] == 13
    a.close()
    b.close()


def test_checkpoint_resume_bitwise():
    case = small_case(150, 40, 0.8, 60, 90, [(75, 0.5, 15.0)])
    a = gpu_sim(case)
    a.step(20)
    st = a.get_state()
    a.step(17)
    want = a.populations()
    b = gpu_sim(case, init=False)
    b.set_state(st)
    b.step(17)
    assert np.array_equal(b.populations(), want)
    a.close()
    b.close()


def test_nonfinite_is_reported():
    import paper_1501_05430_amd as P
    case = small_case(100, 30, 0.8, 90, 90, [(50, 0.5, 10.0)])
    sim = gpu_sim(case, check_every=5)
    f = sim.populations()
    f[3, 10, 20] = np.nan
    sim.set_populations(f)
    with pytest.raises(P.LbmError) as e:
        sim.step(10)
    assert e.value.code == 4
    assert sim.diag()["nonfinite"] > 0
    sim.close()


@pytest.mark.parametrize("precision", ["f32", "f32_shifted"])
def test_fp32_modes_track_fp64(precision):
    case = small_case(256, 96, 0.7, 60, 90, [(128, W.wall_cap_centre(30.0, math.radians(60)), 30.0)])
    ref = oracle_sim(case)
    sim = gpu_sim(case, precision=precision)
    # a 100-step slice of the spreading transient; longer runs are compared near steady state elsewhere
    for n in (1, 99):
        sim.step(n)
        ref.run(n)
    rho_ref, _ = ref.density()
    rho = sim.rho()
    rv, rl = ref.coexistence()
    err = np.abs(rho[1:-1] - rho_ref[1:-1]).max() / rl
    assert err < 1e-5, err
    sim.close()


@pytest.mark.parametrize("precision", ["f32", "f32_shifted"])
def test_batched_equals_single_instances_bitwise(precision):
    import paper_1501_05430_amd as P
    cases = W.c4_batch(n=12)
    params = [P.make_params(c.nx, c.ny, c.T_over_Tc, precision=precision, check_every=50,
                            **P.fp32_options(c.T_over_Tc, precision)) for c in cases]
    batch = P.LBM(params)
    singles = []
    for i, c in enumerate(cases):
        batch.apply_wetting(c.theta_bottom, c.theta_top, inst=i)
        batch.init_droplet(c.xc, c.yc, c.R, inst=i)
    batch.step(100, inst=-1)
    for i, c in enumerate(cases):
        s = P.LBM(params[i])
        s.apply_wetting(c.theta_bottom, c.theta_top)
        s.init_droplet(c.xc, c.yc, c.R)
        s.step(100)
        assert np.array_equal(batch.populations(inst=i), s.populations()), i
        s.close()
    batch.close()


@pytest.mark.parametrize("inst", [-1, 3])
def test_autotune_keeps_state_and_results(inst):
    import paper_1501_05430_amd as P
    cases = W.c4_batch(n=10)
    params = [P.make_params(c.nx, c.ny, c.T_over_Tc, precision="f32_shifted", check_every=20,
                            **P.fp32_options(c.T_over_Tc, "f32_shifted")) for c in cases]
    sims = [P.LBM(params), P.LBM(params)]
    for s in sims:
        for i, c in enumerate(cases):
            s.apply_wetting(c.theta_bottom, c.theta_top, inst=i)
            s.init_droplet(c.xc, c.yc, c.R, inst=i)
        s.step(7, inst=-1)
    before = [sims[0].populations(inst=i) for i in range(len(cases))]
    rows = sims[0].autotune(inst=inst, trial_steps=2)
    assert rows >= 1
    for i in range(len(cases)):
        assert np.array_equal(sims[0].populations(inst=i), before[i]), i
    for s in sims:
        s.step(40, inst=-1)
    for i in range(len(cases)):
        assert np.array_equal(sims[0].populations(inst=i), sims[1].populations(inst=i)), i
    for s in sims:
        s.close()
