"""The piecewise-linear EOS (Eq. 11, break points from Eq. 12-13) through the C-ABI: the host break points against
the reference's and Table 1, the step against the FP64 CPU reference at the three density ratios of Table 1 (a
semicircle droplet on the bottom wall, Sec. 3.1's setup, with a different contact angle in every column), an FP32
slice, the periodic mode, and one adjoint step against the reference's complex-step derivatives."""
import math

import numpy as np
import pytest

from gpu_helpers import oracle_pops

pytestmark = pytest.mark.gpu

# Table 1: (theta_v, theta_m, theta_l, rho_v, rho_l), the vapour density taken as 1
TABLE1 = {10: (0.25, -0.02, 0.3, 1.0, 10.0),
          100: (0.1633, -0.02, 0.33333, 1.0, 100.0),
          1000: (0.2, -0.01, 0.33333, 1.0, 1000.0)}
PRINTED = {10: (1.122, 9.54), 100: (1.486, 94.65), 1000: (1.325, 971.1017)}


@pytest.mark.parametrize("pw", list(TABLE1.values()) + [(0.25, -0.02, 1.0, 1.0, 10.0)],
                         ids=["ratio10", "ratio100", "ratio1000", "liquid_slope_1"])
def test_break_points_and_cap_match_reference(ora, pw):
    import paper_1501_05430_amd as P
    with P.LBM(P.make_params(16, 8, 0.5, piecewise=pw)) as sim:
        info = sim.eos_info()
    r1, r2 = ora.pw_breakpoints(*pw)
    assert info["rho_v"] == pw[3] and info["rho_l"] == pw[4]
    assert info["rho_1"] == pytest.approx(r1, rel=1e-12)
    assert info["rho_2"] == pytest.approx(r2, rel=1e-12)
    assert info["rho_cap"] == pytest.approx(ora.pw_rho_cap(*pw[:3], r1, r2), rel=1e-12)
    ratio = int(pw[4])
    if pw[2] < 1 / 3:
        assert info["rho_1"] == pytest.approx(PRINTED[ratio][0], rel=1e-3)
        assert info["rho_2"] == pytest.approx(PRINTED[ratio][1], rel=1e-4)


def wall_pair(ora, ratio, nx=200, ny=100, precision="f64", R=30.0, **kw):
    import paper_1501_05430_amd as P
    pw = TABLE1[ratio]
    th_b = np.radians(np.linspace(30.0, 150.0, nx))
    th_t = np.radians(np.linspace(120.0, 60.0, nx))
    ref = ora.Sim(nx, ny, 1.0, theta_bottom=th_b, theta_top=th_t, piecewise=pw, **kw)
    ref.init_droplets([nx / 2], [0.5], [R])
    sim = P.LBM(P.make_params(nx, ny, 1.0, precision=precision, piecewise=pw,
                              **P.fp32_options(1.0, precision, piecewise=pw), **kw))
    sim.apply_wetting(th_b, th_t)
    sim.init_droplet(nx / 2, 0.5, R)
    return ref, sim


@pytest.mark.parametrize("ratio", [10, 100, 1000])
def test_wall_droplet_fp64_matches_reference(ora, ratio):
    """200 x 100 (three full 64-column tiles and a ragged one), 300 steps."""
    ref, sim = wall_pair(ora, ratio)
    for n in (1, 299):
        ref.run(n)
        sim.step(n)
        f_ref = oracle_pops(ref)
        err = np.abs(sim.populations() - f_ref).max() / np.abs(f_ref).max()
        assert err <= 1e-12, (n, err)
    assert sim.mass() == pytest.approx(ref.mass(), rel=1e-12)
    assert sim.diag()["psi_clamps"] == 0
    sim.close()


@pytest.mark.parametrize("ratio,kw", [
    (10, dict(wet_iters=0, A=0.0)),                          # Eq. 19 ghost density, plain Shan-Chen force
    (10, dict(tau=0.8, A=-0.3, body_force=(0.0, -1e-5))),
    (100, dict(wet_iters=0)),
    (100, dict(tau=0.8, body_force=(0.0, -1e-5))),
], ids=["r10_eq19_shan_chen", "r10_tau08_gravity", "r100_eq19", "r100_tau08_gravity"])
def test_wall_droplet_fp64_other_settings(ora, ratio, kw):
    ref, sim = wall_pair(ora, ratio, nx=130, ny=60, R=20.0, **kw)
    ref.run(200)
    sim.step(200)
    f_ref = oracle_pops(ref)
    err = np.abs(sim.populations() - f_ref).max() / np.abs(f_ref).max()
    sim.close()
    assert err <= 1e-12, err


@pytest.mark.parametrize("ratio", [100, 1000])
def test_wall_droplet_fp32_shifted_slice(ora, ratio):
    ref, sim = wall_pair(ora, ratio, precision="f32_shifted")
    ref.run(100)
    sim.step(100)
    r_ref, _ = ref.density()
    err = np.abs(sim.rho()[1:-1] - r_ref[1:-1]).max() / TABLE1[ratio][4]
    sim.close()
    assert err <= 1e-5, err


def test_periodic_free_droplet_matches_reference(ora):
    import paper_1501_05430_amd as P
    pw = TABLE1[100]
    ref = ora.Sim(96, 80, 1.0, periodic_y=True, piecewise=pw)
    ref.init_droplets([48.0], [40.0], [20.0])
    sim = P.LBM(P.make_params(96, 82, 1.0, boundary="periodic", piecewise=pw))
    sim.init_droplet(48.0, 41.0, 20.0)
    ref.run(200)
    sim.step(200)
    r_ref, _ = ref.density()
    err = np.abs(sim.rho()[1:-1] - r_ref).max() / np.abs(r_ref).max()
    sim.close()
    assert err <= 1e-12, err


@pytest.mark.parametrize("ratio", [10, 100])
def test_adjoint_step_dot_product(ora, ratio):
    """lambda_1 . (J v) from the reference's complex step equals the adjoint's lambda_0 . v + theta_bar . v_theta
    + G_bar . v_G for random directions v."""
    import torch
    import paper_1501_05430_amd as P
    nx, ny = 40, 14
    pw = TABLE1[ratio]
    rng = np.random.default_rng(ratio)
    tb, tt = np.radians(rng.uniform(40, 140, nx)), np.radians(rng.uniform(40, 140, nx))
    ref = ora.Sim(nx, ny, 1.0, theta_bottom=tb, theta_top=tt, piecewise=pw)
    ref.init_droplets([nx / 2, nx / 5], [0.5, ny * 0.6], [10.0, 3.0])
    ref.run(15)
    f0 = ref.f.copy()
    sim = P.LBM(P.make_params(nx, ny, 1.0, piecewise=pw, enable_adjoint=True))
    sim.apply_wetting(tb, tt)
    dev = sim.device
    lam1 = rng.standard_normal((9, ny - 2, nx))
    lib = lambda f: np.ascontiguousarray(np.moveaxis(f[1:-1], 2, 0))
    t_l0 = torch.empty((9, ny - 2, nx), dtype=torch.float64, device=dev)
    t_th = torch.zeros((2, nx), dtype=torch.float64, device=dev)
    t_G = torch.zeros(2, dtype=torch.float64, device=dev)
    sim.adjoint_step(torch.tensor(lib(f0), device=dev), torch.tensor(lam1, device=dev), t_l0, t_th, t_G)
    sim.stream.synchronize()
    lam0, thb, Gb = t_l0.cpu().numpy(), t_th.cpu().numpy(), t_G.cpu().numpy()
    sim.close()
    h = 1e-30
    bad = []
    for k in range(3):
        v = rng.standard_normal(f0.shape) * 1e-3
        v[0] = v[-1] = 0
        vb, vt, vgf, vgp = rng.standard_normal(nx), rng.standard_normal(nx), rng.standard_normal(), rng.standard_normal()
        fc = ref.run_cplx(1, f0 + 1j * h * v, tb + 1j * h * vb, tt + 1j * h * vt, -1.0 + 1j * h * vgf,
                          -1.0 + 1j * h * vgp)
        lhs = float((lam1 * lib(fc.imag / h)).sum())
        terms = np.array([(lam0 * lib(v)).sum(), (thb[0] * vb).sum(), (thb[1] * vt).sum(), Gb[0] * vgf, Gb[1] * vgp])
        scale = abs(lhs) + np.abs(terms).sum()
        if abs(lhs - terms.sum()) > 1e-10 * scale:
            bad.append((k, lhs, terms.sum()))
    assert not bad, bad
