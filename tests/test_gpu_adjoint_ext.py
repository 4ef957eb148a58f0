"""The adjoint step beyond BGK with geometric walls: the MRT collision with the surface-tension source (Eq. 15-17),
the piecewise-linear EOS in the paper's setting, and Martys-Chen walls (Eq. 14). Dot-product tests against the
reference's complex-step directional derivatives: lambda_1 . (J v) = lambda_0 . v + theta_bar . v_theta
+ G_bar . v_G for random directions in every input, and for each input alone."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

PW10 = (0.25, -0.02, 0.3, 1.0, 10.0)

CASES = {
    # name: (nx, ny, T, keyword arguments shared by the reference and the library)
    "mrt_kappa": (40, 14, 0.75, dict(tau=0.8, mrt=(1.2, 1.4, 1.1), kappa=0.5)),
    "paper_setting_pw10": (40, 14, 1.0, dict(piecewise=PW10, kappa=0.5)),
    "kappa_eq19_sc": (33, 6, 0.75, dict(kappa=0.3, wet_iters=0, A=0.0)),
    "mrt_only_ny4": (64, 4, 0.75, dict(tau=1.3, mrt=(1.6, 1.5, 1.9), wet_iters=7)),
    "martys_chen": (40, 14, 0.75, dict(G_w=(-0.3, -0.2))),
    "smallest_lattice": (2, 4, 0.75, dict(tau=0.9)),
    "martys_chen_mrt_kappa_pw10": (40, 14, 1.0, dict(piecewise=PW10, kappa=0.5, G_w=(-1.5, -1.2), tau=0.9,
                                                    mrt=(1.2, 1.4, 1.1), body_force=(1e-5, -2e-6))),
}


def to_lib(f):
    return np.ascontiguousarray(np.moveaxis(f[1:-1], 2, 0))


@pytest.mark.parametrize("name", list(CASES))
def test_adjoint_step_dot_product(ora, name):
    import torch
    import paper_1501_05430_amd as P
    nx, ny, T, kw = CASES[name]
    rng = np.random.default_rng(len(name))
    tb, tt = np.radians(rng.uniform(40, 140, nx)), np.radians(rng.uniform(40, 140, nx))
    ref = ora.Sim(nx, ny, T, theta_bottom=tb, theta_top=tt, **kw)
    ref.init_droplets([nx / 2, nx / 5], [0.5, ny * 0.6], [min(nx, 2 * ny) * 0.25, 2.0])
    ref.run(15)
    f0 = ref.f.copy()
    lib_kw = {k: v for k, v in kw.items() if k != "G_w"}
    if "G_w" in kw:
        lib_kw.update(boundary="martys_chen", G_w=kw["G_w"])
    sim = P.LBM(P.make_params(nx, ny, T, enable_adjoint=True, **lib_kw))
    sim.apply_wetting(tb, tt)
    dev = sim.device
    lam1 = rng.standard_normal((9, ny - 2, nx))
    t_l0 = torch.empty((9, ny - 2, nx), dtype=torch.float64, device=dev)
    t_th = torch.zeros((2, nx), dtype=torch.float64, device=dev)
    t_G = torch.zeros(2, dtype=torch.float64, device=dev)
    sim.adjoint_step(torch.tensor(to_lib(f0), device=dev), torch.tensor(lam1, device=dev), t_l0, t_th, t_G)
    sim.stream.synchronize()
    lam0, thb, Gb = t_l0.cpu().numpy(), t_th.cpu().numpy(), t_G.cpu().numpy()
    sim.close()
    if "G_w" in kw:
        assert np.all(thb == 0.0)   # the walls do not depend on the angles
    h = 1e-30
    dirs = []
    for _ in range(3):
        v = rng.standard_normal(f0.shape) * 1e-3
        v[0] = v[-1] = 0
        dirs.append((v, rng.standard_normal(nx), rng.standard_normal(nx), rng.standard_normal(), rng.standard_normal()))
    z = np.zeros(f0.shape)
    dirs += [(z, rng.standard_normal(nx), np.zeros(nx), 0.0, 0.0), (z, np.zeros(nx), rng.standard_normal(nx), 0.0, 0.0),
             (z, np.zeros(nx), np.zeros(nx), 1.0, 0.0), (z, np.zeros(nx), np.zeros(nx), 0.0, 1.0)]
    bad = []
    for k, (v, vb, vt, vgf, vgp) in enumerate(dirs):
        fc = ref.run_cplx(1, f0 + 1j * h * v, tb + 1j * h * vb, tt + 1j * h * vt, -1.0 + 1j * h * vgf,
                          -1.0 + 1j * h * vgp)
        lhs = float((lam1 * to_lib(fc.imag / h)).sum())
        terms = np.array([(lam0 * to_lib(v)).sum(), (thb[0] * vb).sum(), (thb[1] * vt).sum(), Gb[0] * vgf, Gb[1] * vgp])
        scale = abs(lhs) + np.abs(terms).sum() + 1e-300
        if abs(lhs - terms.sum()) > 1e-10 * scale:
            bad.append((k, lhs, float(terms.sum()), (lhs - terms.sum()) / scale))
    assert not bad, bad


def test_rollout_gradient_in_the_papers_setting_vs_central_fd():
    """End to end in the paper's own model (Table 1 EOS at a density ratio of 10, kappa = 0.5 with the relaxation
    matrix diag(0,1,...,1), A = -0.6): a semicircle R = 20 on a 128 x 64 lattice with wall angles 90 deg +- N(0, 10 deg)
    per node, 1000 steps, loss ||rho - rho_target|| against the run with 60 deg walls. The checkpointed rollout's
    gradient with respect to the wall angles matches central finite differences (h = 1e-6) of the GPU forward run
    at the contact lines, at random columns and on the top wall; dL/dG_f + dL/dG_psi = 0 (geometric walls)."""
    import torch
    import paper_1501_05430_amd as P
    from paper_1501_05430_amd.autograd import Rollout, rollout
    nx, ny, steps = 128, 64, 1000
    rng = np.random.default_rng(1501)
    tb0 = np.radians(90.0 + rng.normal(0.0, 10.0, nx))
    tt0 = np.radians(90.0 + rng.normal(0.0, 10.0, nx))
    sim = P.LBM(P.make_params(nx, ny, 1.0, piecewise=PW10, kappa=0.5, enable_adjoint=True))
    sim.apply_wetting(tb0, tt0)
    sim.init_droplet(nx / 2, 0.5, 20.0)
    f0 = sim.populations(device=True)
    th60 = np.full(nx, np.radians(60.0))
    sim.apply_wetting(th60, th60)
    sim.set_populations(f0)
    sim.step(steps)
    target = sim.rho(device=True)[1:-1].clone()

    def loss(b, t):
        sim.apply_wetting(b, t)
        sim.set_populations(f0)
        sim.step(steps)
        return float(torch.linalg.norm(sim.rho(device=True)[1:-1] - target))

    tb = torch.tensor(tb0, dtype=torch.float64, requires_grad=True)
    tt = torch.tensor(tt0, dtype=torch.float64, requires_grad=True)
    rho = rollout(tb, tt, -1.0, sim, f0, steps, seg=100)
    L = torch.linalg.norm(rho - target.to(rho.device))
    L.backward()
    gb, gt = tb.grad.numpy(), tt.grad.numpy()
    assert float(L.detach()) == pytest.approx(loss(tb0, tt0), rel=1e-13)
    h = 1e-6
    fd, ad = [], []
    for wall, cols in ((0, [42, 43, 44, 45, 83, 84, 85, 86, 10, 110]), (1, [5, 64])):
        for c in cols:
            vals = []
            for sgn in (1, -1):
                b, t = tb0.copy(), tt0.copy()
                (b if wall == 0 else t)[c] += sgn * h
                vals.append(loss(b, t))
            fd.append((vals[0] - vals[1]) / (2 * h))
            ad.append((gb if wall == 0 else gt)[c])
    sim.close()
    fd, ad = np.array(fd), np.array(ad)
    print("\n  max |adjoint - FD| / max |FD| =", np.abs(ad - fd).max() / np.abs(fd).max())
    assert np.abs(fd).max() > 0
    assert np.abs(ad - fd).max() <= 1e-4 * np.abs(fd).max(), np.c_[ad, fd]
    gf, gpsi = Rollout.last_G_parts
    assert abs(gf + gpsi) <= 1e-9 * abs(gf)


@pytest.mark.parametrize("nx,ny,T,kw", [
    (40, 12, 0.75, dict(tau=0.8, body_force=(1e-5, -2e-6))),
    (33, 5, 0.75, dict(A=0.0)),
    (40, 12, 1.0, dict(piecewise=PW10, kappa=0.5, tau=0.9, mrt=(1.2, 1.4, 1.1))),
], ids=["bgk", "shan_chen_5rows", "mrt_kappa_pw10"])
def test_adjoint_step_dot_product_periodic_rows(ora, nx, ny, T, kw):
    """Periodic rows (the library's ny + 2 rows with rows 1 .. ny fluid, the reference's ny rows): a droplet across
    the wrap in y; the same dot-product test, the wall angles taking no part."""
    import torch
    import paper_1501_05430_amd as P
    rng = np.random.default_rng(ny)
    ref = ora.Sim(nx, ny, T, periodic_y=True, **kw)
    ref.init_droplets([nx / 2, nx / 5], [1.0, ny * 0.6], [min(nx, 2 * ny) * 0.3, 2.0])
    ref.run(15)
    f0 = ref.f.copy()
    lib = lambda f: np.ascontiguousarray(np.moveaxis(f, 2, 0))   # [ny][nx][9] -> [9][ny][nx], every row fluid
    sim = P.LBM(P.make_params(nx, ny + 2, T, boundary="periodic", enable_adjoint=True, **kw))
    dev = sim.device
    lam1 = rng.standard_normal((9, ny, nx))
    t_l0 = torch.empty((9, ny, nx), dtype=torch.float64, device=dev)
    t_th = torch.zeros((2, nx), dtype=torch.float64, device=dev)
    t_G = torch.zeros(2, dtype=torch.float64, device=dev)
    sim.adjoint_step(torch.tensor(lib(f0), device=dev), torch.tensor(lam1, device=dev), t_l0, t_th, t_G)
    sim.stream.synchronize()
    lam0, thb, Gb = t_l0.cpu().numpy(), t_th.cpu().numpy(), t_G.cpu().numpy()
    sim.close()
    assert np.all(thb == 0.0)
    h = 1e-30
    th = np.full(nx, np.pi / 2)
    bad = []
    for k in range(4):
        v = rng.standard_normal(f0.shape) * 1e-3 if k < 3 else np.zeros(f0.shape)
        vgf, vgp = (rng.standard_normal(), rng.standard_normal()) if k != 3 else (1.0, 0.0)
        fc = ref.run_cplx(1, f0 + 1j * h * v, th, th, -1.0 + 1j * h * vgf, -1.0 + 1j * h * vgp)
        lhs = float((lam1 * lib(fc.imag / h)).sum())
        terms = np.array([(lam0 * lib(v)).sum(), Gb[0] * vgf, Gb[1] * vgp])
        scale = abs(lhs) + np.abs(terms).sum() + 1e-300
        if abs(lhs - terms.sum()) > 1e-10 * scale:
            bad.append((k, lhs, float(terms.sum()), (lhs - terms.sum()) / scale))
    assert not bad, bad


def test_wall_angles_recovered_by_gradient_descent():
    """The adjoint put to its use: from walls at 90 deg, Adam on the rollout gradient finds wall angles that
    reproduce the density field of a 60 deg run (128 x 64, 0.7 T_c, semicircle R = 20, 1000 steps). Measured: the
    loss falls from 3.90 to 0.016 in 20 iterations, where over the wetted columns (|x - 64| < 30) the angle averages
    64.8 deg (columns under the droplet, which the density barely depends on, move less)."""
    import math
    import torch
    import paper_1501_05430_amd as P
    from paper_1501_05430_amd.autograd import rollout
    nx, ny, steps = 128, 64, 1000
    sim = P.LBM(P.make_params(nx, ny, 0.7, enable_adjoint=True))
    sim.apply_wetting(math.pi / 2, math.pi / 2)
    sim.init_droplet(nx / 2, 0.5, 20.0)
    f0 = sim.populations(device=True)
    sim.apply_wetting(np.full(nx, math.radians(60.0)), np.full(nx, math.pi / 2))
    sim.set_populations(f0)
    sim.step(steps)
    target = sim.rho(device=True)[1:-1].clone()
    tb = torch.full((nx,), math.pi / 2, dtype=torch.float64, requires_grad=True)
    tt = torch.full((nx,), math.pi / 2, dtype=torch.float64)
    opt = torch.optim.Adam([tb], lr=0.03)
    losses, thetas = [], []
    for _ in range(24):
        opt.zero_grad()
        rho = rollout(tb, tt, -1.0, sim, f0, steps, seg=100)
        L = torch.linalg.norm(rho - target.to(rho.device))
        L.backward()
        losses.append(float(L.detach()))
        thetas.append(np.degrees(tb.detach().numpy().copy()))
        opt.step()
        with torch.no_grad():
            tb.clamp_(0.2, math.pi - 0.2)
    sim.close()
    best = int(np.argmin(losses))
    wetted = thetas[best][34:94].mean()
    print(f"\n  loss {losses[0]:.3f} -> {losses[best]:.4f} at iteration {best}; wetted-column mean {wetted:.2f} deg")
    assert losses[best] < 0.05 * losses[0], losses
    assert abs(wetted - 60.0) <= 5.0, wetted


def _adjoint_pair(sim, f64, lam1_32, nx):
    """The reverse step through both entry points at the same FP32-representable state and cotangent."""
    import torch
    dev = f64.device
    out = []
    for dt in (torch.float64, torch.float32):
        l0 = torch.empty(lam1_32.shape, dtype=dt, device=dev)
        th = torch.zeros((2, nx), dtype=torch.float64, device=dev)
        G = torch.zeros(2, dtype=torch.float64, device=dev)
        sim.adjoint_step(f64.to(dt).contiguous(), lam1_32.to(dt).contiguous(), l0, th, G)
        sim.stream.synchronize()
        out.append((l0.cpu().numpy(), th.cpu().numpy(), G.cpu().numpy()))
    return out


@pytest.mark.parametrize("kw,periodic", [(dict(), False), (dict(tau=0.8, mrt=(1.2, 1.4, 1.1), kappa=0.5), False),
                                         (dict(boundary="martys_chen", G_w=(-0.3, -0.2)), False),
                                         (dict(kappa=0.3), True)], ids=["bgk", "mrt_kappa", "martys_chen", "periodic"])
def test_fp32_entry_point_rounds_only_the_output(kw, periodic):
    """lbm_adjoint_step_f32 evaluates the same FP64 arithmetic on the FP32 state and cotangent: theta_bar and G_bar
    equal the FP64 entry point's bit for bit (given the same FP32-representable inputs), and lambda_n is the FP64
    result rounded to FP32 (one extra rounding on the four wall rows that receive the wetting terms: within 2 ulp
    of their largest value)."""
    import math
    import torch
    import paper_1501_05430_amd as P
    nx, ny = 96, 40 if not periodic else 42
    if periodic:
        kw = dict(kw, boundary="periodic")
    sim = P.LBM(P.make_params(nx, ny, 0.75, enable_adjoint=True, **kw))
    rng = np.random.default_rng(3)
    if not periodic:
        sim.apply_wetting(np.radians(rng.uniform(40, 140, nx)), np.radians(rng.uniform(40, 140, nx)))
    sim.init_droplet([48.0, 20.0], [0.5 if not periodic else 20.0, 25.0], [16.0, 4.0])
    sim.step(30)
    f64 = sim.populations(device=True).float().double()
    lam1 = torch.tensor(rng.standard_normal(f64.shape), dtype=torch.float32, device=f64.device)
    (l64, th64, G64), (l32, th32, G32) = _adjoint_pair(sim, f64, lam1, nx)
    sim.close()
    assert np.array_equal(th64, th32) and np.array_equal(G64, G32)
    rounded = l64.astype(np.float32)
    rows = np.ones(ny - 2, bool)
    if not periodic:
        rows[[0, 1, ny - 4, ny - 3]] = False      # fluid rows 1, 2, ny-3, ny-2
    assert np.array_equal(l32[:, rows], rounded[:, rows])
    if not periodic:
        # the wall rows add the wetting terms to the already rounded value: a second rounding of the sum
        w = rounded[:, ~rows]
        assert np.abs(l32[:, ~rows] - w).max() <= 2 * np.spacing(np.float32(np.abs(w).max()))


def test_fp32_reverse_rollout_tracks_fp64():
    """200 reverse steps along an FP32 forward trajectory (128 x 64, 0.7 T_c, heterogeneous walls, cotangent of a
    weighted density sum): the wall-angle gradient accumulated through the FP32 entry point stays within 1e-5 of
    the one through the FP64 entry point (lambda is rounded to FP32 once per step)."""
    import math
    import torch
    import paper_1501_05430_amd as P
    nx, ny, steps = 128, 64, 200
    rng = np.random.default_rng(11)
    tb, tt = np.radians(90 + rng.normal(0, 10, nx)), np.radians(90 + rng.normal(0, 10, nx))
    sim = P.LBM(P.make_params(nx, ny, 0.7, precision="f32", enable_adjoint=True, **P.fp32_options(0.7, "f32")))
    sim.apply_wetting(tb, tt)
    sim.init_droplet(nx / 2, 0.5, 20.0)
    states = []
    for _ in range(steps):
        states.append(sim.populations(device=True).float())
        sim.step(1)
    wgt = torch.tensor(rng.standard_normal((ny - 2, nx)), device=states[0].device)
    res = {}
    for dt in (torch.float64, torch.float32):
        lam = wgt.to(dt).expand(9, ny - 2, nx).contiguous()
        th = torch.zeros((2, nx), dtype=torch.float64, device=lam.device)
        G = torch.zeros(2, dtype=torch.float64, device=lam.device)
        nxt = torch.empty_like(lam)
        for n in range(steps - 1, -1, -1):
            sim.adjoint_step(states[n].to(dt).contiguous(), lam, nxt, th, G)
            lam, nxt = nxt, lam
        sim.stream.synchronize()
        res[dt] = th.cpu().numpy()
    sim.close()
    a, b = res[torch.float32], res[torch.float64]
    err = np.abs(a - b).max() / np.abs(b).max()
    print(f"\n  FP32 vs FP64 reverse rollout: max |dtheta_bar| / max |theta_bar| = {err:.2e}")
    assert np.abs(b).max() > 0 and err <= 1e-5, err
