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
