"""Pins of the reference's complex-step derivative path, which the GPU adjoint is checked against: its real part
is the real step, its imaginary part matches central finite differences of the real step, and the two roles of
G (force prefactor, psi inversion) cancel exactly in the total derivative."""
import math

import numpy as np
import pytest

W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def developed_state(ora, iters=4, A=-0.6, tau=1.0):
    nx, ny = 40, 14
    rng = np.random.default_rng(4)
    tb = np.radians(rng.uniform(50, 130, nx))
    tt = np.radians(rng.uniform(50, 130, nx))
    sim = ora.Sim(nx, ny, 0.75, theta_bottom=tb, theta_top=tt, wet_iters=iters, A=A, tau=tau)
    sim.init_droplets([20.0, 8.0], [0.5, 9.0], [9.0, 3.0])
    sim.run(15)
    return sim, tb, tt


def fluid_direction(sim, rng):
    v = rng.standard_normal(sim.f.shape) * 1e-3
    v[0] = 0
    v[-1] = 0
    return v


@pytest.mark.parametrize("iters,A,tau", [(4, -0.6, 1.0), (0, 0.0, 1.0), (2, -0.3, 0.8)])
def test_complex_step_matches_central_differences(ora, iters, A, tau):
    sim, tb, tt = developed_state(ora, iters, A, tau)
    rng = np.random.default_rng(9)
    f0 = sim.f.copy()
    v = fluid_direction(sim, rng)
    vtb, vtt = rng.standard_normal(sim.nx), rng.standard_normal(sim.nx)
    h = 1e-30
    fc = sim.run_cplx(1, f0 + 1j * h * v, tb + 1j * h * vtb, tt + 1j * h * vtt, -1.0, -1.0)
    # real part is the real step
    sim.run(1)
    np.testing.assert_allclose(fc.real, sim.f, rtol=0, atol=1e-15)
    jvp = fc.imag / h
    eps = 1e-6
    outs = []
    for s in (1, -1):
        t = ora.Sim(sim.nx, sim.ny, 0.75, theta_bottom=tb + s * eps * vtb, theta_top=tt + s * eps * vtt,
                    wet_iters=iters, A=A, tau=tau)
        t.f[:] = f0 + s * eps * v
        t.run(1)
        outs.append(t.f.copy())
    fd = (outs[0] - outs[1]) / (2 * eps)
    assert np.abs(jvp - fd).max() <= 1e-6 * np.abs(fd).max()


def test_force_prefactor_and_psi_roles_cancel(ora):
    sim, tb, tt = developed_state(ora)
    h = 1e-30
    a = sim.run_cplx(1, sim.f, tb, tt, -1.0 + 1j * h, -1.0).imag / h  # d/dG_f
    b = sim.run_cplx(1, sim.f, tb, tt, -1.0, -1.0 + 1j * h).imag / h  # d/dG_psi
    assert np.abs(a).max() > 1e-6
    assert np.abs(a + b).max() <= 1e-12 * np.abs(a).max()


PW10 = (0.25, -0.02, 0.3, 1.0, 10.0)


@pytest.mark.parametrize("T,kw", [
    (0.75, dict(tau=0.8, mrt=(1.2, 1.4, 1.1), kappa=0.5)),
    (1.0, dict(piecewise=PW10, kappa=0.5)),
    (0.75, dict(G_w=(-0.3, -0.2))),
    (1.0, dict(piecewise=PW10, G_w=(-1.5, -1.2), mrt=(1.2, 1.4, 1.1), tau=0.9, kappa=0.5)),
    (0.75, dict(periodic_y=True, kappa=0.3)),
], ids=["mrt_kappa", "paper_setting_pw10", "martys_chen", "martys_chen_mrt_kappa_pw10", "periodic_kappa"])
def test_complex_step_matches_central_differences_for_every_option(ora, T, kw):
    """The complex-step path through the MRT collision with the source, the piecewise-linear EOS, Martys-Chen walls
    and periodic rows: the real part is the real step, and the derivative along a random direction in the state,
    the wall angles and G_f matches central differences of the real step."""
    nx, ny = 40, 14
    rng = np.random.default_rng(5)
    tb = np.radians(rng.uniform(50, 130, nx))
    tt = np.radians(rng.uniform(50, 130, nx))
    sim = ora.Sim(nx, ny, T, theta_bottom=tb, theta_top=tt, **kw)
    sim.init_droplets([20.0, 8.0], [0.5 if not kw.get("periodic_y") else 7.0, 9.0], [9.0, 3.0])
    sim.run(15)
    f0 = sim.f.copy()
    v = rng.standard_normal(f0.shape) * 1e-3
    if not kw.get("periodic_y"):
        v[0] = 0
        v[-1] = 0
    vtb, vtt, vg = rng.standard_normal(nx), rng.standard_normal(nx), rng.standard_normal()
    h = 1e-30
    fc = sim.run_cplx(1, f0 + 1j * h * v, tb + 1j * h * vtb, tt + 1j * h * vtt, -1.0 + 1j * h * vg, -1.0)
    sim.run(1)
    np.testing.assert_allclose(fc.real, sim.f, rtol=0, atol=1e-14 * np.abs(sim.f).max())
    jvp = fc.imag / h
    eps = 1e-6
    # the real step at perturbed inputs (G_f moves alone, so it goes through the complex path with real values,
    # whose real part is the real step as just checked)
    outs = [sim.run_cplx(1, f0 + s * eps * v, tb + s * eps * vtb, tt + s * eps * vtt, -1.0 + s * eps * vg, -1.0).real
            for s in (1, -1)]
    fd = (outs[0] - outs[1]) / (2 * eps)
    assert np.abs(jvp - fd).max() <= 1e-6 * np.abs(fd).max()
