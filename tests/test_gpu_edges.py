"""Edge cases through the C-ABI: an empty lattice (no droplet), the smallest lattices, the largest lattice the
in-plane 32-bit offsets allow (checked through properties that hold at any size), and calls out of order."""
import math

import numpy as np
import pytest

from gpu_helpers import oracle_pops

pytestmark = pytest.mark.gpu


def test_no_droplet_matches_reference_and_stays_uniform(ora):
    import paper_1501_05430_amd as P
    nx, ny = 96, 40
    th = np.radians(np.linspace(30.0, 150.0, nx))
    ref = ora.Sim(nx, ny, 0.7, theta_bottom=th, theta_top=th[::-1].copy())
    ref.init_droplets([], [], [])
    sim = P.LBM(P.make_params(nx, ny, 0.7))
    sim.apply_wetting(th, th[::-1].copy())
    sim.init_droplet([], [], [])
    ref.run(200)
    sim.step(200)
    rv, _ = ref.coexistence()
    r = sim.rho()[1:-1]
    assert np.abs(sim.populations() - oracle_pops(ref)).max() <= 1e-12 * rv
    assert np.abs(r - rv).max() <= 1e-12 * rv   # a uniform vapour: no interface, no force, no flow
    sim.close()


@pytest.mark.parametrize("nx,ny,steps,drop", [
    (2, 4, 60, (1.0, 0.5, 1.5)),
    (3, 5, 60, (1.5, 0.5, 2.0)),
    (65, 4, 60, (32.0, 0.5, 6.0)),
    (129, 7, 60, (64.0, 0.5, 20.0)),
])
def test_smallest_lattices_match_reference(ora, nx, ny, steps, drop):
    import paper_1501_05430_amd as P
    th = np.full(nx, math.radians(70.0))
    ref = ora.Sim(nx, ny, 0.8, theta_bottom=th, theta_top=th)
    ref.init_droplets([drop[0]], [drop[1]], [drop[2]])
    sim = P.LBM(P.make_params(nx, ny, 0.8))
    sim.apply_wetting(th, th)
    sim.init_droplet(drop[0], drop[1], drop[2])
    ref.run(steps)
    sim.step(steps)
    f_ref = oracle_pops(ref)
    err = np.abs(sim.populations() - f_ref).max() / np.abs(f_ref).max()
    sim.close()
    assert err <= 1e-12, err


@pytest.mark.parametrize("precision,nx,nyf", [("f32_shifted", 32768, 65535), ("f64", 16384, 32768)])
def test_largest_lattice(precision, nx, nyf):
    """Lattices past the 2^31 elements of a whole state: in FP32 the largest one the in-plane 32-bit offsets allow
    (32768 x 65535 fluid rows, pitch x rows just below 2^31: 2.1e9 nodes, 155 GB of populations), in FP64 16384 x
    32768 (5.4e8 nodes, 77 GB). 20 steps with a droplet centred at x = nx/2 run without a fault or a non-finite
    value, conserve mass and stay mirror-symmetric bit for bit; one more row (or a wider plane) is refused."""
    import torch
    import paper_1501_05430_amd as P
    kw = P.fp32_options(0.7, precision)
    if precision == "f32_shifted":   # one more row exceeds the offsets
        with pytest.raises(P.LbmError):
            P.workspace_bytes(P.make_params(nx + 64, nyf + 2, 0.7, precision=precision, **kw))
    sim = P.LBM(P.make_params(nx, nyf + 2, 0.7, precision=precision, check_every=10, **kw))
    R = nyf / 5
    sim.apply_wetting(math.radians(60.0), math.radians(90.0))
    sim.init_droplet([nx / 2, nx / 2], [0.5 - R * math.cos(math.radians(60.0)), 3 * R], [R, R / 2])
    m0 = sim.mass()
    sim.step(20)
    d = sim.diag()
    m1 = sim.mass()
    r = sim.rho(device=True)[1:-1]
    mirror = torch.remainder(-torch.arange(nx, device=r.device), nx)
    symmetric = all(bool(torch.equal(r[k:k + 4096], r[k:k + 4096].index_select(1, mirror)))
                    for k in range(0, r.shape[0], 4096))
    finite = bool(torch.isfinite(r).all())
    del r
    sim.close()
    torch.cuda.empty_cache()
    assert d["nonfinite"] == 0 and finite
    assert abs(m1 - m0) / m0 <= (1e-12 if precision == "f64" else 1e-6)
    assert symmetric


def test_calls_out_of_order_are_errors():
    import paper_1501_05430_amd as P
    sim = P.LBM(P.make_params(20, 10, 0.8))
    with pytest.raises(P.LbmError) as e:
        sim.step(1)                      # no state yet
    assert e.value.code == 5
    with pytest.raises(P.LbmError) as e:
        sim.step(1, inst=1)              # no such instance
    assert e.value.code == 1
    sim.init_droplet(10.0, 0.5, 4.0)
    sim.step(0)                          # a no-op
    import ctypes as C
    buf = C.c_void_p(sim._ws_ptr)        # any device address: the call must refuse before using it
    rc = sim.lib.lbm_adjoint_step(sim.ctx, 0, buf, buf, buf, buf, buf)
    assert rc == 5                       # created without enable_adjoint
    rc = sim.lib.lbm_adjoint_step(sim.ctx, 0, None, buf, buf, buf, buf)
    assert rc == 1                       # NULL buffer
    sim.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_adjoint_at_the_largest_lattice(storage):
    """16384 columns x 14563 fluid rows (2.4e8 nodes, FP64 state; up to about 130 GB of device memory), both
    storage forms of the reverse step, two exact properties at every node. The step conserves mass, so the
    cotangent lambda = 1 (the derivative of the total mass) comes back as lambda = 1 with no angle or G gradient;
    and the reverse step is linear, so doubling lambda doubles every output bit for bit."""
    import torch
    import paper_1501_05430_amd as P
    nx = 16384
    nyf = (2 ** 31 - 1) // (9 * nx)
    sim = P.LBM(P.make_params(nx, nyf + 2, 0.7, enable_adjoint=True))
    sim.apply_wetting(math.radians(60.0), math.radians(120.0))
    sim.init_droplet([nx / 2, 3000.0], [0.5 - 3000 * math.cos(math.radians(60.0)), 9000.0], [3000.0, 1500.0])
    sim.step(5)
    f = sim.populations(device=True)
    if storage == "f32":   # lbm_adjoint_step_f32: the same indexing over FP32 arrays
        f = f.float()
    lam1 = torch.ones_like(f)
    lam0 = torch.empty_like(f)
    thb = torch.zeros((2, nx), dtype=torch.float64, device=f.device)
    Gb = torch.zeros(2, dtype=torch.float64, device=f.device)
    sim.adjoint_step(f, lam1, lam0, thb, Gb)
    torch.cuda.synchronize()
    err = float((lam0 - 1.0).abs().max())
    assert err <= 1e-11, err
    assert float(thb.abs().max()) <= 1e-9 and float(Gb.abs().max()) <= 1e-6 * nx * nyf * 1e-6, (thb.abs().max(), Gb)
    g = torch.Generator(device=f.device)
    g.manual_seed(7)
    torch.randn(lam1.shape, generator=g, device=f.device, dtype=lam1.dtype, out=lam1)
    sim.adjoint_step(f, lam1, lam0, thb.zero_(), Gb.zero_())
    first = (lam0.clone(), thb.clone(), Gb.clone())
    lam1.mul_(2.0)
    sim.adjoint_step(f, lam1, lam0, thb.zero_(), Gb.zero_())
    torch.cuda.synchronize()
    assert bool(torch.isfinite(first[0]).all())
    assert torch.equal(lam0, 2.0 * first[0]) and torch.equal(thb, 2.0 * first[1])
    sim.close()


def test_density_above_the_psi_cap_is_clamped_and_counted(ora):
    """A droplet started above the largest density with real psi (0.5 against 0.458 at 0.85 T_c): psi is clamped
    at 0 there and the ghost densities at rho_cap, and the device checks (every step) count exactly the clamps the
    reference counts (1058 fluid and 162 ghost over 20 steps, the density then relaxing below the cap), with the
    state still matching the reference."""
    import paper_1501_05430_amd as P
    nx, ny = 96, 40
    th = np.radians(np.linspace(40.0, 140.0, nx))
    ref = ora.Sim(nx, ny, 0.85, theta_bottom=th, theta_top=th[::-1].copy())
    ref.init_droplets([48.0], [0.5], [14.0], rho_l=0.5)
    ref.run(20)
    sim = P.LBM(P.make_params(nx, ny, 0.85, check_every=1))
    sim.apply_wetting(th, th[::-1].copy())
    sim.init_droplet(48.0, 0.5, 14.0, rho_l=0.5)
    sim.step(20)
    d = sim.diag()
    f_ref = oracle_pops(ref)
    err = np.abs(sim.populations() - f_ref).max() / np.abs(f_ref).max()
    sim.close()
    assert ref.counters[1] > 0 and ref.counters[0] > 0
    assert d["psi_clamps"] == ref.counters[1] and d["ghost_clamps"] == ref.counters[0], (d, ref.counters)
    assert d["nonfinite"] == 0 and err <= 1e-12, err


def test_binding_refuses_wrong_sizes_before_the_library():
    """The C-ABI takes raw device pointers, so the binding checks sizes: a cotangent of the wrong size or a
    host-side state buffer is refused before anything reaches the GPU."""
    import torch
    import paper_1501_05430_amd as P
    sim = P.LBM(P.make_params(20, 10, 0.8, enable_adjoint=True))
    sim.init_droplet(10.0, 0.5, 4.0)
    f = sim.populations(device=True)
    small = torch.zeros(9 * 8 * 19, dtype=torch.float64, device=f.device)
    th = torch.zeros((2, 20), dtype=torch.float64, device=f.device)
    G = torch.zeros(2, dtype=torch.float64, device=f.device)
    with pytest.raises(AssertionError):
        sim.adjoint_step(f, small, torch.empty_like(f), th, G)
    with pytest.raises(AssertionError):
        sim.adjoint_step(f, f.clone(), torch.empty_like(f), th[:, :10].contiguous(), G)
    with pytest.raises(AssertionError):
        sim.set_state(sim.get_state().cpu())
    sim.close()
