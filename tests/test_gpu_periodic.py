"""Periodic rows (LBM_PERIODIC_Y): the step with no walls against the FP64 CPU reference in its periodic mode, and
the Laplace law for free droplets on the GPU path. A periodic lattice of N rows is ny = N + 2 for the library (fluid
rows 1..N) and ny = N for the reference (rows 0..N-1)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def periodic_pair(ora, n_x, n_y, T, drops, precision="f64", **kw):
    import paper_1501_05430_amd as P
    ref = ora.Sim(n_x, n_y, T, periodic_y=True, **kw)
    ref.init_droplets([d[0] for d in drops], [d[1] for d in drops], [d[2] for d in drops])
    p = P.make_params(n_x, n_y + 2, T, precision=precision, boundary="periodic",
                      **P.fp32_options(T, precision), **kw)
    sim = P.LBM(p)
    sim.init_droplet([d[0] for d in drops], [d[1] + 1.0 for d in drops], [d[2] for d in drops])
    return ref, sim


@pytest.mark.parametrize("n_x,n_y,steps,drops,kw", [
    (96, 80, 300, [(48.0, 40.0, 20.0)], {}),
    (70, 33, 200, [(10.0, 16.0, 9.0), (45.0, 5.0, 8.0)], dict(A=0.0)),        # droplet across the wrap in y
    (130, 64, 200, [(65.0, 32.0, 18.0)], dict(tau=0.8, body_force=(2e-6, -1e-6))),
])
def test_periodic_fp64_matches_reference(ora, n_x, n_y, steps, drops, kw):
    ref, sim = periodic_pair(ora, n_x, n_y, 0.8, drops, **kw)
    for n in (1, steps - 1):
        ref.run(n)
        sim.step(n)
        r_ref, _ = ref.density()
        r = sim.rho()
        err = np.abs(r[1:-1] - r_ref).max() / np.abs(r_ref).max()
        assert err <= 1e-12, (n, err)
        assert np.all(r[0] == 0) and np.all(r[-1] == 0)
    assert sim.mass() == pytest.approx(ref.mass(), rel=1e-12)
    sim.close()


def test_periodic_fp32_shifted_slice(ora):
    ref, sim = periodic_pair(ora, 128, 128, 0.7, [(64.0, 64.0, 24.0)], precision="f32_shifted")
    ref.run(100)
    sim.step(100)
    rv, rl = ref.coexistence()
    err = np.abs(sim.rho()[1:-1] - ref.density()[0]).max() / rl
    sim.close()
    assert err <= 1e-5, err


@pytest.mark.parametrize("precision", ["f64", "f32_shifted"])
def test_periodic_free_droplet_mirror_symmetric_bitwise(ora, precision):
    import paper_1501_05430_amd as P
    p = P.make_params(128, 130, 0.7, precision=precision, boundary="periodic", **P.fp32_options(0.7, precision))
    sim = P.LBM(p)
    sim.init_droplet(64.0, 65.0, 24.0)        # centre on a lattice node: mirrors x -> 128 - x, y -> 130 - y
    sim.step(1500)
    r = sim.rho()[1:-1]
    sim.close()
    mx = r[:, (-np.arange(128)) % 128]
    my = np.roll(r[::-1], 1, axis=0)          # fluid row y (1..128) <-> 130 - y, with row 129 = row 1
    assert np.array_equal(r, mx)
    assert np.array_equal(r, my)


def test_laplace_law_on_the_gpu(ora):
    """Free droplets in a periodic 128 x 128 box: p_in - p_out is linear in 1/R through the origin (R the equimolar
    radius), the pressure being the Carnahan-Starling p of the bulk densities."""
    import paper_1501_05430_amd as P
    res = []
    for R in [12, 15, 18, 21, 24]:
        sim = P.LBM(P.make_params(128, 130, 0.85, boundary="periodic"))
        sim.init_droplet(64.0, 65.0, float(R))
        sim.step(4000)
        T = sim.eos_info()["T"]
        r = sim.rho()[1:-1]
        sim.close()
        rin, rout = r[64, 64], r[0, 0]
        Reff = np.sqrt((r - rout).sum() / (np.pi * (rin - rout)))
        res.append((Reff, ora.cs_pressure(rin, T) - ora.cs_pressure(rout, T)))
    res = np.array(res)
    x, y = 1 / res[:, 0], res[:, 1]
    A = np.stack([x, np.ones_like(x)], 1)
    (k, b), *_ = np.linalg.lstsq(A, y, rcond=None)
    fit = A @ [k, b]
    r2 = 1 - ((y - fit) ** 2).sum() / ((y - y.mean()) ** 2).sum()
    print(f"\n  Laplace: sigma = {k:.4e}, intercept {b:.2e} (smallest dp {y.min():.2e}), R^2 = {r2:.6f}")
    assert k > 0 and r2 > 0.999 and abs(b) < 0.05 * y.min()
