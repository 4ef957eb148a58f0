"""One batched launch over instances that differ in every per-instance choice (EOS, collision, surface-tension
source, wall kind, periodic rows, size, temperature) gives, bit for bit, what each instance gives in a context of
its own. Every instance runs at tau != 1, so that all take the general step kernel in both settings."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SPECS = [
    dict(nx=96, ny=48, T=0.8, kw=dict(tau=0.8), walls=(60.0, 120.0), drop=(48.0, 0.5, 14.0)),
    dict(nx=130, ny=60, T=1.0, kw=dict(piecewise=(0.25, -0.02, 0.3, 1.0, 10.0), kappa=0.5, tau=0.9), walls=(45.0, 90.0),
         drop=(65.0, 0.5, 18.0)),
    dict(nx=70, ny=40, T=0.85, kw=dict(boundary="martys_chen", G_w=(-0.3, -0.25), mrt=(1.2, 1.4, 1.1)), walls=None,
         drop=(35.0, 0.5, 12.0)),
    dict(nx=64, ny=66, T=0.85, kw=dict(boundary="periodic", kappa=0.3, tau=0.9), walls=None, drop=(32.0, 33.0, 14.0)),
]


def params(spec, precision):
    import paper_1501_05430_amd as P
    pw = spec["kw"].get("piecewise")
    return P.make_params(spec["nx"], spec["ny"], spec["T"], precision=precision, check_every=50,
                         **P.fp32_options(spec["T"], precision, piecewise=pw), **spec["kw"])


def prepare(sim, spec, inst=0):
    if spec["walls"] is not None:
        sim.apply_wetting(math.radians(spec["walls"][0]), math.radians(spec["walls"][1]), inst=inst)
    x, y, R = spec["drop"]
    sim.init_droplet(x, y, R, inst=inst)


@pytest.mark.parametrize("precision", ["f64", "f32_shifted"])
def test_mixed_feature_batch_equals_single_contexts_bitwise(precision):
    import paper_1501_05430_amd as P
    batch = P.LBM([params(s, precision) for s in SPECS])
    for i, s in enumerate(SPECS):
        prepare(batch, s, inst=i)
    batch.step(200, inst=-1)
    for i, s in enumerate(SPECS):
        single = P.LBM(params(s, precision))
        prepare(single, s)
        single.step(200)
        a, b = batch.populations(inst=i), single.populations()
        single.close()
        assert np.isfinite(a).all(), i
        assert np.array_equal(a, b), (i, np.abs(a - b).max())
    batch.close()


def test_mixed_feature_batch_matches_reference(ora):
    """The same batched launch (FP64) against the CPU reference, instance by instance, after 200 steps: 1e-12."""
    import paper_1501_05430_amd as P
    batch = P.LBM([params(s, "f64") for s in SPECS])
    for i, s in enumerate(SPECS):
        prepare(batch, s, inst=i)
    batch.step(200, inst=-1)
    for i, s in enumerate(SPECS):
        kw = {k: v for k, v in s["kw"].items() if k != "boundary"}
        periodic = s["kw"].get("boundary") == "periodic"
        ny = s["ny"] - 2 if periodic else s["ny"]
        th = s["walls"] or (90.0, 90.0)
        ref = ora.Sim(s["nx"], ny, s["T"], theta_bottom=math.radians(th[0]), theta_top=math.radians(th[1]),
                      periodic_y=periodic, **kw)
        x, y, R = s["drop"]
        ref.init_droplets([x], [y - 1.0 if periodic else y], [R])
        ref.run(200)
        f_ref = np.moveaxis(ref.f if periodic else ref.f[1:-1], 2, 0)
        f = batch.populations(inst=i)
        err = np.abs(f - f_ref).max() / np.abs(f_ref).max()
        assert err <= 1e-12, (i, err)
    batch.close()
