"""Entry points of the boundary beyond the step itself: the coexistence densities, the timed step and graph replay
of short runs, and the adjoint of the density readout, all through the C-ABI."""
import math

import numpy as np
import pytest

from paper_1501_05430_amd import workloads as W
from gpu_helpers import gpu_sim

pytestmark = pytest.mark.gpu


def small_case(nx, ny, T, th_b_deg, th_t_deg, drops):
    return W.Case(f"small_{nx}x{ny}", nx, ny, T, np.full(nx, math.radians(th_b_deg)),
                  np.full(nx, math.radians(th_t_deg)), [d[0] for d in drops], [d[1] for d in drops],
                  [d[2] for d in drops], 0)


@pytest.mark.parametrize("T", [0.5, 0.7, 0.85])
def test_coexistence_matches_reference(ora, T):
    import paper_1501_05430_amd as P
    with P.LBM(P.make_params(16, 8, T)) as sim:
        rv, rl = sim.coexistence()
        info = sim.eos_info()
    _, tc, _ = ora.cs_critical()
    rv_ref, rl_ref = ora.cs_maxwell(T * tc)
    assert (rv, rl) == (info["rho_v"], info["rho_l"])
    assert rv == pytest.approx(rv_ref, rel=1e-11) and rl == pytest.approx(rl_ref, rel=1e-12)


def test_coexistence_of_the_piecewise_eos_is_its_pair():
    import paper_1501_05430_amd as P
    with P.LBM(P.make_params(16, 8, 0.7, piecewise=(0.2, -0.01, 0.33333, 1.0, 1000.0))) as sim:
        assert sim.coexistence() == (1.0, 1000.0)


@pytest.mark.parametrize("steps,check", [(20, 100), (37, 8), (1, 0), (150, 100)])
def test_short_runs_replay_graphs_bitwise(steps, check):
    """Runs shorter than a graph chunk (and chunk remainders) replay a graph of their own length, with the final
    device check in it: the state equals plain single launches bit for bit, and the checks count as before."""
    case = small_case(150, 40, 0.8, 60, 90, [(75, 0.5, 15.0)])
    a = gpu_sim(case, check_every=check)
    ms = a.step_timed(steps)
    assert ms > 0
    b = gpu_sim(case, check_every=0)
    for _ in range(steps):
        b.step(1)
    assert np.array_equal(a.populations(), b.populations())
    if check > 0:
        assert a.diag()["checks"] == steps // check + (1 if steps % check else 0)
    assert a.diag()["steps"] == steps
    a.close()
    b.close()


def test_timed_step_equals_step():
    case = small_case(130, 30, 0.75, 45, 120, [(65, 0.5, 12.0)])
    a = gpu_sim(case, check_every=10)
    b = gpu_sim(case, check_every=10)
    t = a.step_timed(55)
    b.step(55)
    assert t > 0 and np.array_equal(a.populations(), b.populations())
    a.close()
    b.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_adjoint_seed_of_the_density_readout(dtype):
    import torch
    case = small_case(96, 24, 0.8, 60, 120, [(48, 0.5, 10.0)])
    sim = gpu_sim(case, enable_adjoint=True)
    g = torch.randn((case.ny - 2, case.nx), dtype=torch.float64, device="cuda",
                    generator=torch.Generator("cuda").manual_seed(3))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    lam = torch.full((9, case.ny - 2, case.nx), 7.0, dtype=tdt, device="cuda")
    tb = torch.full((2, case.nx), 5.0, dtype=torch.float64, device="cuda")
    Gb = torch.full((2,), 5.0, dtype=torch.float64, device="cuda")
    sim.adjoint_seed_rho(g, lam, tb, Gb)
    torch.cuda.synchronize()
    want = g.to(tdt).unsqueeze(0).expand(9, -1, -1)
    assert torch.equal(lam, want)
    assert torch.count_nonzero(tb).item() == 0 and torch.count_nonzero(Gb).item() == 0
    sim.close()


def test_rollout_gradient_unchanged_by_the_library_seed():
    """The checkpointed rollout seeds lambda_N in the library; the gradient equals, bit for bit, the one from the
    readout adjoint broadcast by hand (dL/df_i = dL/drho for every i)."""
    import torch
    from paper_1501_05430_amd.autograd import rollout
    case = small_case(64, 32, 0.7, 80, 95, [(32, 0.5, 9.0)])
    sim = gpu_sim(case, enable_adjoint=True)
    f0 = sim.populations(device=True)
    nsteps = 120
    rng = np.random.default_rng(5)
    tgt = torch.tensor(rng.uniform(0.0, 0.3, (case.ny - 2, case.nx)), dtype=torch.float64)
    tb = torch.tensor(case.theta_bottom, dtype=torch.float64, requires_grad=True)
    tt = torch.tensor(case.theta_top, dtype=torch.float64, requires_grad=True)
    rho = rollout(tb, tt, -1.0, sim, f0, nsteps, seg=50)
    seen = []
    rho.register_hook(lambda g: seen.append(g.detach().clone()))
    L = torch.linalg.norm(rho - tgt)
    L.backward()
    # by hand: lambda_N broadcast from the same dL/drho, then the adjoint steps in reverse over recomputed states
    grad_rho = seen[0].to("cuda", torch.float64)
    lam = grad_rho.unsqueeze(0).expand(9, -1, -1).contiguous()
    lam_prev = torch.empty_like(lam)
    theta_bar = torch.zeros((2, case.nx), dtype=torch.float64, device="cuda")
    G_bar = torch.zeros(2, dtype=torch.float64, device="cuda")
    sim.apply_wetting(case.theta_bottom, case.theta_top)
    sim.set_populations(f0)
    states = []
    for _ in range(nsteps):
        states.append(sim.populations(device=True))
        sim.step(1)
    for st in reversed(states):
        sim.adjoint_step(st, lam, lam_prev, theta_bar, G_bar)
        lam, lam_prev = lam_prev, lam
    torch.cuda.synchronize()
    tbar = theta_bar.cpu()
    assert torch.equal(tb.grad, tbar[0]) and torch.equal(tt.grad, tbar[1])
    sim.close()


def _batch(precision="f32_shifted"):
    import paper_1501_05430_amd as P
    rng = np.random.default_rng(21)
    cases = []
    for k, (nx, ny) in enumerate([(128, 64), (256, 128), (64, 32), (256, 128)]):
        th = math.radians(rng.uniform(40, 140))
        cases.append(W.Case(f"t{k}", nx, ny, 0.75, np.full(nx, th), np.full(nx, math.pi / 2), [nx / 2],
                            [W.wall_cap_centre(0.3 * ny, th)], [0.3 * ny], 0))
    params = [P.make_params(c.nx, c.ny, c.T_over_Tc, precision=precision, **P.fp32_options(c.T_over_Tc, precision))
              for c in cases]
    sim = P.LBM(params)
    for i, c in enumerate(cases):
        sim.apply_wetting(c.theta_bottom, c.theta_top, inst=i)
        sim.init_droplet(c.xc, c.yc, c.R, inst=i)
    return sim


def test_autotune_cache_records_and_reapplies_the_shape(tmp_path):
    """lbm_autotune's choice is kept in a JSON cache (the binding's autotune(cache=...)): a second context with the
    same instances applies the recorded shape without the trials (lbm_set_tuning), gets the same rows per strip,
    and steps to the same state bit for bit as the tuned context and as an untuned one."""
    import json
    import time
    path = str(tmp_path / "tuning.json")
    a = _batch()
    t0 = time.perf_counter()
    chosen = a.autotune(inst=-1, trial_steps=4, cache=path)
    t_search = time.perf_counter() - t0
    rec = a.tuning()
    data = json.load(open(path))
    assert len(data) == 1 and list(data.values())[0] == rec
    b = _batch()
    t0 = time.perf_counter()
    assert b.autotune(inst=-1, trial_steps=4, cache=path) == chosen
    t_cached = time.perf_counter() - t0
    assert b.tuning() == rec
    c = _batch()                         # library defaults
    for s in (a, b, c):
        s.step(37, inst=-1)
    for i in range(4):
        pa = a.populations(inst=i)
        assert np.array_equal(pa, b.populations(inst=i)) and np.array_equal(pa, c.populations(inst=i)), i
    print(f"\n  search {t_search:.2f} s, from the cache {t_cached:.3f} s; shape {rec}")
    assert t_cached < t_search
    for s in (a, b, c):
        s.close()


def test_set_tuning_rejects_bad_shapes_and_changes_nothing():
    import paper_1501_05430_amd as P
    sim = _batch()
    rec = sim.tuning()
    for bad in (dict(waves=3), dict(waves2=16), dict(prefetch=2), dict(two_step=-1),
                dict(strip_rows=[0, 8, 8, 8]), dict(strip_rows2=[8, 8, -1, 8])):
        with pytest.raises(P.LbmError) as e:
            sim.set_tuning(dict(rec, **bad))
        assert e.value.code == 1
        assert sim.tuning() == rec
    # a valid other shape: one-step launches with two wavefronts, 5-row strips; the state still steps bitwise alike
    ref = _batch()
    sim.set_tuning(dict(rec, two_step=0, waves=2, prefetch=1, strip_rows=[5, 5, 5, 5]))
    assert sim.tuning()["waves"] == 2 and sim.tuning()["two_step"] == 0
    sim.step(21, inst=-1)
    ref.step(21, inst=-1)
    for i in range(4):
        assert np.array_equal(sim.populations(inst=i), ref.populations(inst=i)), i
    sim.close()
    ref.close()
