"""Helpers shared by the GPU tests: run one workload on the GPU library and on the CPU reference."""
import math

import numpy as np


def rel_max(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def gpu_sim(case, precision="f64", wet_iters=4, A=-0.6, check_every=0, strip_rows=0, rho0_shift=None,
            rho_fp64_below=None, enable_adjoint=False, init=True, **kw):
    import paper_1501_05430_amd as P
    extra = {}
    sim_probe = None
    if precision != "f64":
        # reference densities for the FP32 options come from the library's own coexistence solve
        probe = P.LBM(P.make_params(case.nx, case.ny, case.T_over_Tc, precision="f64"))
        info = probe.eos_info()
        probe.close()
        if precision == "f32_shifted":
            extra["rho0_shift"] = info["rho_l"] if rho0_shift is None else rho0_shift
        extra["rho_fp64_below"] = (math.sqrt(info["rho_v"] * info["rho_l"]) if rho_fp64_below is None
                                   else rho_fp64_below)
    del sim_probe
    p = P.make_params(case.nx, case.ny, case.T_over_Tc, precision=precision, wet_iters=wet_iters, A=A,
                      check_every=check_every, strip_rows=strip_rows, enable_adjoint=enable_adjoint, **extra, **kw)
    sim = P.LBM(p)
    sim.apply_wetting(case.theta_bottom, case.theta_top)
    if init:
        sim.init_droplet(case.xc, case.yc, case.R)
    return sim


def oracle_sim(case, wet_iters=4, A=-0.6, **kw):
    import oracle
    s = oracle.Sim(case.nx, case.ny, case.T_over_Tc, theta_bottom=case.theta_bottom, theta_top=case.theta_top,
                   wet_iters=wet_iters, A=A, **kw)
    s.init_droplets(case.xc, case.yc, case.R)
    return s


def oracle_pops(s):
    """Reference populations in the library's layout [9, ny-2, nx]."""
    return np.moveaxis(s.f[1:-1], 2, 0)
