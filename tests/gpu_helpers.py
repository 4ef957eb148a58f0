"""Helpers shared by the GPU tests: run one workload on the GPU library and on the CPU reference."""
import math

import numpy as np


def rel_max(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def gpu_sim(case, precision="f64", wet_iters=4, A=-0.6, check_every=0, strip_rows=0, shift="rho_v",
            rho_fp64_below=None, enable_adjoint=False, init=True, **kw):
    """The library on one workload. FP32 modes take their EOS threshold and shift density from the library's own
    coexistence solve (fp32_options); shift is 'rho_v', 'rho_l' or a number."""
    import paper_1501_05430_amd as P
    extra = P.fp32_options(case.T_over_Tc, precision, shift=shift)
    if rho_fp64_below is not None and precision != "f64":
        extra["rho_fp64_below"] = rho_fp64_below
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
