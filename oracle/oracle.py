"""ctypes front end of liblbm_oracle.so (test infrastructure).

Array layout on this side: populations f[ny, nx, 9] (all rows, ghost rows unused), densities rho[ny, nx].
Angles are in radians.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


class OraParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("periodic_y", C.c_int32), ("wet_iters", C.c_int32),
        ("tau", C.c_double), ("G", C.c_double), ("A", C.c_double),
        ("eos_a", C.c_double), ("eos_b", C.c_double), ("eos_R", C.c_double), ("T", C.c_double),
        ("body_fx", C.c_double), ("body_fy", C.c_double),
        ("eos_kind", C.c_int32), ("pad", C.c_int32),
        ("pw_theta_v", C.c_double), ("pw_theta_m", C.c_double), ("pw_theta_l", C.c_double),
        ("pw_rho1", C.c_double), ("pw_rho2", C.c_double),
        ("mrt", C.c_int32), ("pad2", C.c_int32),
        ("s_e", C.c_double), ("s_eps", C.c_double), ("s_q", C.c_double), ("kappa", C.c_double),
        ("wall_mode", C.c_int32), ("pad3", C.c_int32), ("G_w", C.c_double * 2),
    ]


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(path)
        d, i32, i64, p = C.c_double, C.c_int32, C.c_int64, C.c_void_p
        pp = C.POINTER(OraParams)
        L.ora_cs_pressure.argtypes = [d, d, d, d, d]; L.ora_cs_pressure.restype = d
        L.ora_cs_dpdrho.argtypes = [d, d, d, d, d]; L.ora_cs_dpdrho.restype = d
        L.ora_cs_d2pdrho2.argtypes = [d, d, d, d, d]; L.ora_cs_d2pdrho2.restype = d
        L.ora_cs_mu.argtypes = [d, d, d, d, d]; L.ora_cs_mu.restype = d
        L.ora_cs_critical.argtypes = [d, d, d, p, p, p]; L.ora_cs_critical.restype = C.c_int
        L.ora_cs_maxwell.argtypes = [d, d, d, d, p, p]; L.ora_cs_maxwell.restype = C.c_int
        L.ora_cs_rho_cap.argtypes = [d, d, d, d, d]; L.ora_cs_rho_cap.restype = d
        L.ora_run.argtypes = [pp, p, i64, p, p, p]; L.ora_run.restype = C.c_int
        L.ora_run_cplx.argtypes = [pp, p, i64, p, p, p, p]; L.ora_run_cplx.restype = C.c_int
        L.ora_density.argtypes = [pp, p, p, p, p, p]; L.ora_density.restype = C.c_int
        L.ora_force.argtypes = [pp, p, p, p, p, p]; L.ora_force.restype = C.c_int
        L.ora_force_psi.argtypes = [pp, p, p, p]; L.ora_force_psi.restype = C.c_int
        L.ora_collide_node.argtypes = [pp, p, d, d, p]; L.ora_collide_node.restype = C.c_int
        L.ora_ghost_density.argtypes = [d, d, d, d, d, i32]; L.ora_ghost_density.restype = d
        L.ora_psi.argtypes = [pp, d]; L.ora_psi.restype = d
        L.ora_init_droplets.argtypes = [pp, p, i32, p, p, p, d, d, d]; L.ora_init_droplets.restype = C.c_int
        L.ora_mass.argtypes = [pp, p]; L.ora_mass.restype = d
        L.ora_num_threads.argtypes = []; L.ora_num_threads.restype = i32
        L.ora_pw_pressure.argtypes = [d, d, d, d, d, d]; L.ora_pw_pressure.restype = d
        L.ora_pw_breakpoints.argtypes = [d, d, d, d, d, p, p]; L.ora_pw_breakpoints.restype = C.c_int
        L.ora_pw_rho_cap.argtypes = [d, d, d, d, d]; L.ora_pw_rho_cap.restype = d
        L.ora_collide_mrt_node.argtypes = [pp, p, d, d, p, p]; L.ora_collide_mrt_node.restype = C.c_int
        L.ora_qtensor.argtypes = [pp, p, p]; L.ora_qtensor.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


# ------------------------------------------------------------------------------------------------ EOS helpers
def cs_pressure(rho, T, a=1.0, b=4.0, R=1.0):
    return lib().ora_cs_pressure(a, b, R, T, float(rho))


def cs_dpdrho(rho, T, a=1.0, b=4.0, R=1.0):
    return lib().ora_cs_dpdrho(a, b, R, T, float(rho))


def cs_d2pdrho2(rho, T, a=1.0, b=4.0, R=1.0):
    return lib().ora_cs_d2pdrho2(a, b, R, T, float(rho))


def cs_mu(rho, T, a=1.0, b=4.0, R=1.0):
    return lib().ora_cs_mu(a, b, R, T, float(rho))


def cs_critical(a=1.0, b=4.0, R=1.0):
    """(rho_c, T_c, p_c) of the Carnahan-Starling EOS."""
    rc, tc, pc = C.c_double(), C.c_double(), C.c_double()
    rc_ = lib().ora_cs_critical(a, b, R, C.byref(rc), C.byref(tc), C.byref(pc))
    if rc_:
        raise ValueError("critical point: no root")
    return rc.value, tc.value, pc.value


def cs_maxwell(T, a=1.0, b=4.0, R=1.0):
    """Maxwell coexistence densities (rho_v, rho_l) at absolute temperature T."""
    rv, rl = C.c_double(), C.c_double()
    rc_ = lib().ora_cs_maxwell(a, b, R, T, C.byref(rv), C.byref(rl))
    if rc_:
        raise ValueError(f"maxwell: failed ({rc_})")
    return rv.value, rl.value


def cs_rho_cap(T, G=-1.0, a=1.0, b=4.0, R=1.0):
    return lib().ora_cs_rho_cap(a, b, R, T, G)


def pw_breakpoints(theta_v, theta_m, theta_l, rho_v, rho_l):
    """(rho_1, rho_2) of the piecewise-linear EOS (Eq. 11) from Eq. (12)-(13)."""
    r1, r2 = C.c_double(), C.c_double()
    rc_ = lib().ora_pw_breakpoints(theta_v, theta_m, theta_l, rho_v, rho_l, C.byref(r1), C.byref(r2))
    if rc_:
        raise ValueError(f"no break points ({rc_})")
    return r1.value, r2.value


def pw_pressure(theta_v, theta_m, theta_l, rho1, rho2, rho):
    return lib().ora_pw_pressure(theta_v, theta_m, theta_l, rho1, rho2, float(rho))


def pw_rho_cap(theta_v, theta_m, theta_l, rho1, rho2):
    return lib().ora_pw_rho_cap(theta_v, theta_m, theta_l, rho1, rho2)


def ghost_density(r_im1_1, r_ip1_1, r_i_1, r_i_2, theta, iters):
    return lib().ora_ghost_density(float(r_im1_1), float(r_ip1_1), float(r_i_1), float(r_i_2), float(theta),
                                   int(iters))


# ------------------------------------------------------------------------------------------------ simulation
class Sim:
    """One lattice (state in self.f, [ny, nx, 9] float64) advanced by the reference step."""

    def __init__(self, nx, ny, T_over_Tc, theta_bottom=np.pi / 2, theta_top=np.pi / 2, *, wet_iters=4, tau=1.0,
                 G=-1.0, A=-0.6, a=1.0, b=4.0, R=1.0, body_force=(0.0, 0.0), periodic_y=False, piecewise=None,
                 mrt=None, kappa=0.0, G_w=None):
        """piecewise = (theta_v, theta_m, theta_l, rho_v, rho_l) selects the EOS of Eq. (11) with the break points
        of Eq. (12)-(13) (T_over_Tc is then unused); None selects Carnahan-Starling. mrt = (s_e, s_eps, s_q) selects
        the MRT collision of Eq. (15) (the stress relaxes at 1/tau); kappa != 0 adds the source of Eq. (16)-(17) and
        implies MRT (rates 1/tau where mrt is None). G_w = (bottom, top) selects Martys-Chen walls (Eq. 14) in place
        of the geometric wetting (the contact angles are then unused)."""
        if piecewise is None:
            rc, tc, pc = cs_critical(a, b, R)
            self.T_c = tc
            self.T = T_over_Tc * tc
        else:
            self.T_c = self.T = 1.0
        self.p = OraParams(nx, ny, 1 if periodic_y else 0, wet_iters, tau, G, A, a, b, R, self.T,
                           body_force[0], body_force[1])
        self.piecewise = piecewise
        if mrt is not None or kappa != 0.0:
            rates = mrt if mrt is not None else (1.0 / tau,) * 3
            self.p.mrt = 1
            self.p.s_e, self.p.s_eps, self.p.s_q = (float(r) for r in rates)
            self.p.kappa = float(kappa)
        if G_w is not None:
            self.p.wall_mode = 1
            self.p.G_w[0], self.p.G_w[1] = float(G_w[0]), float(G_w[1])
        if piecewise is not None:
            tv, tm, tl, rv, rl = piecewise
            r1, r2 = pw_breakpoints(tv, tm, tl, rv, rl)
            self.p.eos_kind = 1
            self.p.pw_theta_v, self.p.pw_theta_m, self.p.pw_theta_l = tv, tm, tl
            self.p.pw_rho1, self.p.pw_rho2 = r1, r2
        self.nx, self.ny = nx, ny
        self.f = np.zeros((ny, nx, 9), dtype=np.float64)
        self.theta_b = np.ascontiguousarray(np.broadcast_to(np.asarray(theta_bottom, np.float64), (nx,)))
        self.theta_t = np.ascontiguousarray(np.broadcast_to(np.asarray(theta_top, np.float64), (nx,)))
        self.counters = np.zeros(2, dtype=np.int64)
        self.steps = 0

    def coexistence(self):
        if self.piecewise is not None:  # the densities Eq. (12)-(13) were solved for
            return self.piecewise[3], self.piecewise[4]
        return cs_maxwell(self.T, self.p.eos_a, self.p.eos_b, self.p.eos_R)

    def init_droplets(self, xc, yc, R, width=5.0, rho_l=None, rho_v=None):
        xc = np.ascontiguousarray(np.atleast_1d(np.asarray(xc, np.float64)))
        yc = np.ascontiguousarray(np.atleast_1d(np.asarray(yc, np.float64)))
        R = np.ascontiguousarray(np.atleast_1d(np.asarray(R, np.float64)))
        if rho_l is None or rho_v is None:
            rv, rl = self.coexistence()
            rho_l = rl if rho_l is None else rho_l
            rho_v = rv if rho_v is None else rho_v
        rc_ = lib().ora_init_droplets(C.byref(self.p), _ptr(self.f), len(xc), _ptr(xc), _ptr(yc), _ptr(R),
                                      float(width), float(rho_l), float(rho_v))
        if rc_:
            raise ValueError("init_droplets failed")
        self.steps = 0

    def run(self, nsteps):
        rc_ = lib().ora_run(C.byref(self.p), _ptr(self.f), int(nsteps), _ptr(self.theta_b), _ptr(self.theta_t),
                            _ptr(self.counters))
        if rc_:
            raise ValueError("run failed")
        self.steps += nsteps

    def density(self):
        """(rho, psi), [ny, nx] each; ghost rows hold the wetting densities of the current state."""
        rho = np.zeros((self.ny, self.nx))
        psi = np.zeros((self.ny, self.nx))
        rc_ = lib().ora_density(C.byref(self.p), _ptr(self.f), _ptr(self.theta_b), _ptr(self.theta_t), _ptr(rho),
                                _ptr(psi))
        if rc_:
            raise ValueError("density failed")
        return rho, psi

    def force(self):
        Fx = np.zeros((self.ny, self.nx))
        Fy = np.zeros((self.ny, self.nx))
        lib().ora_force(C.byref(self.p), _ptr(self.f), _ptr(self.theta_b), _ptr(self.theta_t), _ptr(Fx), _ptr(Fy))
        return Fx, Fy

    def mass(self):
        return lib().ora_mass(C.byref(self.p), _ptr(self.f))

    def fluid_rows(self):
        return slice(0, self.ny) if self.p.periodic_y else slice(1, self.ny - 1)

    def run_cplx(self, nsteps, f, theta_b, theta_t, G_f, G_psi):
        """Complex-step run from complex inputs; returns the complex populations."""
        fc = np.ascontiguousarray(f, dtype=np.complex128).copy()
        tb = np.ascontiguousarray(np.broadcast_to(theta_b, (self.nx,)), dtype=np.complex128)
        tt = np.ascontiguousarray(np.broadcast_to(theta_t, (self.nx,)), dtype=np.complex128)
        gf = np.array([complex(G_f)], dtype=np.complex128)
        gp = np.array([complex(G_psi)], dtype=np.complex128)
        rc_ = lib().ora_run_cplx(C.byref(self.p), _ptr(fc), int(nsteps), _ptr(tb), _ptr(tt), _ptr(gf), _ptr(gp))
        if rc_:
            raise ValueError("run_cplx failed")
        return fc


def collide_mrt_node(sim, f_in, Fx, Fy, Q=(0.0, 0.0, 0.0)):
    """One MRT collision (Eq. 15) of one node with total force (Fx, Fy) and Q = (Q_xx, Q_yy, Q_xy)."""
    f_in = np.ascontiguousarray(f_in, dtype=np.float64)
    q = np.ascontiguousarray(Q, dtype=np.float64)
    out = np.zeros(9)
    if lib().ora_collide_mrt_node(C.byref(sim.p), _ptr(f_in), float(Fx), float(Fy), _ptr(q), _ptr(out)):
        raise ValueError("bad parameters (MRT off?)")
    return out


def qtensor(sim, psi):
    """Q of Eq. (17) at every node of a psi field [ny, nx]: array [3, ny, nx] of Q_xx, Q_yy, Q_xy."""
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    q = np.zeros((3,) + psi.shape)
    if lib().ora_qtensor(C.byref(sim.p), _ptr(psi), _ptr(q)):
        raise ValueError("bad parameters")
    return q


def force_psi(sim, psi):
    """The interaction force of Eq. (9) (no body force) on a given psi field [ny, nx]: (Fx, Fy), [ny, nx] each,
    zero outside the fluid rows."""
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    assert psi.shape == (sim.ny, sim.nx)
    Fx = np.zeros_like(psi)
    Fy = np.zeros_like(psi)
    if lib().ora_force_psi(C.byref(sim.p), _ptr(psi), _ptr(Fx), _ptr(Fy)):
        raise ValueError("bad parameters")
    return Fx, Fy


def collide_node(sim, f_in, Fx, Fy):
    f_in = np.ascontiguousarray(f_in, np.float64)
    out = np.zeros(9)
    lib().ora_collide_node(C.byref(sim.p), _ptr(f_in), float(Fx), float(Fy), _ptr(out))
    return out


def num_threads():
    """OpenMP threads the reference uses."""
    return int(lib().ora_num_threads())


def psi(sim, rho):
    return lib().ora_psi(C.byref(sim.p), float(rho))


__all__ = ["OraParams", "lib", "cs_pressure", "cs_dpdrho", "cs_d2pdrho2", "cs_mu", "cs_critical", "cs_maxwell",
           "cs_rho_cap", "pw_breakpoints", "pw_pressure", "pw_rho_cap", "ghost_density", "Sim", "collide_node",
           "collide_mrt_node", "qtensor", "psi", "force_psi", "num_threads"]
