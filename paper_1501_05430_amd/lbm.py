"""Python front end of liblbm: torch owns the device workspace and the stream; every step of the method runs in
the library's HIP kernels. Argument marshalling only."""
import ctypes as C
import json
import math
import os

import numpy as np

from . import _lib
from ._lib import LbmError, Params, check, PRECISIONS


BOUNDARIES = {"walls": 0, "periodic": 1, "martys_chen": 2}


def make_params(nx, ny, T_over_Tc, *, precision="f64", wet_iters=4, check_every=0, strip_rows=0,
                enable_adjoint=False, step_variant=0, tau=1.0, G=-1.0, A=-0.6, eos_a=1.0, eos_b=4.0, eos_R=1.0, rho0_shift=0.0,
                rho_fp64_below=0.0, body_force=(0.0, 0.0), boundary="walls", piecewise=None, mrt=None, kappa=0.0,
                G_w=(0.0, 0.0)):
    """lbm_params of one lattice (see include/lbm.h). precision: 'f64', 'f32', 'f32_shifted' or 'f32_shifted_mixed'
    (FP32 storage, FP64 force and equilibrium); boundary: 'walls'
    (ghost rows 0 and ny-1 with the geometric wetting), 'periodic' (fluid rows 1..ny-2 wrap around) or
    'martys_chen' (solid walls with the fluid-solid force of Eq. 14, strengths G_w = (bottom, top)).
    piecewise = (theta_v, theta_m, theta_l, rho_v, rho_l) selects the piecewise-linear EOS of Eq. 11 (break points
    from Eq. 12-13; T_over_Tc and eos_a/b/R are then unused); None selects Carnahan-Starling. mrt = (s_e, s_eps,
    s_q) selects the MRT collision of Eq. 15 (0 entries mean 1/tau); kappa != 0 adds the surface-tension source of
    Eq. 16-17 (and implies MRT)."""
    p = Params()
    if mrt is not None:
        for k in range(3):
            p.mrt_rates[k] = float(mrt[k])
    p.kappa = float(kappa)
    p.G_w[0], p.G_w[1] = float(G_w[0]), float(G_w[1])
    if piecewise is not None:
        p.eos = 1
        for k in range(3):
            p.pw_theta[k] = float(piecewise[k])
        p.pw_rho[0], p.pw_rho[1] = float(piecewise[3]), float(piecewise[4])
    p.boundary = BOUNDARIES[boundary] if isinstance(boundary, str) else int(boundary)
    p.nx, p.ny = int(nx), int(ny)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.wet_iters = int(wet_iters)
    p.check_every = int(check_every)
    p.strip_rows = int(strip_rows)
    p.enable_adjoint = 1 if enable_adjoint else 0
    p.step_variant = int(step_variant)
    p.tau, p.G, p.A = float(tau), float(G), float(A)
    p.eos_a, p.eos_b, p.eos_R = float(eos_a), float(eos_b), float(eos_R)
    p.T_over_Tc = float(T_over_Tc)
    p.rho0_shift = float(rho0_shift)
    p.rho_fp64_below = float(rho_fp64_below)
    p.body_force[0], p.body_force[1] = float(body_force[0]), float(body_force[1])
    return p


def eos_coexistence(T_over_Tc, device="cuda:0", **eos):
    """(rho_v, rho_l) of the library's EOS (a 16 x 8 probe context): the Maxwell construction at T_over_Tc, or the
    pair given with piecewise=."""
    with LBM(make_params(16, 8, T_over_Tc, **eos), device=device) as probe:
        info = probe.eos_info()
    return info["rho_v"], info["rho_l"]


def fp32_options(T_over_Tc, precision, shift="rho_v", device="cuda:0", **eos):
    """make_params keywords of the FP32 modes: the EOS in FP64 below the geometric mean of the coexistence
    densities, and for 'f32_shifted' and 'f32_shifted_mixed' the reference density rho0 of the stored f_i - w_i rho0
    ('rho_v', 'rho_l' or a number). The vapour density is the default shift: it keeps the vapour's populations small (their relative
    rounding is then that of the deviation from rho_v), while the liquid's populations are no larger than
    unshifted ones."""
    if precision == "f64":
        return {}
    rv, rl = eos_coexistence(T_over_Tc, device=device, **eos)
    out = {"rho_fp64_below": math.sqrt(rv * rl)}
    if precision in ("f32_shifted", "f32_shifted_mixed"):
        out["rho0_shift"] = {"rho_v": rv, "rho_l": rl}.get(shift, shift)
    return out


def workspace_bytes(params):
    params = params if isinstance(params, (list, tuple)) else [params]
    arr = (Params * len(params))(*params)
    lib = _lib.load()
    n = lib.lbm_workspace_bytes(arr, len(params))
    if n == 0:
        raise LbmError(_lib.LBM_E_INVALID, lib.lbm_last_error().decode())
    return n


def _dptr(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


class LBM:
    """A context over one or more lattice instances (one launch per step covers every instance when
    `step(n, inst=-1)`)."""

    def __init__(self, params, device="cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("liblbm needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.lib = _lib.load()
        self.params = list(params) if isinstance(params, (list, tuple)) else [params]
        self.n = len(self.params)
        self.device = torch.device(device)
        arr = (Params * self.n)(*self.params)
        nbytes = workspace_bytes(self.params)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self._take_over()
        ctx = C.c_void_p()
        check(self.lib.lbm_create(arr, self.n, C.c_void_p(self._ws_ptr), nbytes, C.c_void_p(self.stream.cuda_stream),
                                  C.byref(ctx)))
        self.ctx = ctx

    # ------------------------------------------------------------------------------------------- lifecycle
    def close(self):
        if getattr(self, "ctx", None):
            self.stream.synchronize()
            check(self.lib.lbm_destroy(self.ctx))
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------------------------------- setup
    def eos_info(self, inst=0):
        out = (C.c_double * 6)()
        check(self.lib.lbm_eos_info(self.ctx, inst, out))
        keys = ["rho_v", "rho_l", "T", "T_c", "rho_c", "rho_cap"]
        if self.params[inst].eos == 1:
            keys = ["rho_v", "rho_l", "rho_1", "rho_2", "_", "rho_cap"]
        return dict(zip(keys, list(out)))

    def coexistence(self, inst=0):
        """(rho_v, rho_l) the library solved for instance inst."""
        out = (C.c_double * 2)()
        check(self.lib.lbm_coexistence(self.ctx, inst, out))
        return out[0], out[1]

    def init_droplet(self, xc, yc, R, inst=0, width=5.0, rho_l=0.0, rho_v=0.0):
        xa, xp = _dptr(np.atleast_1d(xc))
        ya, yp = _dptr(np.atleast_1d(yc))
        ra, rp = _dptr(np.atleast_1d(R))
        assert len(xa) == len(ya) == len(ra), "xc, yc and R need one entry per droplet"
        check(self.lib.lbm_init_droplet(self.ctx, inst, len(xa), xp, yp, rp, float(width), float(rho_l),
                                        float(rho_v)))

    def apply_wetting(self, theta_bottom=None, theta_top=None, inst=0):
        nx = self.params[inst].nx
        args = []
        keep = []
        for th in (theta_bottom, theta_top):
            if th is None:
                args.append(None)
            else:
                a, p = _dptr(np.broadcast_to(np.asarray(th, np.float64), (nx,)))
                keep.append(a)
                args.append(p)
        check(self.lib.lbm_apply_wetting(self.ctx, inst, args[0], args[1]))

    # ------------------------------------------------------------------------------------------- stepping
    def step(self, nsteps, inst=0):
        check(self.lib.lbm_step(self.ctx, inst, int(nsteps)))

    def step_timed(self, nsteps, inst=0):
        """Advance nsteps and return the device time of the queued steps in ms (HIP events on the library's stream).
        Raises LbmError as step() does."""
        ms = C.c_double()
        rc = self.lib.lbm_step_timed(self.ctx, inst, int(nsteps), C.byref(ms))
        check(rc)
        return ms.value

    def autotune(self, inst=0, trial_steps=20, cache=None):
        """lbm_autotune on instance inst (-1: all of them); returns the chosen rows per strip. With cache (a JSON
        file path), a shape recorded there for the same device, library and instances is applied without the
        trials, and a new search's result is recorded (the file is replaced atomically)."""
        key = self._tuning_key(inst, trial_steps) if cache is not None else None
        if key is not None and os.path.exists(cache):
            with open(cache) as f:
                rec = json.load(f).get(key)
            if rec is not None:
                self.set_tuning(rec)
                i0 = max(inst, 0)
                return rec["strip_rows2" if rec["two_step"] and self._two_step_applies(inst) else "strip_rows"][i0]
        out = C.c_int32()
        check(self.lib.lbm_autotune(self.ctx, inst, int(trial_steps), C.byref(out)))
        if key is not None:
            data = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    data = json.load(f)
            data[key] = self.tuning()
            tmp = f"{cache}.{os.getpid()}.tmp"
            with open(tmp, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return out.value

    def tuning(self):
        """The step shape (lbm_get_tuning): two_step, waves, prefetch, waves2 and each instance's rows per strip."""
        n = len(self.params)
        t = _lib.Tuning()
        rows, rows2 = (C.c_int32 * n)(), (C.c_int32 * n)()
        check(self.lib.lbm_get_tuning(self.ctx, C.byref(t), rows, rows2))
        return {"two_step": t.two_step, "waves": t.waves, "prefetch": t.prefetch, "waves2": t.waves2,
                "strip_rows": list(rows), "strip_rows2": list(rows2)}

    def set_tuning(self, rec):
        """Apply a shape from tuning() (lbm_set_tuning); results do not depend on it."""
        n = len(self.params)
        if len(rec["strip_rows"]) != n or len(rec["strip_rows2"]) != n:
            raise ValueError(f"tuning record for {len(rec['strip_rows'])} instances, context has {n}")
        t = _lib.Tuning(int(rec["two_step"]), int(rec["waves"]), int(rec["prefetch"]), int(rec["waves2"]))
        rows = (C.c_int32 * n)(*[int(v) for v in rec["strip_rows"]])
        rows2 = (C.c_int32 * n)(*[int(v) for v in rec["strip_rows2"]])
        check(self.lib.lbm_set_tuning(self.ctx, C.byref(t), rows, rows2))

    def _two_step_applies(self, inst):
        sel = self.params if inst < 0 else [self.params[inst]]
        return all(p.boundary != BOUNDARIES["periodic"] for p in sel)

    def _tuning_key(self, inst, trial_steps):
        """Device, library build and everything about the instances that decides a launch's time."""
        import hashlib
        import torch
        props = torch.cuda.get_device_properties(self.device)
        h = hashlib.sha256()
        with open(_lib.LIB_PATH, "rb") as f:
            h.update(f.read())
        fields = [f for f, _ in _lib.Params._fields_]
        inst_desc = [[list(v) if hasattr(v, "__len__") else v for v in (getattr(p, f) for f in fields)]
                     for p in self.params]
        desc = json.dumps({"device": props.name, "cus": props.multi_processor_count, "lib": h.hexdigest()[:16],
                           "inst": inst, "trial_steps": int(trial_steps), "params": inst_desc}, sort_keys=True)
        return hashlib.sha256(desc.encode()).hexdigest()[:24]

    # ------------------------------------------------------------------------------------------- readout
    def mass(self, inst=0):
        out = C.c_double()
        check(self.lib.lbm_mass(self.ctx, inst, C.byref(out)))
        return out.value

    def diag(self, inst=0):
        d = _lib.Diag()
        check(self.lib.lbm_get_diag(self.ctx, inst, C.byref(d)))
        return {k: getattr(d, k) for k, _ in _lib.Diag._fields_}

    def rho(self, inst=0, device=False):
        """Density [ny, nx] (FP64) with the ghost rows; numpy array, or a torch tensor when device=True."""
        import torch
        p = self.params[inst]
        if device:
            with torch.cuda.stream(self.stream):
                out = torch.empty((p.ny, p.nx), dtype=torch.float64, device=self.device)
            check(self.lib.lbm_get_rho(self.ctx, inst, C.c_void_p(out.data_ptr()), 1))
            self._hand_over()
            return out
        out = np.empty((p.ny, p.nx), dtype=np.float64)
        check(self.lib.lbm_get_rho(self.ctx, inst, out.ctypes.data_as(C.c_void_p), 0))
        return out

    def populations(self, inst=0, device=False):
        """Populations [9, ny-2, nx] (FP64, unshifted)."""
        import torch
        p = self.params[inst]
        if device:
            with torch.cuda.stream(self.stream):
                out = torch.empty((9, p.ny - 2, p.nx), dtype=torch.float64, device=self.device)
            check(self.lib.lbm_get_populations(self.ctx, inst, C.c_void_p(out.data_ptr()), 1))
            self._hand_over()
            return out
        out = np.empty((9, p.ny - 2, p.nx), dtype=np.float64)
        check(self.lib.lbm_get_populations(self.ctx, inst, out.ctypes.data_as(C.c_void_p), 0))
        return out

    def set_populations(self, f, inst=0):
        import torch
        p = self.params[inst]
        if isinstance(f, torch.Tensor):
            assert f.shape == (9, p.ny - 2, p.nx) and f.dtype == torch.float64 and f.is_cuda
            f = f.contiguous()
            self._take_over()
            check(self.lib.lbm_set_populations(self.ctx, inst, C.c_void_p(f.data_ptr()), 1))
            f.record_stream(self.stream)
        else:
            a = np.ascontiguousarray(f, dtype=np.float64)
            assert a.shape == (9, p.ny - 2, p.nx)
            check(self.lib.lbm_set_populations(self.ctx, inst, a.ctypes.data_as(C.c_void_p), 0))

    def state_bytes(self, inst=0):
        return self.lib.lbm_state_bytes(self.ctx, inst)

    def get_state(self, inst=0):
        import torch
        with torch.cuda.stream(self.stream):
            out = torch.empty(self.state_bytes(inst), dtype=torch.uint8, device=self.device)
        check(self.lib.lbm_get_state(self.ctx, inst, C.c_void_p(out.data_ptr())))
        self._hand_over()
        return out

    def set_state(self, state, inst=0):
        import torch
        assert state.is_cuda and state.is_contiguous() and state.dtype == torch.uint8
        assert state.numel() == self.state_bytes(inst)
        self._take_over()
        check(self.lib.lbm_set_state(self.ctx, inst, C.c_void_p(state.data_ptr())))
        state.record_stream(self.stream)

    def measure_contact_angle(self, box, wall=0, inst=0):
        """(theta [rad], R, xc, yc, npoints) of the droplet in box = (x_lo, x_hi, y_lo, y_hi)."""
        b = (C.c_int32 * 4)(*[int(v) for v in box])
        out = (C.c_double * 5)()
        check(self.lib.lbm_measure_contact_angle(self.ctx, inst, int(wall), b, out))
        return out[0], out[1], out[2], out[3], int(out[4])

    def adjoint_step(self, f_n, lam_np1, lam_n, theta_bar, G_bar, inst=0):
        """lam_n = (df_{n+1}/df_n)^T lam_np1; theta_bar [2, nx] and G_bar [2] accumulate (device FP64 tensors).
        f_n, lam_np1 and lam_n are all FP64 (lbm_adjoint_step) or all FP32 (lbm_adjoint_step_f32)."""
        import torch
        dt = f_n.dtype
        assert dt in (torch.float64, torch.float32)
        p = self.params[inst]
        for t in (f_n, lam_np1, lam_n):   # the library takes raw pointers: sizes are checked here
            assert t.is_cuda and t.is_contiguous() and t.dtype == dt and t.numel() == 9 * (p.ny - 2) * p.nx
        for t, size in ((theta_bar, 2 * p.nx), (G_bar, 2)):
            assert t.is_cuda and t.is_contiguous() and t.dtype == torch.float64 and t.numel() == size
        self._take_over()
        fn = self.lib.lbm_adjoint_step if dt == torch.float64 else self.lib.lbm_adjoint_step_f32
        check(fn(self.ctx, inst, C.c_void_p(f_n.data_ptr()), C.c_void_p(lam_np1.data_ptr()),
                 C.c_void_p(lam_n.data_ptr()), C.c_void_p(theta_bar.data_ptr()), C.c_void_p(G_bar.data_ptr())))
        self._hand_over()

    def adjoint_seed_rho(self, grad_rho, lam, theta_bar, G_bar, inst=0):
        """lam = dL/df_N from grad_rho = dL/drho_N [ny-2, nx] (device FP64) on every population plane; theta_bar and
        G_bar set to zero. lam is FP64 or FP32 [9, ny-2, nx] (the FP32 form feeds the FP32 adjoint step)."""
        import torch
        p = self.params[inst]
        assert grad_rho.is_cuda and grad_rho.is_contiguous() and grad_rho.dtype == torch.float64
        assert grad_rho.numel() == (p.ny - 2) * p.nx
        assert lam.is_cuda and lam.is_contiguous() and lam.dtype in (torch.float64, torch.float32)
        assert lam.numel() == 9 * (p.ny - 2) * p.nx
        for t, size in ((theta_bar, 2 * p.nx), (G_bar, 2)):
            assert t.is_cuda and t.is_contiguous() and t.dtype == torch.float64 and t.numel() == size
        self._take_over()
        fn = self.lib.lbm_adjoint_seed_rho if lam.dtype == torch.float64 else self.lib.lbm_adjoint_seed_rho_f32
        check(fn(self.ctx, inst, C.c_void_p(grad_rho.data_ptr()), C.c_void_p(lam.data_ptr()),
                 C.c_void_p(theta_bar.data_ptr()), C.c_void_p(G_bar.data_ptr())))
        self._hand_over()

    def _take_over(self):
        """Make the library's stream wait for the work queued on torch's current stream (device inputs). Nothing to
        do when that stream is the library's own (inside `with torch.cuda.stream(sim.stream)`): a wait across two
        streams costs a round trip between two hardware queues on every call."""
        import torch
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)

    def _hand_over(self):
        """Make torch's current stream wait for the work queued on the library's stream (device outputs)."""
        import torch
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            cur.wait_stream(self.stream)


def deg(rad):
    return rad * 180.0 / math.pi
