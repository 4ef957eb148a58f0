"""Seeded synthetic workloads (geometry and random draws only; none of the method's arithmetic).

Shared by the tests, the smoke check and the benchmark, for both the GPU library and the CPU reference. The
paper's own setup (Sec. 3.1) is one droplet of radius 30 on the middle of the bottom wall; the workloads below
scale that setup. A wall droplet starts as the circular cap that meets the wall plane y_w = 0.5 at its prescribed
angle (centre at y_w - R cos(theta)), which is the paper's semicircle when theta = 90 deg.
"""
import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

SEED = 1501
WIDTH = 5.0          # tanh interface width of the initial profile
Y_WALL = 0.5         # bottom wall plane (between ghost row 0 and fluid row 1)


@dataclass
class Case:
    name: str
    nx: int
    ny: int
    T_over_Tc: float
    theta_bottom: np.ndarray          # [nx] radians
    theta_top: np.ndarray             # [nx] radians
    xc: List[float] = field(default_factory=list)
    yc: List[float] = field(default_factory=list)
    R: List[float] = field(default_factory=list)
    steps: int = 0

    @property
    def fluid_nodes(self):
        return self.nx * (self.ny - 2)


def wall_cap_centre(R, theta):
    """y of the centre of a circle of radius R meeting the bottom wall plane at angle theta (through the liquid)."""
    return Y_WALL - R * math.cos(theta)


def _uniform(nx, theta):
    return np.full(nx, float(theta))


def c1_neutral():
    """200 x 100, T = 0.85 T_c, theta = 90 deg, semicircle R = 30 centred on the bottom wall, 2000 steps."""
    nx, ny = 200, 100
    return Case("c1_200x100_T0.85_theta90", nx, ny, 0.85, _uniform(nx, math.pi / 2), _uniform(nx, math.pi / 2),
                [nx / 2], [Y_WALL], [30.0], 2000)


def c2_angle(theta_deg):
    """1024 x 512, T = 0.7 T_c, R = 120 cap at theta on the bottom wall, 20000 steps."""
    nx, ny = 1024, 512
    th = math.radians(theta_deg)
    return Case(f"c2_1024x512_T0.7_theta{theta_deg:g}", nx, ny, 0.7, _uniform(nx, th), _uniform(nx, math.pi / 2),
                [nx / 2], [wall_cap_centre(120.0, th)], [120.0], 20000)


def c3_large(seed=SEED, nx=4096, ny=2048, R_main=400.0, n_sat=64):
    """4096 x 2048, T = 0.5 T_c, theta = 45 deg: cap R = 400 at x = nx/2 plus n_sat free satellites with radius
    ~ U[10, 40] and centres ~ U over the fluid rows (y in [r+W+1, ny-2-r-W]), rejected when within 2W of another
    droplet or of the main cap (nearest periodic image in x); 10000 steps."""
    th = math.radians(45.0)
    rng = np.random.default_rng(seed)
    xs, ys, rs = [nx / 2], [wall_cap_centre(R_main, th)], [R_main]
    tries = 0
    while len(xs) < 1 + n_sat:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place satellites")
        r = rng.uniform(10.0, 40.0)
        x = rng.uniform(0.0, nx)
        y = rng.uniform(r + WIDTH + 1, ny - 2 - r - WIDTH)
        ok = True
        for (x2, y2, r2) in zip(xs, ys, rs):
            dx = x - x2
            dx -= nx * math.floor(dx / nx + 0.5)
            if math.hypot(dx, y - y2) < r + r2 + 2 * WIDTH:
                ok = False
                break
        if ok:
            xs.append(x)
            ys.append(y)
            rs.append(r)
    return Case(f"c3_{nx}x{ny}_T0.5_theta45_sat{n_sat}", nx, ny, 0.5, _uniform(nx, th), _uniform(nx, math.pi / 2),
                xs, ys, rs, 10000)


C4_SIZES = [(64, 32), (128, 64), (256, 128), (512, 256)]


def c4_batch(n=256, seed=SEED):
    """n instances: size uniform over C4_SIZES, theta ~ U[20, 160] deg, T/T_c ~ U[0.6, 0.9], cap of radius
    0.3 ny on the bottom wall at x = nx/2; 5000 steps."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        nx, ny = C4_SIZES[int(rng.integers(0, len(C4_SIZES)))]
        th = math.radians(rng.uniform(20.0, 160.0))
        t = rng.uniform(0.6, 0.9)
        R = 0.3 * ny
        out.append(Case(f"c4_{k}_{nx}x{ny}", nx, ny, t, _uniform(nx, th), _uniform(nx, math.pi / 2), [nx / 2],
                        [wall_cap_centre(R, th)], [R], 5000))
    return out


def c5_adjoint(seed=SEED):
    """256 x 128, T = 0.7 T_c, theta(x) = 90 deg + N(0, 10 deg) per wall node on both walls, semicircle of radius
    0.3 ny = 38.4 on the bottom wall; 2000 steps; target field from theta = 60 deg on both walls."""
    nx, ny = 256, 128
    rng = np.random.default_rng(seed)
    tb = np.radians(90.0 + rng.normal(0.0, 10.0, nx))
    tt = np.radians(90.0 + rng.normal(0.0, 10.0, nx))
    return Case("c5_256x128_T0.7_adjoint", nx, ny, 0.7, tb, tt, [nx / 2], [Y_WALL], [0.3 * ny], 2000)


def c5_target_angle():
    return math.radians(60.0)
