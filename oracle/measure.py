"""Contact-angle measurement on a density field (test infrastructure).

The paper quotes measured angles (Sec. 4.2.1 and 4.2.2) without saying how they were read off the droplet. The
reading taken here: inside a box around the droplet, take rho_mid = (max + min)/2 over the box, locate the
rho_mid crossings on horizontal and vertical lattice links by linear interpolation, drop points within 3 lattice
units of the wall plane, fit a circle algebraically (Kasa: least squares of x^2 + y^2 + D x + E y + F = 0), and
take the angle through the liquid between the wall and the circle, theta = acos((y_w - y_c)/R) on the bottom wall
(y_w = 0.5) and acos((y_c - y_w)/R) on the top wall (y_w = ny - 1.5).
"""
import numpy as np


def interface_points(rho, box, wall, ny):
    """rho_mid crossing points [(x, y)] inside box = (x_lo, x_hi, y_lo, y_hi) (half-open node ranges)."""
    x_lo, x_hi, y_lo, y_hi = box
    sub = rho[y_lo:y_hi, x_lo:x_hi]
    m = 0.5 * (sub.max() + sub.min())
    pts = []
    # horizontal links (x, y) - (x + 1, y)
    a, b = sub[:, :-1], sub[:, 1:]
    cross = (a < m) != (b < m)
    yy, xx = np.nonzero(cross)
    t = (m - a[yy, xx]) / (b[yy, xx] - a[yy, xx])
    pts.append(np.stack([x_lo + xx + t, y_lo + yy.astype(np.float64)], axis=1))
    # vertical links (x, y) - (x, y + 1)
    a, b = sub[:-1, :], sub[1:, :]
    cross = (a < m) != (b < m)
    yy, xx = np.nonzero(cross)
    t = (m - a[yy, xx]) / (b[yy, xx] - a[yy, xx])
    pts.append(np.stack([x_lo + xx.astype(np.float64), y_lo + yy + t], axis=1))
    pts = np.concatenate(pts, axis=0)
    y_w = 0.5 if wall == 0 else ny - 1.5
    keep = pts[:, 1] >= y_w + 3.0 if wall == 0 else pts[:, 1] <= y_w - 3.0
    return pts[keep], m


def kasa_fit(pts):
    """Algebraic circle fit; returns (xc, yc, R)."""
    x, y = pts[:, 0], pts[:, 1]
    Amat = np.stack([x, y, np.ones_like(x)], axis=1)
    rhs = -(x * x + y * y)
    (D, E, F), *_ = np.linalg.lstsq(Amat, rhs, rcond=None)
    xc, yc = -D / 2.0, -E / 2.0
    return xc, yc, np.sqrt(xc * xc + yc * yc - F)


def measure_contact_angle(rho, box, wall=0):
    """(theta [rad], R, xc, yc, npoints) of the droplet inside box on the given wall (0 bottom, 1 top).

    rho: [ny, nx] density with row 0 / ny-1 the ghost rows (their values are not used unless the box covers them).
    """
    ny = rho.shape[0]
    pts, _ = interface_points(rho, box, wall, ny)
    if len(pts) < 3:
        raise ValueError("too few interface points in the box")
    xc, yc, R = kasa_fit(pts)
    y_w = 0.5 if wall == 0 else ny - 1.5
    c = (y_w - yc) / R if wall == 0 else (yc - y_w) / R
    return float(np.arccos(np.clip(c, -1.0, 1.0))), float(R), float(xc), float(yc), int(len(pts))
