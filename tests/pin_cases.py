"""Small validation setups for the closed-form pins (flags and initial fields only)."""
import numpy as np

from inputs import default_params
from inputs.presets import ELECTRODE0, FLUID, GROUND, NEUMANN


def grid(n):
    nx, ny, nz = n
    idx = np.arange(nx * ny * nz)
    return idx % nx, (idx // nx) % ny, idx // (nx * ny)


def flat_interface(nx=64, ny=4, lo=16, hi=48, **p):
    """Periodic strip, slab of phase 1 (droplet) in phase 3 (ambient), sharp start."""
    n = (nx, ny, 1)
    x, y, z = grid(n)
    flags = np.zeros(nx * ny, np.uint8)
    p1 = ((x >= lo) & (x < hi)).astype(np.float64)
    phi = np.stack([p1, np.zeros_like(p1), 1 - p1])
    return n, (1, 1, 0), default_params(2, **p), flags, phi


def periodic_droplet(n=(64, 64, 1), radius=12.0, W=4.0, **p):
    """Droplet of phase 1 in phase 3, fully periodic, tanh profile."""
    x, y, z = grid(n)
    c = [v / 2.0 for v in n]
    r2 = (x - c[0] + 0.5) ** 2 + (y - c[1] + 0.5) ** 2
    if n[2] > 1:
        r2 = r2 + (z - c[2] + 0.5) ** 2
    r = np.sqrt(r2)
    p1 = 0.5 * (1 + np.tanh(2 * (radius - r) / W))
    phi = np.stack([p1, np.zeros_like(p1), 1 - p1])
    dim = 3 if n[2] > 1 else 2
    periodic = (1, 1, 1) if dim == 3 else (1, 1, 0)
    return n, periodic, default_params(dim, width=W, **p), np.zeros(x.size, np.uint8), phi


def wall_droplet(nx=96, ny=40, radius=14.0, W=4.0, theta0_deg=90.0, **p):
    """Droplet of phase 1 in phase 3 on the bottom wall (walls at y = 0, ny-1): a circular cap
    meeting the wall plane y = 0.5 at angle theta0 (measured through the droplet)."""
    n = (nx, ny, 1)
    x, y, z = grid(n)
    flags = np.zeros(nx * ny, np.uint8)
    flags[y == 0] = GROUND
    flags[y == ny - 1] = NEUMANN
    yc = 0.5 - radius * np.cos(np.radians(theta0_deg))
    r = np.sqrt((x - nx / 2.0) ** 2 + (y - yc) ** 2)
    p1 = 0.5 * (1 + np.tanh(2 * (radius - r) / W))
    phi = np.stack([p1, np.zeros_like(p1), 1 - p1])
    phi[:, flags != FLUID] = 0
    return n, (1, 0, 0), default_params(2, width=W, **p), flags, phi


def channel(nx=4, ny=18, **p):
    """Single ambient phase between walls at y = 0 and y = ny-1 (Poiseuille)."""
    n = (nx, ny, 1)
    x, y, z = grid(n)
    flags = np.zeros(nx * ny, np.uint8)
    flags[y == 0] = GROUND
    flags[y == ny - 1] = NEUMANN
    phi = np.zeros((3, nx * ny))
    phi[2] = 1.0
    phi[:, flags != FLUID] = 0
    return n, (1, 0, 0), default_params(2, **p), flags, phi


def capacitor(nx=4, ny=34, top=ELECTRODE0, bottom=GROUND, layer=None, **p):
    """Plates at y = 0 and y = ny-1; ambient fluid, optionally phase 1 below row `layer`."""
    n = (nx, ny, 1)
    x, y, z = grid(n)
    flags = np.zeros(nx * ny, np.uint8)
    flags[y == 0] = bottom
    flags[y == ny - 1] = top
    phi = np.zeros((3, nx * ny))
    if layer is None:
        phi[2] = 1.0
    else:
        phi[0] = (y < layer).astype(np.float64)
        phi[2] = 1.0 - phi[0]
    phi[:, flags != FLUID] = 0
    return n, (1, 0, 0), default_params(2, **p), flags, phi


def strip(nx=262, ny=42, e_lo=21, **p):
    """Grounded bottom (y = 0), insulating top and left end, electrode on the right end wall
    for rows y >= e_lo (the semi-infinite strip behind the paper's electric-force model)."""
    n = (nx, ny, 1)
    x, y, z = grid(n)
    flags = np.zeros(nx * ny, np.uint8)
    flags[x == 0] = NEUMANN
    flags[x == nx - 1] = NEUMANN
    flags[(x == nx - 1) & (y >= e_lo)] = ELECTRODE0
    flags[y == 0] = GROUND
    flags[y == ny - 1] = NEUMANN
    phi = np.zeros((3, nx * ny))
    phi[2] = 1.0
    phi[:, flags != FLUID] = 0
    return n, (0, 0, 0), default_params(2, **p), flags, phi


def contact_angle(phi1_2d, wall_y=0.5, min_y=2.0):
    """Angle (degrees, through phase 1) where a circle fitted to the Phi_1 = 1/2 contour
    meets the wall plane."""
    import math
    f = phi1_2d
    ny, nx = f.shape
    pts = []
    for yy in range(1, ny - 1):
        row = f[yy]
        for xx in range(nx - 1):
            a, b = row[xx], row[xx + 1]
            if (a - 0.5) * (b - 0.5) < 0:
                pts.append((xx + (0.5 - a) / (b - a), yy))
    for xx in range(nx):
        col = f[:, xx]
        for yy in range(1, ny - 2):
            a, b = col[yy], col[yy + 1]
            if (a - 0.5) * (b - 0.5) < 0:
                pts.append((xx, yy + (0.5 - a) / (b - a)))
    P = np.array(pts)
    P = P[P[:, 1] >= min_y]
    A = np.c_[2 * P[:, 0], 2 * P[:, 1], np.ones(len(P))]
    xc, yc, cc = np.linalg.lstsq(A, (P ** 2).sum(1), rcond=None)[0]
    R = math.sqrt(cc + xc * xc + yc * yc)
    return math.degrees(math.acos((wall_y - yc) / R)), R


def lens(nx=160, ny=112, area=628.3185307179587, W=4.0, **p):
    """A droplet (phase 1) at the flat interface between a lubricant layer (phase 2, below
    y0 = ny/2) and the ambient (phase 3, above): a disc of the given area centred on the
    interface, tanh profiles.  Periodic in x; walls at y = 0 and ny-1, each touched by one
    phase only (so the wetting condition does not act)."""
    n = (nx, ny, 1)
    x, y, z = grid(n)
    flags = np.zeros(nx * ny, np.uint8)
    flags[y == 0] = GROUND
    flags[y == ny - 1] = NEUMANN
    y0 = ny / 2.0
    r0 = np.sqrt(area / np.pi)
    r = np.sqrt((x - nx / 2.0) ** 2 + (y - y0) ** 2)
    p1 = 0.5 * (1 + np.tanh(2 * (r0 - r) / W))
    below = 0.5 * (1 + np.tanh(2 * (y0 - y) / W))
    p2 = (1 - p1) * below
    phi = np.stack([p1, p2, 1 - p1 - p2])
    phi[:, flags != FLUID] = 0
    return n, (1, 0, 0), default_params(2, width=W, **p), flags, phi


def contour_points(f, level=0.5):
    """Crossings of the level set of a 2D field (rows y, columns x) along rows and columns,
    by linear interpolation: an (n, 2) array of (x, y)."""
    ny, nx = f.shape
    pts = []
    for yy in range(ny):
        row = f[yy]
        for xx in range(nx - 1):
            a, b = row[xx], row[xx + 1]
            if (a - level) * (b - level) < 0:
                pts.append((xx + (level - a) / (b - a), yy))
    for xx in range(nx):
        col = f[:, xx]
        for yy in range(ny - 1):
            a, b = col[yy], col[yy + 1]
            if (a - level) * (b - level) < 0:
                pts.append((xx, yy + (level - a) / (b - a)))
    return np.asarray(pts, dtype=np.float64)


def fit_circle(P):
    """Least-squares circle through the points P (n, 2): centre (xc, yc) and radius."""
    import math
    A = np.c_[2 * P[:, 0], 2 * P[:, 1], np.ones(len(P))]
    xc, yc, cc = np.linalg.lstsq(A, (P ** 2).sum(1), rcond=None)[0]
    return xc, yc, math.sqrt(cc + xc * xc + yc * yc)


def lens_geometry(phi3d):
    """Geometry of a lens of phase 1 at the 2-3 interface from the fields (3, ny, nx): the level
    y0 of the 2-3 interface far from the lens (Phi_2 = Phi_3 in the 15 outermost columns on
    each side), and circles fitted to the Phi_1 = 1/2 contour above (upper cap, in phase 3) and
    below (lower cap, in phase 2) y0 +- 3.  Returns y0 and per cap: the angle between its chord
    on y = y0 and its arc at the triple points (degrees, inside phase 1), its height and chord,
    and its radius."""
    import math
    f1, f2, f3 = phi3d
    ny, nx = f1.shape
    lv = []
    for c in list(range(0, 15)) + list(range(nx - 15, nx)):
        d = f2[:, c] - f3[:, c]
        for yy in range(ny - 1):
            if d[yy] * d[yy + 1] < 0:
                lv.append(yy + d[yy] / (d[yy] - d[yy + 1]))
    y0 = float(np.mean(lv))
    P = contour_points(f1)
    out = dict(y0=y0)
    for name, sel, sgn in (("upper", P[:, 1] > y0 + 3, 1.0), ("lower", P[:, 1] < y0 - 3, -1.0)):
        xc, yc, r = fit_circle(P[sel])
        d = sgn * (y0 - yc)                # distance of the centre behind the chord
        out[name] = dict(angle=math.degrees(math.acos(d / r)), height=r - d,
                         chord=2 * math.sqrt(r * r - d * d), radius=r)
    return out
