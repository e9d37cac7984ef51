"""Workload recipes: the droplet / lubricant / ambient configurations, in lattice units.

Geometry of the workloads follows the paper's problem statement (Results, Fig. 1
and its text): a droplet resting on a lubricant layer that infuses a micropillar
array on the bottom wall, an electrode segment on the opposite wall, grounded
pillars and substrate, Neumann (insulating) walls elsewhere.  Pillars of width
w and pitch p give solid fraction (w/p)^2 = 0.25 in 3D, as in the paper.

Arrays use the node index  node = x + Nx*(y + Ny*z)  (x fastest); 2D cases have
Nz = 1.  Flags: 0 fluid, 1 grounded solid, 2 insulating (Neumann) solid,
3 + k electrode k.  Phase arrays are float64 of shape (3, N): droplet,
lubricant, ambient.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FLUID, GROUND, NEUMANN, ELECTRODE0 = 0, 1, 2, 3
MAX_ELECTRODES = 4

_M64 = (1 << 64) - 1


def splitmix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (Steele, Lea & Flood 2014; Vigna's public-domain
    reference), vectorised over uint64 states; the state increment is applied first."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, node: np.ndarray, comp: int) -> np.ndarray:
    """Counter-based uniform draw in [0, 1): top 53 bits of splitmix64(seed*2^40 + 4*node + comp)."""
    base = (int(seed) << 40) & _M64
    ctr = (np.uint64(base) + np.asarray(node, dtype=np.uint64) * np.uint64(4) + np.uint64(comp))
    return (splitmix64(ctr) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def voltage_schedule(seed: int, n_seg: int, lo: float = 0.0, hi: float = 0.08) -> np.ndarray:
    """Piecewise-constant electrode voltages drawn uniform[lo, hi) from numpy's default generator."""
    return np.random.default_rng(seed).uniform(lo, hi, n_seg)


def default_params(dim: int, **over) -> dict:
    """Parameter set in lattice units.  Index 0 = droplet, 1 = lubricant, 2 = ambient.

    Defaults: tau = 1 in all phases, interface width 4, equal tensions 1e-3,
    mobility 0.0025 (Methods, text after Eq. 8), contact angles theta_13 = 100 deg
    (droplet on solid in ambient) and theta_23 = 5 deg (lubricant on solid in
    ambient) as in the paper's Fig. 2 case; theta_12 follows from Young's relation.
    """
    g12 = over.pop("gamma12", 1e-3)
    g13 = over.pop("gamma13", 1e-3)
    g23 = over.pop("gamma23", 1e-3)
    th13 = over.pop("theta13_deg", 100.0)
    th23 = over.pop("theta23_deg", 5.0)
    c13 = math.cos(math.radians(th13))
    c23 = math.cos(math.radians(th23))
    # Young: gamma12 cos(theta12) = gamma_s2 - gamma_s1 = gamma13 cos(theta13) - gamma23 cos(theta23)
    c12 = (g13 * c13 - g23 * c23) / g12
    p = dict(
        dim=dim,
        tau_flow=(1.0, 1.0, 1.0),
        mobility=0.0025,
        width=4.0,
        gamma12=g12, gamma13=g13, gamma23=g23,
        cos12=c12, cos13=c13, cos23=c23,
        ehd=0,
        eps=(80.0, 2.5, 1.0),
        cond=(0.1, 1e-4, 1e-4),
        charge_diffusion=0.0,
        body_force=(0.0, 0.0, 0.0),
        electrode_volts=(0.0,) * MAX_ELECTRODES,
        poisson_tol=1e-13,
        poisson_max_iter=400,
        poisson_check_every=1,
        s_high=1.0,
        rho=(1.0, 1.0, 1.0),
    )
    for k, v in over.items():
        if k not in p:
            raise KeyError(f"unknown parameter {k}")
        p[k] = v
    return p


@dataclass
class Case:
    name: str
    dim: int
    n: tuple            # (Nx, Ny, Nz)
    periodic: tuple     # per axis, 1 = wraps
    precision: str      # "fp64" or "fp32"
    params: dict
    flags: np.ndarray   # uint8 (N,)
    phi: np.ndarray     # float64 (3, N)
    steps: int
    schedule: np.ndarray | None = None   # volts per segment for electrode 0
    t_total: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    def coords(self):
        nx, ny, nz = self.n
        z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        return x.ravel(), y.ravel(), z.ravel()


def _grid(n):
    nx, ny, nz = n
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.ravel().astype(np.float64), y.ravel().astype(np.float64), z.ravel().astype(np.float64)


def _lis_geometry(dim, n, pillar_w, pillar_pitch, pillar_h, electrode_x):
    """Walls on the two ends of the vertical axis (y in 2D, z in 3D): bottom grounded,
    top insulating except an electrode segment.  Pillars on the bottom wall, grounded."""
    x, y, z = _grid(n)
    vert = y if dim == 2 else z
    nv = n[1] if dim == 2 else n[2]
    flags = np.zeros(x.size, dtype=np.uint8)
    if pillar_w > 0:
        inx = np.mod(x, pillar_pitch) < pillar_w
        if dim == 3:
            inx &= np.mod(y, pillar_pitch) < pillar_w
        pil = inx & (vert >= 1) & (vert <= pillar_h)
        flags[pil] = GROUND
    flags[vert == 0] = GROUND
    top = vert == nv - 1
    flags[top] = NEUMANN
    if electrode_x is not None:
        e0, e1 = electrode_x
        flags[top & (x >= e0) & (x < e1)] = ELECTRODE0
    return flags


def _droplet_on_film(dim, n, flags, center, radius, level, width):
    """Initial phase fields: a droplet cap centred on the lubricant level, lubricant below
    the level, ambient elsewhere; tanh profiles of width W across every interface."""
    x, y, z = _grid(n)
    if dim == 2:
        r = np.sqrt((x - center[0]) ** 2 + (y - level) ** 2)
        vert = y
    else:
        r = np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - level) ** 2)
        vert = z
    above = 0.5 * (1.0 + np.tanh(2.0 * (vert - level) / width))
    below = 0.5 * (1.0 + np.tanh(2.0 * (level - vert) / width))
    p1 = 0.5 * (1.0 + np.tanh(2.0 * (radius - r) / width)) * above
    p2 = (1.0 - p1) * below
    phi = np.stack([p1, p2, 1.0 - p1 - p2])
    phi[:, flags != FLUID] = 0.0
    return phi


def _jitter(phi, flags, seed, amp=1e-6):
    node = np.arange(phi.shape[1], dtype=np.uint64)
    out = phi.copy()
    for comp in (0, 1):
        u = uniform01(seed, node, comp)
        out[comp] += (2.0 * u - 1.0) * amp
    out[2] = 1.0 - out[0] - out[1]
    out[:, flags != FLUID] = 0.0
    return out


def _charge_diffusion(alpha_star, eps_w, radius, volts, height, tau_w):
    """alpha from alpha* = alpha mu_w / (eps_w R0^2 E0^2) with E0 = phi0 / L (text after Eq. 14
    and the potential boundary conditions of the Results), mu_w = rho nu = (tau - 1/2)/3."""
    mu_w = (tau_w - 0.5) / 3.0
    e0 = volts / height
    return alpha_star * eps_w * radius ** 2 * e0 ** 2 / mu_w


def make_case(name: str, seed: int = 0, precision: str | None = None, **over) -> Case:
    """Build a named workload.

    c1  2D 128x64 FP64, flat walls, 6-cell lubricant film, droplet R=20, no field.
    c2  2D 512x256 EHD, pillars 8/16/12, droplet R=40, electrode 64 cells 40 lu ahead.
    c3  3D 256x128x96 EHD, pillars 6x6x10 pitch 12, droplet R=30, electrode strip.
    c4  c2 geometry, FP32, 64-segment voltage schedule over T=4000 (adjoint workload).
    c5  3D 384x192x128 EHD, droplet R=48, 32-segment schedule over T=2000.
    Reduced-size variants with the same structure (for oracle-speed tests):
    c1s 2D 64x32, c2s 2D 128x64, c3s 3D 48x32x24, c4s 2D 96x48 with a schedule.
    """
    alpha_star = over.pop("alpha_star", 1e-4)
    volts = over.pop("volts", None)
    if volts is None:
        volts = {"m2": 1.0, "m2s": 0.7}.get(name, 0.05)
    jitter = over.pop("jitter", None)
    if name in ("c1", "c1s"):
        n = (128, 64, 1) if name == "c1" else (64, 32, 1)
        film = 6 if name == "c1" else 4
        radius = 20.0 if name == "c1" else 10.0
        dim = 2
        flags = _lis_geometry(dim, n, 0, 1, 0, None)
        level = film + 0.5
        center = (n[0] / 2.0,)
        params = default_params(2)
        phi = _droplet_on_film(dim, n, flags, center, radius, level, params["width"])
        phi = _jitter(phi, flags, seed)
        steps = 1000
        prec = "fp64"
        sched = None
        t_total = 0
        electrode = None
    elif name in ("c2", "c2s", "c4", "c4s"):
        dim = 2
        if name in ("c2", "c4"):
            n, pw, pp, ph, radius, xc = (512, 256, 1), 8, 16, 12, 40.0, 128.0
        elif name == "c2s":
            n, pw, pp, ph, radius, xc = (128, 64, 1), 4, 8, 6, 12.0, 40.0
        else:
            n, pw, pp, ph, radius, xc = (96, 48, 1), 4, 8, 5, 10.0, 30.0
        gap = 40 if name in ("c2", "c4") else 10
        elen = 64 if name in ("c2", "c4") else 24
        e0 = int(xc + radius) + gap
        electrode = (e0, e0 + elen)
        flags = _lis_geometry(dim, n, pw, pp, ph, electrode)
        level = ph + 0.5
        params = default_params(2)
        phi = _droplet_on_film(dim, n, flags, (xc,), radius, level, params["width"])
        alpha = _charge_diffusion(alpha_star, params["eps"][0], radius, volts, n[1], params["tau_flow"][0])
        params.update(ehd=1, charge_diffusion=alpha, electrode_volts=(volts, 0.0, 0.0, 0.0))
        if name == "c2":
            steps, prec = 20000, "fp64"
        elif name == "c2s":
            steps, prec = 1000, "fp64"
        elif name == "c4":
            steps, prec = 4000, "fp32"
        else:
            steps, prec = 400, "fp64"
        sched, t_total = None, 0
        if name in ("c4", "c4s"):
            n_seg = 64 if name == "c4" else 8
            sched = voltage_schedule(seed, n_seg)
            t_total = steps
    elif name in ("c3", "c3s", "c5"):
        dim = 3
        if name == "c3":
            n, radius, xc, yc, steps = (256, 128, 96), 30.0, 64.0, 64.0, 5000
        elif name == "c5":
            n, radius, xc, yc, steps = (384, 192, 128), 48.0, 96.0, 96.0, 2000
        else:
            n, radius, xc, yc, steps = (48, 32, 24), 8.0, 14.0, 16.0, 200
        if name == "c3s":
            pw, pp, ph = 3, 6, 4
        else:
            pw, pp, ph = 6, 12, 10
        gap = 40 if name != "c3s" else 8
        elen = 64 if name != "c3s" else 16
        e0 = int(xc + radius) + gap
        electrode = (e0, e0 + elen)
        flags = _lis_geometry(dim, n, pw, pp, ph, electrode)
        level = ph + 0.5
        params = default_params(3)
        phi = _droplet_on_film(dim, n, flags, (xc, yc), radius, level, params["width"])
        alpha = _charge_diffusion(alpha_star, params["eps"][0], radius, volts, n[2], params["tau_flow"][0])
        params.update(ehd=1, charge_diffusion=alpha, electrode_volts=(volts, 0.0, 0.0, 0.0))
        prec = "fp32" if name in ("c3", "c5") else "fp64"
        sched, t_total = None, 0
        if name == "c5":
            sched = voltage_schedule(seed, 32)
            t_total = steps
    elif name in ("m2", "m2s"):
        # migrating workload: a droplet sliding on a flat lubricant film (the lubricant wets the
        # solid and the film is thicker than the interface, so the droplet never touches it: the
        # regime I_os(w)/I_s < 0 of the drag model), pulled by top-wall electrodes; tensions and
        # voltage raised so that it travels 3 R0 in about 2e5 steps at an electric capillary
        # number eps_a (V/L)^2 R0 / gamma ~ 0.3 (m2: 1.0 lu; m2s: 0.7 lu).  Electrode 0 lies 3 R0 ahead of the droplet's
        # front, electrode 1 as far behind its back (for two-electrode switching).
        dim = 2
        n, radius, xc, film = ((384, 64, 1), 12.0, 120.0, 8) if name == "m2" else ((192, 48, 1), 8.0, 64.0, 6)
        gap, elen = int(3 * radius), 64 if name == "m2" else 32
        e0 = int(xc + radius) + gap
        e1_hi = int(xc - radius) - gap
        electrode = (e0, e0 + elen)
        x, y, z = _grid(n)
        flags = _lis_geometry(dim, n, 0, 1, 0, electrode)
        top = y == n[1] - 1
        flags[top & (x >= e1_hi - elen) & (x < e1_hi)] = ELECTRODE0 + 1
        level = film + 0.5
        g = 0.01
        params = default_params(2, gamma12=g, gamma13=g, gamma23=g)
        phi = _droplet_on_film(dim, n, flags, (xc,), radius, level, params["width"])
        # charge diffusion 1e-4 (alpha* = 1e-4 would give 1.7e-3 here: a charge layer that
        # spreads over the droplet and stalls its motion in these lattice units)
        params.update(ehd=1, charge_diffusion=1e-4, electrode_volts=(volts, 0.0, 0.0, 0.0))
        steps, prec = (200000, "fp32") if name == "m2" else (60000, "fp32")
        sched, t_total = None, 0
    else:
        raise KeyError(name)
    if jitter is not None:
        phi = _jitter(phi, flags, jitter)
    for k, v in over.items():
        params[k] = v
    periodic = (1, 1, 0) if dim == 3 else (1, 0, 0)
    meta = dict(radius=radius, electrode=electrode)
    if name in ("m2", "m2s"):
        meta.update(electrode2=(e1_hi - elen, e1_hi), film=film, channel=n[1] - 2)
    return Case(name=name, dim=dim, n=n, periodic=periodic, precision=precision or prec,
                params=params, flags=flags, phi=phi, steps=steps, schedule=sched,
                t_total=t_total, meta=meta)


def case_names():
    return ["c1", "c2", "c3", "c4", "c5", "c1s", "c2s", "c3s", "c4s", "m2", "m2s"]
