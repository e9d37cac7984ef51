"""Per-term formulas of the ternary EHD model (oracle; test infrastructure only).

Each function is one equation or one reading, written in the paper's notation.
Shapes: populations (Q, N), vectors (3, N) (z component zero in 2D), scalars (N,).
"""
import torch

DELTA_N = 1e-12   # regulariser of the interface normal where grad(Phi) vanishes


# ---------------------------------------------------------------- Eq. 11
def upsilons(g12, g13, g23):
    """Upsilon_1..3 and Upsilon_T from the three tensions (Eq. 11)."""
    u1 = g12 + g13 - g23
    u2 = g12 + g23 - g13
    u3 = g13 + g23 - g12
    ut = 3.0 / (1.0 / u1 + 1.0 / u2 + 1.0 / u3)
    return (u1, u2, u3), ut


# ---------------------------------------------------------------- Eq. 10
def chemical_potentials(phi, lap, ups, upsT, W):
    """mu_i = 24 U_i/W Phi_i (Phi_i - 1)(Phi_i - 1/2) - 24 U_T/W Phi1 Phi2 Phi3 - 3/4 U_i W lap Phi_i."""
    triple = phi[0] * phi[1] * phi[2]
    mus = []
    for i in range(3):
        p = phi[i]
        mus.append(24.0 * ups[i] / W * p * (p - 1.0) * (p - 0.5)
                   - 24.0 * upsT / W * triple
                   - 0.75 * ups[i] * W * lap[i])
    return torch.stack(mus)


# ---------------------------------------------------------------- isotropic stencils
def gather(field, nbr, q):
    """field at x + e_q for every node x."""
    return field[..., nbr[q]]


def grad_iso(field, lat, nbr):
    """grad F(x) = (1/cs2) sum_q w_q e_q F(x + e_q); field (..., N) -> (..., 3, N)."""
    acc = 0.0
    for q in range(1, lat.Q):
        fq = gather(field, nbr, q)
        acc = acc + (lat.w[q] / lat.cs2) * lat.e[q].reshape(3, 1) * fq.unsqueeze(-2)
    return acc


def lap_iso(field, lat, nbr):
    """lap F(x) = (2/cs2) sum_q w_q (F(x + e_q) - F(x))."""
    acc = 0.0
    for q in range(1, lat.Q):
        acc = acc + (2.0 * lat.w[q] / lat.cs2) * (gather(field, nbr, q) - field)
    return acc


def normals(grad):
    """n_i = grad Phi_i / sqrt(|grad Phi_i|^2 + delta^2)   (definition after Eq. 8, regularised)."""
    mag = torch.sqrt((grad ** 2).sum(-2, keepdim=True) + DELTA_N ** 2)
    return grad / mag


# ---------------------------------------------------------------- Eq. 18
def phase_flux(phi, nrm, W):
    """F_Phi_i = 4 n_i/W |Phi_i(1-Phi_i)| - Phi_i^2/sum_j Phi_j^2 * sum_j 4 n_j/W |Phi_j(1-Phi_j)|."""
    a = (4.0 / W) * torch.abs(phi * (1.0 - phi)).unsqueeze(-2) * nrm     # (3, 3, N)
    total = a.sum(0)                                                     # (3, N)
    den = (phi ** 2).sum(0, keepdim=True)
    den = torch.where(den > 0, den, torch.ones_like(den))                # solid nodes hold Phi = 0
    share = phi ** 2 / den                                               # (3, N)
    return a - share.unsqueeze(-2) * total.unsqueeze(0)


# ---------------------------------------------------------------- Eq. 20 (wetting)
def wetting_rhs(phi, cos12, cos13, cos23, W):
    """Right-hand sides of the energy-based wetting condition: n . grad Phi_i at the solid."""
    p1, p2, p3 = phi[0], phi[1], phi[2]
    r1 = (4.0 / W) * (-cos13 * p1 * p3 - cos12 * p1 * p2)
    r2 = (4.0 / W) * (cos12 * p1 * p2 - cos23 * p2 * p3)
    r3 = (4.0 / W) * (cos23 * p2 * p3 + cos13 * p1 * p3)
    return torch.stack([r1, r2, r3])


# ---------------------------------------------------------------- equilibria and sources
def edot(lat, vec):
    """e_q . v for every q: (3, N) -> (Q, N)."""
    return lat.e @ vec


def phase_equilibrium(phi_i, u, lat):
    """Eq. 16: f_eq = Phi w (1 + e.u/cs2)."""
    return lat.w.reshape(-1, 1) * phi_i * (1.0 + edot(lat, u) / lat.cs2)


def vector_source(G, lat):
    """Eq. 17 form: C_q = (w_q/cs2) e_q . G  (first moment G, zero mass)."""
    return lat.w.reshape(-1, 1) / lat.cs2 * edot(lat, G)


def flow_equilibrium(drho, u, lat):
    """Incompressible (rho0 = 1) equilibrium as a deviation from w:
    dg_eq = w [drho + e.u/cs2 + (e.u)^2/(2cs4) - u.u/(2cs2)]."""
    eu = edot(lat, u)
    uu = (u * u).sum(0)
    cs2 = lat.cs2
    return lat.w.reshape(-1, 1) * (drho + eu / cs2 + eu * eu / (2 * cs2 * cs2) - uu / (2 * cs2))


def guo_source(u, F, lat):
    """Guo forcing: F_q = w [(e - u).F/cs2 + (e.u)(e.F)/cs4]."""
    cs2 = lat.cs2
    eu = edot(lat, u)
    eF = edot(lat, F)
    uF = (u * F).sum(0)
    return lat.w.reshape(-1, 1) * ((eF - uF) / cs2 + eu * eF / (cs2 * cs2))


def second_moments(f, lat):
    """Pi_ab = sum_q e_qa e_qb f_q: (Q, N) -> (3, 3, N)."""
    return torch.einsum("qa,qb,qn->abn", lat.e, lat.e, f)


def mrt_collide(f, feq, C, rates, lat):
    """Raw-moment MRT, literally (Eq. 15 / Eq. 20b):
    m = M f, m_eq = M f_eq, m* = (I - S) m + S m_eq + (I - S/2) M C, f* = M^-1 m*.
    rates: (Q,) or (Q, N) diagonal of S."""
    M, Minv = lat.M, lat.Minv
    m = M @ f
    meq = M @ feq
    mc = M @ C
    if rates.dim() == 1:
        rates = rates.reshape(-1, 1)
    mstar = (1.0 - rates) * m + rates * meq + (1.0 - 0.5 * rates) * mc
    return Minv @ mstar


def moment_rates(lat, by_order, N=None, default=1.0):
    """Diagonal of S from a map order -> rate (scalar or (N,) tensor); unlisted orders relax at
    `default` (the rate of the moments the paper leaves unspecified, 1 unless chosen)."""
    rows = []
    for k in range(lat.Q):
        r = by_order.get(lat.order[k], default)
        if torch.is_tensor(r):
            rows.append(r)
        else:
            rows.append(torch.full((N,), float(r), dtype=torch.float64) if N is not None
                        else torch.tensor(float(r), dtype=torch.float64))
    return torch.stack(rows)
