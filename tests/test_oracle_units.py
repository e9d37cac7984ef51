"""Pins of the oracle's individual terms against identities and closed forms the model fixes.

Each check is independent of the code it tests: an algebraic identity, a
reduction to the binary (two-phase) textbook case, an exact moment, or a
second derivation of the same collision.
"""
import math

import numpy as np
import pytest
import torch

from oracle import model
from oracle.lattice import Lattice

F64 = torch.float64


@pytest.fixture(params=[2, 3], ids=["D2Q9", "D3Q19"])
def lat(request):
    return Lattice(request.param)


def _rand_phi(n, seed=0, ternary=True):
    g = torch.Generator().manual_seed(seed)
    a = torch.rand(3, n, generator=g, dtype=F64)
    if not ternary:
        a[1] = 0
    return a / a.sum(0, keepdim=True)


# ------------------------------------------------------------------ lattice
def test_lattice_isotropy(lat):
    """sum w = 1, sum w e e = cs2 I, fourth moment cs4 (dd + dd + dd), odd moments 0."""
    e, w, cs2 = lat.e, lat.w, lat.cs2
    assert abs(float(w.sum()) - 1.0) < 1e-15
    d = lat.dim
    I = torch.eye(3, dtype=F64)
    I[d:, d:] = 0
    second = torch.einsum("q,qa,qb->ab", w, e, e)
    assert torch.allclose(second, cs2 * I, atol=1e-15)
    third = torch.einsum("q,qa,qb,qc->abc", w, e, e, e)
    assert third.abs().max() < 1e-15
    fourth = torch.einsum("q,qa,qb,qc,qd->abcd", w, e, e, e, e)
    iso = (torch.einsum("ab,cd->abcd", I, I) + torch.einsum("ac,bd->abcd", I, I)
           + torch.einsum("ad,bc->abcd", I, I)) * cs2 * cs2
    assert torch.allclose(fourth, iso, atol=1e-15)


def test_moment_basis_invertible(lat):
    assert torch.linalg.matrix_rank(lat.M) == lat.Q
    assert torch.allclose(lat.M @ lat.Minv, torch.eye(lat.Q, dtype=F64), atol=1e-13)
    for q in range(lat.Q):
        assert torch.equal(lat.e[lat.opp[q]], -lat.e[q])


# ------------------------------------------------------------------ stencils
def _periodic_nbr(lat, n):
    nx, ny, nz = n
    idx = np.arange(nx * ny * nz)
    x, y, z = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    nb = np.stack([((x + ex) % nx) + nx * (((y + ey) % ny) + ny * ((z + ez) % nz))
                   for ex, ey, ez in lat.e_int])
    return torch.from_numpy(nb), torch.from_numpy(np.stack([x, y, z]).astype(np.float64))


def test_isotropic_stencils_exact_on_polynomials(lat):
    """grad of a linear field and lap of a quadratic field are exact away from the wrap."""
    n = (8, 8, 8 if lat.dim == 3 else 1)
    nbr, xyz = _periodic_nbr(lat, n)
    x, y, z = xyz
    lin = 0.3 * x - 0.7 * y + (0.2 * z if lat.dim == 3 else 0)
    quad = x * x + 2 * y * y + (3 * z * z if lat.dim == 3 else 0) + x * y
    inner = (x > 0) & (x < n[0] - 1) & (y > 0) & (y < n[1] - 1)
    if lat.dim == 3:
        inner &= (z > 0) & (z < n[2] - 1)
    g = model.grad_iso(lin, lat, nbr)
    assert torch.allclose(g[0][inner], torch.full_like(g[0][inner], 0.3), atol=1e-13)
    assert torch.allclose(g[1][inner], torch.full_like(g[1][inner], -0.7), atol=1e-13)
    lap = model.lap_iso(quad, lat, nbr)
    expect = 2 + 4 + (6 if lat.dim == 3 else 0)
    assert torch.allclose(lap[inner], torch.full_like(lap[inner], float(expect)), atol=1e-12)


# ------------------------------------------------------------------ Eqs. 10-11
def test_upsilon_pairwise_tensions():
    """Binary tension between phases i, j is (U_i + U_j)/2 = gamma_ij."""
    g12, g13, g23 = 0.7e-3, 1.3e-3, 0.9e-3
    (u1, u2, u3), ut = model.upsilons(g12, g13, g23)
    assert math.isclose((u1 + u2) / 2, g12, rel_tol=1e-14)
    assert math.isclose((u1 + u3) / 2, g13, rel_tol=1e-14)
    assert math.isclose((u2 + u3) / 2, g23, rel_tol=1e-14)
    assert math.isclose(3.0 / ut, 1 / u1 + 1 / u2 + 1 / u3, rel_tol=1e-14)


def test_chemical_potentials_sum_identity():
    """sum_i mu_i / U_i = 0 whenever sum Phi_i = 1 (and hence sum lap Phi_i = 0)."""
    (u1, u2, u3), ut = model.upsilons(0.7e-3, 1.3e-3, 0.9e-3)
    phi = _rand_phi(500)
    g = torch.Generator().manual_seed(1)
    lap = torch.randn(3, 500, generator=g, dtype=F64)
    lap[2] = -lap[0] - lap[1]
    mu = model.chemical_potentials(phi, lap, (u1, u2, u3), ut, 4.0)
    s = mu[0] / u1 + mu[1] / u2 + mu[2] / u3
    assert s.abs().max() < 1e-12 * mu.abs().max()


def test_chemical_potential_vanishes_on_tanh_profile():
    """Binary case: Phi = (1 + tanh(2x/W))/2 with its exact second derivative gives mu = 0."""
    W = 5.0
    x = torch.linspace(-12, 12, 241, dtype=F64)
    p = 0.5 * (1 + torch.tanh(2 * x / W))
    d1 = (1 - torch.tanh(2 * x / W) ** 2) / W
    d2 = (4.0 / W) * (1 - 2 * p) * d1
    phi = torch.stack([p, torch.zeros_like(p), 1 - p])
    lap = torch.stack([d2, torch.zeros_like(p), -d2])
    (u1, u2, u3), ut = model.upsilons(1e-3, 1e-3, 1e-3)
    mu = model.chemical_potentials(phi, lap, (u1, u2, u3), ut, W)
    assert mu.abs().max() < 1e-17


# ------------------------------------------------------------------ Eq. 18
def test_phase_flux_sums_to_zero_and_reduces_to_binary():
    phi = _rand_phi(300)
    g = torch.Generator().manual_seed(2)
    grad = torch.randn(3, 3, 300, generator=g, dtype=F64)
    nrm = model.normals(grad)
    F = model.phase_flux(phi, nrm, 4.0)
    assert F.sum(0).abs().max() < 1e-15
    # binary: Phi_2 = 0, Phi_3 = 1 - Phi_1, n_3 = -n_1  ->  F_1 = (4/W) Phi(1-Phi) n_1
    p = phi[0]
    phib = torch.stack([p, torch.zeros_like(p), 1 - p])
    n1 = nrm[0]
    nb = torch.stack([n1, torch.zeros_like(n1), -n1])
    Fb = model.phase_flux(phib, nb, 4.0)
    assert torch.allclose(Fb[0], (4.0 / 4.0) * (p * (1 - p)) * n1, atol=1e-15)
    assert Fb[1].abs().max() == 0


# ------------------------------------------------------------------ Eq. 20 (wetting)
def test_wetting_rhs_sum_and_binary():
    phi = _rand_phi(200)
    c12, c13, c23 = -0.3, 0.5, 0.8
    r = model.wetting_rhs(phi, c12, c13, c23, 4.0)
    assert r.sum(0).abs().max() < 1e-16
    p = phi[0]
    phib = torch.stack([p, torch.zeros_like(p), 1 - p])
    rb = model.wetting_rhs(phib, c12, c13, c23, 4.0)
    assert torch.allclose(rb[0], -(4.0 / 4.0) * c13 * p * (1 - p), atol=1e-16)


# ------------------------------------------------------------------ equilibria (Eq. 16, flow, Guo)
def _moments(lat, f):
    m0 = f.sum(0)
    m1 = lat.e.T @ f
    m2 = torch.einsum("qa,qb,qn->abn", lat.e, lat.e, f)
    return m0, m1, m2


def test_phase_equilibrium_moments(lat):
    g = torch.Generator().manual_seed(3)
    n = 50
    phi = torch.rand(n, generator=g, dtype=F64)
    u = 0.05 * torch.randn(3, n, generator=g, dtype=F64)
    u[lat.dim:] = 0
    feq = model.phase_equilibrium(phi, u, lat)
    m0, m1, m2 = _moments(lat, feq)
    assert torch.allclose(m0, phi, atol=1e-15)
    assert torch.allclose(m1, phi * u, atol=1e-15)
    I = torch.eye(3, dtype=F64)
    I[lat.dim:, lat.dim:] = 0
    assert torch.allclose(m2, lat.cs2 * I.unsqueeze(-1) * phi, atol=1e-15)


def test_flow_equilibrium_and_guo_moments(lat):
    g = torch.Generator().manual_seed(4)
    n = 50
    drho = 1e-3 * torch.randn(n, generator=g, dtype=F64)
    u = 0.05 * torch.randn(3, n, generator=g, dtype=F64)
    F = 1e-4 * torch.randn(3, n, generator=g, dtype=F64)
    u[lat.dim:] = 0
    F[lat.dim:] = 0
    geq = model.flow_equilibrium(drho, u, lat)
    m0, m1, m2 = _moments(lat, geq)
    I = torch.eye(3, dtype=F64)
    I[lat.dim:, lat.dim:] = 0
    assert torch.allclose(m0, drho, atol=1e-16)
    assert torch.allclose(m1, u, atol=1e-16)
    uu = torch.einsum("an,bn->abn", u, u)
    assert torch.allclose(m2, lat.cs2 * I.unsqueeze(-1) * drho + uu, atol=1e-16)
    src = model.guo_source(u, F, lat)
    s0, s1, s2 = _moments(lat, src)
    assert s0.abs().max() < 1e-18
    assert torch.allclose(s1, F, atol=1e-18)
    assert torch.allclose(s2, torch.einsum("an,bn->abn", u, F) + torch.einsum("an,bn->abn", F, u), atol=1e-18)


# ------------------------------------------------------------------ Eq. 15 literal MRT
def test_mrt_equal_rates_is_bgk(lat):
    g = torch.Generator().manual_seed(5)
    n = 40
    f = torch.rand(lat.Q, n, generator=g, dtype=F64)
    feq = torch.rand(lat.Q, n, generator=g, dtype=F64)
    C = 1e-3 * torch.randn(lat.Q, n, generator=g, dtype=F64)
    s = 1.37
    out = model.mrt_collide(f, feq, C, torch.full((lat.Q,), s, dtype=F64), lat)
    assert torch.allclose(out, f - s * (f - feq) + (1 - s / 2) * C, atol=1e-14)


def test_mrt_two_rate_closed_form(lat):
    """First-order raw moments at rate s, all others at 1: the literal moment-space collision
    equals f_eq + C/2 + (1 - s)/2 (e_q . J) on the axis links only, with
    J = sum f e - sum f_eq e + (sum C e)/2.  Derived by hand from the columns of M^-1
    of the monomial basis (the first-order columns are +-1/2 on the +-axis links)."""
    g = torch.Generator().manual_seed(6)
    n = 40
    f = torch.rand(lat.Q, n, generator=g, dtype=F64)
    phi = torch.rand(n, generator=g, dtype=F64)
    u = 0.05 * torch.randn(3, n, generator=g, dtype=F64)
    G = 1e-3 * torch.randn(3, n, generator=g, dtype=F64)
    u[lat.dim:] = 0
    G[lat.dim:] = 0
    feq = model.phase_equilibrium(phi, u, lat)
    C = model.vector_source(G, lat)
    s = 1.9704
    lit = model.mrt_collide(f, feq, C, model.moment_rates(lat, {1: s}), lat)
    J = lat.e.T @ f - phi * u + 0.5 * G
    axis = (lat.e.abs().sum(1) == 1).to(F64).reshape(-1, 1)
    closed = feq + 0.5 * C + axis * (1 - s) * 0.5 * (lat.e @ J)
    assert torch.allclose(lit, closed, atol=1e-15)
