"""Electric potential: the discrete Gauss law solved exactly (oracle; test infrastructure only).

The paper (Eq. 21) reaches the steady state of a D3Q7 single-relaxation LB
inner iteration every time step; its equilibrium and source are deferred to
other papers.  Reading taken here: the fixed point is the conservative
finite-volume form of Eq. 13 on the axis faces of every fluid node,

    sum_faces c_f (phi_nb - phi_x) = -rho_e(x),
    c_f = (eps_x + eps_nb)/2              fluid neighbour,
    c_f = 2 eps_x, phi_nb -> phi_D       grounded (phi_D = 0) or electrode (phi_D = V_k)
                                         solid neighbour: Dirichlet on the half-cell face,
    no flux                              insulating solid neighbour, or an electrode whose
                                         voltage is NaN (switched off and left floating),

with the boundary conditions stated with Fig. 1 (pillars and substrate at zero
potential, electrode at its potential, Neumann on the other walls).  The oracle
solves A phi = b exactly up to rounding: by a sparse LU factorisation in 2D,
and in 3D (where LU fill-in is prohibitive) by Jacobi-preconditioned conjugate
gradients run until the residual is at rounding level.  The autograd backward
solves with the same (symmetric) matrix.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch

from .geometry import FLUID, GROUND, NEUMANN, ELECTRODE0


class PotentialSystem:
    def __init__(self, geom, lat):
        self.geom = geom
        fl = geom.fluid_np
        self.fidx = np.nonzero(fl)[0]
        self.nf = self.fidx.size
        uid = -np.ones(geom.N, dtype=np.int64)
        uid[self.fidx] = np.arange(self.nf)
        self.uid = uid
        ff_i, ff_j = [], []
        dir_i, dir_k = [], []          # Dirichlet faces: fluid unknown, electrode index (-1 = ground)
        for a in range(lat.dim):
            qp, qm = lat.axis_dirs[a]
            for q in (qp, qm):
                y = geom.nbr_np[q, self.fidx]
                fy = geom.flags_np[y]
                # fluid-fluid faces counted once, from the + side
                if q == qp:
                    m = fy == FLUID
                    ff_i.append(uid[self.fidx[m]])
                    ff_j.append(uid[y[m]])
                m = fy == GROUND
                dir_i.append(uid[self.fidx[m]])
                dir_k.append(np.full(m.sum(), -1, dtype=np.int64))
                m = fy >= ELECTRODE0
                dir_i.append(uid[self.fidx[m]])
                dir_k.append(fy[m].astype(np.int64) - ELECTRODE0)
        self.ff_i = np.concatenate(ff_i) if ff_i else np.zeros(0, np.int64)
        self.ff_j = np.concatenate(ff_j) if ff_j else np.zeros(0, np.int64)
        self.dir_i = np.concatenate(dir_i)
        self.dir_k = np.concatenate(dir_k)

    def assemble(self, eps_f, rho_f, volts):
        """Matrix and right-hand side over the fluid unknowns (numpy float64).  An electrode
        whose voltage is NaN is floating: its faces carry no flux (insulating)."""
        nf = self.nf
        volts = np.asarray(volts, dtype=np.float64)
        el = self.dir_k >= 0
        floating = np.zeros(self.dir_k.size, dtype=bool)
        if el.any():
            floating[el] = np.isnan(volts[self.dir_k[el]])
        c = 0.5 * (eps_f[self.ff_i] + eps_f[self.ff_j])
        cd = np.where(floating, 0.0, 2.0 * eps_f[self.dir_i])
        diag = np.zeros(nf)
        np.add.at(diag, self.ff_i, c)
        np.add.at(diag, self.ff_j, c)
        np.add.at(diag, self.dir_i, cd)
        rows = np.concatenate([np.arange(nf), self.ff_i, self.ff_j])
        cols = np.concatenate([np.arange(nf), self.ff_j, self.ff_i])
        vals = np.concatenate([diag, -c, -c])
        A = sp.csc_matrix((vals, (rows, cols)), shape=(nf, nf))
        phid = np.where(el & ~floating, volts[np.maximum(self.dir_k, 0)], 0.0)
        b = rho_f.copy()
        np.add.at(b, self.dir_i, cd * phid)
        return A, b, c, cd, phid

    def solve(self, eps, rho, volts):
        """phi (N,) as a differentiable function of eps (N,), rho_e (N,), volts (E,)."""
        return _Solve.apply(eps, rho, volts, self)

    def residual(self, phi, eps, rho, volts):
        """max|b - A phi| and max|b| (float64), for checking a solution."""
        A, b, *_ = self.assemble(eps.detach().numpy()[self.fidx], rho.detach().numpy()[self.fidx],
                                 volts.detach().numpy())
        r = b - A @ phi.detach().numpy()[self.fidx]
        return float(np.abs(r).max()), float(np.abs(b).max())


CG_RTOL = 1e-15
# Progress lines from the 3D conjugate-gradient solve every so many iterations (0: none), for the
# long oracle runs that write stored references of the large lattices; no effect on the result.
PROGRESS_EVERY = 0


class _Factor:
    """A^-1 applied exactly (2D: sparse LU) or to rounding level (3D: Jacobi-PCG)."""

    def __init__(self, A, dim):
        self.A = A
        self.dim = dim
        if dim == 2:
            self.lu = spla.splu(A, permc_spec="MMD_AT_PLUS_A", options=dict(SymmetricMode=True))
        else:
            d = A.diagonal()
            self.Minv = spla.LinearOperator(A.shape, matvec=lambda v: v / d, dtype=np.float64)

    def solve(self, b):
        if self.dim == 2:
            return self.lu.solve(b)
        nb = np.linalg.norm(b)
        if nb == 0.0:
            return np.zeros_like(b)
        count = [0]

        def progress(_x):
            count[0] += 1
            if count[0] % PROGRESS_EVERY == 0:
                print(f"  oracle CG iteration {count[0]}", flush=True)

        x, info = spla.cg(self.A, b, rtol=CG_RTOL, atol=0.0, maxiter=50 * b.size, M=self.Minv,
                          callback=progress if PROGRESS_EVERY > 0 else None)
        if info != 0:
            raise RuntimeError(f"oracle CG did not converge (info={info})")
        return x


class _Solve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps, rho, volts, system):
        fidx = system.fidx
        eps_f = eps.detach().numpy()[fidx]
        rho_f = rho.detach().numpy()[fidx]
        A, b, c, cd, phid = system.assemble(eps_f, rho_f, volts.detach().numpy())
        lu = _Factor(A, system.geom.lat.dim)
        x = lu.solve(b)
        phi = torch.zeros(system.geom.N, dtype=torch.float64)
        phi[torch.from_numpy(fidx)] = torch.from_numpy(x)
        ctx.system = system
        ctx.lu = lu
        ctx.x = x
        ctx.phid = phid
        ctx.cd = cd
        ctx.active = cd != 0.0
        ctx.nvolts = volts.numel()
        return phi

    @staticmethod
    def backward(ctx, gphi):
        s = ctx.system
        fidx = s.fidx
        lam = ctx.lu.solve(gphi.detach().numpy()[fidx])        # A symmetric: A^T lam = dL/dphi
        x = ctx.x
        N = s.geom.N
        g_rho = np.zeros(N)
        g_rho[fidx] = lam                                        # dL/db = lam
        g_eps_f = np.zeros(s.nf)
        # fluid-fluid faces: dL/dc = -(lam_i - lam_j)(x_i - x_j); dc/deps = 1/2 each side
        dc = -(lam[s.ff_i] - lam[s.ff_j]) * (x[s.ff_i] - x[s.ff_j])
        np.add.at(g_eps_f, s.ff_i, 0.5 * dc)
        np.add.at(g_eps_f, s.ff_j, 0.5 * dc)
        # Dirichlet faces: A_ii += c, b_i += c phi_D -> dL/dc = lam_i (phi_D - x_i); c = 2 eps_i
        dcd = np.where(ctx.active, lam[s.dir_i] * (ctx.phid - x[s.dir_i]), 0.0)   # floating faces: none
        np.add.at(g_eps_f, s.dir_i, 2.0 * dcd)
        g_eps = np.zeros(N)
        g_eps[fidx] = g_eps_f
        return (torch.from_numpy(g_eps), torch.from_numpy(g_rho), _volt_grad(ctx, lam), None)


def _volt_grad(ctx, lam):
    """Electrode voltages enter only b: b_i += c_d V_k on electrode faces, so dL/dV_k = sum c_d lam_i."""
    s = ctx.system
    g_v = np.zeros(ctx.nvolts)
    el = s.dir_k >= 0
    if el.any():
        np.add.at(g_v, s.dir_k[el], ctx.cd[el] * lam[s.dir_i[el]])
    return torch.from_numpy(g_v)
