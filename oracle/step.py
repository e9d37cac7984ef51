"""One time step of the ternary EHD lattice-Boltzmann scheme (oracle; test infrastructure only).

Order of operations within a step t -> t+1 (the paper lists the pieces of its
Methods section but not their order; this is the reading used):

  O1  moments: Phi_i = sum f_i (Eq. 19), rho_e = sum h, drho = sum dg, j = sum dg e
  O2  wetting ghosts at solid nodes next to fluid (Eq. 20, energy-based wetting)
  O3  isotropic grad Phi_i, lap Phi_i, normals n_i
  O4  chemical potentials (Eqs. 10-11) and capillary force F_s = sum_i mu_i grad Phi_i
  O5  permittivity and conductivity linear in Phi; potential from the discrete
      Gauss law (Eq. 13), solved exactly (poisson.py)
  O6  E = -grad phi (axis central differences), F_e = rho_e E - |E|^2 grad(eps)/2 (Eq. 12)
  O7  flow: u = j + F/2; raw-moment MRT (Eq. 20b first line), Guo forcing; stream
  O8  phase fields (Eqs. 15-18); stream
  O9  charge (Eq. 14 / Eq. 20b second line) with the Ohmic source; stream
  O10 keep Phi, u, rho_e, Q for the next step's time derivatives

Readings (paper silent or garbled):
  * Eq. 17 first moment is G_i = cs2 F_Phi_i + d(Phi_i u)/dt; with the printed
    form (no cs2) the Chapman-Enskog limit is not Eq. 8 (it yields
    M div(grad Phi - F_Phi/cs2)).  Relaxation: first-order raw moments at
    s = 1/tau_Phi with M = cs2 (tau_Phi - 1/2); all higher moments at 1.
  * Flow (equilibrium and forcing deferred by the paper): incompressible
    He-Luo equilibrium with rho0 = 1 stored as the deviation dg = g - w; Guo
    forcing; u = j + F/2; p = cs2 drho.  Unequal phase densities (Eq. 9 with
    rho(Phi) = sum rho_i Phi_i): the same populations in the velocity-based
    form, whose zeroth moment is p* = p / (rho cs2); the acceleration F / rho
    replaces F, with F adding -cs2 p* grad(rho) and nu (grad u + grad u^T).grad(rho).  Second-order raw moments relax at
    1/tau(x) with tau = 1/2 + nu/cs2, nu linear in Phi; higher moments at
    s_high (1 unless chosen; also for orders >= 2 of the phase fields and charge).
  * Charge: equilibrium rho_e w (1 + e.u/cs2); R = (w/cs2) e.d(rho_e u)/dt
    inside the MRT; C = w Q added after the collision with the half time
    derivative; first-order moments at 1/tau_e, alpha = cs2 (tau_e - 1/2).
    Q = sum_faces sigma_f (phi_nb - phi) with Ohmic flux 2 sigma (phi_D - phi)
    through Dirichlet faces and none through insulating ones.
  * Time derivatives are first-order backward differences of the previous
    step's stored values and vanish on the first step (t = 0).
  * Solid boundaries: halfway bounce-back for every population family.
  * Interface normal regularised as grad/sqrt(|grad|^2 + 1e-24).
  * All three phase fields are evolved (sum Phi_i = 1 is not enforced).
"""
from dataclasses import dataclass

import torch

from . import model
from .geometry import Geometry
from .lattice import Lattice
from .poisson import PotentialSystem

F64 = torch.float64


@dataclass
class State:
    g: torch.Tensor          # (Q, N) flow populations, deviation from w
    f: torch.Tensor          # (3, Q, N) phase populations
    h: torch.Tensor          # (Q, N) charge populations (zeros when the field is off)
    phi_prev: torch.Tensor   # (3, N)
    u_prev: torch.Tensor     # (3, N)
    rho_prev: torch.Tensor   # (N,)
    q_prev: torch.Tensor     # (N,)
    t: int


class Oracle:
    def __init__(self, dim, n, periodic, params, flags):
        self.lat = Lattice(dim)
        self.geom = Geometry(self.lat, n, periodic, flags)
        self.p = dict(params)
        self.ehd = bool(self.p.get("ehd", 0))
        self.N = self.geom.N
        self.fl = self.geom.fluid.to(F64)          # fluid mask as float
        self.pot = PotentialSystem(self.geom, self.lat) if self.ehd else None
        p = self.p
        self.W = float(p["width"])
        self.ups, self.upsT = model.upsilons(p["gamma12"], p["gamma13"], p["gamma23"])
        cs2 = self.lat.cs2
        self.s_phi = 1.0 / (0.5 + p["mobility"] / cs2)
        self.s_e = 1.0 / (0.5 + p["charge_diffusion"] / cs2) if self.ehd else 1.0
        # rate of every raw moment not named by the scheme (orders >= 2 of the phase fields and
        # the charge, >= 3 of the flow; Eq. 15 and Eq. 20b leave S unspecified): 1 by default
        self.s_high = float(p.get("s_high", 1.0) or 1.0)
        # density per phase (mixed linearly); unequal densities select the velocity-based
        # variable-density form of the flow (the paper's Eq. 9 with rho(Phi))
        self.rho = [float(v) or 1.0 for v in p.get("rho", (1.0, 1.0, 1.0))]
        self.var_rho = not (self.rho[0] == self.rho[1] == self.rho[2] == 1.0)
        self.nu = [cs2 * (t - 0.5) for t in p["tau_flow"]]
        self.eps = [float(v) for v in p["eps"]]
        self.cond = [float(v) for v in p["cond"]]
        self.body = torch.tensor(p["body_force"], dtype=F64).reshape(3, 1)
        # streaming source (x - e_q) and whether it is fluid, per direction
        lat, geom = self.lat, self.geom
        self.src = torch.stack([geom.nbr[lat.opp[q]] for q in range(lat.Q)])      # (Q, N)
        self.src_fluid = geom.fluid[self.src]                                       # (Q, N)

    # ------------------------------------------------------------ state
    def init_state(self, phi0, rho0=None):
        """Populations at equilibrium with u = 0 and drho = 0; rho_e = 0 (no bulk free
        charge initially, Methods assumptions) unless a test charge rho0 is given;
        previous-step fields set to the t = 0 moments."""
        phi0 = torch.as_tensor(phi0, dtype=F64) * self.fl
        lat = self.lat
        zero_u = torch.zeros(3, self.N, dtype=F64)
        f = torch.stack([model.phase_equilibrium(phi0[i], zero_u, lat) for i in range(3)]) * self.fl
        g = torch.zeros(lat.Q, self.N, dtype=F64)
        r0 = torch.zeros(self.N, dtype=F64) if rho0 is None else torch.as_tensor(rho0, dtype=F64) * self.fl
        h = model.phase_equilibrium(r0, zero_u, lat) * self.fl
        return State(g=g, f=f, h=h, phi_prev=phi0.clone(), u_prev=zero_u,
                     rho_prev=r0.clone(), q_prev=torch.zeros(self.N, dtype=F64), t=0)

    # ------------------------------------------------------------ O1
    def moments(self, s):
        lat = self.lat
        phi = s.f.sum(1)
        rho = s.h.sum(0)
        drho = s.g.sum(0)
        j = lat.e.T @ s.g
        return phi, rho, drho, j

    # ------------------------------------------------------------ O2
    def ghosts(self, phi):
        """Phi at boundary solid nodes: Phi(s) = Phi(s+e*) - |e*| (n . grad Phi_i from Eq. 20)."""
        geom, p = self.geom, self.p
        out = phi * self.fl
        if geom.ghost_nodes.numel() == 0:
            return out
        src = phi[:, geom.ghost_src]
        rhs = model.wetting_rhs(src, p["cos12"], p["cos13"], p["cos23"], self.W)
        val = src - geom.ghost_len * rhs
        return out.index_put((torch.arange(3).reshape(3, 1), geom.ghost_nodes.reshape(1, -1)), val)

    # ------------------------------------------------------------ O6 helper
    def axis_values(self, pot, volts):
        """phi at x +- e_a for every axis a < dim, with solid neighbours replaced by their
        mirror across the face: 2 phi_D - phi(x) (Dirichlet) or phi(x) (insulating, and an
        electrode whose voltage is NaN: switched off and floating)."""
        geom, lat = self.geom, self.lat
        off = torch.isnan(volts)
        vs = torch.where(off, torch.zeros_like(volts), volts)
        out = []
        for a in range(lat.dim):
            pair = []
            for q in lat.axis_dirs[a]:
                y = geom.nbr[q]
                fy = geom.flags[y]
                vy = pot[y]
                phid = torch.zeros(self.N, dtype=F64)
                k = (fy - 3).clamp(min=0)
                el = (fy >= 3) & ~off[k]
                if el.any():
                    phid = torch.where(el, vs[k], phid)
                dirich = (fy == 1) | el
                v = torch.where(fy == 0, vy, torch.where(dirich, 2.0 * phid - pot, pot))
                pair.append((v, fy, phid, dirich))
            out.append(pair)
        return out

    def ohmic_source(self, pot, sig, volts, axes):
        """Q = sum over axis faces of sigma_f (phi_nb - phi): face mean on fluid faces,
        2 sigma(x)(phi_D - phi) on Dirichlet faces, 0 on insulating faces."""
        geom, lat = self.geom, self.lat
        Q = torch.zeros(self.N, dtype=F64)
        for a in range(lat.dim):
            for k, q in enumerate(lat.axis_dirs[a]):
                y = geom.nbr[q]
                _, fy, phid, dirich = axes[a][k]
                fluid_face = 0.5 * (sig + sig[y]) * (pot[y] - pot)
                dir_face = 2.0 * sig * (phid - pot)
                Q = Q + torch.where(fy == 0, fluid_face, torch.where(dirich, dir_face, torch.zeros_like(pot)))
        return Q * self.fl

    # ------------------------------------------------------------ streaming
    def stream(self, fstar):
        """Pull from x - e_q; halfway bounce-back (f_q(x) <- f*_opp(q)(x)) when x - e_q is solid."""
        lat = self.lat
        q_idx = torch.arange(lat.Q).reshape(-1, 1)
        pulled = fstar[..., q_idx, self.src]
        bounced = fstar[..., lat.opp, :]
        out = torch.where(self.src_fluid, pulled, bounced)
        return torch.where(self.geom.fluid, out, torch.zeros_like(out))

    # ------------------------------------------------------------ one step
    def step(self, s, volts=None):
        lat, geom, p = self.lat, self.geom, self.p
        cs2 = lat.cs2
        N = self.N
        nbr = geom.nbr
        dt_on = 0.0 if s.t == 0 else 1.0
        if volts is None:
            volts = torch.tensor(p["electrode_volts"], dtype=F64)
        # O1
        phi, rho, drho, j = self.moments(s)
        # O2
        phig = self.ghosts(phi)
        # O3
        grad = model.grad_iso(phig, lat, nbr)            # (3 comps, 3 axes, N)
        lap = model.lap_iso(phig, lat, nbr)              # (3, N)
        nrm = model.normals(grad)
        # O4
        mu = model.chemical_potentials(phi, lap, self.ups, self.upsT, self.W)
        Fs = (mu.unsqueeze(1) * grad).sum(0)             # (3, N)
        F = Fs + self.body
        aux = {}
        if self.ehd:
            # O5
            epsn = sum(self.eps[i] * phi[i] for i in range(3)) * self.fl
            sig = sum(self.cond[i] * phi[i] for i in range(3)) * self.fl
            pot = self.pot.solve(epsn, rho * self.fl, volts)
            # O6
            axes = self.axis_values(pot, volts)
            E = torch.zeros(3, N, dtype=F64)
            Ecomp = []
            for a in range(3):
                if a < lat.dim:
                    Ecomp.append(-0.5 * (axes[a][0][0] - axes[a][1][0]))
                else:
                    Ecomp.append(torch.zeros(N, dtype=F64))
            E = torch.stack(Ecomp)
            grad_eps = sum(self.eps[i] * grad[i] for i in range(3))
            Fe = rho * E - 0.5 * (E * E).sum(0) * grad_eps
            F = F + Fe
            Qsrc = self.ohmic_source(pot, sig, volts, axes)
            aux.update(pot=pot, E=E, Q=Qsrc, Fe=Fe * self.fl, eps=epsn, sigma=sig)
        F = F * self.fl
        # O7 flow
        nu = sum(self.nu[i] * phi[i] for i in range(3))
        tau = 0.5 + nu / cs2
        if self.var_rho:
            # density linear in the phase fields; the flow populations carry p* = p / (rho cs2)
            # and the velocity, so the momentum equation divided by rho needs, besides F / rho,
            # the pressure force -cs2 p* grad(rho) and the viscous force nu (grad u + grad u^T)
            # . grad(rho), the latter from the non-equilibrium second moments of a provisional
            # collision with the other forces: nu S_ab = -(nu / (cs2 tau)) Pi_ab
            rho_m = sum(self.rho[i] * phi[i] for i in range(3)) * self.fl + (1.0 - self.fl)
            grad_rho = sum(self.rho[i] * grad[i] for i in range(3))
            u1 = (j + 0.5 * F / rho_m) * self.fl
            pi_neq = model.second_moments(s.g - model.flow_equilibrium(drho, u1, lat)
                                          + 0.5 * model.guo_source(u1, F / rho_m, lat), lat)
            F_mu = -(nu / (cs2 * tau)) * (pi_neq * grad_rho.unsqueeze(0)).sum(1)
            F_p = -cs2 * drho * grad_rho
            F = (F + F_p + F_mu) * self.fl
            acc = F / rho_m
        else:
            acc = F
        u = (j + 0.5 * acc) * self.fl
        geq = model.flow_equilibrium(drho, u, lat)
        Fg = model.guo_source(u, acc, lat)
        rates_g = model.moment_rates(lat, {2: 1.0 / tau}, N, default=self.s_high)
        gstar = model.mrt_collide(s.g, geq, Fg, rates_g, lat)
        g_new = self.stream(gstar)
        # O8 phase fields
        Fphi = model.phase_flux(phi, nrm, self.W)          # (3 comps, 3 axes, N)
        rates_f = model.moment_rates(lat, {1: self.s_phi}, default=self.s_high)
        f_new = []
        for i in range(3):
            dphiu = dt_on * (phi[i] * u - s.phi_prev[i] * s.u_prev)
            G = cs2 * Fphi[i] + dphiu
            C = model.vector_source(G, lat)
            feq = model.phase_equilibrium(phi[i], u, lat)
            fstar = model.mrt_collide(s.f[i], feq, C, rates_f, lat)
            f_new.append(self.stream(fstar))
        f_new = torch.stack(f_new)
        # O9 charge
        if self.ehd:
            drhou = dt_on * (rho * u - s.rho_prev * s.u_prev)
            R = model.vector_source(drhou, lat)
            heq = model.phase_equilibrium(rho, u, lat)
            rates_h = model.moment_rates(lat, {1: self.s_e}, default=self.s_high)
            hstar = model.mrt_collide(s.h, heq, R, rates_h, lat)
            hstar = hstar + lat.w.reshape(-1, 1) * (Qsrc + 0.5 * dt_on * (Qsrc - s.q_prev))
            h_new = self.stream(hstar)
            q_keep = Qsrc
        else:
            h_new = s.h
            q_keep = s.q_prev
        # O10
        new = State(g=g_new, f=f_new, h=h_new, phi_prev=phi * self.fl, u_prev=u,
                    rho_prev=rho * self.fl, q_prev=q_keep, t=s.t + 1)
        aux.update(u=u, F=F, phi=phi, rho=rho, drho=drho, mu=mu, phig=phig)
        return new, aux

    # ------------------------------------------------------------ observables (a10)
    def observables(self, s):
        """Masses, droplet centroid (node coordinates, plain Phi_1-weighted mean), droplet
        velocity from the last collided step, total charge, max |sum Phi_i - 1|."""
        phi, rho, drho, j = self.moments(s)
        fl = self.geom.fluid
        m = (phi * self.fl).sum(1)
        xc = (self.geom.xyz * phi[0] * self.fl).sum(1) / m[0]
        w1 = s.phi_prev[0] * self.fl
        mp = w1.sum()
        vc = (s.u_prev * w1).sum(1) / mp
        drift = ((phi.sum(0) - 1.0).abs() * self.fl).max()
        return dict(mass=m, centroid=xc, velocity=vc, charge=(rho * self.fl).sum(),
                    sum_phi_drift=drift, pressure_mean=(drho * self.fl).sum() / self.fl.sum() * self.lat.cs2)

    def fields(self, s):
        phi, rho, drho, j = self.moments(s)
        return dict(phi=phi * self.fl, rho_e=rho * self.fl, p=self.lat.cs2 * drho * self.fl,
                    u=s.u_prev, q=s.q_prev)

    def run(self, s, steps, volts_fn=None):
        aux = None
        for _ in range(steps):
            v = volts_fn(s.t) if volts_fn is not None else None
            s, aux = self.step(s, v)
        return s, aux
