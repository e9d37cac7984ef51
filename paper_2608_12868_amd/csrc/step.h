// Fused collide-stream kernel of the ternary EHD lattice-Boltzmann step (gfx950): the
// dominant kernel of the path.  One thread per fluid node: isotropic phase stencils,
// chemical potentials and capillary force (Eqs. 10-11), electric force and Ohmic source
// (Eqs. 12-14), flow / phase / charge collisions in raw-moment MRT closed form (Eqs. 15-18,
// 20b) and push streaming with halfway bounce-back.
#pragma once
#include "kernels.h"

namespace ehd {

// ----------------------------------------------------------------------------- fused collide-stream
// NT: population loads with the non-temporal hint (as in k_moments).  HIGH: the higher moments
// relax at p.s_high instead of 1.  With S the diagonal of rates, the raw-moment MRT
// m* = m - S(m - m_eq) + (I - S/2) M C is f* = f_eq + C/2 + M^-1 (I - S) M d with
// d = f - f_eq + C/2, whose zeroth moment vanishes (and, for the flow, its first moment too:
// j - u + F/2 = 0), so M^-1 (I - S) M d = (1 - s_high) d + (s_high - s_k) P_k d with P_k the
// projection on the moments of the one order k relaxing at its own rate s_k (first order for
// the phase fields and the charge, second order for the flow).
//
// VRHO: unequal phase densities (Eq. 9 with rho(Phi) = sum rho_i Phi_i) in the velocity-based
// form: the flow populations carry p* = p / (rho cs2) (their zeroth moment) and the velocity;
// the momentum equation divided by rho needs the acceleration F / rho with F adding the pressure
// force -cs2 p* grad(rho) and the viscous force nu (grad u + grad u^T) . grad(rho), the strain
// rate taken from the non-equilibrium second moments of a provisional collision with the other
// forces (nu S_ab = -3 nu s_nu Pi_ab).  grad(rho) = sum rho_i grad(Phi_i) reuses the stencils.
template <class L, class T, bool EHD, bool STORE, bool NT, bool HIGH, bool VRHO>
__global__ __launch_bounds__(kBlock) void k_step(StepArgs<T> a) {
  using ML = MomLayout<L>;
  constexpr int Q = L::Q;
  constexpr int D = L::D;
  if (a.gate != nullptr && *a.gate == 0) return;
  const int64_t node = D == 3 ? band_idx(a.d) : gidx();
  if (node >= a.d.N) return;
  if (a.flags[node] != 0) return;
  const int64_t N = a.d.N;
  const Phys<T>& p = a.p;
  const T cs2 = T(1) / T(3);

  int nb[Q];
  neighbours<L>(a.d, node, nb);

  // ---- a3: isotropic gradient and Laplacian of the three phase fields
  T pc[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) pc[i] = a.phi[(int64_t)i * N + node];
  T gr[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  T lap[3] = {0, 0, 0};
  uint32_t solid = 0;
  T sig_ax[2 * D];  // conductivity at the axis neighbours (+a, -a)
  uint8_t fl_ax[2 * D];
#pragma unroll
  for (int q = 1; q < Q; ++q) {
    const int m = nb[q];
    const uint8_t fm = a.flags[m];
    if (fm) solid |= 1u << q;
    const T w = T(L::w36[q]) / T(36);
    T v[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      v[i] = a.phi[(int64_t)i * N + m];
      gr[i][0] += w * T(L::ex[q]) * v[i];
      gr[i][1] += w * T(L::ey[q]) * v[i];
      if (D == 3) gr[i][2] += w * T(L::ez[q]) * v[i];
      lap[i] += w * (v[i] - pc[i]);
    }
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      if (q == L::axp[ax] || q == L::axm[ax]) {
        const int k = 2 * ax + (q == L::axp[ax] ? 0 : 1);
        sig_ax[k] = p.cond[0] * v[0] + p.cond[1] * v[1] + p.cond[2] * v[2];
        fl_ax[k] = fm;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int c = 0; c < 3; ++c) gr[i][c] *= T(3);
    lap[i] *= T(6);
  }

  // ---- a4: chemical potentials (Eq. 10) and capillary force F_s = sum mu_i grad Phi_i
  const T triple = pc[0] * pc[1] * pc[2];
  T F[3] = {p.body[0], p.body[1], p.body[2]};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const T mu = T(24) * p.ups[i] / p.W * pc[i] * (pc[i] - T(1)) * (pc[i] - T(0.5)) -
                 T(24) * p.upsT / p.W * triple - T(0.75) * p.ups[i] * p.W * lap[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) F[c] += mu * gr[i][c];
  }

  // ---- a6: electric force (Eq. 12) and Ohmic source of the charge equation
  T Qs = 0;
  if (EHD) {
    const T phx = a.pot[node];
    const T sigx = p.cond[0] * pc[0] + p.cond[1] * pc[1] + p.cond[2] * pc[2];
    T E[3] = {0, 0, 0};
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      T side[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int q = k == 0 ? L::axp[ax] : L::axm[ax];
        const uint8_t fm = fl_ax[2 * ax + k];
        if (fm == 0) {
          const T v = a.pot[nb[q]];
          side[k] = v;
          Qs += T(0.5) * (sigx + sig_ax[2 * ax + k]) * (v - phx);
        } else if (dirichlet_face(fm, a.volts)) {
          const T pd = fm == 1 ? T(0) : a.volts.v[fm - 3];
          side[k] = T(2) * pd - phx;
          Qs += T(2) * sigx * (pd - phx);
        } else {
          side[k] = phx;
        }
      }
      E[ax] = -T(0.5) * (side[0] - side[1]);
    }
    const T e2 = E[0] * E[0] + E[1] * E[1] + E[2] * E[2];
    const T rq = a.rho[node];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T ge = p.eps[0] * gr[0][c] + p.eps[1] * gr[1][c] + p.eps[2] * gr[2][c];
      F[c] += rq * E[c] - T(0.5) * e2 * ge;
    }
  }

  auto emit = [&](int fam, int q, T val) {
    if ((solid >> q) & 1u)
      a.pop_out[((int64_t)fam * Q + L::opp[q]) * N + node] = val;
    else
      a.pop_out[((int64_t)fam * Q + q) * N + nb[q]] = val;
  };

  // ---- a7: flow.  u = j + F/2, incompressible equilibrium, Guo source, raw-moment MRT
  // with second-order moments at 1/tau(x) and all higher moments at 1.
  T u[3];
  {
    T gq[Q];
    T drho = 0, j[3] = {0, 0, 0};
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      gq[q] = ld_pop<NT>(&a.pop_in[(int64_t)q * N + node]);
      drho += gq[q];
      j[0] += T(L::ex[q]) * gq[q];
      j[1] += T(L::ey[q]) * gq[q];
      j[2] += T(L::ez[q]) * gq[q];
    }
    const T nu = p.nu[0] * pc[0] + p.nu[1] * pc[1] + p.nu[2] * pc[2];
    const T s_nu = T(1) / (T(0.5) + T(3) * nu);
    if (VRHO) {
      const T irho = T(1) / (p.rho[0] * pc[0] + p.rho[1] * pc[1] + p.rho[2] * pc[2]);
      T grho[3], u1[3], a1[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        grho[c] = p.rho[0] * gr[0][c] + p.rho[1] * gr[1][c] + p.rho[2] * gr[2][c];
        a1[c] = F[c] * irho;
        u1[c] = j[c] + T(0.5) * a1[c];
      }
      const T uu1 = u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2];
      const T ua1 = u1[0] * a1[0] + u1[1] * a1[1] + u1[2] * a1[2];
      // second-order moments of g - g_eq + F_q/2 of the provisional collision (xx yy zz xy xz yz)
      T P[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const T exq = T(L::ex[q]), eyq = T(L::ey[q]), ezq = T(L::ez[q]);
        const T w = T(L::w36[q]) / T(36);
        const T eu = exq * u1[0] + eyq * u1[1] + ezq * u1[2];
        const T ea = exq * a1[0] + eyq * a1[1] + ezq * a1[2];
        const T dq = gq[q] - w * (drho + T(3) * eu + T(4.5) * eu * eu - T(1.5) * uu1) +
                     T(0.5) * w * (T(3) * (ea - ua1) + T(9) * eu * ea);
        P[0] += exq * exq * dq;
        P[1] += eyq * eyq * dq;
        P[2] += ezq * ezq * dq;
        P[3] += exq * eyq * dq;
        P[4] += exq * ezq * dq;
        P[5] += eyq * ezq * dq;
      }
      const T cmu = -T(3) * nu * s_nu;
      const T cp = -cs2 * drho;
      F[0] += cp * grho[0] + cmu * (P[0] * grho[0] + P[3] * grho[1] + P[4] * grho[2]);
      F[1] += cp * grho[1] + cmu * (P[3] * grho[0] + P[1] * grho[1] + P[5] * grho[2]);
      F[2] += cp * grho[2] + cmu * (P[4] * grho[0] + P[5] * grho[1] + P[2] * grho[2]);
#pragma unroll
      for (int c = 0; c < 3; ++c) F[c] *= irho;  // from here on the acceleration
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c] = j[c] + T(0.5) * F[c];
    const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const T uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    // second-order raw moments of g - g_eq + F_q/2
    T Pxx = 0, Pyy = 0, Pzz = 0, Pxy = 0, Pxz = 0, Pyz = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const T exq = T(L::ex[q]), eyq = T(L::ey[q]), ezq = T(L::ez[q]);
      const T w = T(L::w36[q]) / T(36);
      const T eu = exq * u[0] + eyq * u[1] + ezq * u[2];
      const T eF = exq * F[0] + eyq * F[1] + ezq * F[2];
      const T geq = w * (drho + T(3) * eu + T(4.5) * eu * eu - T(1.5) * uu);
      const T fq = w * (T(3) * (eF - uF) + T(9) * eu * eF);
      const T dq = gq[q] - geq + T(0.5) * fq;
      Pxx += exq * exq * dq;
      Pyy += eyq * eyq * dq;
      Pxy += exq * eyq * dq;
      if (D == 3) {
        Pzz += ezq * ezq * dq;
        Pxz += exq * ezq * dq;
        Pyz += eyq * ezq * dq;
      }
    }
    const T om = (HIGH ? p.s_high : T(1)) - s_nu;
    if (STORE) {
      T* r = a.rec;
      r[(int64_t)ML::DRHO * N + node] = drho;
#pragma unroll
      for (int c = 0; c < D; ++c) r[(int64_t)(ML::J + c) * N + node] = j[c];
      // the second moments of g - g_eq + F_q/2; with unequal densities the raw second moments of g
      // instead (the adjoint rebuilds the provisional collision's from them): add back the
      // equilibrium's drho/3 delta + u u and take off half the forcing's u F + F u
      T sxx = Pxx, syy = Pyy, szz = Pzz, sxy = Pxy, sxz = Pxz, syz = Pyz;
      if (VRHO) {
        const T d3 = drho / T(3);
        sxx += d3 + u[0] * u[0] - u[0] * F[0];
        syy += d3 + u[1] * u[1] - u[1] * F[1];
        szz += d3 + u[2] * u[2] - u[2] * F[2];
        sxy += u[0] * u[1] - T(0.5) * (u[0] * F[1] + u[1] * F[0]);
        sxz += u[0] * u[2] - T(0.5) * (u[0] * F[2] + u[2] * F[0]);
        syz += u[1] * u[2] - T(0.5) * (u[1] * F[2] + u[2] * F[1]);
      }
      r[(int64_t)(ML::PI + 0) * N + node] = sxx;
      r[(int64_t)(ML::PI + 1) * N + node] = syy;
      if (D == 2) {
        r[(int64_t)(ML::PI + 2) * N + node] = sxy;
      } else {
        r[(int64_t)(ML::PI + 2) * N + node] = szz;
        r[(int64_t)(ML::PI + 3) * N + node] = sxy;
        r[(int64_t)(ML::PI + 4) * N + node] = sxz;
        r[(int64_t)(ML::PI + 5) * N + node] = syz;
      }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int ix = L::ex[q], iy = L::ey[q], iz = L::ez[q];
      const T exq = T(ix), eyq = T(iy), ezq = T(iz);
      const T w = T(L::w36[q]) / T(36);
      const T eu = exq * u[0] + eyq * u[1] + ezq * u[2];
      const T eF = exq * F[0] + eyq * F[1] + ezq * F[2];
      const T geq = w * (drho + T(3) * eu + T(4.5) * eu * eu - T(1.5) * uu);
      const T fq = w * (T(3) * (eF - uF) + T(9) * eu * eF);
      // columns of M^-1 of the monomial basis for the second-order moments:
      // xx: +1/2 on the +-x links, -1 at rest; xy: e_x e_y / 4 on the xy-plane diagonals
      T corr;
      const int l2 = ix * ix + iy * iy + iz * iz;
      if (l2 == 0) {
        corr = -(Pxx + Pyy + Pzz);
      } else if (l2 == 1) {
        corr = T(0.5) * (ix ? Pxx : (iy ? Pyy : Pzz));
      } else {
        corr = T(0.25) * (iz == 0 ? exq * eyq * Pxy : (iy == 0 ? exq * ezq * Pxz : eyq * ezq * Pyz));
      }
      if (HIGH)
        emit(0, q, p.s_high * geq + (T(1) - T(0.5) * p.s_high) * fq + (T(1) - p.s_high) * gq[q] + om * corr);
      else
        emit(0, q, geq + T(0.5) * fq + om * corr);
    }
  }

  // ---- a8: phase fields (Eqs. 15-18).  G_i = cs2 F_Phi_i + d(Phi_i u)/dt; first-order raw
  // moments at s_phi, others at 1: f* = f_eq + C/2 + (1 - s_phi)/2 e.J on the axis links
  // (HIGH: f* = s_high f_eq + (1 - s_high/2) C + (1 - s_high) f + (s_high - s_phi)/2 e.J).
  {
    T nrm[3][3], amag[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T m2 = gr[i][0] * gr[i][0] + gr[i][1] * gr[i][1] + gr[i][2] * gr[i][2];
      const T inv = T(1) / sqrt(m2 + T(1e-24));
#pragma unroll
      for (int c = 0; c < 3; ++c) nrm[i][c] = gr[i][c] * inv;
      amag[i] = T(4) / p.W * fabs(pc[i] * (T(1) - pc[i]));
    }
    T tot[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) tot[c] = amag[0] * nrm[0][c] + amag[1] * nrm[1][c] + amag[2] * nrm[2][c];
    T den = pc[0] * pc[0] + pc[1] * pc[1] + pc[2] * pc[2];
    if (!(den > T(0))) den = T(1);
    const T om = (HIGH ? p.s_high : T(1)) - p.s_phi;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T share = pc[i] * pc[i] / den;
      const T php = a.phi_prev[(int64_t)i * N + node];
      T G[3], J[3];
      T jf[3] = {0, 0, 0};
      T fq[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        fq[q] = ld_pop<NT>(&a.pop_in[((int64_t)(1 + i) * Q + q) * N + node]);
        jf[0] += T(L::ex[q]) * fq[q];
        jf[1] += T(L::ey[q]) * fq[q];
        jf[2] += T(L::ez[q]) * fq[q];
      }
      if (STORE) {
#pragma unroll
        for (int c = 0; c < D; ++c) a.rec[(int64_t)(ML::JF + D * i + c) * N + node] = jf[c];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T up = c < D ? a.u_prev[(int64_t)c * N + node] : T(0);
        const T Fphi = amag[i] * nrm[i][c] - share * tot[c];
        G[c] = cs2 * Fphi + a.dt_on * (pc[i] * u[c] - php * up);
        J[c] = jf[c] - pc[i] * u[c] + T(0.5) * G[c];
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int ix = L::ex[q], iy = L::ey[q], iz = L::ez[q];
        const T w = T(L::w36[q]) / T(36);
        const T eu = T(ix) * u[0] + T(iy) * u[1] + T(iz) * u[2];
        const T eG = T(ix) * G[0] + T(iy) * G[1] + T(iz) * G[2];
        T val;
        if (HIGH)
          val = p.s_high * w * pc[i] * (T(1) + T(3) * eu) + (T(3) - T(1.5) * p.s_high) * w * eG +
                (T(1) - p.s_high) * fq[q];
        else
          val = w * pc[i] * (T(1) + T(3) * eu) + T(1.5) * w * eG;
        if (ix * ix + iy * iy + iz * iz == 1) val += T(0.5) * om * (T(ix) * J[0] + T(iy) * J[1] + T(iz) * J[2]);
        emit(1 + i, q, val);
      }
    }
  }

  // ---- a9: charge (Eq. 14): equilibrium rho_e w (1 + e.u/cs2), R = (w/cs2) e.d(rho_e u)/dt
  // inside the MRT, Ohmic source w (Q + dQ/dt / 2) after the collision.
  if (EHD) {
    const T rq = a.rho[node];
    const T rp = a.rho_prev[node];
    T dru[3], J[3], jh[3] = {0, 0, 0};
    T hq[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      hq[q] = ld_pop<NT>(&a.pop_in[((int64_t)4 * Q + q) * N + node]);
      jh[0] += T(L::ex[q]) * hq[q];
      jh[1] += T(L::ey[q]) * hq[q];
      jh[2] += T(L::ez[q]) * hq[q];
    }
    if (STORE) {
#pragma unroll
      for (int c = 0; c < D; ++c) a.rec[(int64_t)(ML::JH + c) * N + node] = jh[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T up = c < D ? a.u_prev[(int64_t)c * N + node] : T(0);
      dru[c] = a.dt_on * (rq * u[c] - rp * up);
      J[c] = jh[c] - rq * u[c] + T(0.5) * dru[c];
    }
    const T src = Qs + T(0.5) * a.dt_on * (Qs - a.q_prev[node]);
    const T om = (HIGH ? p.s_high : T(1)) - p.s_e;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int ix = L::ex[q], iy = L::ey[q], iz = L::ez[q];
      const T w = T(L::w36[q]) / T(36);
      const T eu = T(ix) * u[0] + T(iy) * u[1] + T(iz) * u[2];
      const T eR = T(ix) * dru[0] + T(iy) * dru[1] + T(iz) * dru[2];
      T val;
      if (HIGH)
        val = p.s_high * w * rq * (T(1) + T(3) * eu) + (T(3) - T(1.5) * p.s_high) * w * eR +
              (T(1) - p.s_high) * hq[q] + w * src;
      else
        val = w * rq * (T(1) + T(3) * eu) + T(1.5) * w * eR + w * src;
      if (ix * ix + iy * iy + iz * iz == 1) val += T(0.5) * om * (T(ix) * J[0] + T(iy) * J[1] + T(iz) * J[2]);
      emit(4, q, val);
    }
    a.q_out[node] = Qs;
  }
#pragma unroll
  for (int c = 0; c < D; ++c) a.u_out[(int64_t)c * N + node] = u[c];
}

}  // namespace ehd
