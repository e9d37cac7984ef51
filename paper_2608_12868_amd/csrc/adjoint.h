// Hand-written discrete adjoint of one time step (reverse mode), gfx950.
//
// State of step t: populations P_t and the previous-step fields (Phi, u, rho_e, Q of step
// t-1).  One forward step maps (P_t, prev_t, V(t)) to (P_t+1, prev_t+1); the adjoint maps the
// cotangents of the outputs back to those of the inputs and accumulates dL/dV(t).  The
// potential solve is treated as exact: its adjoint is one solve with the same symmetric
// matrix.  Everything the collision needs from the populations is carried by a few moments
// (MomLayout), which the forward recompute stores per step together with Phi (with wetting
// ghosts), rho_e, the potential and the previous step's Phi, u and rho_e (the previous step's
// Ohmic source enters the charge source linearly, so its value is not needed).
//
// Passes per step (all gathers, no atomics, fixed summation order):
//   A   per fluid node: recompute the forward quantities, gather the streamed population
//       cotangents (transpose of push streaming = pull), reverse the collision, the forces
//       and the electric terms; write stencil cotangents (grad, lap, neighbour sigma and phi)
//       and local ones
//   B   per node: apply the transposed stencils as gathers -> lambda_Phi, lambda_phi
//   G   per fluid node that is a wetting-link source: fold in the ghosts' cotangents
//   S   solve A lambda_b = lambda_phi
//   CD  per fluid node: permittivity/charge cotangents from lambda_b, then the population
//       cotangents of step t
#pragma once
#include "kernels.h"
#include "step.h"

namespace ehd {

// per-step record of the recompute: [RecLayout::COUNT][N]
template <class L>
struct RecLayout {
  static constexpr int D = L::D;
  static constexpr int PHI = 0, RHO = 3, POT = 4, PHIP = 5, UP = 8, RHOP = 8 + D, MOM = 9 + D;
  static constexpr int COUNT = MOM + MomLayout<L>::COUNT;
};

template <class T>
struct AdjArgs {
  Dims d;
  const uint8_t* flags;
  const T* rec;        // record of step t
  const T* lP_next;    // population cotangents of step t+1 [F][Q][N]
  const T* lphip_next; // cotangents of the previous-step fields of step t+1
  const T* lup_next;
  const T* lrhop_next;
  const T* lqp_next;
  T* lphip;            // ... of step t (written by pass A)
  T* lup;
  T* lrhop;
  T* lqp;
  T* lgr;              // [3][D][N]
  T* llap;             // [3][N]
  T* lsig;             // [2D][N] cotangent of sigma at the axis neighbours
  T* lpnb;             // [2D][N] cotangent of phi at the axis neighbours
  T* lphi_loc;         // [3][N]
  T* lpot_loc;         // [N]
  T* lrho_loc;         // [N]
  T* lmom;             // [MomLayout::COUNT][N]
  double* vpart;       // per-block partials of dL/dV_k [nblocks][kMaxE], accumulated over a segment's steps
  Phys<T> p;
  Volts<T> volts;
  T dt_on;
};

// ----------------------------------------------------------------------------- pass A
// HIGH: the higher moments relax at p.s_high (see k_step): every equilibrium and source term
// of the collision is scaled accordingly, and the population cotangents of step t receive
// (1 - s_high) times the streamed cotangents directly (pass CD).
// VRHO: unequal phase densities (see k_step): the force becomes the acceleration
// F' = (F + cp grad rho + cmu P grad rho) / rho with the provisional collision's second moments
// P = S - (drho/3 delta + u1 u1) + (u1 a1 + a1 u1)/2 (S the raw second moments of g, which the
// record holds in this case; a1 = F / rho, u1 = j + a1/2), cp = -cs2 drho, cmu = -3 nu s_nu;
// its reverse maps the cotangent of F' to that of F and adds the cotangents of S, drho, j, the
// phase fields at the node and their gradients.
template <class L, class T, bool EHD, bool HIGH, bool VRHO>
__device__ __forceinline__ void adj_a_body(const AdjArgs<T>& a) {
  using ML = MomLayout<L>;
  using RL = RecLayout<L>;
  constexpr int Q = L::Q;
  constexpr int D = L::D;
  constexpr int P = ML::P;
  const int64_t node = D == 3 ? band_idx(a.d) : gidx();
  double vloc[kMaxE] = {0.0, 0.0, 0.0, 0.0};
  const int64_t N = a.d.N;
  const bool active = node < N && a.flags[node] == 0;
  if (active) {
    const Phys<T>& p = a.p;
    const T cs2 = T(1) / T(3);
    const T dt = a.dt_on;
    const T* rec = a.rec;
    auto R = [&](int f, int64_t i) -> T { return rec[(int64_t)f * N + i]; };
    // neighbour indices on demand (keeping all Q of them live costs occupancy)
    const int nx_ = (int)node % a.d.nx, ny_ = ((int)node / a.d.nx) % a.d.ny, nz_ = ((int)node / a.d.nx) / a.d.ny;
    auto NB = [&](int q) -> int { return neighbour<L>(a.d, nx_, ny_, nz_, q); };
    uint32_t solid = 0;

    // ---------------------------------------------------------- forward recompute
    T pc[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) pc[i] = R(RL::PHI + i, node);
    T gr[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    T lap[3] = {0, 0, 0};
#pragma unroll
    for (int q = 1; q < Q; ++q) {
      const int m = NB(q);
      const uint8_t fm = a.flags[m];
      if (fm) solid |= 1u << q;
      const T w = T(L::w36[q]) / T(36);
      T v[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        v[i] = R(RL::PHI + i, m);
        gr[i][0] += w * T(L::ex[q]) * v[i];
        gr[i][1] += w * T(L::ey[q]) * v[i];
        if (D == 3) gr[i][2] += w * T(L::ez[q]) * v[i];
        lap[i] += w * (v[i] - pc[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int c = 0; c < 3; ++c) gr[i][c] *= T(3);
      lap[i] *= T(6);
    }
    const T triple = pc[0] * pc[1] * pc[2];
    T mu[3];
    T F[3] = {p.body[0], p.body[1], p.body[2]};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      mu[i] = T(24) * p.ups[i] / p.W * pc[i] * (pc[i] - T(1)) * (pc[i] - T(0.5)) -
              T(24) * p.upsT / p.W * triple - T(0.75) * p.ups[i] * p.W * lap[i];
#pragma unroll
      for (int c = 0; c < 3; ++c) F[c] += mu[i] * gr[i][c];
    }
    // face kk = 2 ax + k (k = 0: +axis, 1: -axis): neighbour flag, conductivity, potential and
    // Dirichlet value, recomputed wherever needed instead of being kept live
    struct Face {
      uint8_t fm;
      T sig, pn, pd;
    };
    auto face = [&](int kk) -> Face {
      const int ax = kk >> 1;
      const int q = (kk & 1) == 0 ? L::axp[ax] : L::axm[ax];
      const int m = NB(q);
      Face f;
      f.fm = a.flags[m];
      f.sig = p.cond[0] * R(RL::PHI, m) + p.cond[1] * R(RL::PHI + 1, m) + p.cond[2] * R(RL::PHI + 2, m);
      f.pn = f.fm == 0 ? R(RL::POT, m) : T(0);
      f.pd = dirichlet_face(f.fm, a.volts) ? (f.fm == 1 ? T(0) : a.volts.v[f.fm - 3]) : T(0);
      return f;
    };
    T E[3] = {0, 0, 0}, ge[3] = {0, 0, 0};
    T phx = 0, sigx = 0, rq = 0, Qs = 0, e2 = 0;
    if (EHD) {
      phx = R(RL::POT, node);
      sigx = p.cond[0] * pc[0] + p.cond[1] * pc[1] + p.cond[2] * pc[2];
      rq = R(RL::RHO, node);
#pragma unroll
      for (int ax = 0; ax < D; ++ax) {
        T side[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const Face f = face(2 * ax + k);
          if (f.fm == 0) {
            side[k] = f.pn;
            Qs += T(0.5) * (sigx + f.sig) * (f.pn - phx);
          } else if (dirichlet_face(f.fm, a.volts)) {
            side[k] = T(2) * f.pd - phx;
            Qs += T(2) * sigx * (f.pd - phx);
          } else {
            side[k] = phx;
          }
        }
        E[ax] = -T(0.5) * (side[0] - side[1]);
      }
      e2 = E[0] * E[0] + E[1] * E[1] + E[2] * E[2];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        ge[c] = p.eps[0] * gr[0][c] + p.eps[1] * gr[1][c] + p.eps[2] * gr[2][c];
        F[c] += rq * E[c] - T(0.5) * e2 * ge[c];
      }
    }
    const T drho = R(RL::MOM + ML::DRHO, node);
    T j[3] = {0, 0, 0}, u[3], up[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < D; ++c) {
      j[c] = R(RL::MOM + ML::J + c, node);
      up[c] = R(RL::UP + c, node);
    }
    const T nu = p.nu[0] * pc[0] + p.nu[1] * pc[1] + p.nu[2] * pc[2];
    const T s_nu = T(1) / (T(0.5) + T(3) * nu);
    T Pi[P];
#pragma unroll
    for (int k = 0; k < P; ++k) Pi[k] = R(RL::MOM + ML::PI + k, node);
    // unequal densities: symmetric tensors as (xx yy zz xy xz yz); vs = the raw second moments
    // (record), vp = the provisional collision's, vG = F + cp grad rho + cmu vp grad rho
    T Fpre[3] = {F[0], F[1], F[2]}, vs[6] = {0, 0, 0, 0, 0, 0}, vp[6] = {0, 0, 0, 0, 0, 0};
    T vG[3] = {0, 0, 0}, grho[3] = {0, 0, 0}, a1[3] = {0, 0, 0}, u1[3] = {0, 0, 0};
    T irho = T(1), cp_ = T(0), cmu = T(0);
    if (VRHO) {
      if (D == 2) {
        vs[0] = Pi[0];
        vs[1] = Pi[1];
        vs[3] = Pi[2];
      } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) vs[k] = Pi[k < P ? k : 0];
      }
      irho = T(1) / (p.rho[0] * pc[0] + p.rho[1] * pc[1] + p.rho[2] * pc[2]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        grho[c] = p.rho[0] * gr[0][c] + p.rho[1] * gr[1][c] + p.rho[2] * gr[2][c];
        a1[c] = Fpre[c] * irho;
        u1[c] = j[c] + T(0.5) * a1[c];
      }
      const T d3 = drho / T(3);
      vp[0] = vs[0] - d3 - u1[0] * u1[0] + u1[0] * a1[0];
      vp[1] = vs[1] - d3 - u1[1] * u1[1] + u1[1] * a1[1];
      vp[3] = vs[3] - u1[0] * u1[1] + T(0.5) * (u1[0] * a1[1] + u1[1] * a1[0]);
      if (D == 3) {
        vp[2] = vs[2] - d3 - u1[2] * u1[2] + u1[2] * a1[2];
        vp[4] = vs[4] - u1[0] * u1[2] + T(0.5) * (u1[0] * a1[2] + u1[2] * a1[0]);
        vp[5] = vs[5] - u1[1] * u1[2] + T(0.5) * (u1[1] * a1[2] + u1[2] * a1[1]);
      }
      cmu = -T(3) * nu * s_nu;
      cp_ = -cs2 * drho;
      vG[0] = Fpre[0] + cp_ * grho[0] + cmu * (vp[0] * grho[0] + vp[3] * grho[1] + vp[4] * grho[2]);
      vG[1] = Fpre[1] + cp_ * grho[1] + cmu * (vp[3] * grho[0] + vp[1] * grho[1] + vp[5] * grho[2]);
      vG[2] = Fpre[2] + cp_ * grho[2] + cmu * (vp[4] * grho[0] + vp[5] * grho[1] + vp[2] * grho[2]);
#pragma unroll
      for (int c = 0; c < 3; ++c) F[c] = vG[c] * irho;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c] = j[c] + T(0.5) * F[c];
    const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const T uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    if (VRHO) {
      // the non-equilibrium second moments of the collision, with the final u and F
      const T d3 = drho / T(3);
      const T pn[6] = {vs[0] - d3 - u[0] * u[0] + u[0] * F[0], vs[1] - d3 - u[1] * u[1] + u[1] * F[1],
                       vs[2] - d3 - u[2] * u[2] + u[2] * F[2],
                       vs[3] - u[0] * u[1] + T(0.5) * (u[0] * F[1] + u[1] * F[0]),
                       vs[4] - u[0] * u[2] + T(0.5) * (u[0] * F[2] + u[2] * F[0]),
                       vs[5] - u[1] * u[2] + T(0.5) * (u[1] * F[2] + u[2] * F[1])};
      if (D == 2) {
        Pi[0] = pn[0];
        Pi[1] = pn[1];
        Pi[P - 1] = pn[3];
      } else {
#pragma unroll
        for (int k = 0; k < P; ++k) Pi[k] = pn[k];
      }
    }

    // ---------------------------------------------------------- cotangents of the outputs
    // streamed populations: the value pushed from node along q landed on node + e_q (or on
    // node's opposite slot when bounced back)
    auto lout = [&](int fam, int q) -> T {
      if ((solid >> q) & 1u) return a.lP_next[((int64_t)fam * Q + L::opp[q]) * N + node];
      return a.lP_next[((int64_t)fam * Q + q) * N + NB(q)];
    };
    T lu[3] = {0, 0, 0}, lF[3] = {0, 0, 0}, lphi[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < D; ++c) lu[c] = a.lup_next[(int64_t)c * N + node];
    T lQs = EHD ? a.lqp_next[node] : T(0);
    T lrho = EHD ? a.lrhop_next[node] : T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) lphi[i] = a.lphip_next[(int64_t)i * N + node];
    T lgr[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    T lphip[3] = {0, 0, 0}, lup[3] = {0, 0, 0}, lrhop = 0, lqp = 0;
    T* lm = a.lmom;

    // ---------------------------------------------------------- charge (reverse)
    if (EHD) {
      const T rp = R(RL::RHOP, node);
      T dru[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) dru[c] = dt * (rq * u[c] - rp * up[c]);
      T lsrc = 0, ldru[3] = {0, 0, 0}, lJe[3] = {0, 0, 0};
      const T sh = HIGH ? p.s_high : T(1);
      const T om = sh - p.s_e;
      const T cR = T(3) - T(1.5) * sh;  // (1 - s_high/2) times the 3 w e of the source
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int ix = L::ex[q], iy = L::ey[q], iz = L::ez[q];
        const T w = T(L::w36[q]) / T(36);
        const T lo = lout(4, q);
        const T los = HIGH ? sh * lo : lo;
        const T eu = T(ix) * u[0] + T(iy) * u[1] + T(iz) * u[2];
        lsrc += lo * w;
        lrho += los * w * (T(1) + T(3) * eu);
        lu[0] += los * w * rq * T(3) * T(ix);
        lu[1] += los * w * rq * T(3) * T(iy);
        lu[2] += los * w * rq * T(3) * T(iz);
        ldru[0] += lo * cR * w * T(ix);
        ldru[1] += lo * cR * w * T(iy);
        ldru[2] += lo * cR * w * T(iz);
        if (ix * ix + iy * iy + iz * iz == 1) {
          lJe[0] += lo * T(0.5) * om * T(ix);
          lJe[1] += lo * T(0.5) * om * T(iy);
          lJe[2] += lo * T(0.5) * om * T(iz);
        }
      }
      // Je = jh - rho u + dru/2
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        ldru[c] += T(0.5) * lJe[c];
        lrho -= lJe[c] * u[c];
        lu[c] -= rq * lJe[c];
      }
#pragma unroll
      for (int c = 0; c < D; ++c) lm[(int64_t)(ML::JH + c) * N + node] = lJe[c];
      // dru = dt (rho u - rho_p u_p)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        lrho += dt * ldru[c] * u[c];
        lu[c] += dt * rq * ldru[c];
        lrhop -= dt * ldru[c] * up[c];
        lup[c] -= dt * rp * ldru[c];
      }
      // src = Qs + dt (Qs - Qp)/2
      lQs += lsrc * (T(1) + T(0.5) * dt);
      lqp -= T(0.5) * dt * lsrc;
    }

    // ---------------------------------------------------------- phase fields (reverse)
    {
      T nrm[3][3], amag[3], msz[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const T m2 = gr[i][0] * gr[i][0] + gr[i][1] * gr[i][1] + gr[i][2] * gr[i][2];
        msz[i] = sqrt(m2 + T(1e-24));
#pragma unroll
        for (int c = 0; c < 3; ++c) nrm[i][c] = gr[i][c] / msz[i];
        amag[i] = T(4) / p.W * fabs(pc[i] * (T(1) - pc[i]));
      }
      T tot[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) tot[c] = amag[0] * nrm[0][c] + amag[1] * nrm[1][c] + amag[2] * nrm[2][c];
      T den = pc[0] * pc[0] + pc[1] * pc[1] + pc[2] * pc[2];
      if (!(den > T(0))) den = T(1);
      const T sh = HIGH ? p.s_high : T(1);
      const T om = sh - p.s_phi;
      const T cC = T(3) - T(1.5) * sh;  // (1 - s_high/2) times the 3 w e of the source
      T lFphi[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const T php = R(RL::PHIP + i, node);
        T lG[3] = {0, 0, 0}, lJ[3] = {0, 0, 0};
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int ix = L::ex[q], iy = L::ey[q], iz = L::ez[q];
          const T w = T(L::w36[q]) / T(36);
          const T lo = lout(1 + i, q);
          const T los = HIGH ? sh * lo : lo;
          const T eu = T(ix) * u[0] + T(iy) * u[1] + T(iz) * u[2];
          lphi[i] += los * w * (T(1) + T(3) * eu);
          lu[0] += los * w * pc[i] * T(3) * T(ix);
          lu[1] += los * w * pc[i] * T(3) * T(iy);
          lu[2] += los * w * pc[i] * T(3) * T(iz);
          lG[0] += lo * cC * w * T(ix);
          lG[1] += lo * cC * w * T(iy);
          lG[2] += lo * cC * w * T(iz);
          if (ix * ix + iy * iy + iz * iz == 1) {
            lJ[0] += lo * T(0.5) * om * T(ix);
            lJ[1] += lo * T(0.5) * om * T(iy);
            lJ[2] += lo * T(0.5) * om * T(iz);
          }
        }
        // J = jf - Phi u + G/2
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          lG[c] += T(0.5) * lJ[c];
          lphi[i] -= lJ[c] * u[c];
          lu[c] -= pc[i] * lJ[c];
        }
#pragma unroll
        for (int c = 0; c < D; ++c) lm[(int64_t)(ML::JF + D * i + c) * N + node] = lJ[c];
        // G = cs2 F_Phi + dt (Phi u - Phi_p u_p)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          lFphi[i][c] = cs2 * lG[c];
          lphi[i] += dt * lG[c] * u[c];
          lu[c] += dt * pc[i] * lG[c];
          lphip[i] -= dt * lG[c] * up[c];
          lup[c] -= dt * php * lG[c];
        }
      }
      // F_Phi_i = a_i n_i - share_i tot,  tot = sum_j a_j n_j,  share_i = Phi_i^2 / den
      T ltot[3];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        ltot[c] = -(pc[0] * pc[0] * lFphi[0][c] + pc[1] * pc[1] * lFphi[1][c] + pc[2] * pc[2] * lFphi[2][c]) / den;
      T lden = 0;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const T lshare = -(lFphi[i][0] * tot[0] + lFphi[i][1] * tot[1] + lFphi[i][2] * tot[2]);
        lphi[i] += lshare * T(2) * pc[i] / den;
        lden -= lshare * pc[i] * pc[i] / (den * den);
        T ln[3], la = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T g = lFphi[i][c] + ltot[c];
          ln[c] = amag[i] * g;
          la += nrm[i][c] * g;
        }
        const T s = pc[i] * (T(1) - pc[i]);
        const T sg = s > T(0) ? T(1) : (s < T(0) ? T(-1) : T(0));
        lphi[i] += la * T(4) / p.W * sg * (T(1) - T(2) * pc[i]);
        const T nl = nrm[i][0] * ln[0] + nrm[i][1] * ln[1] + nrm[i][2] * ln[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) lgr[i][c] += (ln[c] - nrm[i][c] * nl) / msz[i];
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) lphi[i] += T(2) * pc[i] * lden;
    }

    // ---------------------------------------------------------- flow (reverse)
    {
      T C[6] = {0, 0, 0, 0, 0, 0};  // C_k = sum_q lambda_g*_q P_k[q]  (xx yy zz xy xz yz)
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int ix = L::ex[q], iy = L::ey[q], iz = L::ez[q];
        const T lo = lout(0, q);
        const int l2 = ix * ix + iy * iy + iz * iz;
        if (l2 == 0) {
          C[0] -= lo;
          C[1] -= lo;
          C[2] -= lo;
        } else if (l2 == 1) {
          if (ix) C[0] += T(0.5) * lo;
          if (iy) C[1] += T(0.5) * lo;
          if (iz) C[2] += T(0.5) * lo;
        } else {
          if (iz == 0) C[3] += T(0.25) * T(ix * iy) * lo;
          else if (iy == 0) C[4] += T(0.25) * T(ix * iz) * lo;
          else C[5] += T(0.25) * T(iy * iz) * lo;
        }
      }
      // Pi layout: 2D (xx, yy, xy); 3D (xx, yy, zz, xy, xz, yz)
      T Ck[6], Pk[6];
      if (D == 2) {
        Ck[0] = C[0]; Ck[1] = C[1]; Ck[2] = C[3];
        Pk[0] = Pi[0]; Pk[1] = Pi[1]; Pk[2] = Pi[P - 1];
      } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          Ck[k] = C[k];
          Pk[k] = Pi[k < P ? k : 0];
        }
      }
      const T sh = HIGH ? p.s_high : T(1);
      const T omn = sh - s_nu;
      T ls = 0;
#pragma unroll
      for (int k = 0; k < P; ++k) {
        lm[(int64_t)(ML::PI + k) * N + node] = omn * Ck[k];
        ls -= Pk[k] * Ck[k];
      }
      // lambda_d_q = sum_k m_k(e_q) lambda_Pi_k
      T ldrho = 0;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int ix = L::ex[q], iy = L::ey[q], iz = L::ez[q];
        const T exq = T(ix), eyq = T(iy), ezq = T(iz);
        T ld;
        if (D == 2) {
          ld = omn * (exq * exq * Ck[0] + eyq * eyq * Ck[1] + exq * eyq * Ck[2]);
        } else {
          ld = omn * (exq * exq * Ck[0] + eyq * eyq * Ck[1] + ezq * ezq * Ck[2] + exq * eyq * Ck[3] +
                      exq * ezq * Ck[4] + eyq * ezq * Ck[5]);
        }
        const T w = T(L::w36[q]) / T(36);
        const T lq = lout(0, q);  // re-read (cache hit) rather than kept live
        const T lgeq = (HIGH ? sh * lq : lq) - ld;
        const T lFq = (HIGH ? (T(1) - T(0.5) * sh) * lq : T(0.5) * lq) + T(0.5) * ld;
        const T eu = exq * u[0] + eyq * u[1] + ezq * u[2];
        const T eF = exq * F[0] + eyq * F[1] + ezq * F[2];
        ldrho += lgeq * w;
        const T e3[3] = {exq, eyq, ezq};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          lu[c] += lgeq * w * (T(3) * e3[c] + T(9) * eu * e3[c] - T(3) * u[c]);
          lF[c] += lFq * w * (T(3) * (e3[c] - u[c]) + T(9) * eu * e3[c]);
          lu[c] += lFq * w * (-T(3) * F[c] + T(9) * eF * e3[c]);
        }
      }
      (void)uu;
      (void)uF;
      // s_nu = 1 / (1/2 + 3 nu), nu = sum nu_i Phi_i
      const T lnu = ls * (-T(3) * s_nu * s_nu);
#pragma unroll
      for (int i = 0; i < 3; ++i) lphi[i] += p.nu[i] * lnu;
      // u = j + F/2  (lu now complete)
#pragma unroll
      for (int c = 0; c < 3; ++c) lF[c] += T(0.5) * lu[c];
      if (VRHO) {
        // reverse of F' = vG / rho (lF: cotangent of F'; afterwards that of the force F)
        T lG[3], lvp[6], la1[3], lu1[3];
        T lirho = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          lG[c] = irho * lF[c];
          lirho += lF[c] * vG[c];
        }
        const T lcp = lG[0] * grho[0] + lG[1] * grho[1] + lG[2] * grho[2];
        const T pg[3] = {vp[0] * grho[0] + vp[3] * grho[1] + vp[4] * grho[2],
                         vp[3] * grho[0] + vp[1] * grho[1] + vp[5] * grho[2],
                         vp[4] * grho[0] + vp[5] * grho[1] + vp[2] * grho[2]};
        const T lcmu = lG[0] * pg[0] + lG[1] * pg[1] + lG[2] * pg[2];
        const T gl[3] = {vp[0] * lG[0] + vp[3] * lG[1] + vp[4] * lG[2],
                         vp[3] * lG[0] + vp[1] * lG[1] + vp[5] * lG[2],
                         vp[4] * lG[0] + vp[5] * lG[1] + vp[2] * lG[2]};
        T lgrho[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) lgrho[c] = cp_ * lG[c] + cmu * gl[c];
        lvp[0] = cmu * lG[0] * grho[0];
        lvp[1] = cmu * lG[1] * grho[1];
        lvp[2] = cmu * lG[2] * grho[2];
        lvp[3] = cmu * (lG[0] * grho[1] + lG[1] * grho[0]);
        lvp[4] = cmu * (lG[0] * grho[2] + lG[2] * grho[0]);
        lvp[5] = cmu * (lG[1] * grho[2] + lG[2] * grho[1]);
        // vp = vs - (drho/3 delta + u1 u1) + (u1 a1 + a1 u1)/2
        ldrho += -cs2 * lcp - (lvp[0] + lvp[1] + lvp[2]) / T(3);
        lu1[0] = lvp[0] * (-T(2) * u1[0] + a1[0]) + lvp[3] * (-u1[1] + T(0.5) * a1[1]) +
                 lvp[4] * (-u1[2] + T(0.5) * a1[2]);
        lu1[1] = lvp[1] * (-T(2) * u1[1] + a1[1]) + lvp[3] * (-u1[0] + T(0.5) * a1[0]) +
                 lvp[5] * (-u1[2] + T(0.5) * a1[2]);
        lu1[2] = lvp[2] * (-T(2) * u1[2] + a1[2]) + lvp[4] * (-u1[0] + T(0.5) * a1[0]) +
                 lvp[5] * (-u1[1] + T(0.5) * a1[1]);
        la1[0] = lvp[0] * u1[0] + T(0.5) * (lvp[3] * u1[1] + lvp[4] * u1[2]);
        la1[1] = lvp[1] * u1[1] + T(0.5) * (lvp[3] * u1[0] + lvp[5] * u1[2]);
        la1[2] = lvp[2] * u1[2] + T(0.5) * (lvp[4] * u1[0] + lvp[5] * u1[1]);
        // u1 = j + a1/2, a1 = F / rho
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          lu[c] += lu1[c];  // the cotangent of j below
          la1[c] += T(0.5) * lu1[c];
          lirho += Fpre[c] * la1[c];
          lF[c] = lG[c] + irho * la1[c];
        }
        // the raw second moments: their cotangent maps to the populations as that of Pi does
        if (D == 2) {
          lm[(int64_t)(ML::PI + 0) * N + node] += lvp[0];
          lm[(int64_t)(ML::PI + 1) * N + node] += lvp[1];
          lm[(int64_t)(ML::PI + 2) * N + node] += lvp[3];
        } else {
#pragma unroll
          for (int k = 0; k < 6; ++k) lm[(int64_t)(ML::PI + k) * N + node] += lvp[k];
        }
        // 1/rho and nu of the phase fields at the node, grad rho of their gradients
        const T lnu_v = lcmu * (-T(1.5) * s_nu * s_nu);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          lphi[i] += -p.rho[i] * irho * irho * lirho + p.nu[i] * lnu_v;
#pragma unroll
          for (int c = 0; c < 3; ++c) lgr[i][c] += p.rho[i] * lgrho[c];
        }
      }
      lm[(int64_t)ML::DRHO * N + node] = ldrho;
#pragma unroll
      for (int c = 0; c < D; ++c) lm[(int64_t)(ML::J + c) * N + node] = lu[c];
    }

    // ---------------------------------------------------------- forces (reverse)
    T llap[3];
    {
      T S = 0;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const T lmu = lF[0] * gr[i][0] + lF[1] * gr[i][1] + lF[2] * gr[i][2];
#pragma unroll
        for (int c = 0; c < 3; ++c) lgr[i][c] += mu[i] * lF[c];
        const T pp = pc[i];
        lphi[i] += lmu * T(24) * p.ups[i] / p.W * (T(3) * pp * pp - T(3) * pp + T(0.5));
        S += lmu;
        llap[i] = -T(0.75) * p.ups[i] * p.W * lmu;
      }
      const T c3 = T(24) * p.upsT / p.W;
      lphi[0] -= S * c3 * pc[1] * pc[2];
      lphi[1] -= S * c3 * pc[0] * pc[2];
      lphi[2] -= S * c3 * pc[0] * pc[1];
    }
    T lpot = 0, lsigx = 0;
    if (EHD) {
      T lE[3];
      const T lFge = lF[0] * ge[0] + lF[1] * ge[1] + lF[2] * ge[2];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        lrho += lF[c] * E[c];
        lE[c] = rq * lF[c] - lFge * E[c];
        const T lge = -T(0.5) * e2 * lF[c];
#pragma unroll
        for (int i = 0; i < 3; ++i) lgr[i][c] += p.eps[i] * lge;
      }
#pragma unroll
      for (int ax = 0; ax < D; ++ax) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int kk = 2 * ax + k;
          const T lside = (k == 0 ? -T(0.5) : T(0.5)) * lE[ax];
          const Face f = face(kk);
          const uint8_t fm = f.fm;
          T lsn = 0, lpn = 0;
          if (fm == 0) {
            const T hs = T(0.5) * (sigx + f.sig);
            const T dphi = f.pn - phx;
            lsigx += T(0.5) * dphi * lQs;
            lsn = T(0.5) * dphi * lQs;
            lpn = hs * lQs + lside;
            lpot -= hs * lQs;
          } else if (dirichlet_face(fm, a.volts)) {
            lsigx += T(2) * (f.pd - phx) * lQs;
            lpot -= T(2) * sigx * lQs + lside;
            if (fm >= 3) vloc[fm - 3] += (double)(T(2) * sigx * lQs + T(2) * lside);
          } else {
            lpot += lside;
          }
          a.lsig[(int64_t)kk * N + node] = lsn;
          a.lpnb[(int64_t)kk * N + node] = lpn;
        }
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) lphi[i] += p.cond[i] * lsigx;
    }

    // ---------------------------------------------------------- write
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int c = 0; c < D; ++c) a.lgr[(int64_t)(D * i + c) * N + node] = lgr[i][c];
      a.llap[(int64_t)i * N + node] = llap[i];
      a.lphi_loc[(int64_t)i * N + node] = lphi[i];
      a.lphip[(int64_t)i * N + node] = lphip[i];
    }
#pragma unroll
    for (int c = 0; c < D; ++c) a.lup[(int64_t)c * N + node] = lup[c];
    if (EHD) {
      a.lpot_loc[node] = lpot;
      a.lrho_loc[node] = lrho;
      a.lrhop[node] = lrhop;
      a.lqp[node] = lqp;
    }
  } else if (node < N) {
    // solid nodes: zero stencil cotangents so that pass B can gather unconditionally
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int c = 0; c < D; ++c) a.lgr[(int64_t)(D * i + c) * N + node] = T(0);
      a.llap[(int64_t)i * N + node] = T(0);
      a.lphi_loc[(int64_t)i * N + node] = T(0);
      a.lphip[(int64_t)i * N + node] = T(0);
    }
#pragma unroll
    for (int c = 0; c < D; ++c) a.lup[(int64_t)c * N + node] = T(0);
    if (EHD) {
#pragma unroll
      for (int k = 0; k < 2 * D; ++k) {
        a.lsig[(int64_t)k * N + node] = T(0);
        a.lpnb[(int64_t)k * N + node] = T(0);
      }
      a.lpot_loc[node] = T(0);
      a.lrho_loc[node] = T(0);
      a.lrhop[node] = T(0);
      a.lqp[node] = T(0);
    }
  }
  if (EHD) block_reduce<kMaxE, false>(vloc, a.vpart + (int64_t)blockIdx.x * kMaxE, 1, true);
}

template <class L, class T, bool EHD, bool HIGH, bool VRHO>
__global__ __launch_bounds__(kBlock) void k_adj_a(AdjArgs<T> a) {
  adj_a_body<L, T, EHD, HIGH, VRHO>(a);
}
// FP32: capped at 256 registers so that two waves fit per SIMD (one 8-byte spill in 3D);
// uncapped, the kernel needs just over 256 and runs one wave per SIMD.  The FP64 variants
// would spill heavily under the same cap.
template <class L, bool EHD, bool HIGH, bool VRHO>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_adj_a32(AdjArgs<float> a) {
  adj_a_body<L, float, EHD, HIGH, VRHO>(a);
}

// ----------------------------------------------------------------------------- pass B
// Transposed stencils as gathers.  lphi_out at every node (ghost solids included),
// lpot_out at fluid nodes.
template <class L, class T, bool EHD>
__global__ __launch_bounds__(kBlock) void k_adj_b(Dims d, const uint8_t* __restrict__ flags, Phys<T> p,
                                                   const T* __restrict__ lgr, const T* __restrict__ llap,
                                                   const T* __restrict__ lsig, const T* __restrict__ lpnb,
                                                   const T* __restrict__ lphi_loc, const T* __restrict__ lpot_loc,
                                                   T* __restrict__ lphi_out, T* __restrict__ lpot_out) {
  constexpr int Q = L::Q;
  constexpr int D = L::D;
  const int64_t y = D == 3 ? band_idx(d) : sidx();  // XCD-aware orders: gathered neighbours share an L2
  if (y >= d.N) return;
  const int64_t N = d.N;
  const bool fluid = flags[y] == 0;
  int nb[Q];
  neighbours<L>(d, y, nb);
  T acc[3] = {0, 0, 0};
  T lp = 0;
  if (fluid) {
    const T wsum = T(36 - L::w36[0]) / T(36);
#pragma unroll
    for (int i = 0; i < 3; ++i) acc[i] = lphi_loc[(int64_t)i * N + y] - T(6) * wsum * llap[(int64_t)i * N + y];
    if (EHD) lp = lpot_loc[y];
  }
#pragma unroll
  for (int q = 1; q < Q; ++q) {
    const int x = nb[L::opp[q]];  // y = x + e_q
    // no test of flags[x]: pass A wrote zero stencil cotangents at solid nodes, so the
    // gathers are unconditional and their loads independent
    const T w = T(L::w36[q]) / T(36);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      T g = T(L::ex[q]) * lgr[(int64_t)(D * i + 0) * N + x] + T(L::ey[q]) * lgr[(int64_t)(D * i + 1) * N + x];
      if (D == 3) g += T(L::ez[q]) * lgr[(int64_t)(D * i + 2) * N + x];
      acc[i] += T(3) * w * g + T(6) * w * llap[(int64_t)i * N + x];
    }
    if (EHD && fluid) {
#pragma unroll
      for (int ax = 0; ax < D; ++ax) {
        if (q == L::axp[ax] || q == L::axm[ax]) {
          const int kk = 2 * ax + (q == L::axp[ax] ? 0 : 1);
          const T ls = lsig[(int64_t)kk * N + x];
#pragma unroll
          for (int i = 0; i < 3; ++i) acc[i] += p.cond[i] * ls;
          lp += lpnb[(int64_t)kk * N + x];
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) lphi_out[(int64_t)i * N + y] = acc[i];
  if (EHD) lpot_out[y] = fluid ? lp : T(0);
}

// ----------------------------------------------------------------------------- pass G
// Ghost cotangents into their link sources.  Links are sorted by source; one thread per
// distinct source sums its ghosts in order.
template <class T>
__global__ __launch_bounds__(kBlock) void k_adj_ghost(int64_t N, int nsrc, const int32_t* __restrict__ src_node,
                                                       const int32_t* __restrict__ src_start,
                                                       const int32_t* __restrict__ gnode_sorted,
                                                       const T* __restrict__ glen_sorted, const T* __restrict__ phi,
                                                       Phys<T> p, T* __restrict__ lphi) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nsrc) return;
  const int64_t f = src_node[k];
  const T p1 = phi[f], p2 = phi[N + f], p3 = phi[2 * N + f];
  const T a4 = T(4) / p.W;
  // dR_i/dp_j
  const T dR[3][3] = {{a4 * (-p.cos13 * p3 - p.cos12 * p2), -a4 * p.cos12 * p1, -a4 * p.cos13 * p1},
                      {a4 * p.cos12 * p2, a4 * (p.cos12 * p1 - p.cos23 * p3), -a4 * p.cos23 * p2},
                      {a4 * p.cos13 * p3, a4 * p.cos23 * p3, a4 * (p.cos23 * p2 + p.cos13 * p1)}};
  T acc[3] = {0, 0, 0};
  for (int g = src_start[k]; g < src_start[k + 1]; ++g) {
    const int64_t s = gnode_sorted[g];
    const T l = glen_sorted[g];
    const T ls[3] = {lphi[s], lphi[N + s], lphi[2 * N + s]};
#pragma unroll
    for (int jx = 0; jx < 3; ++jx)
      acc[jx] += ls[jx] - l * (ls[0] * dR[0][jx] + ls[1] * dR[1][jx] + ls[2] * dR[2][jx]);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) lphi[(int64_t)i * N + f] += acc[i];
}

// ----------------------------------------------------------------------------- pass CD
// Permittivity and charge cotangents from the potential adjoint lb, then the population
// cotangents of step t.  HIGH: plus (1 - s_high) times the streamed cotangents of step t+1
// (lP_next, gathered as in pass A).
template <class L, class T, bool EHD, bool HIGH>
__global__ __launch_bounds__(kBlock) void k_adj_cd(Dims d, const uint8_t* __restrict__ flags, Phys<T> p,
                                                    Volts<T> volts, const T* __restrict__ rec,
                                                    const T* __restrict__ lphi, const T* __restrict__ lrho_loc,
                                                    const T* __restrict__ lb, const T* __restrict__ lmom,
                                                    const T* __restrict__ lP_next, T* __restrict__ lP,
                                                    double* __restrict__ vpart) {
  using ML = MomLayout<L>;
  using RL = RecLayout<L>;
  constexpr int Q = L::Q;
  constexpr int D = L::D;
  const int64_t x = D == 3 ? band_idx(d) : gidx();
  double vloc[kMaxE] = {0.0, 0.0, 0.0, 0.0};
  const int64_t N = d.N;
  if (x < N) {
    const int F = EHD ? 5 : 4;
    if (flags[x] != 0) {
      for (int f = 0; f < F; ++f)
#pragma unroll
        for (int q = 0; q < Q; ++q) lP[((int64_t)f * Q + q) * N + x] = T(0);
    } else {
      T lph[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) lph[i] = lphi[(int64_t)i * N + x];
      T lrho = 0;
      if (EHD) {
        int nb[Q];
        neighbours<L>(d, x, nb);
        const T ex = p.eps[0] * rec[(int64_t)(RL::PHI) * N + x] + p.eps[1] * rec[(int64_t)(RL::PHI + 1) * N + x] +
                     p.eps[2] * rec[(int64_t)(RL::PHI + 2) * N + x];
        const T phx = rec[(int64_t)RL::POT * N + x];
        const T lbx = lb[x];
        T leps = 0;
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            const int m = nb[k == 0 ? L::axp[ax] : L::axm[ax]];
            const uint8_t fm = flags[m];
            if (fm == 0) {
              leps += -T(0.5) * (lbx - lb[m]) * (phx - rec[(int64_t)RL::POT * N + m]);
            } else if (dirichlet_face(fm, volts)) {
              const T pd = fm == 1 ? T(0) : volts.v[fm - 3];
              leps += T(2) * lbx * (pd - phx);
              if (fm >= 3) vloc[fm - 3] += (double)(T(2) * ex * lbx);
            }
          }
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) lph[i] += p.eps[i] * leps;
        lrho = lrho_loc[x] + lbx;
      }
      const T ldrho = lmom[(int64_t)ML::DRHO * N + x];
      T lj[3] = {0, 0, 0}, ljh[3] = {0, 0, 0}, Pk[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int c = 0; c < D; ++c) {
        lj[c] = lmom[(int64_t)(ML::J + c) * N + x];
        if (EHD) ljh[c] = lmom[(int64_t)(ML::JH + c) * N + x];
      }
#pragma unroll
      for (int k = 0; k < ML::P; ++k) Pk[k] = lmom[(int64_t)(ML::PI + k) * N + x];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const T exq = T(L::ex[q]), eyq = T(L::ey[q]), ezq = T(L::ez[q]);
        T ld;
        if (D == 2)
          ld = exq * exq * Pk[0] + eyq * eyq * Pk[1] + exq * eyq * Pk[2];
        else
          ld = exq * exq * Pk[0] + eyq * eyq * Pk[1] + ezq * ezq * Pk[2] + exq * eyq * Pk[3] + exq * ezq * Pk[4] +
               eyq * ezq * Pk[5];
        lP[(int64_t)q * N + x] = ldrho + exq * lj[0] + eyq * lj[1] + ezq * lj[2] + ld;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          T v = lph[i];
          v += exq * lmom[(int64_t)(ML::JF + D * i + 0) * N + x] + eyq * lmom[(int64_t)(ML::JF + D * i + 1) * N + x];
          if (D == 3) v += ezq * lmom[(int64_t)(ML::JF + D * i + 2) * N + x];
          lP[((int64_t)(1 + i) * Q + q) * N + x] = v;
        }
        if (EHD) lP[((int64_t)4 * Q + q) * N + x] = lrho + exq * ljh[0] + eyq * ljh[1] + ezq * ljh[2];
      }
      if (HIGH) {
        int nb[Q];
        neighbours<L>(d, x, nb);
        const T k1 = T(1) - p.s_high;
        for (int f = 0; f < F; ++f) {
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            const T lo = flags[nb[q]] != 0 ? lP_next[((int64_t)f * Q + L::opp[q]) * N + x]
                                           : lP_next[((int64_t)f * Q + q) * N + nb[q]];
            lP[((int64_t)f * Q + q) * N + x] += k1 * lo;
          }
        }
      }
    }
  }
  if (EHD) block_reduce<kMaxE, false>(vloc, vpart + (int64_t)blockIdx.x * kMaxE, 1, true);
}

// ----------------------------------------------------------------------------- terminal cotangent
// L depends on x_c(T) (phase-1 moments of the populations at T) and on v_c(T) (previous-
// step Phi_1 and u in the state at T).  s = {M1, x_c[3], Mp, v_c[3]} in FP64.
template <class L, class T, bool EHD>
__global__ __launch_bounds__(kBlock) void k_adj_terminal(Dims d, const uint8_t* __restrict__ flags,
                                                          const T* __restrict__ phi_prev, const T* __restrict__ u_prev,
                                                          const double* __restrict__ s, double gx0, double gx1,
                                                          double gx2, double gv0, double gv1, double gv2,
                                                          T* __restrict__ lP, T* __restrict__ lphip,
                                                          T* __restrict__ lup, T* __restrict__ lrhop,
                                                          T* __restrict__ lqp) {
  constexpr int Q = L::Q;
  constexpr int D = L::D;
  const int64_t x = gidx();
  if (x >= d.N) return;
  const int64_t N = d.N;
  const int F = EHD ? 5 : 4;
  const bool fluid = flags[x] == 0;
  const double cx[3] = {(double)(x % d.nx), (double)((x / d.nx) % d.ny), (double)(x / ((int64_t)d.nx * d.ny))};
  const double gx[3] = {gx0, gx1, gx2}, gv[3] = {gv0, gv1, gv2};
  double l1 = 0.0, lpp = 0.0;
  double lu[3] = {0.0, 0.0, 0.0};
  if (fluid) {
    for (int a = 0; a < D; ++a) l1 += gx[a] * (cx[a] - s[1 + a]) / s[0];
    const double pp = phi_prev[x];
    for (int a = 0; a < D; ++a) {
      const double ua = u_prev[(int64_t)a * N + x];
      lpp += gv[a] * (ua - s[5 + a]) / s[4];
      lu[a] = gv[a] * pp / s[4];
    }
  }
  for (int f = 0; f < F; ++f)
    for (int q = 0; q < Q; ++q) lP[((int64_t)f * Q + q) * N + x] = f == 1 ? (T)l1 : T(0);
  lphip[x] = (T)lpp;
  lphip[N + x] = T(0);
  lphip[2 * N + x] = T(0);
  for (int a = 0; a < D; ++a) lup[(int64_t)a * N + x] = (T)lu[a];
  lrhop[x] = T(0);
  lqp[x] = T(0);
}

}  // namespace ehd
