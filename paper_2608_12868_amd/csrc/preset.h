// Host-only workload presets (ehdlb_preset): lattice, parameters, node flags and initial phase
// fields of the droplet / lubricant / ambient configurations, from the paper's problem
// statement (Results, Fig. 1: micropillars of solid fraction 0.25 infused with lubricant to
// their tops, a droplet cap on the lubricant, an electrode segment on the opposite wall,
// grounded pillars and substrate, insulating walls elsewhere) and its Methods parameters.
// Every value is computed in the same order of operations as the seeded input generator the
// tests use, so both give the same bits (the tanh of the interface profiles is the C
// library's).
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>

#include "../../include/ehdlb.h"

namespace ehd_preset {

struct Spec {
  int dim;
  int n[3];
  int precision;
  double radius, xc, yc;
  int pillar_w, pillar_pitch, pillar_h;  // pillar_w = 0: flat wall
  int film;                              // flat-film cases: lubricant rows 1..film
  int gap, elen;                         // electrode: starts gap lu ahead of the droplet front
  bool ehd, jitter;
};

inline bool spec_of(int id, Spec& s) {
  std::memset(&s, 0, sizeof(s));
  switch (id) {
    case EHDLB_PRESET_C1:
      s = Spec{2, {128, 64, 1}, EHDLB_FP64, 20.0, 64.0, 0.0, 0, 1, 0, 6, 0, 0, false, true};
      return true;
    case EHDLB_PRESET_C1S:
      s = Spec{2, {64, 32, 1}, EHDLB_FP64, 10.0, 32.0, 0.0, 0, 1, 0, 4, 0, 0, false, true};
      return true;
    case EHDLB_PRESET_C2:
      s = Spec{2, {512, 256, 1}, EHDLB_FP64, 40.0, 128.0, 0.0, 8, 16, 12, 0, 40, 64, true, false};
      return true;
    case EHDLB_PRESET_C4:
      s = Spec{2, {512, 256, 1}, EHDLB_FP32_DEV, 40.0, 128.0, 0.0, 8, 16, 12, 0, 40, 64, true, false};
      return true;
    case EHDLB_PRESET_C2S:
      s = Spec{2, {128, 64, 1}, EHDLB_FP64, 12.0, 40.0, 0.0, 4, 8, 6, 0, 10, 24, true, false};
      return true;
    case EHDLB_PRESET_C4S:
      s = Spec{2, {96, 48, 1}, EHDLB_FP64, 10.0, 30.0, 0.0, 4, 8, 5, 0, 10, 24, true, false};
      return true;
    case EHDLB_PRESET_C3:
      s = Spec{3, {256, 128, 96}, EHDLB_FP32_DEV, 30.0, 64.0, 64.0, 6, 12, 10, 0, 40, 64, true, false};
      return true;
    case EHDLB_PRESET_C5:
      s = Spec{3, {384, 192, 128}, EHDLB_FP32_DEV, 48.0, 96.0, 96.0, 6, 12, 10, 0, 40, 64, true, false};
      return true;
    case EHDLB_PRESET_C3S:
      s = Spec{3, {48, 32, 24}, EHDLB_FP64, 8.0, 14.0, 16.0, 3, 6, 4, 0, 8, 16, true, false};
      return true;
    default:
      return false;
  }
}

// SplitMix64 output function (Steele, Lea & Flood 2014), the state increment applied first
inline uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// counter-based uniform draw in [0, 1): top 53 bits of splitmix64(seed 2^40 + 4 node + comp)
inline double uniform01(uint64_t seed, uint64_t node, uint64_t comp) {
  const uint64_t ctr = (seed << 40) + node * 4u + comp;
  return (double)(splitmix64(ctr) >> 11) * 0x1p-53;
}

// the Methods / Fig. 2 parameter set in lattice units, contact angles by Young's relation
inline void default_params(int dim, ehdlb_params& p) {
  (void)dim;
  std::memset(&p, 0, sizeof(p));
  for (int i = 0; i < 3; ++i) p.tau_flow[i] = 1.0;
  p.mobility = 0.0025;
  p.width = 4.0;
  p.gamma12 = p.gamma13 = p.gamma23 = 1e-3;
  const double deg = 3.141592653589793 / 180.0;
  p.cos13 = std::cos(100.0 * deg);
  p.cos23 = std::cos(5.0 * deg);
  p.cos12 = (p.gamma13 * p.cos13 - p.gamma23 * p.cos23) / p.gamma12;
  p.ehd = 0;
  p.eps[0] = 80.0;
  p.eps[1] = 2.5;
  p.eps[2] = 1.0;
  p.cond[0] = 0.1;
  p.cond[1] = 1e-4;
  p.cond[2] = 1e-4;
  p.poisson_tol = 1e-13;
  p.poisson_max_iter = 400;
  p.poisson_check_every = 1;
  p.s_high = 1.0;
  for (int i = 0; i < 3; ++i) p.rho[i] = 1.0;
}

inline ehdlb_status preset(int id, ehdlb_lattice* L, ehdlb_params* P, uint8_t* flags, double* phi, uint64_t seed) {
#pragma clang fp contract(off)
  Spec s;
  if (!spec_of(id, s) || !L || !P) return EHDLB_EINVAL;
  std::memset(L, 0, sizeof(*L));
  L->dim = s.dim;
  for (int a = 0; a < 3; ++a) L->n[a] = s.n[a];
  L->periodic[0] = 1;
  L->periodic[1] = s.dim == 3 ? 1 : 0;
  L->periodic[2] = 0;
  L->precision = s.precision;
  default_params(s.dim, *P);
  const int nv = s.dim == 2 ? s.n[1] : s.n[2];
  const double level = s.pillar_w > 0 ? s.pillar_h + 0.5 : s.film + 0.5;
  int e0 = 0, e1 = 0;
  if (s.ehd) {
    // charge diffusion from alpha* = alpha mu_w / (eps_w R0^2 E0^2) = 1e-4 (text after Eq. 14), E0 = V / L
    const double volts = 0.05, mu_w = (1.0 - 0.5) / 3.0, e = volts / nv;
    P->ehd = 1;
    P->charge_diffusion = 1e-4 * P->eps[0] * std::pow(s.radius, 2.0) * std::pow(e, 2.0) / mu_w;
    P->electrode_volts[0] = volts;
    e0 = (int)(s.xc + s.radius) + s.gap;
    e1 = e0 + s.elen;
  }
  const int64_t N = (int64_t)s.n[0] * s.n[1] * s.n[2];
  if (!flags && !phi) return EHDLB_OK;
  for (int64_t i = 0; i < N; ++i) {
    const int x = (int)(i % s.n[0]), y = (int)((i / s.n[0]) % s.n[1]), z = (int)(i / ((int64_t)s.n[0] * s.n[1]));
    const int vert = s.dim == 2 ? y : z;
    uint8_t f = EHDLB_FLUID;
    if (s.pillar_w > 0) {
      bool in = x % s.pillar_pitch < s.pillar_w;
      if (s.dim == 3) in = in && y % s.pillar_pitch < s.pillar_w;
      if (in && vert >= 1 && vert <= s.pillar_h) f = EHDLB_GROUND;
    }
    if (vert == 0) f = EHDLB_GROUND;
    if (vert == nv - 1) {
      f = EHDLB_INSULATOR;
      if (s.ehd && x >= e0 && x < e1) f = EHDLB_ELECTRODE0;
    }
    if (flags) flags[i] = f;
    if (!phi) continue;
    const double xd = x, yd = y, zd = z, vd = vert, W = P->width;
    double r;
    if (s.dim == 2) {
      const double dx = xd - s.xc, dy = yd - level;
      r = std::sqrt(dx * dx + dy * dy);
    } else {
      const double dx = xd - s.xc, dy = yd - s.yc, dz = zd - level;
      r = std::sqrt(dx * dx + dy * dy + dz * dz);
    }
    const double above = 0.5 * (1.0 + std::tanh(2.0 * (vd - level) / W));
    const double below = 0.5 * (1.0 + std::tanh(2.0 * (level - vd) / W));
    double p1 = 0.5 * (1.0 + std::tanh(2.0 * (s.radius - r) / W)) * above;
    double p2 = (1.0 - p1) * below;
    double p3 = 1.0 - p1 - p2;
    if (s.jitter) {
      // +-1e-6 on Phi_1 and Phi_2 (the 128x64 case), Phi_3 recomputed
      p1 += (2.0 * uniform01(seed, (uint64_t)i, 0) - 1.0) * 1e-6;
      p2 += (2.0 * uniform01(seed, (uint64_t)i, 1) - 1.0) * 1e-6;
      p3 = 1.0 - p1 - p2;
    }
    if (f != EHDLB_FLUID) p1 = p2 = p3 = 0.0;
    phi[i] = p1;
    phi[N + i] = p2;
    phi[2 * N + i] = p3;
  }
  return EHDLB_OK;
}

}  // namespace ehd_preset
