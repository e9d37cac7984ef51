// Host side of the ternary EHD lattice-Boltzmann library: validation, geometry tables,
// workspace layout, the time-step driver and the C ABI declared in include/ehdlb.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>
#include <type_traits>

#include "../../include/ehdlb.h"
#include "kernels.h"
#include "step.h"
#include "adjoint.h"
#include "preset.h"

using namespace ehd;

namespace {

struct Status {
  ehdlb_status code;
};

size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }
int nblocks(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }
// grid of the grid-stride reduction kernels (fixed, so the reduction order is fixed)
constexpr int kRedBlocks = 1024;
constexpr int kZeroBlocks = 256;  // grid of k_cg_zero (grid-stride; returns at once unless b == 0)
// levels with at most this many cells whose working vectors, with those of every coarser
// level, fit the tail's LDS run inside the single-workgroup V-cycle tail
constexpr int64_t kTailMaxCells = 2048;
constexpr int kSolverParts = 7;
// earlier solutions spanning the projected warm starts: forward (potentials of steps t-1..t-5)
// and adjoint (adjoint potentials of steps t+1..t+6, which alternate in sign)
constexpr int kProjFwd = 5, kProjAdj = 6;
// steps between rebuilds of the forward solves' coarse hierarchy (a preconditioner: the coarse
// operators of a few steps back still precondition the current fine operator well)
constexpr int64_t kHierLag = 8;
// saved-state header tag (its layout: t, tag, N, bytes per value, hierarchy step)
constexpr int64_t kStateMagic = 0x45484443;
// grid of the projection's Gram pass: its per-block partials (up to 27 FP64 each) are summed by
// one workgroup, whose read bandwidth bounds the solve (4096 blocks: 65 us at 384x192x128,
// 1024: 28 us, with the Gram pass no slower)
constexpr int kProjBlocks = 1024;
// MI355X's Infinity Cache (memory-side last-level cache)
constexpr size_t kInfinityCacheBytes = (size_t)256 << 20;
int rblocks(int64_t n) { return std::min(nblocks(n), kRedBlocks); }

struct MGLevel {
  Level L;
  size_t cp, diag, dinv, r, z, t;  // byte offsets
  size_t acp, adiag, adinv;        // the adjoint solves' own coarse operators (levels >= 1)
};

}  // namespace

// ---------------------------------------------------------------------------- library-held scratch
// Device scratch of ehdlb_observables_device (for callers that cannot allocate): the observables'
// per-block FP64 partials (kObs sums and one maximum per block of kBlock nodes) and the final
// sums, for lattices of at most kNoAllocMaxNodes nodes (9 MiB per device, held until the process
// ends).  Host code never passes the array's name to a kernel: each device's address comes from
// hipGetSymbolAddress at ehdlb_bind, with that device current, and is kept in g_scratch.
constexpr int64_t kNoAllocMaxNodes = (int64_t)1 << 24;
constexpr int64_t kNoAllocBlocks = kNoAllocMaxNodes / ehd::kBlock;
constexpr int64_t kNoAllocRed = 64;  // final sums (kObs) and maximum
constexpr size_t kNoAllocDoubles = (size_t)kNoAllocBlocks * (ehd::kObs + 1) + kNoAllocRed;
static __device__ __align__(256) double scratch[kNoAllocDoubles];
constexpr int kMaxDevices = 64;
static double* g_scratch[kMaxDevices] = {};
static std::mutex g_scratch_mu;

struct ehdlb_ctx {
  ehdlb_lattice lat{};
  ehdlb_params prm{};
  int D = 2, Q = 9, F = 4;
  int64_t N = 0;
  size_t tsize = 8;
  bool ehd = false;
  std::string err;
  // host tables
  std::vector<uint8_t> flags;
  std::vector<int32_t> ghost_node, ghost_src;
  std::vector<int32_t> ghost_dir;
  bool have_geometry = false;
  bool have_state = false;
  // schedules
  struct Sched {
    std::vector<double> v;
    int64_t t_total = 0;
  } sched[EHDLB_MAX_ELECTRODES];
  // device
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  bool bound = false;
  int64_t t = 0;
  int cur = 0;
  int sticky = 0;
  // forward generation: bumped by every public call that changes the state or what a step
  // computes (set_geometry, set_phase, set_charge, set_schedule, set_solver_options, step with
  // n > 0, load_state); the checkpointed forward records it and the adjoint requires it unchanged
  uint64_t gen = 0;
  double last_resid = 0.0, last_resid0 = 0.0;
  int last_iters = 0;
  // iteration counts of the last potential solves of each kind (0: forward, 1: adjoint): they
  // decide how much work is queued before the host looks at the control block (speed only)
  struct CgHistory {
    int last = 0, last_nonzero = 1;
    unsigned zeros = 0;  // bit k: the solve k solves ago took no iteration (last 8 solves)
    unsigned over = 0;   // bit k: the solve k solves ago took more iterations than first queued
    int64_t solves = 0, iters = 0;  // statistics (ehdlb_solver_stats)
    double max_rel0 = 0.0;
  } cg_hist[2];
  int device = -1;     // HIP device current at ehdlb_bind
  ehd::CgCtl hctl{};  // host copy of the solve's control block
  ehd::CgCtl* hctl_pin = nullptr;  // pinned staging of the control block (allocated at bind)
  hipEvent_t ev_ctl = nullptr;     // marks the control block's copy in the stream
  int64_t hier_t = -1;  // step whose operator the coarse hierarchy was built from (-1: none); saved
  // the adjoint solves' hierarchy (own storage, swapped in for their solves): the step it was built
  // from, and the step of the solve in progress
  int64_t adj_hier_t = -1, adj_step = 0;
  size_t off_inv_adj = 0;
  // layout (byte offsets into ws)
  size_t off_pop[2]{}, off_phi[2]{}, off_rho[2]{}, off_u[2]{}, off_q[2]{}, off_pot = 0, off_pot_old = 0;
  size_t off_pot_hist[kProjFwd]{};  // potentials of earlier steps for the projected warm start (ring by t)
  // end of the state region that save_state copies after the populations
  size_t off_state_end = 0;  // end of the state region (the saved state)
  size_t state_end() const { return off_state_end; }
  size_t off_flags = 0, off_gnode = 0, off_gsrc = 0, off_glen = 0, off_scratch = 0;
  size_t off_b = 0, off_r = 0, off_z = 0, off_p = 0, off_qv = 0, off_spart = 0;
  size_t off_part = 0, off_red = 0, off_cg = 0, off_inv = 0, off_dbl = 0, off_ppart = 0, off_pcoef = 0;
  size_t state_bytes = 0, total = 0;
  std::vector<MGLevel> mg;
  size_t tail_first = 0;  // first level handled by the single-workgroup tail kernel
  int64_t max_ghost = 0;
  int64_t nparts = 0;
  int64_t hdr[5]{};  // host staging of the state header (kept alive for async copies)
  // wetting links sorted by source (for the adjoint's gather of ghost cotangents)
  std::vector<int32_t> gs_node, src_node, src_start;
  std::vector<double> gs_len;
  size_t off_gs_node = 0, off_gs_len = 0, off_src_node = 0, off_src_start = 0;
  // adjoint: checkpointed forward bookkeeping and workspace layout
  struct Adj {
    char* ws = nullptr;
    size_t bytes = 0;
    int64_t t0 = 0, T = 0;
    int K = 0, nck = 0;
    bool ready = false;
    size_t ckpt = 0, fin = 0, rec = 0, lP[2]{}, lphip[2]{}, lup[2]{}, lrhop[2]{}, lqp[2]{};
    size_t lgr = 0, llap = 0, lsig = 0, lpnb = 0, lphi_loc = 0, lpot_loc = 0, lrho_loc = 0, lmom = 0;
    size_t lphi = 0, lpot = 0, lb = 0, lbr[kProjAdj]{}, vpart = 0, vred = 0, vacc = 0, obs = 0, total = 0, rec_stride = 0;
    int nvseg = 0;
    uint64_t gen = 0;  // forward generation at the end of the checkpointed forward
  } adj;
  // potential-solver options (ehdlb_set_solver_options): degree-2 Chebyshev smoothing of the
  // Jacobi-preconditioned operator on [lo, hi], coarse-correction scale
  double mg_lo = 0.5, mg_hi = 2.0;
  double mg_overcorrect = 2.0;
  bool stream_pops = false;       // population loads with the non-temporal hint
  // forward warm start: 0 previous potential, 1 extrapolated, 2 projected with at least one CG
  // iteration, 3 projected, 4 (default) projected, with at least one CG iteration in the
  // gradient's forward (ehdlb_forward_checkpointed and the adjoint's recompute) only
  int warm_mode = 4;
  bool grad_fwd = false;  // inside ehdlb_forward_checkpointed or ehdlb_adjoint
  // smoothing polynomial z += c1 y - c2 D^-1 A y: p(mu) = 1 - c1 mu + c2 mu^2 = T2(s(mu))/T2(s(0)),
  // s(mu) = (hi + lo - 2 mu)/(hi - lo)
  void poly(double& c1, double& c2) const {
    const double sg = (mg_hi + mg_lo) / (mg_hi - mg_lo), dl = 2.0 / (mg_hi - mg_lo);
    const double t2 = 2.0 * sg * sg - 1.0;
    c1 = 4.0 * sg * dl / t2;
    c2 = 2.0 * dl * dl / t2;
  }
  // optional timing: one event per phase boundary per step (moments | potential | step)
  bool timing = false;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  int64_t timed_steps = 0;
  double acc_ms[3]{};
  double last_mp = 0.0;  // sum of the previous-step Phi_1 at the last observables call

  template <class T>
  T* ptr(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

// ============================================================================ helpers
static ehdlb_status fail(ehdlb_ctx* c, ehdlb_status s, const std::string& m) {
  if (c) c->err = m;
  return s;
}

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(c, EHDLB_EHIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

#define LAUNCHCHK()                                                                        \
  do {                                                                                     \
    hipError_t e_ = hipGetLastError();                                                     \
    if (e_ != hipSuccess) return fail(c, EHDLB_EHIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
  } while (0)

static void upsilons(const ehdlb_params& p, double u[3], double& ut) {
  u[0] = p.gamma12 + p.gamma13 - p.gamma23;
  u[1] = p.gamma12 + p.gamma23 - p.gamma13;
  u[2] = p.gamma13 + p.gamma23 - p.gamma12;
  ut = 3.0 / (1.0 / u[0] + 1.0 / u[1] + 1.0 / u[2]);
}

template <class T>
static Phys<T> make_phys(const ehdlb_params& p) {
  Phys<T> r{};
  double u[3], ut;
  upsilons(p, u, ut);
  r.W = (T)p.width;
  for (int i = 0; i < 3; ++i) r.ups[i] = (T)u[i];
  r.upsT = (T)ut;
  r.cos12 = (T)p.cos12;
  r.cos13 = (T)p.cos13;
  r.cos23 = (T)p.cos23;
  r.s_phi = (T)(1.0 / (0.5 + 3.0 * p.mobility));
  r.s_e = (T)(1.0 / (0.5 + 3.0 * p.charge_diffusion));
  r.s_high = (T)p.s_high;
  for (int i = 0; i < 3; ++i) {
    r.nu[i] = (T)((p.tau_flow[i] - 0.5) / 3.0);
    r.rho[i] = (T)p.rho[i];
    r.eps[i] = (T)p.eps[i];
    r.cond[i] = (T)p.cond[i];
    r.body[i] = (T)p.body_force[i];
  }
  return r;
}

static double volts_at(const ehdlb_ctx* c, int k, int64_t t) {
  const auto& s = c->sched[k];
  if (s.v.empty()) return c->prm.electrode_volts[k];
  // floor(t * n_seg / t_total) in exact integer arithmetic
  int64_t seg = (t * (int64_t)s.v.size()) / s.t_total;
  if (seg >= (int64_t)s.v.size()) seg = (int64_t)s.v.size() - 1;
  if (seg < 0) seg = 0;
  return s.v[(size_t)seg];
}

// electrode voltages of step t for the kernels: NaN (switched off, floating) -> 0 and the
// electrode's bit in off
template <class T>
static Volts<T> volts_of(const ehdlb_ctx* c, int64_t t) {
  Volts<T> v{};
  for (int e = 0; e < kMaxE; ++e) {
    const double x = volts_at(c, e, t);
    const bool floating = std::isnan(x);
    v.v[e] = floating ? T(0) : (T)x;
    if (floating) v.off |= 1u << e;
  }
  return v;
}

// lattice tables on the host (same canonical order as the device)
static void host_lattice(int dim, std::vector<int>& ex, std::vector<int>& ey, std::vector<int>& ez,
                         std::vector<int>& w36) {
  if (dim == 2) {
    ex.assign(D2Q9::ex, D2Q9::ex + 9);
    ey.assign(D2Q9::ey, D2Q9::ey + 9);
    ez.assign(D2Q9::ez, D2Q9::ez + 9);
    w36.assign(D2Q9::w36, D2Q9::w36 + 9);
  } else {
    ex.assign(D3Q19::ex, D3Q19::ex + 19);
    ey.assign(D3Q19::ey, D3Q19::ey + 19);
    ez.assign(D3Q19::ez, D3Q19::ez + 19);
    w36.assign(D3Q19::w36, D3Q19::w36 + 19);
  }
}

// ============================================================================ layout
// dimensions of the potential solver's levels: aggregation of 2 cells per axis down to at most
// kCoarseMax cells (or until a level stops shrinking)
static std::vector<Level> mg_levels(const ehdlb_ctx* c) {
  std::vector<Level> v;
  v.push_back(Level{{c->lat.n[0], c->lat.n[1], c->lat.n[2]}, c->N});
  while (v.back().N > kCoarseMax) {
    const Level f = v.back();
    Level l{};
    for (int a = 0; a < 3; ++a) l.n[a] = (a < c->D) ? (f.n[a] + 1) / 2 : 1;
    l.N = (int64_t)l.n[0] * l.n[1] * l.n[2];
    if (l.N == f.N) break;
    v.push_back(l);
  }
  return v;
}

static void plan_layout(ehdlb_ctx* c) {
  const int64_t N = c->N;
  const size_t ts = c->tsize;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align_up(o + bytes);
    return r;
  };
  // --- state region (save/load copies [state_begin, state_end))
  for (int k = 0; k < 2; ++k) c->off_pop[k] = take((size_t)c->F * c->Q * N * ts);
  // populations that cannot stay in the Infinity Cache between steps are loaded with the
  // non-temporal hint (faster there; slightly slower where they stay resident)
  c->stream_pops = 2 * (size_t)c->F * c->Q * N * ts > kInfinityCacheBytes;
  for (int k = 0; k < 2; ++k) c->off_phi[k] = take(3 * N * ts);
  for (int k = 0; k < 2; ++k) c->off_rho[k] = take(N * ts);
  for (int k = 0; k < 2; ++k) c->off_u[k] = take((size_t)c->D * N * ts);
  for (int k = 0; k < 2; ++k) c->off_q[k] = take(N * ts);
  c->off_pot = take(N * ts);
  c->off_pot_old = take(N * ts);  // potential of the previous step (warm-start extrapolation)
  for (int k = 0; k < kProjFwd; ++k) c->off_pot_hist[k] = take(N * ts);
  // the coarse levels of the potential solver's hierarchy (Galerkin operators, inverse
  // diagonals, dense coarsest inverse) belong to the state: the forward solves rebuild them
  // every kHierLag steps, and a replay from a saved state must precondition with the same ones
  std::vector<Level> levels;
  std::vector<size_t> hcp, hdiag, hdinv;
  if (c->ehd) {
    levels = mg_levels(c);
    for (size_t l = 1; l < levels.size(); ++l) {
      hcp.push_back(take((size_t)c->D * levels[l].N * ts));
      hdiag.push_back(take(levels[l].N * ts));
      hdinv.push_back(take(levels[l].N * ts));
    }
    const int64_t nc = levels.back().N;
    c->off_inv = take((size_t)nc * nc * 8);
  }
  c->off_state_end = o;
  // --- geometry
  c->off_flags = take(N);
  c->max_ghost = N;  // upper bound; actual count known at set_geometry
  c->off_gnode = take(N * 4);
  c->off_gsrc = take(N * 4);
  c->off_glen = take(N * ts);
  c->off_gs_node = take(N * 4);
  c->off_gs_len = take(N * ts);
  c->off_src_node = take(N * 4);
  c->off_src_start = take((N + 1) * 4);
  c->off_scratch = take(N * ts);
  c->off_dbl = take(N * 8);
  // --- potential solver
  c->mg.clear();
  if (c->ehd) {
    c->off_b = take(N * ts);
    c->off_r = take(N * ts);
    c->off_z = take(N * ts);
    c->off_p = take(N * ts);
    c->off_qv = take(N * ts);
    MGLevel m0{};
    m0.L = levels[0];
    m0.cp = take((size_t)c->D * N * ts);
    m0.diag = take(N * ts);
    m0.dinv = take(N * ts);
    m0.r = c->off_r;
    m0.z = take(N * ts);
    m0.t = take(N * ts);
    c->mg.push_back(m0);
    for (size_t l = 1; l < levels.size(); ++l) {
      MGLevel m{};
      m.L = levels[l];
      m.cp = hcp[l - 1];
      m.diag = hdiag[l - 1];
      m.dinv = hdinv[l - 1];
      m.r = take(levels[l].N * ts);
      m.z = take(levels[l].N * ts);
      m.t = take(levels[l].N * ts);
      m.acp = take((size_t)c->D * levels[l].N * ts);
      m.adiag = take(levels[l].N * ts);
      m.adinv = take(levels[l].N * ts);
      c->mg.push_back(m);
    }
    c->off_inv_adj = take((size_t)levels.back().N * levels.back().N * 8);
    c->tail_first = c->mg.size() - 1;
    int64_t tail_cells = c->mg.back().L.N;
    while (c->tail_first > 0) {
      const int64_t n = c->mg[c->tail_first - 1].L.N;
      if (n > kTailMaxCells || 3 * (size_t)(tail_cells + n) * ts > (size_t)kTailLdsBytes) break;
      tail_cells += n;
      --c->tail_first;
    }
  }
  c->nparts = nblocks(N);
  c->off_part = take((size_t)c->nparts * kObs * 8 + 64);
  c->off_red = take(64 * 8);
  c->off_cg = take(sizeof(CgCtl));
  // solver partials: true residual (3 per block), max|r|, p.q, two r.z
  c->off_spart = take((size_t)kSolverParts * kRedBlocks * 8);
  c->off_ppart = take((size_t)std::max(proj_sums<kProjFwd>(), proj_sums<kProjAdj>()) * kProjBlocks * 8);
  c->off_pcoef = take(std::max(kProjFwd, kProjAdj) * 8);
  c->state_bytes = 256 + align_up((size_t)c->F * c->Q * N * ts) + (c->state_end() - c->off_phi[0]);
  c->total = o;
}

// Exchange the coarse operators of levels >= 1 and the dense coarsest inverse with the adjoint
// solves' own copies (called around each adjoint solve).
static void swap_hierarchy(ehdlb_ctx* c) {
  for (size_t l = 1; l < c->mg.size(); ++l) {
    MGLevel& m = c->mg[l];
    std::swap(m.cp, m.acp);
    std::swap(m.diag, m.adiag);
    std::swap(m.dinv, m.adinv);
  }
  std::swap(c->off_inv, c->off_inv_adj);
}

// ============================================================================ validation
static ehdlb_status validate(ehdlb_ctx* c, const ehdlb_lattice* L, const ehdlb_params* p) {
  if (!L || !p) return fail(c, EHDLB_EINVAL, "null lattice or params");
  if (L->dim != 2 && L->dim != 3) return fail(c, EHDLB_EINVAL, "dim must be 2 or 3");
  for (int a = 0; a < 3; ++a)
    if (L->n[a] < 1) return fail(c, EHDLB_EINVAL, "lattice sizes must be >= 1");
  if (L->dim == 2 && L->n[2] != 1) return fail(c, EHDLB_EINVAL, "2D lattices need Nz = 1");
  if ((int64_t)L->n[0] * L->n[1] * L->n[2] >= (int64_t)1 << 31) return fail(c, EHDLB_EINVAL, "too many nodes");
  if (L->precision != EHDLB_FP64 && L->precision != EHDLB_FP32_DEV)
    return fail(c, EHDLB_EINVAL, "unknown precision");
  for (int i = 0; i < 3; ++i) {
    if (!(p->tau_flow[i] > 0.5)) return fail(c, EHDLB_EINVAL, "tau_flow must exceed 1/2");
    if (p->ehd && !(p->eps[i] > 0.0)) return fail(c, EHDLB_EINVAL, "permittivity must be > 0");
    if (p->ehd && !(p->cond[i] >= 0.0)) return fail(c, EHDLB_EINVAL, "conductivity must be >= 0");
  }
  if (!(p->s_high > 0.0 && p->s_high < 2.0)) return fail(c, EHDLB_EINVAL, "s_high must lie in (0, 2)");
  for (int i = 0; i < 3; ++i)
    if (!(p->rho[i] > 0.0)) return fail(c, EHDLB_EINVAL, "densities must be > 0 (or 0 for the default 1)");
  if (!(p->mobility > 0.0)) return fail(c, EHDLB_EINVAL, "mobility must be > 0");
  if (!(p->width > 0.0)) return fail(c, EHDLB_EINVAL, "interface width must be > 0");
  // pair tensions positive; Upsilon_i may be negative (a spreading phase: the lubricant cloaking
  // the droplet when gamma13 > gamma12 + gamma23) but not zero, and Upsilon_T must be finite
  if (!(p->gamma12 > 0.0 && p->gamma13 > 0.0 && p->gamma23 > 0.0))
    return fail(c, EHDLB_EINVAL, "pair tensions must be > 0");
  double u[3], ut;
  upsilons(*p, u, ut);
  for (int i = 0; i < 3; ++i)
    if (u[i] == 0.0) return fail(c, EHDLB_EINVAL, "every Upsilon_i (Eq. 11) must be nonzero");
  if (!std::isfinite(ut)) return fail(c, EHDLB_EINVAL, "Upsilon_T (Eq. 11) must be finite");
  if (p->ehd) {
    if (!(p->charge_diffusion >= 0.0)) return fail(c, EHDLB_EINVAL, "charge diffusion must be >= 0");
    if (!(p->poisson_tol > 0.0)) return fail(c, EHDLB_EINVAL, "poisson_tol must be > 0");
    if (p->poisson_max_iter < 1) return fail(c, EHDLB_EINVAL, "poisson_max_iter must be >= 1");
    if (p->poisson_check_every < 1) return fail(c, EHDLB_EINVAL, "poisson_check_every must be >= 1");
    for (int e = 0; e < EHDLB_MAX_ELECTRODES; ++e)
      if (std::isinf(p->electrode_volts[e])) return fail(c, EHDLB_EINVAL, "electrode voltages must be finite or NaN");
  }
  return EHDLB_OK;
}

// ============================================================================ potential solve
template <class T>
static TailArgs<T> tail_args(ehdlb_ctx* c) {
  TailArgs<T> t{};
  t.first = (int)c->tail_first;
  t.last = (int)c->mg.size() - 1;
  int off = 0;
  for (int l = t.first; l <= t.last; ++l) {
    t.lds[l] = off;
    off += 3 * (int)c->mg[l].L.N;
  }
  for (int l = t.first; l <= t.last; ++l) {
    MGLevel& m = c->mg[l];
    t.L[l] = m.L;
    t.cp[l] = c->ptr<T>(m.cp);
    t.dg[l] = c->ptr<T>(m.diag);
    t.di[l] = c->ptr<T>(m.dinv);
    t.r[l] = c->ptr<T>(m.r);
    t.z[l] = c->ptr<T>(m.z);
    t.t[l] = c->ptr<T>(m.t);
  }
  t.inv = c->ptr<double>(c->off_inv);
  t.stop = &c->ptr<CgCtl>(c->off_cg)->stop;
  double c1, c2;
  c->poly(c1, c2);
  t.c1 = (T)c1;
  t.c2 = (T)c2;
  t.a = (T)c->mg_overcorrect;
  return t;
}

// One symmetric V-cycle z = M r at level lvl.  At level 0 with dot_part != nullptr the last
// post-smoothing sweep also writes per-block partials of r.z (grid of rblocks(N)); returns
// whether it did.
template <int D, class T>
static ehdlb_status vcycle(ehdlb_ctx* c, size_t lvl, T* r, T** zout, double* dot_part, bool* dotted) {
  hipStream_t s = c->stream;
  MGLevel& m = c->mg[lvl];
  const Level L = m.L;
  const int* stop = &c->ptr<CgCtl>(c->off_cg)->stop;
  if (dotted) *dotted = false;
  if (lvl == c->tail_first) {
    TailArgs<T> ta = tail_args<T>(c);
    if (r != ta.r[lvl]) {
      HIPCHK(hipMemcpyAsync(ta.r[lvl], r, L.N * sizeof(T), hipMemcpyDeviceToDevice, s));
    }
    hipLaunchKernelGGL((k_vcycle_tail<D, T>), dim3(1), dim3(kTailThreads), 0, s, ta);
    LAUNCHCHK();
    *zout = ta.z[lvl];
    return EHDLB_OK;
  }
  T* cp = c->ptr<T>(m.cp);
  T* dg = c->ptr<T>(m.diag);
  T* di = c->ptr<T>(m.dinv);
  double c1d, c2d;
  c->poly(c1d, c2d);
  const T c1 = (T)c1d, c2 = (T)c2d, a = (T)c->mg_overcorrect;
  T* z = c->ptr<T>(m.z);
  T* t = c->ptr<T>(m.t);
  const int nb = nblocks(L.N);
  if (lvl > 0 && L.N <= small_level_max<D>()) {
    // small level: two launches (down, up) instead of four; the result is in t
    MGLevel& mc = c->mg[lvl + 1];
    T* rc = c->ptr<T>(mc.r);
    constexpr int TX = restrict_tile_x<D>();
    const int ntx = (L.n[0] + TX - 1) / TX, nty = (L.n[1] + 1) / 2, ntz = D == 3 ? (L.n[2] + 1) / 2 : 1;
    hipLaunchKernelGGL((k_down_small<D, T>), dim3(ntx * nty * ntz), dim3(kBlock), 0, s, stop, L, (const T*)cp,
                       (const T*)dg, (const T*)di, r, z, mc.L, rc, c1, c2);
    LAUNCHCHK();
    T* zc = nullptr;
    ehdlb_status st = vcycle<D, T>(c, lvl + 1, rc, &zc, nullptr, nullptr);
    if (st) return st;
    hipLaunchKernelGGL((k_up_small<D, T>), dim3(nb), dim3(kBlock), 0, s, stop, L, (const T*)cp, (const T*)dg,
                       (const T*)di, (const T*)r, (const T*)z, mc.L, (const T*)zc, a, c1, c2, t);
    LAUNCHCHK();
    *zout = t;
    return EHDLB_OK;
  }
  hipLaunchKernelGGL((k_smooth2<D, T>), dim3(nb), dim3(kBlock), 0, s, stop, L, cp, di, r, z, c1, c2);
  MGLevel& mc = c->mg[lvl + 1];
  T* rc = c->ptr<T>(mc.r);
  {
    constexpr int TX = restrict_tile_x<D>();
    const int ntx = (L.n[0] + TX - 1) / TX, nty = (L.n[1] + 1) / 2, ntz = D == 3 ? (L.n[2] + 1) / 2 : 1;
    hipLaunchKernelGGL((k_restrict_tile<D, T>), dim3(ntx * nty * ntz), dim3(kBlock), 0, s, stop, L, (const T*)cp,
                       (const T*)dg, (const T*)r, (const T*)z, mc.L, rc);
  }
  LAUNCHCHK();
  T* zc = nullptr;
  ehdlb_status st = vcycle<D, T>(c, lvl + 1, rc, &zc, nullptr, nullptr);
  if (st) return st;
  hipLaunchKernelGGL((k_prolong_resid<D, T>), dim3(nb), dim3(kBlock), 0, s, stop, L, cp, dg, di, r, z, mc.L,
                     (const T*)zc, a, t);
  if (dot_part) {
    hipLaunchKernelGGL((k_poly_post<D, T, true>), dim3(rblocks(L.N)), dim3(kBlock), 0, s, stop, L, cp, di, r, z,
                       mc.L, (const T*)zc, a, (const T*)t, c1, c2, z, dot_part);
    if (dotted) *dotted = true;
  } else {
    hipLaunchKernelGGL((k_poly_post<D, T, false>), dim3(nb), dim3(kBlock), 0, s, stop, L, cp, di, r, z, mc.L,
                       (const T*)zc, a, (const T*)t, c1, c2, z, (double*)nullptr);
  }
  LAUNCHCHK();
  *zout = z;
  return EHDLB_OK;
}

// Conjugate gradients on the fine-level operator (already set up in level 0) for A x = b, warm
// started from x, preconditioned by one multigrid V-cycle; converged when the FP64 residual
// max|b - A x| <= tol max|b| or is at the rounding floor of x stored in T.
//
// Every decision is taken on the device (CgCtl): alpha and beta are evaluated by the kernels
// that use them from the fixed-order partials of the previous reductions, the convergence test
// by k_true_resid/k_cg_judge, and once the solve has stopped every queued solver kernel returns
// at once.  How much is queued before the host reads the control block follows the recent
// iteration counts `hist`: after solves that needed no iteration the host looks right after the
// initial check; in a run of iterating solves it queues the hierarchy and as many iterations as
// the last solve took.  Afterwards it continues one iteration at a time.  The iterates do not
// depend on this.
template <class LT, class T>
static ehdlb_status pcg(ehdlb_ctx* c, T* x, const T* b, ehdlb_ctx::CgHistory& hist, int min1 = 0,
                        const std::function<void()>* spec = nullptr, bool projected = false) {
  constexpr int D = LT::D;
  hipStream_t s = c->stream;
  const int64_t N = c->N;
  MGLevel& m0 = c->mg[0];
  T* cp0 = c->ptr<T>(m0.cp);
  T* dg0 = c->ptr<T>(m0.diag);
  T* r = c->ptr<T>(c->off_r);
  T* p = c->ptr<T>(c->off_p);
  T* qv = c->ptr<T>(c->off_qv);
  CgCtl* ctl = c->ptr<CgCtl>(c->off_cg);
  const int* stop = &ctl->stop;
  double* sp = c->ptr<double>(c->off_spart);
  double* ptrue = sp;  // 3 per block
  double* pmax = sp + 3 * kRedBlocks;
  double* ppq = sp + 4 * kRedBlocks;
  double* prz[2] = {sp + 5 * kRedBlocks, sp + 6 * kRedBlocks};  // r.z of preconditioning k in prz[k & 1]
  const int nb0 = nblocks(N), rb0 = rblocks(N);
  const double tol = c->prm.poisson_tol;
  const double eps_t = sizeof(T) == 4 ? 1.1920928955078125e-07 : 2.220446049250313e-16;

  // initial check; x = 0 when b == 0
  hipLaunchKernelGGL((k_true_resid<D, T>), dim3(rb0), dim3(kBlock), 0, s, (const CgCtl*)nullptr,
                     (const double*)nullptr, 0, tol, 0, m0.L, (const T*)cp0, (const T*)dg0, b, (const T*)x, r,
                     ptrue);
  hipLaunchKernelGGL(k_cg_judge, dim3(1), dim3(kBlock), 0, s, ctl, (const double*)ptrue, (const double*)pmax, rb0,
                     tol, eps_t, 0, 0, 1, min1);
  LAUNCHCHK();
  // (a projected start is already 0 then: the Galerkin right-hand side u_i . b vanishes)
  if (!projected)
    hipLaunchKernelGGL(k_cg_zero<T>, dim3(std::min(nb0, kZeroBlocks)), dim3(kBlock), 0, s, (const CgCtl*)ctl, N, x);
  // The host reads the control block after an event that follows its copy, not after the whole
  // stream: `spec` (if given) queues work that depends on the solution behind the copy, gated
  // on the device by the stop flag, so it runs without a host round trip when the solve has
  // stopped by then (and returns at once otherwise).  Every exit below follows a read at which
  // the solve had stopped, so exactly one such launch does its work.
  auto read_ctl = [&]() -> ehdlb_status {
    HIPCHK(hipMemcpyAsync(c->hctl_pin, ctl, sizeof(CgCtl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(c->ev_ctl, s));
    if (spec) (*spec)();
    HIPCHK(hipEventSynchronize(c->ev_ctl));
    c->hctl = *c->hctl_pin;
    return EHDLB_OK;
  };
  bool stopped = false;
  int batch = std::max(hist.last, 1);
  if (__builtin_popcount(hist.zeros & 0xffu) >= 4) {
    // at least half of the last 8 solves took no iteration: look before queueing the hierarchy
    // (otherwise the iterations are queued at once, and return at once if the start already
    // met the tolerance: cheaper than the GPU waiting for the host on most solves)
    ehdlb_status e = read_ctl();
    if (e) return e;
    stopped = c->hctl.stop != 0;
    batch = std::max(hist.last_nonzero - 1, 1);
  }
  // coarse hierarchy (Galerkin aggregation, with inverse diagonals) and the dense coarsest
  // inverse, only when iterating; the fine level's inverse diagonal comes from pois_setup.  The
  // forward solves rebuild it every kHierLag steps (it only preconditions the current fine
  // operator).  The adjoint's solves keep their own hierarchy (swapped in by the caller), rebuilt
  // on the same lag counted in adjoint steps, so that it does not depend on the checkpoint
  // interval (the recompute between them restores the forward's from the checkpoints).
  const bool fwd_solve = &hist == &c->cg_hist[0];
  int64_t& hier_t = fwd_solve ? c->hier_t : c->adj_hier_t;
  const int64_t t_now = fwd_solve ? c->t : c->adj_step;
  const bool rebuild = hier_t < 0 || std::llabs(t_now - hier_t) >= kHierLag;
  if (!stopped && rebuild) {
    for (size_t l = 0; l < c->tail_first; ++l) {
      MGLevel& f = c->mg[l];
      MGLevel& g = c->mg[l + 1];
      hipLaunchKernelGGL((k_coarsen<D, T>), dim3(nblocks(g.L.N)), dim3(kBlock), 0, s, stop, f.L,
                         (const T*)c->ptr<T>(f.cp), (const T*)c->ptr<T>(f.diag), g.L, c->ptr<T>(g.cp),
                         c->ptr<T>(g.diag), c->ptr<T>(g.dinv));
    }
    hipLaunchKernelGGL((k_tail_setup<D, T>), dim3(1), dim3(kTailThreads), 0, s, tail_args<T>(c),
                       c->ptr<double>(c->off_inv));
    LAUNCHCHK();
  }
  // z = M r, with the partials of r.z
  T* z = nullptr;
  auto precondition = [&](double* rz) -> ehdlb_status {
    bool dotted = false;
    ehdlb_status e = vcycle<D, T>(c, 0, r, &z, rz, &dotted);
    if (e) return e;
    if (!dotted) hipLaunchKernelGGL(k_dot<T>, dim3(rb0), dim3(kBlock), 0, s, stop, N, (const T*)r, (const T*)z, rz);
    LAUNCHCHK();
    return EHDLB_OK;
  };
  ehdlb_status st = EHDLB_OK;
  if (!stopped && (st = precondition(prz[0]))) return st;
  const int maxit = c->prm.poisson_max_iter, every = c->prm.poisson_check_every;
  const bool spec_tail = __builtin_popcount(hist.over & 0xffu) >= 4;
  bool overran = false;
  int queued = 0;
  for (; !stopped;) {
    for (int k = 0; k < batch && queued < maxit; ++k) {
      const int it = ++queued;
      // p = z + beta p with beta = rz_{it-1} / rz_{it-2}; q = A p
      hipLaunchKernelGGL(k_cg_dir<T>, dim3(rb0), dim3(kBlock), 0, s, (const CgCtl*)ctl, N,
                         (const double*)prz[(it - 1) & 1], (const double*)prz[it & 1], rb0, it == 1 ? 1 : 0,
                         (const T*)z, p);
      hipLaunchKernelGGL((k_spmv<D, T>), dim3(rb0), dim3(kBlock), 0, s, (const CgCtl*)ctl, m0.L, (const T*)cp0,
                         (const T*)dg0, (const T*)p, qv, ppq);
      hipLaunchKernelGGL(k_cg_update_max<T>, dim3(rb0), dim3(kBlock), 0, s, (const CgCtl*)ctl, N,
                         (const double*)prz[(it - 1) & 1], (const double*)ppq, rb0, (const T*)p, (const T*)qv, x, r,
                         pmax);
      if (it % every == 0 || it == maxit) {
        const int force = it == maxit ? 1 : 0;
        hipLaunchKernelGGL((k_true_resid<D, T>), dim3(rb0), dim3(kBlock), 0, s, (const CgCtl*)ctl,
                           (const double*)pmax, rb0, tol, force, m0.L, (const T*)cp0, (const T*)dg0, b, (const T*)x,
                           r, ptrue);
        hipLaunchKernelGGL(k_cg_judge, dim3(1), dim3(kBlock), 0, s, ctl, (const double*)ptrue, (const double*)pmax,
                           rb0, tol, eps_t, it, force, 0, 0);
      }
      LAUNCHCHK();
      // the preconditioning for the next iteration: within the batch at once; after its last
      // iteration only once the control block shows that the solve goes on (a queued V-cycle
      // that returns at once still costs a launch per kernel), unless recent solves often
      // needed more than their first batch (then it runs while the host reads the block)
      if ((k + 1 < batch || spec_tail) && queued < maxit && (st = precondition(prz[it & 1]))) return st;
    }
    if ((st = read_ctl())) return st;
    if (c->hctl.stop || queued >= maxit) break;
    overran = true;
    if (!spec_tail && (st = precondition(prz[queued & 1]))) return st;
    batch = 1;
  }
  const CgCtl& h = c->hctl;
  // the build kernels ran iff the solve iterated (they return at once once it has stopped)
  if (!stopped && rebuild) hier_t = h.iterated ? t_now : -1;
  c->last_resid0 = h.rel0;
  c->last_iters = h.iterated && !h.zero ? h.iters : 0;
  c->last_resid = h.zero ? 0.0 : h.rel;
  if (!h.zero) {
    if (h.iterated && !h.conv) c->sticky |= 2;
    if (!std::isfinite(h.rel)) c->sticky |= 1;
  }
  hist.zeros = (hist.zeros << 1) | (c->last_iters == 0 ? 1u : 0u);
  hist.over = (hist.over << 1) | (overran ? 1u : 0u);
  hist.last = c->last_iters;
  if (c->last_iters > 0) hist.last_nonzero = c->last_iters;
  ++hist.solves;
  hist.iters += c->last_iters;
  if (!h.zero) hist.max_rel0 = std::max(hist.max_rel0, h.rel0);
  return EHDLB_OK;
}

// Fine-level operator and right-hand side of the discrete Gauss law from the phase fields
// (rho == nullptr: Dirichlet part of b only).
template <class LT, class T>
static ehdlb_status pois_setup(ehdlb_ctx* c, const T* phi, const T* rho, const Volts<T>& volts) {
  const int64_t N = c->N;
  const Dims dm{c->lat.n[0], c->lat.n[1], c->lat.n[2], N};
  MGLevel& m0 = c->mg[0];
  hipLaunchKernelGGL((k_pois_setup<LT, T>), dim3(nblocks(N)), dim3(kBlock), 0, c->stream, dm,
                     c->ptr<uint8_t>(c->off_flags), phi, rho, make_phys<T>(c->prm), volts, c->ptr<T>(m0.cp),
                     c->ptr<T>(m0.diag), c->ptr<T>(m0.dinv), c->ptr<T>(c->off_b));
  LAUNCHCHK();
  return EHDLB_OK;
}

// Warm start of A x = b (the fine operator of the current pois_setup) by Galerkin projection onto
// x's current content h_1 and up to M - 1 earlier solutions (m vectors in all); h_1 is kept in
// `keep` for later solves.
template <int D, class T, int M>
static void project_warm_start(ehdlb_ctx* c, T* x, const T* b, const T* const* older, int m, T* keep,
                               const double (&basis)[M][M]) {
  hipStream_t s = c->stream;
  const MGLevel& m0 = c->mg[0];
  const int64_t N = m0.L.N;
  ProjVecs<T, M> h{};
  h.v[0] = x;
  for (int j = 1; j < M; ++j) h.v[j] = j < m ? older[j - 1] : x;
  for (int r = 0; r < M; ++r)
    for (int k = 0; k < M; ++k) h.B[r][k] = m == M ? basis[r][k] : (r == k && r < m ? 1.0 : 0.0);
  const int rb = std::min(nblocks(N), kProjBlocks);
  double* part = c->ptr<double>(c->off_ppart);
  double* coef = c->ptr<double>(c->off_pcoef);
  hipLaunchKernelGGL((k_proj_gram<D, T, M>), dim3(rb), dim3(kBlock), 0, s, m0.L, (const T*)c->ptr<T>(m0.cp),
                     (const T*)c->ptr<T>(m0.diag), b, h, m, keep, part);
  hipLaunchKernelGGL((k_proj_solve<T, M>), dim3(1), dim3(kFinalWide), 0, s, (const double*)part, rb, m, h, coef);
  hipLaunchKernelGGL((k_proj_combine<T, M>), dim3(nblocks(N)), dim3(kBlock), 0, s, N, (const double*)coef, h, m, x);
}

template <class LT, class T>
static ehdlb_status potential_solve(ehdlb_ctx* c, const T* phi, const T* rho, const Volts<T>& volts,
                                    const std::function<void()>* spec = nullptr) {
  ehdlb_status st = pois_setup<LT, T>(c, phi, rho, volts);
  if (st) return st;
  // warm start (the potential of the previous step is the plain one): extrapolated linearly from
  // the potentials of the two previous steps, or projected onto the potentials of the last five
  // steps (the default; kept in the saved state, so a replay from a checkpoint takes the same
  // iterates)
  T* pot = c->ptr<T>(c->off_pot);
  const int mode = c->warm_mode == 4 ? (c->grad_fwd ? 2 : 3) : c->warm_mode;
  if (mode == 1) {
    hipLaunchKernelGGL(k_extrapolate<T>, dim3(nblocks(c->N)), dim3(kBlock), 0, c->stream, c->N, pot,
                       c->ptr<T>(c->off_pot_old));
  } else if (mode >= 2 && c->t >= 1) {
    const int64_t t = c->t;
    const int m = (int)std::min<int64_t>(t, kProjFwd);
    const T* older[kProjFwd - 1];
    for (int j = 1; j < kProjFwd; ++j) older[j - 1] = j < m ? c->ptr<T>(c->off_pot_hist[(t - 1 - j) % kProjFwd]) : pot;
    // basis: phi(t-1) and its backward differences up to the fourth, u_r = sum_k (-1)^k C(r, k) h_k
    double basis[kProjFwd][kProjFwd];
    for (int r = 0; r < kProjFwd; ++r)
      for (int k = 0; k < kProjFwd; ++k) {
        double binom = 1.0;
        for (int i = 0; i < k; ++i) binom = binom * (r - i) / (i + 1);
        basis[r][k] = k <= r ? ((k & 1) ? -binom : binom) : 0.0;
      }
    project_warm_start<LT::D, T, kProjFwd>(c, pot, c->ptr<T>(c->off_b), older, m,
                                          c->ptr<T>(c->off_pot_hist[(t - 1) % kProjFwd]), basis);
  }
  // mode 2: at least one CG iteration after the projected start (a solve that keeps the start
  // leaves an error that is carried into the next steps' starts, correlated from step to step,
  // and biases the gradients of the trajectory)
  return pcg<LT, T>(c, c->ptr<T>(c->off_pot), c->ptr<T>(c->off_b), c->cg_hist[0], mode == 2 ? 1 : 0, spec,
                    mode >= 2 && c->t >= 1);
}

// ============================================================================ timing
// Sum the elapsed times of the recorded event quadruples (synchronises on the last event).
static ehdlb_status flush_timing(ehdlb_ctx* c) {
  if (c->ev_used == 0) return EHDLB_OK;
  HIPCHK(hipEventSynchronize(c->ev[c->ev_used - 1]));
  for (size_t k = 0; k + 3 < c->ev_used; k += 4) {
    for (int j = 0; j < 3; ++j) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, c->ev[k + j], c->ev[k + j + 1]));
      c->acc_ms[j] += ms;
    }
  }
  c->ev_used = 0;
  return EHDLB_OK;
}

// ============================================================================ launch helpers
template <class LT, class T>
static void launch_moments(const ehdlb_ctx* c, int families, const Dims& dm, const uint8_t* flags, const T* pop,
                           T* phi, T* rho, T* drho, int fam0) {
  const dim3 grid(nblocks(dm.N), families);
  if (c->stream_pops)
    hipLaunchKernelGGL((k_moments<LT, T, true>), grid, dim3(kBlock), 0, c->stream, dm, flags, pop, phi, rho, drho,
                       fam0);
  else
    hipLaunchKernelGGL((k_moments<LT, T, false>), grid, dim3(kBlock), 0, c->stream, dm, flags, pop, phi, rho, drho,
                       fam0);
}

template <class LT, class T, bool EHD, bool STORE, bool HIGH, bool VRHO>
static void launch_step_h(const ehdlb_ctx* c, const StepArgs<T>& a) {
  if (c->stream_pops)
    hipLaunchKernelGGL((k_step<LT, T, EHD, STORE, true, HIGH, VRHO>), dim3(nblocks(a.d.N)), dim3(kBlock), 0,
                       c->stream, a);
  else
    hipLaunchKernelGGL((k_step<LT, T, EHD, STORE, false, HIGH, VRHO>), dim3(nblocks(a.d.N)), dim3(kBlock), 0,
                       c->stream, a);
}

static bool var_rho(const ehdlb_ctx* c) {
  return !(c->prm.rho[0] == 1.0 && c->prm.rho[1] == 1.0 && c->prm.rho[2] == 1.0);
}

// the variants with the higher moments away from rate 1, or with unequal densities, only when
// they are
template <class LT, class T, bool EHD, bool STORE>
static void launch_step(const ehdlb_ctx* c, const StepArgs<T>& a) {
  const bool high = c->prm.s_high != 1.0;
  if (var_rho(c)) {
    if (high)
      launch_step_h<LT, T, EHD, STORE, true, true>(c, a);
    else
      launch_step_h<LT, T, EHD, STORE, false, true>(c, a);
    return;
  }
  if (high)
    launch_step_h<LT, T, EHD, STORE, true, false>(c, a);
  else
    launch_step_h<LT, T, EHD, STORE, false, false>(c, a);
}

// ============================================================================ step
template <class LT, class T, bool EHD>
static ehdlb_status step_impl(ehdlb_ctx* c, int64_t n) {
  hipStream_t s = c->stream;
  const int64_t N = c->N;
  const Dims dm{c->lat.n[0], c->lat.n[1], c->lat.n[2], N};
  const Phys<T> ph = make_phys<T>(c->prm);
  const uint8_t* flags = c->ptr<uint8_t>(c->off_flags);
  const int G = (int)c->ghost_node.size();
  for (int64_t k = 0; k < n; ++k) {
    const int64_t t = c->t;
    const int pi = (int)(t & 1), pp = 1 - pi;
    const Volts<T> v = volts_of<T>(c, t);
    T* phi = c->ptr<T>(c->off_phi[pi]);
    T* rho = c->ptr<T>(c->off_rho[pi]);
    const T* pin = c->ptr<T>(c->off_pop[c->cur]);
    T* pout = c->ptr<T>(c->off_pop[1 - c->cur]);
    hipEvent_t* ev = nullptr;
    if (c->timing) {
      if (c->ev_used + 4 > c->ev.size()) {
        ehdlb_status st = flush_timing(c);
        if (st) return st;
      }
      ev = &c->ev[c->ev_used];
      c->ev_used += 4;
      HIPCHK(hipEventRecord(ev[0], s));
    }
    launch_moments<LT, T>(c, EHD ? 4 : 3, dm, flags, pin, phi, rho, (T*)nullptr, 1);
    if (G > 0)
      hipLaunchKernelGGL(k_ghosts<T>, dim3(nblocks(G)), dim3(kBlock), 0, s, N, G, c->ptr<int32_t>(c->off_gnode),
                         c->ptr<int32_t>(c->off_gsrc), c->ptr<T>(c->off_glen), phi, ph);
    LAUNCHCHK();
    if (ev) HIPCHK(hipEventRecord(ev[1], s));
    StepArgs<T> a{};
    a.d = dm;
    a.flags = flags;
    a.pop_in = pin;
    a.pop_out = pout;
    a.phi = phi;
    a.phi_prev = c->ptr<T>(c->off_phi[pp]);
    a.rho = rho;
    a.rho_prev = c->ptr<T>(c->off_rho[pp]);
    a.u_prev = c->ptr<T>(c->off_u[pp]);
    a.u_out = c->ptr<T>(c->off_u[pi]);
    a.q_prev = c->ptr<T>(c->off_q[pp]);
    a.q_out = c->ptr<T>(c->off_q[pi]);
    a.pot = c->ptr<T>(c->off_pot);
    a.p = ph;
    a.volts = v;
    a.dt_on = t == 0 ? T(0) : T(1);
    if (EHD) {
      // the fused step is queued behind each read of the solve's control block, gated on the
      // device by its stop flag: the launch that follows the solve's end does the work, without
      // waiting for the host to see the control block (the step's timing starts there)
      const int* gate = &c->ptr<CgCtl>(c->off_cg)->stop;
      hipError_t launch_err = hipSuccess;
      const std::function<void()> spec = [&]() {
        if (ev && launch_err == hipSuccess) launch_err = hipEventRecord(ev[2], s);
        a.gate = gate;
        launch_step<LT, T, EHD, false>(c, a);
        if (launch_err == hipSuccess) launch_err = hipGetLastError();
      };
      ehdlb_status st = potential_solve<LT, T>(c, phi, rho, v, &spec);
      if (st) return st;
      if (launch_err != hipSuccess)
        return fail(c, EHDLB_EHIP, std::string("fused step launch: ") + hipGetErrorString(launch_err));
    } else {
      if (ev) HIPCHK(hipEventRecord(ev[2], s));
      launch_step<LT, T, EHD, false>(c, a);
      LAUNCHCHK();
    }
    if (ev) {
      HIPCHK(hipEventRecord(ev[3], s));
      c->timed_steps++;
    }
    c->cur = 1 - c->cur;
    c->t = t + 1;
  }
  return EHDLB_OK;
}

template <class LT, class T, bool EHD>
static ehdlb_status moments_now(ehdlb_ctx* c, T* drho) {
  const int64_t N = c->N;
  const Dims dm{c->lat.n[0], c->lat.n[1], c->lat.n[2], N};
  const int pi = (int)(c->t & 1);
  // with drho also the flow family (read-out of the pressure)
  launch_moments<LT, T>(c, (EHD ? 4 : 3) + (drho ? 1 : 0), dm, c->ptr<uint8_t>(c->off_flags),
                        c->ptr<T>(c->off_pop[c->cur]), c->ptr<T>(c->off_phi[pi]), c->ptr<T>(c->off_rho[pi]), drho,
                        drho ? 0 : 1);
  LAUNCHCHK();
  return EHDLB_OK;
}

// The observables' reductions: moments of the current populations, per-block FP64 partials
// (sums [nblocks][kObs] at psum, maxima [nblocks] at pmax) and their fixed-order sums into red
// (kObs sums, then the maximum).
template <class LT, class T, bool EHD>
static ehdlb_status observables_reduce(ehdlb_ctx* c, double* psum, double* pmax, double* red) {
  ehdlb_status st = moments_now<LT, T, EHD>(c, nullptr);
  if (st) return st;
  const int64_t N = c->N;
  const Dims dm{c->lat.n[0], c->lat.n[1], c->lat.n[2], N};
  const int pi = (int)(c->t & 1), pp = 1 - pi;
  const int nb = nblocks(N);
  hipLaunchKernelGGL((k_obs<LT, T, EHD>), dim3(nb), dim3(kBlock), 0, c->stream, dm, c->ptr<uint8_t>(c->off_flags),
                     c->ptr<T>(c->off_phi[pi]), c->ptr<T>(c->off_phi[pp]), c->ptr<T>(c->off_u[pp]),
                     c->ptr<T>(c->off_rho[pi]), psum, pmax);
  hipLaunchKernelGGL((k_final_wide<kObs, false>), dim3(1), dim3(kFinalWide), 0, c->stream, psum, nb, red);
  hipLaunchKernelGGL((k_final_wide<1, true>), dim3(1), dim3(kFinalWide), 0, c->stream, pmax, nb, red + kObs);
  LAUNCHCHK();
  return EHDLB_OK;
}

template <class LT, class T, bool EHD>
static ehdlb_status observables_impl(ehdlb_ctx* c, ehdlb_obs* o) {
  // partials in the workspace: sums in the FP64 scratch, maxima in the reduction buffer
  double* red = c->ptr<double>(c->off_red);
  ehdlb_status st = observables_reduce<LT, T, EHD>(c, c->ptr<double>(c->off_dbl), c->ptr<double>(c->off_part), red);
  if (st) return st;
  double h[kObs + 1];
  HIPCHK(hipMemcpyAsync(h, red, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  std::memset(o, 0, sizeof(*o));
  o->step = c->t;
  for (int i = 0; i < 3; ++i) o->mass[i] = h[i];
  for (int a = 0; a < 3; ++a) o->centroid[a] = h[3 + a] / h[0];
  for (int a = 0; a < 3; ++a) o->velocity[a] = h[9] != 0.0 ? h[6 + a] / h[9] : 0.0;
  c->last_mp = h[9];
  o->total_charge = h[10];
  o->sum_phi_drift = h[kObs];
  o->poisson_residual = c->last_resid;
  o->poisson_initial_residual = c->last_resid0;
  o->poisson_iters = c->last_iters;
  if (h[11] != 0.0 || !std::isfinite(h[0] + h[1] + h[2])) c->sticky |= 1;
  o->flags = c->sticky;
  return EHDLB_OK;
}

// dispatch on (lattice, precision, field on/off)
template <template <class, class, bool> class Fn, class... A>
static ehdlb_status dispatch(ehdlb_ctx* c, A... args) {
  const bool f32 = c->lat.precision == EHDLB_FP32_DEV;
  if (c->D == 2) {
    if (f32) return c->ehd ? Fn<D2Q9, float, true>::run(c, args...) : Fn<D2Q9, float, false>::run(c, args...);
    return c->ehd ? Fn<D2Q9, double, true>::run(c, args...) : Fn<D2Q9, double, false>::run(c, args...);
  }
  if (f32) return c->ehd ? Fn<D3Q19, float, true>::run(c, args...) : Fn<D3Q19, float, false>::run(c, args...);
  return c->ehd ? Fn<D3Q19, double, true>::run(c, args...) : Fn<D3Q19, double, false>::run(c, args...);
}

template <class LT, class T, bool EHD>
struct StepFn {
  static ehdlb_status run(ehdlb_ctx* c, int64_t n) { return step_impl<LT, T, EHD>(c, n); }
};
template <class LT, class T, bool EHD>
struct ObsFn {
  static ehdlb_status run(ehdlb_ctx* c, ehdlb_obs* o) { return observables_impl<LT, T, EHD>(c, o); }
};
// droplet observables from the final sums, as ehdlb_observables forms them on the host:
// out = mass[3], centroid[3], velocity[3], total charge, max |sum Phi - 1|, non-finite count
__global__ void k_obs_finish(const double* __restrict__ red, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  for (int i = 0; i < 3; ++i) out[i] = red[i];
  for (int a = 0; a < 3; ++a) out[3 + a] = red[3 + a] / red[0];
  for (int a = 0; a < 3; ++a) out[6 + a] = red[9] != 0.0 ? red[6 + a] / red[9] : 0.0;
  out[9] = red[10];
  out[10] = red[kObs];
  out[11] = red[11];
}

template <class LT, class T, bool EHD>
struct ObsDevFn {
  static ehdlb_status run(ehdlb_ctx* c, double* out) {
    double* base = g_scratch[c->device];
    double* psum = base;
    double* pmax = base + (size_t)kNoAllocBlocks * kObs;
    double* red = pmax + kNoAllocBlocks;
    ehdlb_status st = observables_reduce<LT, T, EHD>(c, psum, pmax, red);
    if (st) return st;
    hipLaunchKernelGGL(k_obs_finish, dim3(1), dim3(64), 0, c->stream, (const double*)red, out);
    LAUNCHCHK();
    return EHDLB_OK;
  }
};

template <class LT, class T, bool EHD>
struct InitFn {
  static ehdlb_status run(ehdlb_ctx* c, int dummy) {
    (void)dummy;
    const int64_t N = c->N;
    const Dims dm{c->lat.n[0], c->lat.n[1], c->lat.n[2], N};
    // initial fields were copied into the t = -1 slots (index 1): they serve as the
    // previous-step fields of the first step
    hipLaunchKernelGGL((k_init<LT, T, EHD>), dim3(nblocks(N)), dim3(kBlock), 0, c->stream, dm,
                       c->ptr<uint8_t>(c->off_flags), c->ptr<T>(c->off_pop[0]), c->ptr<T>(c->off_phi[1]),
                       c->ptr<T>(c->off_rho[1]), c->ptr<T>(c->off_u[1]), c->ptr<T>(c->off_q[1]));
    const int64_t npop = (int64_t)c->F * c->Q * N;
    hipLaunchKernelGGL(k_zero<T>, dim3(nblocks(npop)), dim3(kBlock), 0, c->stream, npop, c->ptr<T>(c->off_pop[1]));
    hipLaunchKernelGGL(k_zero<T>, dim3(nblocks(N)), dim3(kBlock), 0, c->stream, N, c->ptr<T>(c->off_pot));
    hipLaunchKernelGGL(k_zero<T>, dim3(nblocks(N)), dim3(kBlock), 0, c->stream, N, c->ptr<T>(c->off_pot_old));
    // the t = 0 slots of u and Q: the steps write them at fluid nodes only, so their solid nodes
    // (read out as zero velocity and source) are set here
    hipLaunchKernelGGL(k_zero<T>, dim3(nblocks((int64_t)c->D * N)), dim3(kBlock), 0, c->stream, (int64_t)c->D * N,
                       c->ptr<T>(c->off_u[0]));
    hipLaunchKernelGGL(k_zero<T>, dim3(nblocks(N)), dim3(kBlock), 0, c->stream, N, c->ptr<T>(c->off_q[0]));
    LAUNCHCHK();
    return EHDLB_OK;
  }
};
template <class LT, class T, bool EHD>
struct MomFn {
  static ehdlb_status run(ehdlb_ctx* c, int dummy) {
    (void)dummy;
    return moments_now<LT, T, EHD>(c, c->ptr<T>(c->off_scratch));
  }
};

template <class T>
static ehdlb_status copy_out(ehdlb_ctx* c, const T* src, int64_t n, double* dst) {
  // convert on the device into the FP64 scratch in chunks of N, then copy
  double* tmp = c->ptr<double>(c->off_dbl);
  for (int64_t o = 0; o < n; o += c->N) {
    const int64_t m = std::min<int64_t>(c->N, n - o);
    hipLaunchKernelGGL(k_to_double<T>, dim3(nblocks(m)), dim3(kBlock), 0, c->stream, m, src + o, tmp);
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(dst + o, tmp, m * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  return EHDLB_OK;
}

template <class T>
static ehdlb_status upload(ehdlb_ctx* c, const double* src, int64_t n, T* dst) {
  std::vector<T> h((size_t)n);
  for (int64_t i = 0; i < n; ++i) h[(size_t)i] = (T)src[i];
  HIPCHK(hipMemcpyAsync(dst, h.data(), n * sizeof(T), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return EHDLB_OK;
}

// copy flags and wetting links to the device
static ehdlb_status upload_geometry(ehdlb_ctx* c) {
  std::vector<int> ex, ey, ez, w36;
  host_lattice(c->D, ex, ey, ez, w36);
  HIPCHK(hipMemcpyAsync(c->ptr<uint8_t>(c->off_flags), c->flags.data(), c->N, hipMemcpyHostToDevice, c->stream));
  const size_t G = c->ghost_node.size();
  if (G) {
    HIPCHK(hipMemcpyAsync(c->ptr<int32_t>(c->off_gnode), c->ghost_node.data(), G * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->ptr<int32_t>(c->off_gsrc), c->ghost_src.data(), G * 4, hipMemcpyHostToDevice, c->stream));
    std::vector<double> len(G);
    for (size_t k = 0; k < G; ++k) {
      const int q = c->ghost_dir[k];
      len[k] = std::sqrt((double)(ex[q] * ex[q] + ey[q] * ey[q] + ez[q] * ez[q]));
    }
    ehdlb_status st = c->tsize == 8 ? upload<double>(c, len.data(), (int64_t)G, c->ptr<double>(c->off_glen))
                                    : upload<float>(c, len.data(), (int64_t)G, c->ptr<float>(c->off_glen));
    if (st) return st;
    HIPCHK(hipMemcpyAsync(c->ptr<int32_t>(c->off_gs_node), c->gs_node.data(), G * 4, hipMemcpyHostToDevice, c->stream));
    st = c->tsize == 8 ? upload<double>(c, c->gs_len.data(), (int64_t)G, c->ptr<double>(c->off_gs_len))
                       : upload<float>(c, c->gs_len.data(), (int64_t)G, c->ptr<float>(c->off_gs_len));
    if (st) return st;
    HIPCHK(hipMemcpyAsync(c->ptr<int32_t>(c->off_src_node), c->src_node.data(), c->src_node.size() * 4,
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->ptr<int32_t>(c->off_src_start), c->src_start.data(), c->src_start.size() * 4,
                          hipMemcpyHostToDevice, c->stream));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  return EHDLB_OK;
}

// ============================================================================ adjoint
static ehdlb_status load_state_impl(ehdlb_ctx* c, const void* src);

static int rec_count(const ehdlb_ctx* c) {
  return c->D == 2 ? RecLayout<D2Q9>::COUNT : RecLayout<D3Q19>::COUNT;
}
static int mom_count(const ehdlb_ctx* c) { return c->D == 2 ? MomLayout<D2Q9>::COUNT : MomLayout<D3Q19>::COUNT; }

static void plan_adjoint(const ehdlb_ctx* c, int64_t T, int K, ehdlb_ctx::Adj& a) {
  const int64_t N = c->N;
  const size_t ts = c->tsize;
  const int D = c->D;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align_up(o + bytes);
    return r;
  };
  a.T = T;
  a.K = K;
  a.nck = (int)((T + K - 1) / K);
  a.ckpt = take((size_t)a.nck * align_up(c->state_bytes));
  a.fin = take(c->state_bytes);
  a.rec_stride = align_up((size_t)rec_count(c) * N * ts);
  a.rec = take((size_t)K * a.rec_stride);
  const size_t F = (size_t)c->F * c->Q;
  for (int k = 0; k < 2; ++k) {
    a.lP[k] = take(F * N * ts);
    a.lphip[k] = take(3 * N * ts);
    a.lup[k] = take((size_t)D * N * ts);
    a.lrhop[k] = take(N * ts);
    a.lqp[k] = take(N * ts);
  }
  a.lgr = take((size_t)3 * D * N * ts);
  a.llap = take(3 * N * ts);
  a.lsig = take((size_t)2 * D * N * ts);
  a.lpnb = take((size_t)2 * D * N * ts);
  a.lphi_loc = take(3 * N * ts);
  a.lpot_loc = take(N * ts);
  a.lrho_loc = take(N * ts);
  a.lmom = take((size_t)mom_count(c) * N * ts);
  a.lphi = take(3 * N * ts);
  a.lpot = take(N * ts);
  a.lb = take(N * ts);
  for (int k = 0; k < kProjAdj; ++k) a.lbr[k] = take(N * ts);
  a.vpart = take((size_t)nblocks(N) * kMaxE * 8);
  a.vred = take(kMaxE * 8);
  a.nvseg = 1 << 16;
  a.vacc = take((size_t)kMaxE * a.nvseg * 8);
  a.obs = take(16 * 8);
  a.total = o;
}

__global__ void k_vacc_add(const double* __restrict__ red, double* __restrict__ vacc, int seg, int nseg) {
  const int e = threadIdx.x;
  if (e < kMaxE) vacc[(int64_t)e * nseg + seg] += red[e];
}

// one forward step that also writes the adjoint's record of step t
template <class LT, class T, bool EHD>
static ehdlb_status step_record(ehdlb_ctx* c, T* rec) {
  using RL = RecLayout<LT>;
  static_assert(3 + 3 + LT::D + 2 <= kMaxRows, "record rows exceed the row-copy kernel's capacity");
  hipStream_t s = c->stream;
  const int64_t N = c->N;
  const Dims dm{c->lat.n[0], c->lat.n[1], c->lat.n[2], N};
  const Phys<T> ph = make_phys<T>(c->prm);
  const uint8_t* flags = c->ptr<uint8_t>(c->off_flags);
  const int G = (int)c->ghost_node.size();
  const int64_t t = c->t;
  const int pi = (int)(t & 1), pp = 1 - pi;
  const Volts<T> v = volts_of<T>(c, t);
  T* phi = c->ptr<T>(c->off_phi[pi]);
  T* rho = c->ptr<T>(c->off_rho[pi]);
  const T* pin = c->ptr<T>(c->off_pop[c->cur]);
  T* pout = c->ptr<T>(c->off_pop[1 - c->cur]);
  launch_moments<LT, T>(c, EHD ? 4 : 3, dm, flags, pin, phi, rho, (T*)nullptr, 1);
  if (G > 0)
    hipLaunchKernelGGL(k_ghosts<T>, dim3(nblocks(G)), dim3(kBlock), 0, s, N, G, c->ptr<int32_t>(c->off_gnode),
                       c->ptr<int32_t>(c->off_gsrc), c->ptr<T>(c->off_glen), phi, ph);
  LAUNCHCHK();
  // the record's fields that do not depend on the potential, in one pass before the solve
  {
    RowCopy<T> rc{};
    int j = 0;
    auto row = [&](const T* src, size_t slot) {
      rc.src[j] = src;
      rc.dst[j] = rec + slot * N;
      ++j;
    };
    for (int k = 0; k < 3; ++k) row(phi + k * N, RL::PHI + k);
    for (int k = 0; k < 3; ++k) row(c->ptr<T>(c->off_phi[pp]) + k * N, RL::PHIP + k);
    for (int d = 0; d < LT::D; ++d) row(c->ptr<T>(c->off_u[pp]) + d * N, RL::UP + d);
    if (EHD) {
      row(rho, RL::RHO);
      row(c->ptr<T>(c->off_rho[pp]), RL::RHOP);
    }
    rc.nrows = j;
    hipLaunchKernelGGL(k_copy_rows<T>, dim3(nblocks(N)), dim3(kBlock), 0, s, N, rc);
    LAUNCHCHK();
  }
  StepArgs<T> a{};
  a.d = dm;
  a.flags = flags;
  a.pop_in = pin;
  a.pop_out = pout;
  a.phi = phi;
  a.phi_prev = c->ptr<T>(c->off_phi[pp]);
  a.rho = rho;
  a.rho_prev = c->ptr<T>(c->off_rho[pp]);
  a.u_prev = c->ptr<T>(c->off_u[pp]);
  a.u_out = c->ptr<T>(c->off_u[pi]);
  a.q_prev = c->ptr<T>(c->off_q[pp]);
  a.q_out = c->ptr<T>(c->off_q[pi]);
  a.pot = c->ptr<T>(c->off_pot);
  a.p = ph;
  a.volts = v;
  a.dt_on = t == 0 ? T(0) : T(1);
  a.rec = rec + (size_t)RL::MOM * N;
  if (EHD) {
    // the potential's record copy and the fused step follow the solve without a host round
    // trip, gated on its stop flag (as in the plain step)
    const int* gate = &c->ptr<CgCtl>(c->off_cg)->stop;
    hipError_t launch_err = hipSuccess;
    const std::function<void()> spec = [&]() {
      hipLaunchKernelGGL(k_copy_gated<T>, dim3(nblocks(N)), dim3(kBlock), 0, s, gate, N,
                         (const T*)c->ptr<T>(c->off_pot), rec + (size_t)RL::POT * N);
      a.gate = gate;
      launch_step<LT, T, EHD, true>(c, a);
      if (launch_err == hipSuccess) launch_err = hipGetLastError();
    };
    ehdlb_status st = potential_solve<LT, T>(c, phi, rho, v, &spec);
    if (st) return st;
    if (launch_err != hipSuccess)
      return fail(c, EHDLB_EHIP, std::string("recompute launch: ") + hipGetErrorString(launch_err));
  } else {
    launch_step<LT, T, EHD, true>(c, a);
    LAUNCHCHK();
  }
  c->cur = 1 - c->cur;
  c->t = t + 1;
  return EHDLB_OK;
}

// adjoint of step t: cotangents of step t+1 in slot nx, of step t written into slot cu.  Passes A
// and CD add their dL/dV contributions to per-block partials, which are summed into segment seg's
// entry (and cleared) when flush is set: at the last step of the sweep within the segment.
template <class LT, class T, bool EHD>
static ehdlb_status adjoint_step(ehdlb_ctx* c, int64_t t, const T* rec, int nx, int cu, int seg, bool flush) {
  using RL = RecLayout<LT>;
  auto& J = c->adj;
  hipStream_t s = c->stream;
  const int64_t N = c->N;
  const Dims dm{c->lat.n[0], c->lat.n[1], c->lat.n[2], N};
  const Phys<T> ph = make_phys<T>(c->prm);
  const uint8_t* flags = c->ptr<uint8_t>(c->off_flags);
  auto A = [&](size_t off) { return reinterpret_cast<T*>(J.ws + off); };
  const Volts<T> v = volts_of<T>(c, t);
  const int nb = nblocks(N);
  const size_t lbx = J.lb;
  AdjArgs<T> a{};
  a.d = dm;
  a.flags = flags;
  a.rec = rec;
  a.lP_next = A(J.lP[nx]);
  a.lphip_next = A(J.lphip[nx]);
  a.lup_next = A(J.lup[nx]);
  a.lrhop_next = A(J.lrhop[nx]);
  a.lqp_next = A(J.lqp[nx]);
  a.lphip = A(J.lphip[cu]);
  a.lup = A(J.lup[cu]);
  a.lrhop = A(J.lrhop[cu]);
  a.lqp = A(J.lqp[cu]);
  a.lgr = A(J.lgr);
  a.llap = A(J.llap);
  a.lsig = A(J.lsig);
  a.lpnb = A(J.lpnb);
  a.lphi_loc = A(J.lphi_loc);
  a.lpot_loc = A(J.lpot_loc);
  a.lrho_loc = A(J.lrho_loc);
  a.lmom = A(J.lmom);
  a.vpart = reinterpret_cast<double*>(J.ws + J.vpart);
  a.p = ph;
  a.volts = v;
  a.dt_on = t == 0 ? T(0) : T(1);
  double* vpart = reinterpret_cast<double*>(J.ws + J.vpart);
  double* vred = reinterpret_cast<double*>(J.ws + J.vred);
  double* vacc = reinterpret_cast<double*>(J.ws + J.vacc);
  const bool high = c->prm.s_high != 1.0;
  const bool vr = var_rho(c);
  if constexpr (std::is_same<T, float>::value) {
    if (vr) {
      if (high)
        hipLaunchKernelGGL((k_adj_a32<LT, EHD, true, true>), dim3(nb), dim3(kBlock), 0, s, a);
      else
        hipLaunchKernelGGL((k_adj_a32<LT, EHD, false, true>), dim3(nb), dim3(kBlock), 0, s, a);
    } else if (high) {
      hipLaunchKernelGGL((k_adj_a32<LT, EHD, true, false>), dim3(nb), dim3(kBlock), 0, s, a);
    } else {
      hipLaunchKernelGGL((k_adj_a32<LT, EHD, false, false>), dim3(nb), dim3(kBlock), 0, s, a);
    }
  } else {
    if (vr) {
      if (high)
        hipLaunchKernelGGL((k_adj_a<LT, T, EHD, true, true>), dim3(nb), dim3(kBlock), 0, s, a);
      else
        hipLaunchKernelGGL((k_adj_a<LT, T, EHD, false, true>), dim3(nb), dim3(kBlock), 0, s, a);
    } else if (high) {
      hipLaunchKernelGGL((k_adj_a<LT, T, EHD, true, false>), dim3(nb), dim3(kBlock), 0, s, a);
    } else {
      hipLaunchKernelGGL((k_adj_a<LT, T, EHD, false, false>), dim3(nb), dim3(kBlock), 0, s, a);
    }
  }
  hipLaunchKernelGGL((k_adj_b<LT, T, EHD>), dim3(nb), dim3(kBlock), 0, s, dm, flags, ph, (const T*)A(J.lgr),
                     (const T*)A(J.llap), (const T*)A(J.lsig), (const T*)A(J.lpnb), (const T*)A(J.lphi_loc),
                     (const T*)A(J.lpot_loc), A(J.lphi), A(J.lpot));
  const int nsrc = (int)c->src_node.size();
  if (nsrc > 0)
    hipLaunchKernelGGL(k_adj_ghost<T>, dim3(nblocks(nsrc)), dim3(kBlock), 0, s, N, nsrc,
                       c->ptr<int32_t>(c->off_src_node), c->ptr<int32_t>(c->off_src_start),
                       c->ptr<int32_t>(c->off_gs_node), (const T*)c->ptr<T>(c->off_gs_len),
                       rec + (size_t)RL::PHI * N, ph, A(J.lphi));
  LAUNCHCHK();
  if (EHD) {
    // potential adjoint: A lb = lambda_phi with the operator of step t
    ehdlb_status st = pois_setup<LT, T>(c, rec + (size_t)RL::PHI * N, (const T*)nullptr, v);
    if (st) return st;
    // right-hand side lambda_phi read in place; warm start projected onto the adjoint potentials
    // of steps t+1..t+6 (they alternate in sign from step to step, following the adjoint of the
    // over-relaxed first moments); zero at the start of the sweep
    {
      const int m = (int)std::min<int64_t>(J.t0 + J.T - 1 - t, kProjAdj);
      if (m > 0) {
        const T* older[kProjAdj - 1];
        for (int j = 1; j < kProjAdj; ++j) older[j - 1] = j < m ? A(J.lbr[(t + 1 + j) % kProjAdj]) : A(lbx);
        // basis (h_k = lambda(t+k)): the even-step sequence h_2, h_4, h_6 and its first and second
        // differences, and the sums of consecutive steps h_1 + h_2, h_3 + h_4, h_5 + h_6 (the
        // alternating part cancels) and their first and second differences
        static constexpr double kBasis[kProjAdj][kProjAdj] = {
            {0, 1, 0, 0, 0, 0}, {0, 1, 0, -1, 0, 0}, {0, 1, 0, -2, 0, 1},
            {1, 1, 0, 0, 0, 0}, {1, 1, -1, -1, 0, 0}, {1, 1, -2, -2, 1, 1}};
        project_warm_start<LT::D, T, kProjAdj>(c, A(lbx), (const T*)A(J.lpot), older, m,
                                              A(J.lbr[(t + 1) % kProjAdj]), kBasis);
      }
    }
    c->adj_step = t;
    swap_hierarchy(c);
    st = pcg<LT, T>(c, A(lbx), (const T*)A(J.lpot), c->cg_hist[1]);
    swap_hierarchy(c);
    if (st) return st;
  }
  if (high)
    hipLaunchKernelGGL((k_adj_cd<LT, T, EHD, true>), dim3(nb), dim3(kBlock), 0, s, dm, flags, ph, v, rec,
                       (const T*)A(J.lphi), (const T*)A(J.lrho_loc), (const T*)A(lbx), (const T*)A(J.lmom),
                       (const T*)A(J.lP[nx]), A(J.lP[cu]), vpart);
  else
    hipLaunchKernelGGL((k_adj_cd<LT, T, EHD, false>), dim3(nb), dim3(kBlock), 0, s, dm, flags, ph, v, rec,
                       (const T*)A(J.lphi), (const T*)A(J.lrho_loc), (const T*)A(lbx), (const T*)A(J.lmom),
                       (const T*)A(J.lP[nx]), A(J.lP[cu]), vpart);
  if (EHD && flush) {
    hipLaunchKernelGGL((k_final_wide<kMaxE, false>), dim3(1), dim3(kFinalWide), 0, s, vpart, nb, vred);
    hipLaunchKernelGGL(k_vacc_add, dim3(1), dim3(64), 0, s, vred, vacc, seg, J.nvseg);
    hipLaunchKernelGGL(k_zero<double>, dim3(nblocks((int64_t)nb * kMaxE)), dim3(kBlock), 0, s, (int64_t)nb * kMaxE,
                       vpart);
  }
  LAUNCHCHK();
  return EHDLB_OK;
}

template <class LT, class T, bool EHD>
struct FwdCkptFn {
  static ehdlb_status run(ehdlb_ctx* c, int dummy) {
    (void)dummy;
    auto& J = c->adj;
    ehdlb_status st;
    for (int64_t k = 0; k < J.T; ++k) {
      if (k % J.K == 0) {
        if ((st = ehdlb_save_state(c, J.ws + J.ckpt + (size_t)(k / J.K) * align_up(c->state_bytes)))) return st;
      }
      if ((st = step_impl<LT, T, EHD>(c, 1))) return st;
    }
    return ehdlb_save_state(c, J.ws + J.fin);
  }
};

template <class LT, class T, bool EHD>
struct AdjFn {
  static ehdlb_status run(ehdlb_ctx* c, const double* gx, const double* gv, int electrode, double* out) {
    auto& J = c->adj;
    hipStream_t s = c->stream;
    const int64_t N = c->N;
    const Dims dm{c->lat.n[0], c->lat.n[1], c->lat.n[2], N};
    ehdlb_status st;
    c->adj_hier_t = -1;  // the adjoint solves' hierarchy is built afresh in every sweep
    // terminal cotangent from the FP64 observables of the final state
    ehdlb_obs ob;
    if ((st = observables_impl<LT, T, EHD>(c, &ob))) return st;
    double M1 = ob.mass[0];
    // Mp = sum of the previous-step Phi_1: recompute from the velocity definition's weights
    double sv[8] = {M1, ob.centroid[0], ob.centroid[1], ob.centroid[2], c->last_mp, ob.velocity[0],
                    ob.velocity[1], ob.velocity[2]};
    double* sd = reinterpret_cast<double*>(J.ws + J.obs);
    HIPCHK(hipMemcpyAsync(sd, sv, sizeof(sv), hipMemcpyHostToDevice, s));
    const int pp = 1 - (int)(c->t & 1);
    auto A = [&](size_t off) { return reinterpret_cast<T*>(J.ws + off); };
    int cu = 0;
    hipLaunchKernelGGL((k_adj_terminal<LT, T, EHD>), dim3(nblocks(N)), dim3(kBlock), 0, s, dm,
                       c->ptr<uint8_t>(c->off_flags), c->ptr<T>(c->off_phi[pp]), c->ptr<T>(c->off_u[pp]), sd,
                       gx[0], gx[1], gx[2], gv[0], gv[1], gv[2], A(J.lP[cu]), A(J.lphip[cu]), A(J.lup[cu]),
                       A(J.lrhop[cu]), A(J.lqp[cu]));
    HIPCHK(hipMemsetAsync(J.ws + J.vacc, 0, (size_t)kMaxE * J.nvseg * 8, s));
    hipLaunchKernelGGL(k_zero<double>, dim3(nblocks((int64_t)nblocks(N) * kMaxE)), dim3(kBlock), 0, s,
                       (int64_t)nblocks(N) * kMaxE, reinterpret_cast<double*>(J.ws + J.vpart));
    hipLaunchKernelGGL(k_zero<T>, dim3(nblocks(N)), dim3(kBlock), 0, s, N, A(J.lb));
    LAUNCHCHK();
    const auto& sch = c->sched[electrode];
    const int nseg = sch.v.empty() ? 1 : (int)sch.v.size();
    for (int j = J.nck - 1; j >= 0; --j) {
      if ((st = load_state_impl(c, J.ws + J.ckpt + (size_t)j * align_up(c->state_bytes)))) return st;
      const int64_t ta = J.t0 + (int64_t)j * J.K;
      const int64_t tb = std::min<int64_t>(ta + J.K, J.t0 + J.T);
      for (int64_t t = ta; t < tb; ++t)
        if ((st = step_record<LT, T, EHD>(c, reinterpret_cast<T*>(J.ws + J.rec + (size_t)(t - ta) * J.rec_stride))))
          return st;
      auto seg_of = [&](int64_t tt) {
        if (sch.v.empty()) return 0;
        return (int)std::min<int64_t>((tt * (int64_t)nseg) / sch.t_total, nseg - 1);
      };
      for (int64_t t = tb - 1; t >= ta; --t) {
        const int seg = seg_of(t);
        const bool flush = t == J.t0 || seg_of(t - 1) != seg;
        const int nx = cu;
        cu = 1 - cu;
        if ((st = adjoint_step<LT, T, EHD>(c, t, reinterpret_cast<T*>(J.ws + J.rec + (size_t)(t - ta) * J.rec_stride),
                                            nx, cu, seg, flush)))
          return st;
      }
    }
    std::vector<double> h((size_t)kMaxE * J.nvseg);
    HIPCHK(hipMemcpyAsync(h.data(), J.ws + J.vacc, h.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int k = 0; k < nseg; ++k) out[k] = h[(size_t)electrode * J.nvseg + k];
    // back to the final state of the checkpointed forward
    return load_state_impl(c, J.ws + J.fin);
  }
};

// ============================================================================ C ABI
extern "C" {

ehdlb_status ehdlb_create(const ehdlb_lattice* lattice, const ehdlb_params* params_in, ehdlb_ctx** out) {
  if (!out) return EHDLB_EINVAL;
  *out = nullptr;
  if (!params_in) return EHDLB_EINVAL;
  // zero means the default for the fields a zero-initialised struct leaves at 0
  ehdlb_params pn = *params_in;
  if (pn.s_high == 0.0) pn.s_high = 1.0;
  for (int i = 0; i < 3; ++i)
    if (pn.rho[i] == 0.0) pn.rho[i] = 1.0;
  const ehdlb_params* params = &pn;
  ehdlb_ctx tmp;
  ehdlb_status st = validate(&tmp, lattice, params);
  if (st) return st;
  ehdlb_ctx* c = new ehdlb_ctx();
  c->lat = *lattice;
  c->prm = *params;
  c->D = lattice->dim;
  c->Q = lattice->dim == 2 ? 9 : 19;
  c->ehd = params->ehd != 0;
  c->F = c->ehd ? 5 : 4;
  c->N = (int64_t)lattice->n[0] * lattice->n[1] * lattice->n[2];
  c->tsize = lattice->precision == EHDLB_FP64 ? 8 : 4;
  plan_layout(c);
  *out = c;
  return EHDLB_OK;
}

size_t ehdlb_workspace_bytes(const ehdlb_ctx* c) { return c ? c->total : 0; }

size_t ehdlb_state_bytes(const ehdlb_ctx* c) { return c ? c->state_bytes : 0; }

size_t ehdlb_num_populations(const ehdlb_ctx* c) { return c ? (size_t)c->F * c->Q * c->N : 0; }

ehdlb_status ehdlb_bind(ehdlb_ctx* c, void* ws, size_t bytes, void* stream) {
  if (!c) return EHDLB_EINVAL;
  if (!ws) return fail(c, EHDLB_EINVAL, "null workspace");
  if (((uintptr_t)ws) % 256 != 0) return fail(c, EHDLB_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < c->total) return fail(c, EHDLB_ENOMEM, "workspace too small");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(c, EHDLB_EINVAL, "device index beyond the library's table");
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
      void* p = nullptr;
      HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
      g_scratch[dev] = static_cast<double*>(p);
    }
  }
  c->device = dev;
  c->ws = (char*)ws;
  c->ws_bytes = bytes;
  c->stream = (hipStream_t)stream;
  if (!c->hctl_pin) HIPCHK(hipHostMalloc((void**)&c->hctl_pin, sizeof(CgCtl), hipHostMallocDefault));
  if (!c->ev_ctl) HIPCHK(hipEventCreateWithFlags(&c->ev_ctl, hipEventDisableTiming));
  c->bound = true;
  c->have_state = false;
  if (c->have_geometry) return upload_geometry(c);
  return EHDLB_OK;
}

ehdlb_status ehdlb_set_geometry(ehdlb_ctx* c, const uint8_t* flags) {
  if (!c) return EHDLB_EINVAL;
  if (!flags) return fail(c, EHDLB_EINVAL, "null flags");
  c->hier_t = -1;
  const int nx = c->lat.n[0], ny = c->lat.n[1], nz = c->lat.n[2];
  const int64_t N = c->N;
  std::vector<int> ex, ey, ez, w36;
  host_lattice(c->D, ex, ey, ez, w36);
  const int Q = c->Q;
  for (int64_t i = 0; i < N; ++i) {
    if (flags[i] > EHDLB_ELECTRODE0 + EHDLB_MAX_ELECTRODES - 1)
      return fail(c, EHDLB_EINVAL, "unknown node flag at node " + std::to_string(i));
  }
  auto nbr = [&](int64_t i, int q) -> int64_t {
    int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
    x = (x + ex[q] + nx) % nx;
    y = (y + ey[q] + ny) % ny;
    z = (z + ez[q] + nz) % nz;
    return x + (int64_t)nx * (y + (int64_t)ny * z);
  };
  // end layers of non-periodic axes must be solid
  for (int64_t i = 0; i < N; ++i) {
    if (flags[i] != EHDLB_FLUID) continue;
    const int xyz[3] = {(int)(i % nx), (int)((i / nx) % ny), (int)(i / ((int64_t)nx * ny))};
    for (int a = 0; a < 3; ++a) {
      if (!c->lat.periodic[a] && c->lat.n[a] > 1 && (xyz[a] == 0 || xyz[a] == c->lat.n[a] - 1))
        return fail(c, EHDLB_EINVAL, "fluid on the end layer of a non-periodic axis");
    }
    bool any = false;
    for (int q = 1; q < Q && !any; ++q) any = flags[nbr(i, q)] == EHDLB_FLUID;
    if (!any) return fail(c, EHDLB_EINVAL, "fluid node without a fluid neighbour: " + std::to_string(i));
  }
  // potential: every fluid region (connected through axis faces) needs a Dirichlet face
  if (c->ehd) {
    std::vector<int32_t> comp((size_t)N, -1);
    std::vector<int64_t> stack;
    for (int64_t s0 = 0; s0 < N; ++s0) {
      if (flags[s0] != EHDLB_FLUID || comp[(size_t)s0] >= 0) continue;
      bool dir = false;
      stack.clear();
      stack.push_back(s0);
      comp[(size_t)s0] = 1;
      while (!stack.empty()) {
        const int64_t i = stack.back();
        stack.pop_back();
        for (int q = 1; q < Q; ++q) {
          if (ex[q] * ex[q] + ey[q] * ey[q] + ez[q] * ez[q] != 1) continue;
          const int64_t j = nbr(i, q);
          const uint8_t f = flags[j];
          if (f == EHDLB_FLUID) {
            if (comp[(size_t)j] < 0) {
              comp[(size_t)j] = 1;
              stack.push_back(j);
            }
          } else if (f == EHDLB_GROUND || f >= EHDLB_ELECTRODE0) {
            dir = true;
          }
        }
      }
      if (!dir) return fail(c, EHDLB_EINVAL, "a fluid region has no grounded or electrode face");
    }
  }
  // wetting links: n* maximises (e.N_s)/|e| over fluid neighbours with e.N_s > 0,
  // N_s = sum over fluid neighbours of 36 w e (exact integers); ties to the lowest index;
  // N_s = 0 -> the first fluid neighbour.
  c->ghost_node.clear();
  c->ghost_src.clear();
  c->ghost_dir.clear();
  for (int64_t s = 0; s < N; ++s) {
    if (flags[s] == EHDLB_FLUID) continue;
    int nsx = 0, nsy = 0, nsz = 0, first = -1;
    for (int q = 1; q < Q; ++q) {
      if (flags[nbr(s, q)] != EHDLB_FLUID) continue;
      if (first < 0) first = q;
      nsx += w36[q] * ex[q];
      nsy += w36[q] * ey[q];
      nsz += w36[q] * ez[q];
    }
    if (first < 0) continue;
    int best = -1;
    long long bd = 0, bl = 1;
    if (nsx == 0 && nsy == 0 && nsz == 0) {
      best = first;
    } else {
      for (int q = 1; q < Q; ++q) {
        if (flags[nbr(s, q)] != EHDLB_FLUID) continue;
        const long long d = (long long)ex[q] * nsx + (long long)ey[q] * nsy + (long long)ez[q] * nsz;
        if (d <= 0) continue;
        const long long l2 = ex[q] * ex[q] + ey[q] * ey[q] + ez[q] * ez[q];
        if (best < 0 || d * d * bl > bd * bd * l2) {
          best = q;
          bd = d;
          bl = l2;
        }
      }
    }
    c->ghost_node.push_back((int32_t)s);
    c->ghost_dir.push_back(best);
    c->ghost_src.push_back((int32_t)nbr(s, best));
  }
  // links sorted by source node (stable), grouped: src_node[k], ghosts src_start[k]..src_start[k+1]
  {
    const size_t G = c->ghost_node.size();
    std::vector<size_t> ord(G);
    for (size_t k = 0; k < G; ++k) ord[k] = k;
    std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return c->ghost_src[a] < c->ghost_src[b]; });
    c->gs_node.resize(G);
    c->gs_len.resize(G);
    c->src_node.clear();
    c->src_start.clear();
    for (size_t k = 0; k < G; ++k) {
      const size_t g = ord[k];
      const int q = c->ghost_dir[g];
      c->gs_node[k] = c->ghost_node[g];
      c->gs_len[k] = std::sqrt((double)(ex[q] * ex[q] + ey[q] * ey[q] + ez[q] * ez[q]));
      if (k == 0 || c->ghost_src[g] != c->ghost_src[ord[k - 1]]) {
        c->src_node.push_back(c->ghost_src[g]);
        c->src_start.push_back((int32_t)k);
      }
    }
    c->src_start.push_back((int32_t)G);
  }
  c->flags.assign(flags, flags + N);
  ++c->gen;
  c->have_geometry = true;
  c->have_state = false;
  c->adj.ready = false;
  if (c->bound) return upload_geometry(c);
  return EHDLB_OK;
}

ehdlb_status ehdlb_set_phase(ehdlb_ctx* c, const double* phi) {
  if (!c) return EHDLB_EINVAL;
  if (!phi) return fail(c, EHDLB_EINVAL, "null phase array");
  if (!c->bound) return fail(c, EHDLB_ESTATE, "set_phase before bind");
  if (!c->have_geometry) return fail(c, EHDLB_ESTATE, "set_phase before set_geometry");
  ehdlb_status st;
  const int64_t N = c->N;
  std::vector<double> zero((size_t)N, 0.0);
  if (c->tsize == 8) {
    if ((st = upload<double>(c, phi, 3 * N, c->ptr<double>(c->off_phi[1])))) return st;
    if ((st = upload<double>(c, zero.data(), N, c->ptr<double>(c->off_rho[1])))) return st;
  } else {
    if ((st = upload<float>(c, phi, 3 * N, c->ptr<float>(c->off_phi[1])))) return st;
    if ((st = upload<float>(c, zero.data(), N, c->ptr<float>(c->off_rho[1])))) return st;
  }
  ++c->gen;
  c->t = 0;
  c->hier_t = -1;
  c->cur = 0;
  c->sticky = 0;
  c->last_iters = 0;
  c->last_resid = 0.0;
  if ((st = dispatch<InitFn>(c, 0))) return st;
  HIPCHK(hipStreamSynchronize(c->stream));
  c->have_state = true;
  return EHDLB_OK;
}

ehdlb_status ehdlb_set_charge(ehdlb_ctx* c, const double* rho) {
  if (!c) return EHDLB_EINVAL;
  if (!rho) return fail(c, EHDLB_EINVAL, "null charge array");
  if (!c->have_state || c->t != 0) return fail(c, EHDLB_ESTATE, "set_charge needs a fresh set_phase");
  if (!c->ehd) return fail(c, EHDLB_EINVAL, "set_charge with the field off");
  ++c->gen;
  // the initial fields sit in the t = -1 slots; replace the charge there and rebuild
  ehdlb_status st;
  if (c->tsize == 8) {
    if ((st = upload<double>(c, rho, c->N, c->ptr<double>(c->off_rho[1])))) return st;
  } else {
    if ((st = upload<float>(c, rho, c->N, c->ptr<float>(c->off_rho[1])))) return st;
  }
  if ((st = dispatch<InitFn>(c, 0))) return st;
  HIPCHK(hipStreamSynchronize(c->stream));
  return EHDLB_OK;
}

ehdlb_status ehdlb_set_schedule(ehdlb_ctx* c, int32_t k, int32_t n_seg, const double* volts, int64_t t_total) {
  if (!c) return EHDLB_EINVAL;
  if (k < 0 || k >= EHDLB_MAX_ELECTRODES) return fail(c, EHDLB_EINVAL, "electrode index out of range");
  ++c->gen;
  if (n_seg == 0) {
    c->sched[k].v.clear();
    return EHDLB_OK;
  }
  if (n_seg < 0 || !volts || t_total < 1) return fail(c, EHDLB_EINVAL, "bad schedule");
  for (int32_t s = 0; s < n_seg; ++s)
    if (std::isinf(volts[s])) return fail(c, EHDLB_EINVAL, "schedule voltages must be finite or NaN (floating)");
  c->sched[k].v.assign(volts, volts + n_seg);
  c->sched[k].t_total = t_total;
  return EHDLB_OK;
}

ehdlb_status ehdlb_step(ehdlb_ctx* c, int64_t n) {
  if (!c) return EHDLB_EINVAL;
  if (n < 0) return fail(c, EHDLB_EINVAL, "negative step count");
  if (!c->have_state) return fail(c, EHDLB_ESTATE, "step before set_phase");
  if (n > 0) ++c->gen;
  return dispatch<StepFn>(c, n);
}

ehdlb_status ehdlb_read_field(ehdlb_ctx* c, int32_t field, void* dst_v, int32_t dst_is_device) {
  if (!c) return EHDLB_EINVAL;
  if (!dst_v) return fail(c, EHDLB_EINVAL, "null destination");
  if (dst_is_device != 0 && dst_is_device != 1) return fail(c, EHDLB_EINVAL, "dst_is_device must be 0 or 1");
  if (dst_is_device && ((uintptr_t)dst_v) % 8) return fail(c, EHDLB_EINVAL, "device destination must be 8-byte aligned");
  if (!c->have_state) return fail(c, EHDLB_ESTATE, "read_field before set_phase");
  if (field < EHDLB_FIELD_PHI1 || field > EHDLB_FIELD_POPS) return fail(c, EHDLB_EINVAL, "unknown field id");
  double* dst = static_cast<double*>(dst_v);
  const int64_t N = c->N;
  const int pi = (int)(c->t & 1), pp = 1 - pi;
  ehdlb_status st;
  // n values from workspace offset off (times scale, if not 1), to the host or the device
  auto out = [&](size_t off, int64_t n, double scale = 1.0) -> ehdlb_status {
    if (!dst_is_device) {
      st = c->tsize == 8 ? copy_out<double>(c, c->ptr<double>(off), n, dst)
                         : copy_out<float>(c, c->ptr<float>(off), n, dst);
      if (st) return st;
      if (scale != 1.0)
        for (int64_t i = 0; i < n; ++i) dst[i] *= scale;
      return EHDLB_OK;
    }
    if (c->tsize == 8)
      hipLaunchKernelGGL(k_to_double_scaled<double>, dim3(nblocks(n)), dim3(kBlock), 0, c->stream, n,
                         (const double*)c->ptr<double>(off), scale, dst);
    else
      hipLaunchKernelGGL(k_to_double_scaled<float>, dim3(nblocks(n)), dim3(kBlock), 0, c->stream, n,
                         (const float*)c->ptr<float>(off), scale, dst);
    LAUNCHCHK();
    return EHDLB_OK;
  };
  auto zeros = [&]() -> ehdlb_status {
    if (!dst_is_device) {
      std::fill(dst, dst + N, 0.0);
      return EHDLB_OK;
    }
    hipLaunchKernelGGL(k_zero<double>, dim3(nblocks(N)), dim3(kBlock), 0, c->stream, N, dst);
    LAUNCHCHK();
    return EHDLB_OK;
  };
  switch (field) {
    case EHDLB_FIELD_PHI1:
    case EHDLB_FIELD_PHI2:
    case EHDLB_FIELD_PHI3:
    case EHDLB_FIELD_RHO_E:
    case EHDLB_FIELD_P:
      if ((st = dispatch<MomFn>(c, 0))) return st;
      if (field == EHDLB_FIELD_RHO_E) return c->ehd ? out(c->off_rho[pi], N) : zeros();
      if (field == EHDLB_FIELD_P) return out(c->off_scratch, N, 1.0 / 3.0);
      return out(c->off_phi[pi] + (size_t)(field - EHDLB_FIELD_PHI1) * N * c->tsize, N);
    case EHDLB_FIELD_UX:
    case EHDLB_FIELD_UY:
    case EHDLB_FIELD_UZ: {
      const int a = field - EHDLB_FIELD_UX;
      return a >= c->D ? zeros() : out(c->off_u[pp] + (size_t)a * N * c->tsize, N);
    }
    case EHDLB_FIELD_POT:
      return c->ehd ? out(c->off_pot, N) : zeros();
    case EHDLB_FIELD_Q:
      return c->ehd ? out(c->off_q[pp], N) : zeros();
    default:  // EHDLB_FIELD_POPS
      return out(c->off_pop[c->cur], (int64_t)c->F * c->Q * N);
  }
}

ehdlb_status ehdlb_preset(int32_t preset_id, ehdlb_lattice* lattice, ehdlb_params* params, uint8_t* flags,
                          double* phi, uint64_t seed) {
  return ehd_preset::preset(preset_id, lattice, params, flags, phi, seed);
}

ehdlb_status ehdlb_observables(ehdlb_ctx* c, ehdlb_obs* o) {
  if (!c) return EHDLB_EINVAL;
  if (!o) return fail(c, EHDLB_EINVAL, "null output");
  if (!c->have_state) return fail(c, EHDLB_ESTATE, "observables before set_phase");
  ehdlb_status st = dispatch<ObsFn>(c, o);
  if (st) return st;
  if (c->sticky & 1) return fail(c, EHDLB_ENONFINITE, "non-finite field");
  if (c->sticky & 2) return fail(c, EHDLB_ENOCONV, "potential solve hit its iteration cap");
  return EHDLB_OK;
}

ehdlb_status ehdlb_observables_device(ehdlb_ctx* c, double* dev_out) {
  if (!c) return EHDLB_EINVAL;
  if (!dev_out || ((uintptr_t)dev_out) % 8) return fail(c, EHDLB_EINVAL, "null or misaligned device output");
  if (!c->have_state) return fail(c, EHDLB_ESTATE, "observables before set_phase");
  if (c->N > kNoAllocMaxNodes)
    return fail(c, EHDLB_EINVAL, "ehdlb_observables_device: the lattice has " + std::to_string(c->N) +
                                     " nodes, more than the library-held scratch serves (" +
                                     std::to_string(kNoAllocMaxNodes) + ")");
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != c->device || !g_scratch[dev])
    return fail(c, EHDLB_ESTATE, "ehdlb_observables_device: call it with the bound device current");
  return dispatch<ObsDevFn>(c, dev_out);
}

// state blob: [256-byte header: t, magic, N, sizeof(T)][current populations][field slots
// phi x2, rho x2, u x2, q x2, pot, in t-parity order]
ehdlb_status ehdlb_save_state(ehdlb_ctx* c, void* dst) {
  if (!c) return EHDLB_EINVAL;
  if (!dst) return fail(c, EHDLB_EINVAL, "null destination");
  if (!c->have_state) return fail(c, EHDLB_ESTATE, "save_state before set_phase");
  char* d = (char*)dst;
  c->hdr[0] = c->t;
  c->hdr[1] = kStateMagic;
  c->hdr[2] = (int64_t)c->N;
  c->hdr[3] = (int64_t)c->tsize;
  c->hdr[4] = c->hier_t;
  HIPCHK(hipMemcpyAsync(d, c->hdr, sizeof(c->hdr), hipMemcpyHostToDevice, c->stream));
  const size_t pop_bytes = (size_t)c->F * c->Q * c->N * c->tsize;
  HIPCHK(hipMemcpyAsync(d + 256, c->ws + c->off_pop[c->cur], pop_bytes, hipMemcpyDeviceToDevice, c->stream));
  const size_t rest = c->state_end() - c->off_phi[0];
  HIPCHK(hipMemcpyAsync(d + 256 + align_up(pop_bytes), c->ws + c->off_phi[0], rest, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return EHDLB_OK;
}

ehdlb_status ehdlb_load_state(ehdlb_ctx* c, const void* src) {
  if (!c) return EHDLB_EINVAL;
  ++c->gen;
  return load_state_impl(c, src);
}

}  // extern "C"

static ehdlb_status load_state_impl(ehdlb_ctx* c, const void* src) {
  if (!src) return fail(c, EHDLB_EINVAL, "null source");
  if (!c->bound || !c->have_geometry) return fail(c, EHDLB_ESTATE, "load_state before bind/set_geometry");
  const char* s = (const char*)src;
  int64_t hdr[5];
  HIPCHK(hipMemcpyAsync(hdr, s, sizeof(hdr), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (hdr[1] != kStateMagic || hdr[2] != c->N || hdr[3] != (int64_t)c->tsize)
    return fail(c, EHDLB_EINVAL, "state blob does not match this context");
  const size_t pop_bytes = (size_t)c->F * c->Q * c->N * c->tsize;
  HIPCHK(hipMemcpyAsync(c->ws + c->off_pop[0], s + 256, pop_bytes, hipMemcpyDeviceToDevice, c->stream));
  const size_t rest = c->state_end() - c->off_phi[0];
  HIPCHK(hipMemcpyAsync(c->ws + c->off_phi[0], s + 256 + align_up(pop_bytes), rest, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->t = hdr[0];
  c->hier_t = hdr[4];
  c->cur = 0;
  c->have_state = true;
  return EHDLB_OK;
}

extern "C" {

int64_t ehdlb_wetting_links(const ehdlb_ctx* c, int64_t* nodes, int32_t* dirs, int64_t cap) {
  if (!c) return EHDLB_EINVAL;
  if (!c->have_geometry) return EHDLB_ESTATE;
  const int64_t G = (int64_t)c->ghost_node.size();
  for (int64_t k = 0; k < std::min(G, cap); ++k) {
    if (nodes) nodes[k] = c->ghost_node[(size_t)k];
    if (dirs) dirs[k] = c->ghost_dir[(size_t)k];
  }
  return G;
}

size_t ehdlb_adjoint_workspace_bytes(const ehdlb_ctx* c, int64_t T, int32_t K) {
  if (!c || T < 1 || K < 1) return 0;
  ehdlb_ctx::Adj a;
  plan_adjoint(c, T, K, a);
  return a.total;
}

ehdlb_status ehdlb_forward_checkpointed(ehdlb_ctx* c, int64_t T, int32_t K, void* ws, size_t bytes) {
  if (!c) return EHDLB_EINVAL;
  if (T < 1 || K < 1) return fail(c, EHDLB_EINVAL, "T and K must be >= 1");
  if (!ws || ((uintptr_t)ws) % 256) return fail(c, EHDLB_EINVAL, "adjoint workspace must be 256-byte aligned");
  if (!c->have_state) return fail(c, EHDLB_ESTATE, "forward_checkpointed before set_phase");
  ehdlb_ctx::Adj a;
  plan_adjoint(c, T, K, a);
  if (bytes < a.total) return fail(c, EHDLB_ENOMEM, "adjoint workspace too small");
  a.ws = (char*)ws;
  a.bytes = bytes;
  a.t0 = c->t;
  c->adj = a;
  ++c->gen;
  c->grad_fwd = true;
  ehdlb_status st = dispatch<FwdCkptFn>(c, 0);
  c->grad_fwd = false;
  if (st) return st;
  c->adj.gen = c->gen;
  c->adj.ready = true;
  return EHDLB_OK;
}

ehdlb_status ehdlb_adjoint(ehdlb_ctx* c, const double* dL_dcentroid, const double* dL_dvelocity, int32_t electrode,
                           double* dL_dvolts) {
  if (!c) return EHDLB_EINVAL;
  if (!dL_dcentroid || !dL_dvelocity || !dL_dvolts) return fail(c, EHDLB_EINVAL, "null argument");
  if (electrode < 0 || electrode >= EHDLB_MAX_ELECTRODES) return fail(c, EHDLB_EINVAL, "electrode index out of range");
  if (!c->ehd) return fail(c, EHDLB_EINVAL, "adjoint with respect to voltages needs the field on");
  if (!c->adj.ready) return fail(c, EHDLB_ESTATE, "adjoint before forward_checkpointed");
  if (c->sched[electrode].v.size() > (size_t)c->adj.nvseg) return fail(c, EHDLB_EINVAL, "too many schedule segments");
  if (c->gen != c->adj.gen || c->t != c->adj.t0 + c->adj.T)
    return fail(c, EHDLB_ESTATE, "state or schedule changed since forward_checkpointed");
  c->grad_fwd = true;  // the recompute replays the checkpointed forward's solves
  const ehdlb_status st = dispatch<AdjFn>(c, dL_dcentroid, dL_dvelocity, (int)electrode, dL_dvolts);
  c->grad_fwd = false;
  return st;
}

ehdlb_status ehdlb_set_solver_options(ehdlb_ctx* c, double lo, double hi, double overcorrect,
                                      int32_t warm_start) {
  if (!c) return EHDLB_EINVAL;
  if (!(lo > 0.0 && hi > lo && hi <= 2.0)) return fail(c, EHDLB_EINVAL, "need 0 < lo < hi <= 2");
  if (!(overcorrect > 0.0 && overcorrect <= 4.0)) return fail(c, EHDLB_EINVAL, "over-correction must lie in (0, 4]");
  if (warm_start < 0 || warm_start > 4) return fail(c, EHDLB_EINVAL, "warm_start must be 0, 1, 2, 3 or 4");
  ++c->gen;
  c->mg_lo = lo;
  c->mg_hi = hi;
  c->mg_overcorrect = overcorrect;
  c->warm_mode = warm_start;
  return EHDLB_OK;
}

ehdlb_status ehdlb_set_timing(ehdlb_ctx* c, int32_t on) {
  if (!c) return EHDLB_EINVAL;
  if (on && c->ev.empty()) {
    c->ev.resize(4 * 256);
    for (auto& e : c->ev) HIPCHK(hipEventCreate(&e));
  }
  c->timing = on != 0;
  c->ev_used = 0;
  c->timed_steps = 0;
  c->acc_ms[0] = c->acc_ms[1] = c->acc_ms[2] = 0.0;
  return EHDLB_OK;
}

ehdlb_status ehdlb_timing(ehdlb_ctx* c, double* ms3, int64_t* steps) {
  if (!c || !ms3) return EHDLB_EINVAL;
  ehdlb_status st = flush_timing(c);
  if (st) return st;
  for (int j = 0; j < 3; ++j) ms3[j] = c->acc_ms[j];
  if (steps) *steps = c->timed_steps;
  return EHDLB_OK;
}

ehdlb_status ehdlb_solver_stats(ehdlb_ctx* c, int32_t reset, int64_t* counts, double* max_rel0) {
  if (!c) return EHDLB_EINVAL;
  for (int k = 0; k < 2; ++k) {
    if (counts) {
      counts[2 * k] = c->cg_hist[k].solves;
      counts[2 * k + 1] = c->cg_hist[k].iters;
    }
    if (max_rel0) max_rel0[k] = c->cg_hist[k].max_rel0;
    if (reset) {
      c->cg_hist[k].solves = c->cg_hist[k].iters = 0;
      c->cg_hist[k].max_rel0 = 0.0;
    }
  }
  return EHDLB_OK;
}

uint64_t ehdlb_generation(const ehdlb_ctx* c) { return c ? c->gen : 0; }

}  // extern "C"

// ============================================================================ bandwidth references
// Kernels with no arithmetic of the method, timed beside the fused step to give its memory
// traffic two ceilings: a copy at a given access width, and the fused step's own population
// access pattern (each population of a node loaded once, stored at the node its velocity points
// to).  They touch only the caller's buffers.
__global__ __launch_bounds__(256) void k_probe_copy16(const float4* __restrict__ a, float4* __restrict__ b,
                                                      size_t n) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

__global__ __launch_bounds__(256) void k_probe_copy4(const float* __restrict__ a, float* __restrict__ b,
                                                     size_t n) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

template <class L, int NF, bool NT>
__global__ __launch_bounds__(256) void k_probe_push(const float* __restrict__ a, float* __restrict__ b, int nx,
                                                    int ny, int nz) {
  const int64_t N = (int64_t)nx * ny * nz;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
  float v[NF * L::Q];
#pragma unroll
  for (int k = 0; k < NF * L::Q; ++k) {
    const float* p = a + (int64_t)k * N + i;
    v[k] = NT ? __builtin_nontemporal_load(p) : *p;
  }
#pragma unroll
  for (int k = 0; k < NF * L::Q; ++k) {
    const int q = k % L::Q;
    int xd = x + L::ex[q], yd = y + L::ey[q], zd = z + L::ez[q];
    xd = xd < 0 ? xd + nx : (xd >= nx ? xd - nx : xd);
    yd = yd < 0 ? yd + ny : (yd >= ny ? yd - ny : yd);
    zd = zd < 0 ? zd + nz : (zd >= nz ? zd - nz : zd);
    b[(int64_t)k * N + ((int64_t)zd * ny + yd) * nx + xd] = v[k];
  }
}

template <class L, bool NT>
static bool launch_probe_push(int nf, const float* a, float* b, const int32_t* n, hipStream_t s) {
  const int64_t N = (int64_t)n[0] * n[1] * n[2];
  const dim3 grid((unsigned)((N + 255) / 256)), block(256);
  switch (nf) {
    case 1: hipLaunchKernelGGL((k_probe_push<L, 1, NT>), grid, block, 0, s, a, b, n[0], n[1], n[2]); return true;
    case 2: hipLaunchKernelGGL((k_probe_push<L, 2, NT>), grid, block, 0, s, a, b, n[0], n[1], n[2]); return true;
    case 3: hipLaunchKernelGGL((k_probe_push<L, 3, NT>), grid, block, 0, s, a, b, n[0], n[1], n[2]); return true;
    case 4: hipLaunchKernelGGL((k_probe_push<L, 4, NT>), grid, block, 0, s, a, b, n[0], n[1], n[2]); return true;
    case 5: hipLaunchKernelGGL((k_probe_push<L, 5, NT>), grid, block, 0, s, a, b, n[0], n[1], n[2]); return true;
    default: return false;
  }
}

extern "C" {

ehdlb_status ehdlb_bandwidth_probe(int32_t kind, const void* src, void* dst, size_t bytes, const int32_t* dims,
                                   int32_t q, int32_t nf, void* stream) {
  if (!src || !dst || kind < 0 || kind > 3) return EHDLB_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (kind == 0) {
    if (bytes % 16 || ((uintptr_t)src | (uintptr_t)dst) % 16) return EHDLB_EINVAL;
    const size_t n = bytes / 16;
    if (n == 0) return EHDLB_OK;
    hipLaunchKernelGGL(k_probe_copy16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (const float4*)src,
                       (float4*)dst, n);
  } else if (kind == 1) {
    if (bytes % 4 || ((uintptr_t)src | (uintptr_t)dst) % 4) return EHDLB_EINVAL;
    const size_t n = bytes / 4;
    if (n == 0) return EHDLB_OK;
    hipLaunchKernelGGL(k_probe_copy4, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (const float*)src,
                       (float*)dst, n);
  } else {
    if (!dims || dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || nf < 1 || nf > 5) return EHDLB_EINVAL;
    if (!((q == 9 && dims[2] == 1) || q == 19)) return EHDLB_EINVAL;
    if (((uintptr_t)src | (uintptr_t)dst) % 4) return EHDLB_EINVAL;
    const int64_t N = (int64_t)dims[0] * dims[1] * dims[2];
    if (N > ((int64_t)1 << 31) || bytes < (size_t)nf * q * N * sizeof(float)) return EHDLB_EINVAL;
    const bool ok = kind == 2 ? (q == 9 ? launch_probe_push<D2Q9, false>(nf, (const float*)src, (float*)dst, dims, s)
                                        : launch_probe_push<D3Q19, false>(nf, (const float*)src, (float*)dst, dims, s))
                              : (q == 9 ? launch_probe_push<D2Q9, true>(nf, (const float*)src, (float*)dst, dims, s)
                                        : launch_probe_push<D3Q19, true>(nf, (const float*)src, (float*)dst, dims, s));
    if (!ok) return EHDLB_EINVAL;
  }
  return hipGetLastError() == hipSuccess ? EHDLB_OK : EHDLB_EHIP;
}

const char* ehdlb_last_error(const ehdlb_ctx* c) { return c ? c->err.c_str() : "null context"; }

void ehdlb_destroy(ehdlb_ctx* c) {
  if (!c) return;
  for (auto& e : c->ev) (void)hipEventDestroy(e);
  if (c->ev_ctl) (void)hipEventDestroy(c->ev_ctl);
  if (c->hctl_pin) (void)hipHostFree(c->hctl_pin);
  delete c;
}

}  // extern "C"
