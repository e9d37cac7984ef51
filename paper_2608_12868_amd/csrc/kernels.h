// Device kernels of the ternary EHD lattice-Boltzmann step (gfx950).
//
// Layout: structure of arrays.  Populations pop[family][q][node] with node =
// x + Nx*(y + Ny*z), families g (flow, stored as the deviation g - w), f1, f2,
// f3 (phase fields), h (charge).  Scalar fields [N], vector fields [D][N].
// One thread per node, x fastest, so every family/direction plane is streamed
// with unit stride.  Streaming is "push": a fluid node collides its own
// populations (aligned loads) and writes each post-collision value to the
// neighbour it moves to, or back into its own opposite slot when that
// neighbour is solid (halfway bounce-back); A/B buffers, so there are no
// in-place races and every fluid slot is written exactly once.
//
// Arithmetic type T is double (FP64 path) or float (FP32 path, flow stored as
// deviations).  Reductions and the potential solve's residual are FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "lattice.h"

namespace ehd {

constexpr int kBlock = 256;
constexpr int kMaxE = 4;
constexpr int kObs = 16;   // observable accumulators per block
constexpr int kCoarseMax = 48;  // cells of the coarsest potential level (dense inverse)

// ----------------------------------------------------------------------------- geometry helpers
struct Dims {
  int nx, ny, nz;
  int64_t N;
};

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on XCD b mod 8).
// Remap so that each XCD processes a contiguous eighth of the logical blocks: the stencil
// neighbours of a block (rows and planes away) then sit in the same XCD's L2.
constexpr int kXcd = 8;
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int per = nb / kXcd;
  if (b >= per * kXcd) return b;
  return (b % kXcd) * per + b / kXcd;
}
// global thread index over nodes, plain block order (kernels without stencils, and the 2D
// lattices, whose fields stay in the Infinity Cache)
__device__ __forceinline__ int64_t gidx() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
// global thread index of the one-thread-per-cell stencil kernels of the potential solver:
// XCD-aware block order, so that the rows above and below a block's cells are read through
// the same XCD's L2 (measured faster for these kernels, unlike the fused step)
__device__ __forceinline__ int64_t sidx() {
  return (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
}
// global thread index of the fused step, the adjoint passes and the potential operator's set-up
// on 3D lattices (plane = nx ny nodes, grid of whole blocks over the lattice): the blocks of each
// z plane form 8 contiguous bands of rows, one per XCD, each walked in order, so the rows above
// and below a block are read through the same XCD's L2, and the same rows of the next plane
// follow an eighth of a plane later (plain order when a plane is not a multiple of 8 blocks)
__device__ __forceinline__ int64_t band_idx(int64_t plane) {
  const int bpp = (int)(plane / blockDim.x);
  int b = blockIdx.x;
  if (plane % blockDim.x == 0 && bpp % kXcd == 0) {
    const int pz = b / bpp, r = b - pz * bpp;
    b = pz * bpp + (r % kXcd) * (bpp / kXcd) + r / kXcd;
  }
  return (int64_t)b * blockDim.x + threadIdx.x;
}
__device__ __forceinline__ int64_t band_idx(const Dims& d) { return band_idx((int64_t)d.nx * d.ny); }
// contiguous chunk [lo, hi) of a grid-stride kernel's index space for this block (fixed, so
// reductions keep a fixed order); chunks are multiples of the block size
__device__ __forceinline__ void chunk_range(int64_t n, int64_t& lo, int64_t& hi) {
  const int64_t nb = gridDim.x;
  const int64_t per = ((n + nb - 1) / nb + blockDim.x - 1) / blockDim.x * blockDim.x;
  lo = (int64_t)xcd_block(blockIdx.x, gridDim.x) * per;
  hi = lo + per < n ? lo + per : n;
}

// neighbour of (x, y, z) along link q (periodic wrap), computed on demand
template <class L>
__device__ __forceinline__ int neighbour(const Dims& d, int x, int y, int z, int q) {
  const int xx = wrap(x + L::ex[q], d.nx);
  const int yy = wrap(y + L::ey[q], d.ny);
  const int zz = wrap(z + L::ez[q], d.nz);
  return xx + d.nx * (yy + d.ny * zz);
}

template <class L>
__device__ __forceinline__ void neighbours(const Dims& d, int64_t node64, int (&nb)[L::Q]) {
  // node counts are validated below 2^31: 32-bit index arithmetic
  const int node = (int)node64;
  const int x = node % d.nx;
  const int t = node / d.nx;
  const int y = t % d.ny;
  const int z = t / d.ny;
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    const int xx = wrap(x + L::ex[q], d.nx);
    const int yy = wrap(y + L::ey[q], d.ny);
    const int zz = wrap(z + L::ez[q], d.nz);
    nb[q] = xx + d.nx * (yy + d.ny * zz);
  }
}

// ----------------------------------------------------------------------------- parameters
template <class T>
struct Phys {
  T W;            // interface width
  T ups[3], upsT; // Eq. 11
  T cos12, cos13, cos23;
  T s_phi;        // first-order rate of the phase fields, 1/(1/2 + M/cs2)
  T s_e;          // first-order rate of the charge, 1/(1/2 + alpha/cs2)
  T s_high;       // rate of the higher moments: order >= 2 (phase, charge), >= 3 (flow)
  T nu[3];        // kinematic viscosity per phase
  T rho[3];       // density per phase (all 1 unless the variable-density flow is selected)
  T eps[3], cond[3];
  T body[3];
};

template <class T>
struct Volts {
  T v[kMaxE];
  unsigned off;  // bit e: electrode e is switched off and floating (its faces insulate; v[e] = 0)
};

// Dirichlet face towards a solid neighbour of flag fm: grounded, or an electrode that is on
template <class T>
__device__ __forceinline__ bool dirichlet_face(uint8_t fm, const Volts<T>& volts) {
  return fm == 1 || (fm >= 3 && !((volts.off >> (fm - 3)) & 1u));
}

template <class T>
struct StepArgs {
  Dims d;
  const uint8_t* flags;
  const T* pop_in;
  T* pop_out;
  const T* phi;       // [3][N] at t, ghosts filled
  const T* phi_prev;  // [3][N] at t-1
  const T* rho;       // [N] at t
  const T* rho_prev;  // [N] at t-1
  const T* u_prev;    // [D][N] at t-1
  T* u_out;           // [D][N] at t
  const T* q_prev;    // [N]
  T* q_out;           // [N]
  const T* pot;       // [N]
  Phys<T> p;
  Volts<T> volts;
  T dt_on;            // 0 on the first step (no time derivatives), 1 afterwards
  T* rec;             // STORE: population moments for the adjoint, [kMom][N] (see mom_layout)
  const int* gate;    // if set, the launch does its work only when *gate != 0 (the solve stopped)
};

// Population moments a step's adjoint needs (the collision depends on the populations only
// through them): drho, j[D], the second-order raw moments Pi[P] of g - g_eq + F_q/2,
// jf[3][D] (first moments of the phase populations), jh[D] (first moment of the charge).
template <class L>
struct MomLayout {
  static constexpr int D = L::D;
  static constexpr int P = D == 2 ? 3 : 6;
  static constexpr int DRHO = 0, J = 1, PI = 1 + D, JF = 1 + D + P, JH = 1 + 4 * D + P;
  static constexpr int COUNT = 1 + 5 * D + P;
};

// Population load, with the non-temporal hint if NT.  Each population is read once per step;
// where the two population arrays exceed the 256 MB Infinity Cache, hinted loads keep them from
// evicting the phase, potential and flag values that neighbouring blocks re-read through L2.
template <bool NT, class T>
__device__ __forceinline__ T ld_pop(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

// ----------------------------------------------------------------------------- moments (Eq. 19)
// Zeroth moment of one population family per thread: blockIdx.y selects the family
// fam0 + blockIdx.y (0: flow deviation -> drho, 1..3: phase fields -> phi, 4: charge -> rho).
// Zero at solid nodes (the wetting kernel then overwrites the solid nodes next to fluid).
// NT: population loads with the non-temporal hint (ld_pop).
template <class L, class T, bool NT>
__global__ __launch_bounds__(kBlock) void k_moments(Dims d, const uint8_t* __restrict__ flags,
                                                     const T* __restrict__ pop, T* __restrict__ phi,
                                                     T* __restrict__ rho, T* __restrict__ drho, int fam0) {
  const int64_t node = gidx();
  if (node >= d.N) return;
  const int64_t N = d.N;
  const int fam = fam0 + (int)blockIdx.y;
  T s = 0;
  if (flags[node] == 0) {
    const T* p = pop + (int64_t)fam * L::Q * N + node;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) s += ld_pop<NT>(&p[(int64_t)q * N]);
  }
  if (fam == 0)
    drho[node] = s;
  else if (fam <= 3)
    phi[(int64_t)(fam - 1) * N + node] = s;
  else
    rho[node] = s;
}

// ----------------------------------------------------------------------------- wetting ghosts (Eq. 20)
// For solid node s with link e*: Phi_i(s) = Phi_i(s + e*) - |e*| * (4/W) * R_i,
// R_i the bracket of Eq. 20 evaluated with the fluid neighbour's values.
template <class T>
__global__ __launch_bounds__(kBlock) void k_ghosts(int64_t N, int G, const int32_t* __restrict__ gnode,
                                                    const int32_t* __restrict__ gsrc,
                                                    const T* __restrict__ glen, T* __restrict__ phi,
                                                    Phys<T> p) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= G) return;
  const int64_t s = gnode[k], f = gsrc[k];
  const T p1 = phi[f], p2 = phi[N + f], p3 = phi[2 * N + f];
  const T a = T(4) / p.W;
  const T r1 = a * (-p.cos13 * p1 * p3 - p.cos12 * p1 * p2);
  const T r2 = a * (p.cos12 * p1 * p2 - p.cos23 * p2 * p3);
  const T r3 = a * (p.cos23 * p2 * p3 + p.cos13 * p1 * p3);
  const T l = glen[k];
  phi[s] = p1 - l * r1;
  phi[N + s] = p2 - l * r2;
  phi[2 * N + s] = p3 - l * r3;
}

// ----------------------------------------------------------------------------- initial state
// Populations at rest equilibrium: f_i = w Phi_i, g - w = 0, h = w rho_e.  phi0/rho0 hold the
// initial fields (they double as the previous-step fields of the first step).
template <class L, class T, bool EHD>
__global__ __launch_bounds__(kBlock) void k_init(Dims d, const uint8_t* __restrict__ flags,
                                                  T* __restrict__ pop, T* __restrict__ phi0,
                                                  T* __restrict__ rho0, T* __restrict__ u_prev,
                                                  T* __restrict__ q_prev) {
  const int64_t node = gidx();
  if (node >= d.N) return;
  const int64_t N = d.N;
  const bool fluid = flags[node] == 0;
  T ph[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    ph[i] = fluid ? phi0[(int64_t)i * N + node] : T(0);
    phi0[(int64_t)i * N + node] = ph[i];
  }
  const T r = (EHD && fluid) ? rho0[node] : T(0);
  if (EHD) {
    rho0[node] = r;
    q_prev[node] = T(0);
  }
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    const T w = T(L::w36[q]) / T(36);
    pop[(int64_t)q * N + node] = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) pop[((int64_t)(1 + i) * L::Q + q) * N + node] = w * ph[i];
    if (EHD) pop[((int64_t)4 * L::Q + q) * N + node] = w * r;
  }
#pragma unroll
  for (int c = 0; c < L::D; ++c) u_prev[(int64_t)c * N + node] = T(0);
}

// ----------------------------------------------------------------------------- block reductions
// out[k * ostride] = the block's sum (or max) of v[k]; accumulate: added to what out holds
template <int K, bool MAX>
__device__ __forceinline__ void block_reduce(double (&v)[K], double* __restrict__ out, int64_t ostride = 1,
                                             bool accumulate = false) {
  __shared__ double sm[kBlock / 64][K];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double x = v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double y = __shfl_down(x, off, 64);
      x = MAX ? fmax(x, y) : x + y;
    }
    if (lane == 0) sm[wv][k] = x;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double x = sm[0][threadIdx.x];
    for (int w = 1; w < kBlock / 64; ++w) x = MAX ? fmax(x, sm[w][threadIdx.x]) : x + sm[w][threadIdx.x];
    out[threadIdx.x * ostride] = accumulate ? out[threadIdx.x * ostride] + x : x;
  }
}

// Sum (or max) of nblk partial rows of width K into out[K]; one block, fixed order.
template <int K, bool MAX>
__global__ __launch_bounds__(kBlock) void k_final(const double* __restrict__ part, int nblk,
                                                   double* __restrict__ out) {
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = MAX ? -INFINITY : 0.0;
  for (int b = threadIdx.x; b < nblk; b += kBlock) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = MAX ? fmax(v[k], part[(int64_t)b * K + k]) : v[k] + part[(int64_t)b * K + k];
  }
  block_reduce<K, MAX>(v, out);
}

// k_final for many partial rows: 1024 threads, fixed order (thread t sums rows t, t + 1024, ...,
// then a fixed tree over the 16 waves).  Row b, entry k is part[b * K + k].
constexpr int kFinalWide = 1024;
template <int K, bool MAX>
__device__ __forceinline__ void final_wide(const double* __restrict__ part, int nblk, double* __restrict__ out) {
  __shared__ double sm[kFinalWide / 64][K];
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = MAX ? -INFINITY : 0.0;
  for (int b = threadIdx.x; b < nblk; b += kFinalWide) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = MAX ? fmax(v[k], part[(int64_t)b * K + k]) : v[k] + part[(int64_t)b * K + k];
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double x = v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double y = __shfl_down(x, off, 64);
      x = MAX ? fmax(x, y) : x + y;
    }
    if (lane == 0) sm[wv][k] = x;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double x = sm[0][threadIdx.x];
    for (int w = 1; w < kFinalWide / 64; ++w) x = MAX ? fmax(x, sm[w][threadIdx.x]) : x + sm[w][threadIdx.x];
    out[threadIdx.x] = x;
  }
}
// Sums of K entries over nblk partial rows stored entry by entry (entry k of row b at
// part[k * nblk + b]), with 1024 threads: wave w reduces entries w, w + 16, ...; lane l adds rows
// l, l + 64, ... in that order (sixteen independent loads at a time), then a fixed shuffle tree.
// Each wave runs one short tree per entry instead of every wave running one per entry.
template <int K>
__device__ __forceinline__ void final_cols(const double* __restrict__ part, int nblk, double* __restrict__ out) {
  constexpr int kWaves = kFinalWide / 64, kRun = 16;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int k = wv; k < K; k += kWaves) {
    const double* col = part + (int64_t)k * nblk;
    double x = 0.0;
    for (int base = 0; base < nblk; base += 64 * kRun) {
      double v[kRun];
#pragma unroll
      for (int j = 0; j < kRun; ++j) {
        const int b = base + lane + 64 * j;
        v[j] = b < nblk ? col[b] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < kRun; ++j) x += v[j];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) out[k] = x;
  }
}

template <int K, bool MAX>
__global__ __launch_bounds__(kFinalWide) void k_final_wide(const double* __restrict__ part, int nblk,
                                                            double* __restrict__ out) {
  final_wide<K, MAX>(part, nblk, out);
}

// Sum (or max) of n per-block partials, evaluated by every block in the same fixed order as
// k_final and returned to every thread (blockDim.x == kBlock).  Lets a kernel consume the
// result of the previous kernel's reduction without a separate one-block launch.
template <bool MAX>
__device__ __forceinline__ double reduce_partials(const double* __restrict__ part, int n) {
  __shared__ double sm[kBlock / 64];
  double x = MAX ? -INFINITY : 0.0;
  for (int b = threadIdx.x; b < n; b += kBlock) x = MAX ? fmax(x, part[b]) : x + part[b];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double y = __shfl_down(x, off, 64);
    x = MAX ? fmax(x, y) : x + y;
  }
  __syncthreads();  // sm may still be read by a previous call
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = x;
  __syncthreads();
  double r = sm[0];
#pragma unroll
  for (int w = 1; w < kBlock / 64; ++w) r = MAX ? fmax(r, sm[w]) : r + sm[w];
  return r;
}

// Device-side state of one conjugate-gradient solve.  Every solver kernel returns at once
// when stop != 0, so the host can queue iterations ahead of the convergence decision.
struct CgCtl {
  double bmax;   // max|b|
  double floor;  // rounding floor of the relative residual (8 eps_T max_i sum_j |A_ij x_j| / max|b|)
  double rel;    // last FP64 relative residual max|b - A x| / max|b|
  double rel0;   // the same before the first iteration
  int stop;      // no further iteration
  int conv;      // stopped converged
  int zero;      // b == 0: x set to zero
  int iterated;  // the initial check did not already satisfy the tolerance
  int iters;     // iteration at which the solve stopped
  int pad[3];
};

// ----------------------------------------------------------------------------- observables (a10)
// Per-block FP64 partials: 0-2 masses, 3-5 sum x Phi1, 6-8 sum Phi1_prev u_prev,
// 9 sum Phi1_prev, 10 total charge, 11 count of non-finite values; block 2 of the
// output (max |sum Phi - 1|) is a separate max-partial.
template <class L, class T, bool EHD>
__global__ __launch_bounds__(kBlock) void k_obs(Dims d, const uint8_t* __restrict__ flags,
                                                 const T* __restrict__ phi, const T* __restrict__ phi_prev,
                                                 const T* __restrict__ u_prev, const T* __restrict__ rho,
                                                 double* __restrict__ part_sum, double* __restrict__ part_max) {
  const int64_t node = gidx();
  double v[kObs];
#pragma unroll
  for (int k = 0; k < kObs; ++k) v[k] = 0.0;
  double mx[1] = {0.0};
  if (node < d.N && flags[node] == 0) {
    const int64_t N = d.N;
    const double p1 = phi[node], p2 = phi[N + node], p3 = phi[2 * N + node];
    const double x = (double)(node % d.nx), y = (double)((node / d.nx) % d.ny),
                 z = (double)(node / ((int64_t)d.nx * d.ny));
    v[0] = p1;
    v[1] = p2;
    v[2] = p3;
    v[3] = x * p1;
    v[4] = y * p1;
    v[5] = z * p1;
    const double pp = phi_prev[node];
    v[6] = pp * (double)u_prev[node];
    v[7] = pp * (double)u_prev[N + node];
    if (L::D == 3) v[8] = pp * (double)u_prev[2 * N + node];
    v[9] = pp;
    if (EHD) v[10] = rho[node];
    const double s = p1 + p2 + p3;
    v[11] = (isfinite(s) && isfinite(v[6] + v[7] + v[8]) && isfinite(v[10])) ? 0.0 : 1.0;
    mx[0] = fabs(s - 1.0);
  }
  block_reduce<kObs, false>(v, part_sum + (int64_t)blockIdx.x * kObs);
  __syncthreads();
  block_reduce<1, true>(mx, part_max + blockIdx.x);
}

// ----------------------------------------------------------------------------- potential solver
// Finite-volume Gauss law on the axis faces: coefficients per level are explicit:
// cp[a][i] couples cell i with i + e_a (0 across solids), diag[i] includes the Dirichlet
// faces.  Level 0 is the lattice; coarser levels aggregate 2 (2D: 2x2, 3D: 2x2x2) cells
// with the Galerkin operator of piecewise-constant interpolation.
struct Level {
  int n[3];
  int64_t N;
};

template <int D>
__device__ __forceinline__ void cell_xyz(const Level& L, int64_t i64, int& x, int& y, int& z) {
  const int i = (int)i64;
  x = i % L.n[0];
  const int t = i / L.n[0];
  if (D == 3) {
    y = t % L.n[1];
    z = t / L.n[1];
  } else {
    y = t;
    z = 0;
  }
}

template <int D>
__device__ __forceinline__ int64_t cell_id(const Level& L, int x, int y, int z) {
  return (int64_t)(x + L.n[0] * (y + L.n[1] * z));
}

// index of the +axis and -axis neighbours of cell i at (x, y, z), periodic wrap, 32-bit
template <int D>
__device__ __forceinline__ void axis_pm(const Level& L, int i, int x, int y, int z, int ax, int& jp, int& jm) {
  if (ax == 0) {
    jp = x + 1 < L.n[0] ? i + 1 : i - (L.n[0] - 1);
    jm = x > 0 ? i - 1 : i + (L.n[0] - 1);
  } else if (ax == 1) {
    const int s = L.n[0];
    jp = y + 1 < L.n[1] ? i + s : i - (L.n[1] - 1) * s;
    jm = y > 0 ? i - s : i + (L.n[1] - 1) * s;
  } else {
    const int s = L.n[0] * L.n[1];
    jp = z + 1 < L.n[2] ? i + s : i - (L.n[2] - 1) * s;
    jm = z > 0 ? i - s : i + (L.n[2] - 1) * s;
  }
}

// Fine-level coefficients, right-hand side and permittivity from the phase fields.
template <class L, class T>
__global__ __launch_bounds__(kBlock) void k_pois_setup(Dims d, const uint8_t* __restrict__ flags,
                                                        const T* __restrict__ phi, const T* __restrict__ rho,
                                                        Phys<T> p, Volts<T> volts,
                                                        T* __restrict__ cp, T* __restrict__ diag,
                                                        T* __restrict__ dinv, T* __restrict__ b) {
  const int64_t node = L::D == 3 ? band_idx(d) : sidx();
  if (node >= d.N) return;
  const int64_t N = d.N;
  if (flags[node] != 0) {
    for (int ax = 0; ax < L::D; ++ax) cp[(int64_t)ax * N + node] = T(0);
    diag[node] = T(0);
    dinv[node] = T(0);
    b[node] = T(0);
    return;
  }
  const int x = (int)node % d.nx, yz = (int)node / d.nx, y = yz % d.ny, z = yz / d.ny;
  const T ex = p.eps[0] * phi[node] + p.eps[1] * phi[N + node] + p.eps[2] * phi[2 * N + node];
  T dg = 0, rhs = rho ? rho[node] : T(0);
  // axis neighbours only; their loads do not wait for the flag test
#pragma unroll
  for (int ax = 0; ax < L::D; ++ax) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int q = k == 0 ? L::axp[ax] : L::axm[ax];
      const int m = neighbour<L>(d, x, y, z, q);
      const uint8_t fm = flags[m];
      const T em = p.eps[0] * phi[m] + p.eps[1] * phi[N + m] + p.eps[2] * phi[2 * N + m];
      const bool fluid = fm == 0, dirichlet = dirichlet_face(fm, volts);
      const T c = fluid ? T(0.5) * (ex + em) : T(0);
      const T cd = T(2) * ex;
      dg += fluid ? c : (dirichlet ? cd : T(0));
      if (fm >= 3 && dirichlet) rhs += cd * volts.v[fm - 3];
      if (k == 0) cp[(int64_t)ax * N + node] = c;
    }
  }
  diag[node] = dg;
  dinv[node] = dg != T(0) ? T(1) / dg : T(0);
  b[node] = rhs;
}

// y = A x at one level (explicit coefficients), optionally with per-block FP64 partials of x.y.
// Grid-stride loop: the grid is capped so the partials stay few.
template <int D, class T>
__device__ __forceinline__ T apply_row(const Level& L, const T* __restrict__ cp, T dg, const T* __restrict__ x,
                                       int64_t i64) {
  const int i = (int)i64;
  int cx, cy, cz;
  cell_xyz<D>(L, i, cx, cy, cz);
  const int N = (int)L.N;
  T r = dg * x[i];
#pragma unroll
  for (int ax = 0; ax < D; ++ax) {
    int jp, jm;
    axis_pm<D>(L, i, cx, cy, cz, ax, jp, jm);
    r -= cp[ax * N + i] * x[jp] + cp[ax * N + jm] * x[jm];
  }
  return r;
}

// Smoothing polynomial of the V-cycle: z <- z + c1 y - c2 D^-1 A y with y = D^-1 (r - A z)
// (degree-2 polynomial in D^-1 A; c1 = 2w, c2 = w^2 is two damped-Jacobi sweeps).
// Pre-smoothing from z = 0 in one pass: z = (c1 - c2) y + c2 dinv sum_faces c y(nb), y = dinv r.
template <int D, class T>
__global__ __launch_bounds__(kBlock) void k_smooth2(const int* __restrict__ stop, Level L, const T* __restrict__ cp,
                                                     const T* __restrict__ dinv, const T* __restrict__ r,
                                                     T* __restrict__ z, T c1, T c2) {
  if (*stop) return;
  const int i = (int)sidx();
  if (i >= (int)L.N) return;
  const T di = dinv[i];
  const int N = (int)L.N;
  int cx, cy, cz;
  cell_xyz<D>(L, i, cx, cy, cz);
  T off = 0;  // absent faces have c = 0 and inactive cells dinv = 0
#pragma unroll
  for (int ax = 0; ax < D; ++ax) {
    int jp, jm;
    axis_pm<D>(L, i, cx, cy, cz, ax, jp, jm);
    off += cp[ax * N + i] * r[jp] * dinv[jp] + cp[ax * N + jm] * r[jm] * dinv[jm];
  }
  z[i] = (c1 - c2) * r[i] * di + c2 * di * off;
}

// Post-smoothing, pass 1: prolongation z' = z + a zc(parent) (on the fly, also at the
// neighbours) and y = dinv (r - A z').
template <int D, class T>
__global__ __launch_bounds__(kBlock) void k_prolong_resid(const int* __restrict__ stop, Level L,
                                                           const T* __restrict__ cp, const T* __restrict__ dg,
                                                           const T* __restrict__ dinv, const T* __restrict__ r,
                                                           const T* __restrict__ z, Level Lc, const T* __restrict__ zc,
                                                           T a, T* __restrict__ y) {
  if (*stop) return;
  const int i = (int)sidx();
  if (i >= (int)L.N) return;
  const T di = dinv[i];
  const int N = (int)L.N;
  int cx, cy, cz;
  cell_xyz<D>(L, i, cx, cy, cz);
  // inactive cells hold z = 0, inactive parents zc = 0 and absent faces c = 0
  auto par = [&](int x, int yy, int zz) -> int { return (x >> 1) + Lc.n[0] * ((yy >> 1) + Lc.n[1] * (zz >> 1)); };
  const T zi = di != T(0) ? z[i] + a * zc[par(cx, cy, cz)] : T(0);
  T az = dg[i] * zi;
#pragma unroll
  for (int ax = 0; ax < D; ++ax) {
    int jp, jm;
    axis_pm<D>(L, i, cx, cy, cz, ax, jp, jm);
    int xp = cx, yp = cy, zp = cz, xm = cx, ym = cy, zm = cz;
    if (ax == 0) { xp = wrap(cx + 1, L.n[0]); xm = wrap(cx - 1, L.n[0]); }
    if (ax == 1) { yp = wrap(cy + 1, L.n[1]); ym = wrap(cy - 1, L.n[1]); }
    if (ax == 2) { zp = wrap(cz + 1, L.n[2]); zm = wrap(cz - 1, L.n[2]); }
    az -= cp[ax * N + i] * (z[jp] + a * zc[par(xp, yp, zp)]) + cp[ax * N + jm] * (z[jm] + a * zc[par(xm, ym, zm)]);
  }
  y[i] = (r[i] - az) * di;
}

// Post-smoothing, pass 2: z_out = z' + (c1 - c2) y + c2 dinv sum_faces c y(nb), z' = z + a zc
// (zc == nullptr: z' = z), optionally with per-block FP64 partials of r.z_out (grid-stride).
template <int D, class T, bool DOT>
__global__ __launch_bounds__(kBlock) void k_poly_post(const int* __restrict__ stop, Level L,
                                                       const T* __restrict__ cp, const T* __restrict__ dinv,
                                                       const T* __restrict__ r, const T* __restrict__ z,
                                                       Level Lc, const T* __restrict__ zc, T a,
                                                       const T* __restrict__ y, T c1, T c2, T* __restrict__ zo,
                                                       double* __restrict__ part) {
  if (*stop) return;
  double acc[1] = {0.0};
  int64_t lo_, hi_;
  if (DOT) {
    chunk_range(L.N, lo_, hi_);
  } else {
    lo_ = sidx();
    hi_ = lo_ < L.N ? lo_ + 1 : lo_;
  }
  const int N = (int)L.N;
  for (int64_t i64 = DOT ? lo_ + threadIdx.x : lo_; i64 < hi_; i64 += DOT ? blockDim.x : 1) {
    const int i = (int)i64;
    const T di = dinv[i];
    int cx, cy, cz;
    cell_xyz<D>(L, i, cx, cy, cz);
    T off = 0;
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      int jp, jm;
      axis_pm<D>(L, i, cx, cy, cz, ax, jp, jm);
      off += cp[ax * N + i] * y[jp] + cp[ax * N + jm] * y[jm];
    }
    T zi = z[i];
    if (zc) zi += a * zc[(cx >> 1) + Lc.n[0] * ((cy >> 1) + Lc.n[1] * (cz >> 1))];
    const T v = di != T(0) ? zi + (c1 - c2) * y[i] + c2 * di * off : T(0);
    zo[i] = v;
    if (DOT) acc[0] += (double)r[i] * (double)v;
  }
  if (DOT) block_reduce<1, false>(acc, part + blockIdx.x);
}

// alpha = rz / pq from the partials of r.z (previous preconditioning) and p.q (this
// iteration's product); x += alpha p, r -= alpha q, with per-block FP64 partials of max|r|
// (grid-stride)
template <class T>
__global__ __launch_bounds__(kBlock) void k_cg_update_max(const CgCtl* __restrict__ ctl, int64_t N,
                                                           const double* __restrict__ prz,
                                                           const double* __restrict__ ppq, int nblk,
                                                           const T* __restrict__ p, const T* __restrict__ q,
                                                           T* __restrict__ x, T* __restrict__ r,
                                                           double* __restrict__ part) {
  if (ctl->stop) return;
  const double rz = reduce_partials<false>(prz, nblk);
  const double pq = reduce_partials<false>(ppq, nblk);
  const T al = (T)(pq != 0.0 ? rz / pq : 0.0);
  double m[1] = {0.0};
  for (int64_t i = gidx(); i < N; i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += al * p[i];
    const T rn = r[i] - al * q[i];
    r[i] = rn;
    m[0] = fmax(m[0], fabs((double)rn));
  }
  block_reduce<1, true>(m, part + blockIdx.x);
}

// p = z + beta p with beta = rz_new / rz_old from the partials of the last two
// preconditionings (first: p = z) (grid-stride)
template <class T>
__global__ __launch_bounds__(kBlock) void k_cg_dir(const CgCtl* __restrict__ ctl, int64_t N,
                                                    const double* __restrict__ prz_new,
                                                    const double* __restrict__ prz_old, int nblk, int first,
                                                    const T* __restrict__ z, T* __restrict__ p) {
  if (ctl->stop) return;
  int64_t lo, hi;
  chunk_range(N, lo, hi);
  if (first) {
    for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) p[i] = z[i];
    return;
  }
  const double rn = reduce_partials<false>(prz_new, nblk);
  const double ro = reduce_partials<false>(prz_old, nblk);
  const T beta = (T)(ro != 0.0 ? rn / ro : 0.0);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) p[i] = z[i] + beta * p[i];
}

// q = A p with per-block FP64 partials of p.q (grid-stride)
template <int D, class T>
__global__ __launch_bounds__(kBlock) void k_spmv(const CgCtl* __restrict__ ctl, Level L, const T* __restrict__ cp,
                                                  const T* __restrict__ diag, const T* __restrict__ p,
                                                  T* __restrict__ q, double* __restrict__ part) {
  if (ctl->stop) return;
  double acc[1] = {0.0};
  int64_t lo, hi;
  chunk_range(L.N, lo, hi);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
    const T dg = diag[i];
    const T r = dg != T(0) ? apply_row<D, T>(L, cp, dg, p, i) : T(0);
    q[i] = r;
    acc[0] += (double)p[i] * (double)r;
  }
  block_reduce<1, false>(acc, part + blockIdx.x);
}

// ---- V-cycle tail: every level from `first` to the coarsest in one workgroup ---------------
// The working vectors r, z, y of the tail levels live in LDS (gfx950: 160 KiB per CU); the
// coefficients stay in global memory, where they are L2-resident.  Only r of level `first` is
// read from and z of level `first` written to global memory.
constexpr int kMaxLevels = 16;
constexpr int kTailThreads = 1024;
constexpr int kTailLdsBytes = 144 * 1024;
template <class T>
struct TailArgs {
  int first, last;  // level indices handled here; last = coarsest
  int lds[kMaxLevels];  // element offset of level l's [r | z | y] in the tail's LDS
  Level L[kMaxLevels];
  T* cp[kMaxLevels];
  T* dg[kMaxLevels];
  T* di[kMaxLevels];
  T* r[kMaxLevels];
  T* z[kMaxLevels];
  T* t[kMaxLevels];
  const double* inv;  // dense inverse of the coarsest operator
  T c1, c2, a;        // smoothing polynomial and coarse-correction scale
  const int* stop;    // the solve's stop flag (nothing to do when set)
};

// One level of the tail, every pass over the level's cells with independent loads only.
// Pre-smoothing from zero: z = (c1 - c2) dinv r + c2 dinv sum_faces c dinv(nb) r(nb).
template <int D, class T>
__device__ __forceinline__ void tail_pre(const Level& L, const T* cp, const T* di, const T* r, T* z, T c1, T c2) {
  const int N = (int)L.N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    int cx, cy, cz;
    cell_xyz<D>(L, i, cx, cy, cz);
    T off = 0;
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      int jp, jm;
      axis_pm<D>(L, i, cx, cy, cz, ax, jp, jm);
      off += cp[ax * N + i] * r[jp] * di[jp] + cp[ax * N + jm] * r[jm] * di[jm];
    }
    const T d = di[i];
    z[i] = (c1 - c2) * r[i] * d + c2 * d * off;
  }
}
// Residual of every cell of the level, y = r - A z' (inactive cells 0), with z' = z + a zc(parent)
// when zc != nullptr (prolongation evaluated on the fly), optionally scaled by dinv.
template <int D, class T>
__device__ __forceinline__ void tail_resid(const Level& L, const T* cp, const T* dg, const T* di, const T* r,
                                           const T* z, const Level& Lc, const T* zc, T a, bool scale, T* y) {
  const int N = (int)L.N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    int cx, cy, cz;
    cell_xyz<D>(L, i, cx, cy, cz);
    auto zp = [&](int j, int x, int yy, int zz) -> T {
      return zc ? z[j] + a * zc[cell_id<D>(Lc, x >> 1, yy >> 1, zz >> 1)] : z[j];
    };
    const T d = dg[i];
    T az = d * zp(i, cx, cy, cz);
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      int jp, jm;
      axis_pm<D>(L, i, cx, cy, cz, ax, jp, jm);
      int xp = cx, yp = cy, zp_ = cz, xm = cx, ym = cy, zm = cz;
      if (ax == 0) { xp = wrap(cx + 1, L.n[0]); xm = wrap(cx - 1, L.n[0]); }
      if (ax == 1) { yp = wrap(cy + 1, L.n[1]); ym = wrap(cy - 1, L.n[1]); }
      if (ax == 2) { zp_ = wrap(cz + 1, L.n[2]); zm = wrap(cz - 1, L.n[2]); }
      az -= cp[ax * N + i] * zp(jp, xp, yp, zp_) + cp[ax * N + jm] * zp(jm, xm, ym, zm);
    }
    const T res = d != T(0) ? r[i] - az : T(0);
    y[i] = scale ? res * di[i] : res;
  }
}
// Restriction: coarse residual = sum of the children's residuals y
template <int D, class T>
__device__ __forceinline__ void tail_restrict(const Level& L, const T* y, const Level& Lc, T* rc) {
  for (int I = threadIdx.x; I < (int)Lc.N; I += blockDim.x) {
    int X, Yc, Zc;
    cell_xyz<D>(Lc, I, X, Yc, Zc);
    T acc = 0;
    for (int dz = 0; dz < (D == 3 ? 2 : 1); ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const int cx = 2 * X + dx, cy = 2 * Yc + dy, cz = 2 * Zc + dz;
          if (cx >= L.n[0] || cy >= L.n[1] || (D == 3 && cz >= L.n[2])) continue;
          acc += y[cell_id<D>(L, cx, cy, cz)];
        }
    rc[I] = acc;
  }
}
// Post-smoothing: z = z' + (c1 - c2) y + c2 dinv sum_faces c y(nb), z' = z + a zc(parent)
template <int D, class T>
__device__ __forceinline__ void tail_post(const Level& L, const T* cp, const T* di, const T* y, T* z,
                                          const Level& Lc, const T* zc, T a, T c1, T c2) {
  const int N = (int)L.N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    int cx, cy, cz;
    cell_xyz<D>(L, i, cx, cy, cz);
    T off = 0;
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      int jp, jm;
      axis_pm<D>(L, i, cx, cy, cz, ax, jp, jm);
      off += cp[ax * N + i] * y[jp] + cp[ax * N + jm] * y[jm];
    }
    const T d = di[i];
    const T zi = z[i] + a * zc[cell_id<D>(Lc, cx >> 1, cy >> 1, cz >> 1)];
    z[i] = d != T(0) ? zi + (c1 - c2) * y[i] + c2 * d * off : T(0);
  }
}

template <int D, class T>
__global__ __launch_bounds__(kTailThreads) void k_vcycle_tail(TailArgs<T> a) {
  if (*a.stop) return;
  __shared__ __align__(16) unsigned char lds_raw[kTailLdsBytes];
  T* const lds = reinterpret_cast<T*>(lds_raw);
  auto R = [&](int l) { return lds + a.lds[l]; };
  auto Z = [&](int l) { return lds + a.lds[l] + a.L[l].N; };
  auto Y = [&](int l) { return lds + a.lds[l] + 2 * a.L[l].N; };
  for (int64_t i = threadIdx.x; i < a.L[a.first].N; i += blockDim.x) R(a.first)[i] = a.r[a.first][i];
  __syncthreads();
  // descend: pre-smooth from zero, residual, restriction
  for (int l = a.first; l < a.last; ++l) {
    const Level& L = a.L[l];
    tail_pre<D, T>(L, a.cp[l], a.di[l], R(l), Z(l), a.c1, a.c2);
    __syncthreads();
    tail_resid<D, T>(L, a.cp[l], a.dg[l], a.di[l], R(l), Z(l), L, (const T*)nullptr, T(0), false, Y(l));
    __syncthreads();
    tail_restrict<D, T>(L, Y(l), a.L[l + 1], R(l + 1));
    __syncthreads();
  }
  // coarsest: dense inverse
  {
    const Level& L = a.L[a.last];
    const int n = (int)L.N;
    const T* rc = R(a.last);
    T* zc = Z(a.last);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      double acc = 0.0;
      for (int j = 0; j < n; ++j) acc += a.inv[i * n + j] * (double)rc[j];
      zc[i] = a.dg[a.last][i] == T(0) ? T(0) : (T)acc;
    }
    __syncthreads();
  }
  // ascend: y = dinv (r - A z') and z = z' + smoothing, the prolongation z' = z + a zc on the fly
  for (int l = a.last - 1; l >= a.first; --l) {
    const Level& L = a.L[l];
    const Level& Lc = a.L[l + 1];
    tail_resid<D, T>(L, a.cp[l], a.dg[l], a.di[l], R(l), Z(l), Lc, Z(l + 1), a.a, true, Y(l));
    __syncthreads();
    tail_post<D, T>(L, a.cp[l], a.di[l], Y(l), Z(l), Lc, Z(l + 1), a.a, a.c1, a.c2);
    __syncthreads();
  }
  for (int64_t i = threadIdx.x; i < a.L[a.first].N; i += blockDim.x) a.z[a.first][i] = Z(a.first)[i];
}

// Tail setup: Galerkin coarsening of levels first+1..last and the dense coarsest inverse
// (Gauss-Jordan, FP64, one workgroup).
template <int D, class T>
__device__ void coarsen_level(const Level& Lf, const T* cpf, const T* diagf, const Level& Lc, T* cpc, T* diagc,
                              T* dinvc) {
  for (int64_t I = threadIdx.x; I < Lc.N; I += blockDim.x) {
    int X, Y, Z;
    cell_xyz<D>(Lc, I, X, Y, Z);
    T dg = 0;
    T c[3] = {0, 0, 0};
    for (int dz = 0; dz < (D == 3 ? 2 : 1); ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const int cx = 2 * X + dx, cy = 2 * Y + dy, cz = 2 * Z + dz;
          if (cx >= Lf.n[0] || cy >= Lf.n[1] || (D == 3 && cz >= Lf.n[2])) continue;
          const int64_t i = cell_id<D>(Lf, cx, cy, cz);
          dg += diagf[i];
          for (int ax = 0; ax < D; ++ax) {
            const T f = cpf[(int64_t)ax * Lf.N + i];
            int jx = cx, jy = cy, jz = cz;
            if (ax == 0) jx = wrap(cx + 1, Lf.n[0]);
            if (ax == 1) jy = wrap(cy + 1, Lf.n[1]);
            if (ax == 2) jz = wrap(cz + 1, Lf.n[2]);
            if ((jx >> 1) == X && (jy >> 1) == Y && (jz >> 1) == Z)
              dg -= T(2) * f;
            else
              c[ax] += f;
          }
        }
    diagc[I] = dg;
    dinvc[I] = dg != T(0) ? T(1) / dg : T(0);
    for (int ax = 0; ax < D; ++ax) cpc[(int64_t)ax * Lc.N + I] = c[ax];
  }
}

template <int D, class T>
__global__ __launch_bounds__(kTailThreads) void k_tail_setup(TailArgs<T> a, double* __restrict__ inv) {
  if (*a.stop) return;
  for (int l = a.first; l < a.last; ++l) {
    coarsen_level<D, T>(a.L[l], a.cp[l], a.dg[l], a.L[l + 1], a.cp[l + 1], a.dg[l + 1], a.di[l + 1]);
    __syncthreads();
  }
  __shared__ double A[kCoarseMax][2 * kCoarseMax + 1];
  const Level& L = a.L[a.last];
  const int n = (int)L.N;
  const T* cp = a.cp[a.last];
  const T* dg = a.dg[a.last];
  // augmented [A | I]
  for (int k = threadIdx.x; k < n * 2 * n; k += blockDim.x) {
    const int r = k / (2 * n), c = k % (2 * n);
    A[r][c] = c >= n ? (c - n == r ? 1.0 : 0.0) : 0.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double d = dg[i];
    A[i][i] = d == 0.0 ? 1.0 : d;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < n; ++i) {
      if (dg[i] == T(0)) continue;
      int cx, cy, cz;
      cell_xyz<D>(L, i, cx, cy, cz);
      for (int ax = 0; ax < D; ++ax) {
        int xp = cx, yp = cy, zp = cz;
        if (ax == 0) xp = wrap(cx + 1, L.n[0]);
        if (ax == 1) yp = wrap(cy + 1, L.n[1]);
        if (ax == 2) zp = wrap(cz + 1, L.n[2]);
        const int j = (int)cell_id<D>(L, xp, yp, zp);
        const double c = cp[(int64_t)ax * L.N + i];
        if (c != 0.0 && j != i) {
          A[i][j] -= c;
          A[j][i] -= c;
        }
      }
    }
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double piv = A[k][k];
    __syncthreads();
    for (int c = threadIdx.x; c < 2 * n; c += blockDim.x) A[k][c] /= piv;
    __syncthreads();
    for (int e = threadIdx.x; e < n * 2 * n; e += blockDim.x) {
      const int r = e / (2 * n), c = e % (2 * n);
      if (r == k || c == k) continue;
      A[r][c] -= A[r][k] * A[k][c];
    }
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += blockDim.x)
      if (r != k) A[r][k] = 0.0;
    __syncthreads();
  }
  for (int k = threadIdx.x; k < n * n; k += blockDim.x) inv[k] = A[k / n][n + k % n];
}

// Restriction of the residual r - A z by fine-cell threads.  A block is a tile of whole
// 2-per-axis aggregates, 64 x 2 x 2 fine cells in 3D (128 x 2 in 2D); each thread forms the
// residual of its own cell (independent loads, like the smoother), x pairs are summed across
// adjacent lanes and the y/z pairs through LDS.  Grid: ceil(nx/TX) x ceil(ny/2) x ceil(nz/2).
template <int D>
constexpr int restrict_tile_x() { return D == 3 ? 64 : 128; }
template <int D, class T>
__global__ __launch_bounds__(kBlock) void k_restrict_tile(const int* __restrict__ stop, Level Lf,
                                                           const T* __restrict__ cp, const T* __restrict__ diag,
                                                           const T* __restrict__ r, const T* __restrict__ z,
                                                           Level Lc, T* __restrict__ rc) {
  if (*stop) return;
  constexpr int TX = restrict_tile_x<D>();
  constexpr int NS = D == 3 ? 4 : 2;  // fine rows per tile: (dy, dz)
  constexpr int NP = TX / 2;          // coarse cells per tile
  const int ntx = (Lf.n[0] + TX - 1) / TX;
  const int nty = (Lf.n[1] + 1) / 2;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int bx = b % ntx;
  const int by = (b / ntx) % nty;
  const int bz = D == 3 ? b / (ntx * nty) : 0;
  const int t = threadIdx.x;
  const int tx = t % TX, sub = t / TX;
  const int cx = bx * TX + tx, cy = 2 * by + (sub & 1), cz = 2 * bz + (sub >> 1);
  T res = 0;
  if (cx < Lf.n[0] && cy < Lf.n[1] && (D == 2 || cz < Lf.n[2])) {
    const int i = (int)cell_id<D>(Lf, cx, cy, cz);
    const T dg = diag[i];
    if (dg != T(0)) res = r[i] - apply_row<D, T>(Lf, cp, dg, z, i);
  }
  res += __shfl_xor(res, 1, 64);
  __shared__ T sm[NS][NP];
  if ((tx & 1) == 0) sm[sub][tx >> 1] = res;
  __syncthreads();
  if (t < NP) {
    T acc = 0;
#pragma unroll
    for (int k = 0; k < NS; ++k) acc += sm[k][t];
    const int X = bx * NP + t;
    if (X < Lc.n[0]) rc[cell_id<D>(Lc, X, by, bz)] = acc;
  }
}

// ---- small levels: the four passes of a level fused into two by recomputation -----------
// On small levels the kernels are launch-latency bound, so each thread can recompute what it
// needs at its neighbours (from L2-resident data) instead of waiting for a separate pass.  The
// values a thread recomputes are bit-identical to those the owning thread stores: both call the
// same device functions.  Measured on MI355X: faster for 2D levels of up to 128K cells (5-point
// stencil), slower for 3D levels (the 7-point recomputation costs more than the launch saved),
// so only 2D levels use it.
template <int D>
constexpr int64_t small_level_max() { return D == 2 ? 131072 : 0; }

// coordinates of the +axis (sgn = 1) or -axis (sgn = -1) neighbour, periodic wrap
template <int D>
__device__ __forceinline__ void nbr_xyz(const Level& L, int x, int y, int z, int ax, int sgn, int& xo, int& yo,
                                        int& zo) {
  xo = x;
  yo = y;
  zo = z;
  if (ax == 0) xo = wrap(x + sgn, L.n[0]);
  if (ax == 1) yo = wrap(y + sgn, L.n[1]);
  if (ax == 2) zo = wrap(z + sgn, L.n[2]);
}

// pre-smoothing from zero at cell p = (x, y, z) (the formula of k_smooth2)
template <int D, class T>
__device__ __forceinline__ T pre_smooth_at(const Level& L, const T* __restrict__ cp, const T* __restrict__ di,
                                           const T* __restrict__ r, int p, int x, int y, int z, T c1, T c2) {
  const int N = (int)L.N;
  T off = 0;
#pragma unroll
  for (int ax = 0; ax < D; ++ax) {
    int jp, jm;
    axis_pm<D>(L, p, x, y, z, ax, jp, jm);
    off += cp[ax * N + p] * r[jp] * di[jp] + cp[ax * N + jm] * r[jm] * di[jm];
  }
  const T d = di[p];
  return (c1 - c2) * r[p] * d + c2 * d * off;
}

// Down pass of a small level: z = pre-smoothing of r (written), and the restriction of
// r - A z (tiles of whole aggregates as in k_restrict_tile; the neighbours' z recomputed).
template <int D, class T>
__global__ __launch_bounds__(kBlock) void k_down_small(const int* __restrict__ stop, Level Lf,
                                                        const T* __restrict__ cp, const T* __restrict__ diag,
                                                        const T* __restrict__ di, const T* __restrict__ r,
                                                        T* __restrict__ z, Level Lc, T* __restrict__ rc, T c1, T c2) {
  if (*stop) return;
  constexpr int TX = restrict_tile_x<D>();
  constexpr int NS = D == 3 ? 4 : 2;
  constexpr int NP = TX / 2;
  const int ntx = (Lf.n[0] + TX - 1) / TX;
  const int nty = (Lf.n[1] + 1) / 2;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int bx = b % ntx;
  const int by = (b / ntx) % nty;
  const int bz = D == 3 ? b / (ntx * nty) : 0;
  const int t = threadIdx.x;
  const int tx = t % TX, sub = t / TX;
  const int cx = bx * TX + tx, cy = 2 * by + (sub & 1), cz = 2 * bz + (sub >> 1);
  T res = 0;
  if (cx < Lf.n[0] && cy < Lf.n[1] && (D == 2 || cz < Lf.n[2])) {
    const int N = (int)Lf.N;
    const int i = (int)cell_id<D>(Lf, cx, cy, cz);
    const T zi = pre_smooth_at<D, T>(Lf, cp, di, r, i, cx, cy, cz, c1, c2);
    z[i] = zi;
    const T dg = diag[i];
    if (dg != T(0)) {
      T az = dg * zi;
#pragma unroll
      for (int ax = 0; ax < D; ++ax) {
        int jp, jm, xp, yp, zp, xm, ym, zm;
        axis_pm<D>(Lf, i, cx, cy, cz, ax, jp, jm);
        nbr_xyz<D>(Lf, cx, cy, cz, ax, 1, xp, yp, zp);
        nbr_xyz<D>(Lf, cx, cy, cz, ax, -1, xm, ym, zm);
        az -= cp[ax * N + i] * pre_smooth_at<D, T>(Lf, cp, di, r, jp, xp, yp, zp, c1, c2) +
              cp[ax * N + jm] * pre_smooth_at<D, T>(Lf, cp, di, r, jm, xm, ym, zm, c1, c2);
      }
      res = r[i] - az;
    }
  }
  res += __shfl_xor(res, 1, 64);
  __shared__ T sm[NS][NP];
  if ((tx & 1) == 0) sm[sub][tx >> 1] = res;
  __syncthreads();
  if (t < NP) {
    T acc = 0;
#pragma unroll
    for (int k = 0; k < NS; ++k) acc += sm[k][t];
    const int X = bx * NP + t;
    if (X < Lc.n[0]) rc[cell_id<D>(Lc, X, by, bz)] = acc;
  }
}

// prolongated correction z' = z + a zc(parent) at cell p = (x, y, zz)
template <int D, class T>
__device__ __forceinline__ T zprime_at(const T* __restrict__ z, const Level& Lc, const T* __restrict__ zc, T a,
                                       int p, int x, int y, int zz) {
  return z[p] + a * zc[(x >> 1) + Lc.n[0] * ((y >> 1) + Lc.n[1] * (zz >> 1))];
}
// y = dinv (r - A z') at cell p = (x, y, zz) (0 on inactive cells)
template <int D, class T>
__device__ __forceinline__ T post_resid_at(const Level& L, const T* __restrict__ cp, const T* __restrict__ dg,
                                           const T* __restrict__ di, const T* __restrict__ r,
                                           const T* __restrict__ z, const Level& Lc, const T* __restrict__ zc, T a,
                                           int p, int x, int y, int zz) {
  const T d = di[p];
  if (d == T(0)) return T(0);
  const int N = (int)L.N;
  T az = dg[p] * zprime_at<D, T>(z, Lc, zc, a, p, x, y, zz);
#pragma unroll
  for (int ax = 0; ax < D; ++ax) {
    int jp, jm, xp, yp, zp, xm, ym, zm;
    axis_pm<D>(L, p, x, y, zz, ax, jp, jm);
    nbr_xyz<D>(L, x, y, zz, ax, 1, xp, yp, zp);
    nbr_xyz<D>(L, x, y, zz, ax, -1, xm, ym, zm);
    az -= cp[ax * N + p] * zprime_at<D, T>(z, Lc, zc, a, jp, xp, yp, zp) +
          cp[ax * N + jm] * zprime_at<D, T>(z, Lc, zc, a, jm, xm, ym, zm);
  }
  return (r[p] - az) * d;
}
// Up pass of a small level: zo = z' + (c1 - c2) y + c2 dinv sum_faces c y(nb), with y and z'
// recomputed at the neighbours; zo is a different buffer from z.
template <int D, class T>
__global__ __launch_bounds__(kBlock) void k_up_small(const int* __restrict__ stop, Level L, const T* __restrict__ cp,
                                                      const T* __restrict__ dg, const T* __restrict__ di,
                                                      const T* __restrict__ r, const T* __restrict__ z, Level Lc,
                                                      const T* __restrict__ zc, T a, T c1, T c2, T* __restrict__ zo) {
  if (*stop) return;
  const int i = (int)sidx();
  if (i >= (int)L.N) return;
  const T d = di[i];
  if (d == T(0)) {
    zo[i] = T(0);
    return;
  }
  const int N = (int)L.N;
  int cx, cy, cz;
  cell_xyz<D>(L, i, cx, cy, cz);
  T off = 0;
#pragma unroll
  for (int ax = 0; ax < D; ++ax) {
    int jp, jm, xp, yp, zp, xm, ym, zm;
    axis_pm<D>(L, i, cx, cy, cz, ax, jp, jm);
    nbr_xyz<D>(L, cx, cy, cz, ax, 1, xp, yp, zp);
    nbr_xyz<D>(L, cx, cy, cz, ax, -1, xm, ym, zm);
    off += cp[ax * N + i] * post_resid_at<D, T>(L, cp, dg, di, r, z, Lc, zc, a, jp, xp, yp, zp) +
           cp[ax * N + jm] * post_resid_at<D, T>(L, cp, dg, di, r, z, Lc, zc, a, jm, xm, ym, zm);
  }
  const T yi = post_resid_at<D, T>(L, cp, dg, di, r, z, Lc, zc, a, i, cx, cy, cz);
  zo[i] = zprime_at<D, T>(z, Lc, zc, a, i, cx, cy, cz) + (c1 - c2) * yi + c2 * d * off;
}

// Galerkin coarse operator of piecewise-constant aggregation: diag_I = sum of the
// children's diagonals minus twice the faces inside I; cp_I(a) = sum of the fine faces
// from I to I + e_a.
template <int D, class T>
__global__ __launch_bounds__(kBlock) void k_coarsen(const int* __restrict__ stop, Level Lf,
                                                     const T* __restrict__ cpf, const T* __restrict__ diagf,
                                                     Level Lc, T* __restrict__ cpc, T* __restrict__ diagc,
                                                     T* __restrict__ dinvc) {
  if (*stop) return;
  const int64_t I = gidx();
  if (I >= Lc.N) return;
  int X, Y, Z;
  cell_xyz<D>(Lc, I, X, Y, Z);
  T dg = 0;
  T c[3] = {0, 0, 0};
  for (int dz = 0; dz < (D == 3 ? 2 : 1); ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const int cx = 2 * X + dx, cy = 2 * Y + dy, cz = 2 * Z + dz;
        if (cx >= Lf.n[0] || cy >= Lf.n[1] || (D == 3 && cz >= Lf.n[2])) continue;
        const int64_t i = cell_id<D>(Lf, cx, cy, cz);
        dg += diagf[i];
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
          const T f = cpf[(int64_t)ax * Lf.N + i];
          int jx = cx, jy = cy, jz = cz;
          if (ax == 0) jx = wrap(cx + 1, Lf.n[0]);
          if (ax == 1) jy = wrap(cy + 1, Lf.n[1]);
          if (ax == 2) jz = wrap(cz + 1, Lf.n[2]);
          const bool inside = (jx >> 1) == X && (jy >> 1) == Y && (jz >> 1) == Z;
          if (inside)
            dg -= T(2) * f;
          else
            c[ax] += f;
        }
      }
  diagc[I] = dg;
  dinvc[I] = dg != T(0) ? T(1) / dg : T(0);
#pragma unroll
  for (int ax = 0; ax < D; ++ax) cpc[(int64_t)ax * Lc.N + I] = c[ax];
}

// per-block FP64 partial of a.b (grid-stride)
template <class T>
__global__ __launch_bounds__(kBlock) void k_dot(const int* __restrict__ stop, int64_t N, const T* __restrict__ a,
                                                 const T* __restrict__ b, double* __restrict__ part) {
  if (*stop) return;
  double v[1] = {0.0};
  for (int64_t i = gidx(); i < N; i += (int64_t)gridDim.x * blockDim.x)
    v[0] += (double)a[i] * (double)b[i];
  block_reduce<1, false>(v, part + blockIdx.x);
}

// Convergence trigger after an iteration, evaluated alike by every block that needs it: the
// recursively updated residual max|r| (partials of k_cg_update_max) against the tolerance and
// the rounding floor, or non-finite, or the iteration cap (force).
__device__ __forceinline__ bool cg_trigger(const CgCtl* __restrict__ ctl, const double* __restrict__ pmax,
                                           int nblk, double tol, int force) {
  const double est = reduce_partials<true>(pmax, nblk) / ctl->bmax;
  return force || est <= tol || est <= ctl->floor || !isfinite(est);
}

// FP64 true residual: r = b - A x (stored in T), per-block partials of max|r|, max|b| and
// max_i sum_j |A_ij x_j| (the rounding floor of the residual of an x stored in T) (grid-stride).
// ctl == nullptr: unconditional (initial check); otherwise only when the solve is running and
// cg_trigger fires.
template <int D, class T>
__global__ __launch_bounds__(kBlock) void k_true_resid(const CgCtl* __restrict__ ctl, const double* __restrict__ pmax,
                                                        int nmax, double tol, int force, Level L,
                                                        const T* __restrict__ cp, const T* __restrict__ diag,
                                                        const T* __restrict__ b, const T* __restrict__ x,
                                                        T* __restrict__ r, double* __restrict__ part) {
  if (ctl) {
    if (ctl->stop) return;
    if (!cg_trigger(ctl, pmax, nmax, tol, force)) return;
  }
  double m[3] = {0.0, 0.0, 0.0};
  for (int64_t i = gidx(); i < L.N; i += (int64_t)gridDim.x * blockDim.x) {
    const double dg = diag[i];
    double res = 0.0;
    if (dg != 0.0) {
      int cx, cy, cz;
      cell_xyz<D>(L, i, cx, cy, cz);
      double ax_ = dg * (double)x[i];
      double mag = fabs(ax_);
#pragma unroll
      for (int ax = 0; ax < D; ++ax) {
        int xp = cx, yp = cy, zp = cz, xm = cx, ym = cy, zm = cz;
        if (ax == 0) { xp = wrap(cx + 1, L.n[0]); xm = wrap(cx - 1, L.n[0]); }
        if (ax == 1) { yp = wrap(cy + 1, L.n[1]); ym = wrap(cy - 1, L.n[1]); }
        if (ax == 2) { zp = wrap(cz + 1, L.n[2]); zm = wrap(cz - 1, L.n[2]); }
        const int64_t jp = cell_id<D>(L, xp, yp, zp), jm = cell_id<D>(L, xm, ym, zm);
        const double tp = (double)cp[(int64_t)ax * L.N + i] * (double)x[jp];
        const double tm = (double)cp[(int64_t)ax * L.N + jm] * (double)x[jm];
        ax_ -= tp + tm;
        mag += fabs(tp) + fabs(tm);
      }
      res = (double)b[i] - ax_;
      m[1] = fmax(m[1], fabs((double)b[i]));
      m[2] = fmax(m[2], mag);
    }
    r[i] = (T)res;
    m[0] = fmax(m[0], fabs(res));
  }
  block_reduce<3, true>(m, part + blockIdx.x, gridDim.x);  // entry k of block b at part[k * blocks + b]
}

// Convergence decision from the true-residual partials (one block).  init != 0: the check
// before the first iteration (sets every field; min1 != 0: iterate at least once even if the
// start already meets the tolerance).  Otherwise runs only when k_true_resid ran, i.e. the
// solve is running and cg_trigger fires; stops on convergence, a non-finite residual or the
// iteration cap (force).
__global__ __launch_bounds__(kBlock) void k_cg_judge(CgCtl* __restrict__ ctl, const double* __restrict__ ptrue,
                                                      const double* __restrict__ pmax, int nblk, double tol,
                                                      double eps_t, int it, int force, int init,
                                                      int min1) {
  if (!init) {
    if (ctl->stop) return;
    if (!cg_trigger(ctl, pmax, nblk, tol, force)) return;
  }
  // entry k of block b at ptrue[k * nblk + b]; wave k (of four) takes the maximum of entry k
  static_assert(kBlock / 64 >= 3, "one wave per entry");
  __shared__ double out[3];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (wv < 3) {
    const double* col = ptrue + (int64_t)wv * nblk;
    double x = -INFINITY;
    for (int base = 0; base < nblk; base += 64 * 16) {
      double v[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int b = base + lane + 64 * j;
        v[j] = b < nblk ? col[b] : -INFINITY;
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) x = fmax(x, v[j]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_down(x, off, 64));
    if (lane == 0) out[wv] = x;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double bmax = out[1];
  const double rel = bmax > 0.0 ? out[0] / bmax : 0.0;
  const double floor = bmax > 0.0 ? 8.0 * eps_t * out[2] / bmax : 0.0;
  const bool done = rel <= tol || rel <= floor;
  ctl->rel = rel;
  ctl->floor = floor;
  if (init) {
    ctl->bmax = bmax;
    ctl->rel0 = rel;
    ctl->zero = bmax == 0.0;
    ctl->iters = 0;
    const bool run = bmax != 0.0 && (!done || min1) && isfinite(rel);
    ctl->iterated = run;
    ctl->stop = !run;
    ctl->conv = bmax == 0.0 || done;
  } else if (done || !isfinite(rel) || force) {
    ctl->stop = 1;
    ctl->conv = done;
    ctl->iters = it;
  }
}

// x = 0 when the right-hand side vanishes
template <class T>
__global__ __launch_bounds__(kBlock) void k_cg_zero(const CgCtl* __restrict__ ctl, int64_t N, T* __restrict__ x) {
  if (!ctl->zero) return;
  for (int64_t i = gidx(); i < N; i += (int64_t)gridDim.x * blockDim.x) x[i] = T(0);
}

// ---- warm start by Galerkin projection onto earlier solutions ------------------------------
// For A x = b and up to M earlier solutions h_1..h_m (h_1 = the current content of x), the
// warm start x0 = sum_j a_j h_j minimising the A-norm of the error over their span (so it is at
// least as good, in that norm, as the previous solution or any extrapolation of the earlier
// ones).  The Galerkin system is formed in the basis u_j = sum_k B_jk h_k (FP64, from the stored
// values): successive solutions are nearly equal (or, for the adjoint, nearly opposite), and
// differences such as h_1 - h_2 resolve what G_ij = h_i . A h_j in FP64 cannot.  With fewer than
// M vectors B is the identity.  Three kernels: partial sums of G_ij = u_i . A u_j and
// g_i = u_i . b (one pass that applies A to every stored h_k in FP64 and forms the basis once per
// cell), a one-block Cholesky solve that maps the coefficients back (a = B^T c), the combination.
template <class T, int M>
struct ProjVecs {
  const T* v[M];
  double B[M][M];
};
template <int M>
constexpr int proj_sums() { return M * (M + 1) / 2 + M; }

// per-block FP64 partials of G (upper triangle, row-major) and g, entry k of block b at
// part[k * blocks + b]; also keep <- h_1
template <int D, class T, int M>
__global__ __launch_bounds__(kBlock) void k_proj_gram(Level L, const T* __restrict__ cp, const T* __restrict__ diag,
                                                      const T* __restrict__ b, ProjVecs<T, M> h, int m,
                                                      T* __restrict__ keep, double* __restrict__ part) {
  constexpr int P = proj_sums<M>();
  double acc[P];
#pragma unroll
  for (int k = 0; k < P; ++k) acc[k] = 0.0;
  int64_t lo, hi;
  chunk_range(L.N, lo, hi);
  const int N = (int)L.N;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
    // A h_k in FP64 for every stored vector (the products of FP32 values are exact in FP64, so
    // the basis differences formed from them below keep their accuracy), then u = B h and
    // A u = B (A h) once per cell.  Every load of the cell is independent of the others (unused
    // slots point at valid vectors and have zero columns in B; inactive cells are masked and
    // their neighbour indices are valid), so one iteration is one memory round trip.
    const T dg = diag[i];
    const double bi = (double)b[i];
    int cx, cy, cz;
    cell_xyz<D>(L, i, cx, cy, cz);
    double hv[M], ah[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
      hv[k] = (double)h.v[k][i];
      ah[k] = (double)dg * hv[k];
    }
    const T h0 = h.v[0][i];
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      int jp, jm;
      axis_pm<D>(L, (int)i, cx, cy, cz, ax, jp, jm);
      const double cpp = (double)cp[(int64_t)ax * N + i], cpm = (double)cp[(int64_t)ax * N + jm];
#pragma unroll
      for (int k = 0; k < M; ++k) ah[k] -= cpp * (double)h.v[k][jp] + cpm * (double)h.v[k][jm];
    }
    double u[M], au[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
      double su = 0.0, sa = 0.0;
#pragma unroll
      for (int k = 0; k < M; ++k) {
        su += h.B[r][k] * hv[k];
        sa += h.B[r][k] * ah[k];
      }
      u[r] = su;
      au[r] = sa;
    }
    if (keep) keep[i] = h0;
    const bool on = dg != T(0);  // selected, not multiplied: inactive cells contribute nothing
#pragma unroll
    for (int r = 0; r < M; ++r) u[r] = on ? u[r] : 0.0;
    int k = 0;
#pragma unroll
    for (int r = 0; r < M; ++r)
#pragma unroll
      for (int c = r; c < M; ++c) acc[k++] += u[r] * au[c];
#pragma unroll
    for (int r = 0; r < M; ++r) acc[k++] += u[r] * bi;
  }
  block_reduce<P, false>(acc, part + blockIdx.x, gridDim.x);  // entry k of block b at part[k * blocks + b]
}

// G c = g from the sums s (upper triangle of G row-major, then g) for the first m vectors
template <int M>
__host__ __device__ inline void proj_coefficients(const double* s, int m, double* coef) {
  // every loop runs to the compile-time M (the vector count m only masks), so the loops unroll
  // and the small arrays stay in registers
  double G[M][M], g[M], Lc[M][M], y[M], c[M];
  bool keepj[M];
  int k = 0;
#pragma unroll
  for (int r = 0; r < M; ++r)
#pragma unroll
    for (int cc = r; cc < M; ++cc) G[r][cc] = G[cc][r] = s[k++];
#pragma unroll
  for (int r = 0; r < M; ++r) g[r] = s[k++];
#pragma unroll
  for (int r = 0; r < M; ++r)
#pragma unroll
    for (int i = 0; i < M; ++i) Lc[r][i] = 0.0;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    double d = G[j][j];
#pragma unroll
    for (int i = 0; i < j; ++i) d -= Lc[j][i] * Lc[j][i];
    keepj[j] = j < m && G[j][j] > 0.0 && d > 1e-12 * G[j][j];
    const double ljj = keepj[j] ? sqrt(d) : 1.0;
    Lc[j][j] = keepj[j] ? ljj : 0.0;
#pragma unroll
    for (int r = j + 1; r < M; ++r) {
      double e = G[r][j];
#pragma unroll
      for (int i = 0; i < j; ++i) e -= Lc[r][i] * Lc[j][i];
      Lc[r][j] = keepj[j] && r < m ? e / ljj : 0.0;
    }
  }
#pragma unroll
  for (int j = 0; j < M; ++j) {
    double e = g[j];
#pragma unroll
    for (int i = 0; i < j; ++i) e -= Lc[j][i] * y[i];
    y[j] = keepj[j] ? e / Lc[j][j] : 0.0;
  }
#pragma unroll
  for (int j = M - 1; j >= 0; --j) {
    double e = y[j];
#pragma unroll
    for (int i = j + 1; i < M; ++i) e -= Lc[i][j] * c[i];
    c[j] = keepj[j] ? e / Lc[j][j] : 0.0;
  }
#pragma unroll
  for (int j = 0; j < M; ++j) coef[j] = c[j] - c[j] == 0.0 ? c[j] : 0.0;  // 0 for inf and NaN
}

// sums the partials in a fixed order (1024 threads) and solves G c = g by Cholesky in FP64; a vector whose
// pivot falls below 1e-12 of its own G_jj (linearly dependent on the earlier ones) gets c_j = 0
template <class T, int M>
__global__ __launch_bounds__(kFinalWide) void k_proj_solve(const double* __restrict__ part, int nblk, int m,
                                                           ProjVecs<T, M> h, double* __restrict__ coef) {
  constexpr int P = proj_sums<M>();
  __shared__ double s[P];
  final_cols<P>(part, nblk, s);
  __syncthreads();
  if (threadIdx.x != 0) return;
  double c[M];
  proj_coefficients<M>(s, m, c);
  for (int k = 0; k < M; ++k) {
    double e = 0.0;
    for (int j = 0; j < M; ++j) e += c[j] * h.B[j][k];
    coef[k] = k < m ? e : 0.0;
  }
}

// x <- sum_j c_j h_j in FP64, rounded once (nearly dependent h_j, such as successive potentials or
// the sign-alternating adjoint potentials, give large coefficients of opposite sign; h_1 may be x
// itself: each element is read before it is written)
template <class T, int M>
__global__ __launch_bounds__(kBlock) void k_proj_combine(int64_t N, const double* __restrict__ coef,
                                                         ProjVecs<T, M> h, int m, T* x) {
  const int64_t i = gidx();
  if (i >= N) return;
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < M; ++j) s += coef[j] * (double)h.v[j][i];  // coef[j] = 0 for j >= m
  x[i] = (T)s;
}

// Linear extrapolation of a warm start from two earlier solutions: x <- 2 x - older, older <- x
template <class T>
__global__ __launch_bounds__(kBlock) void k_extrapolate(int64_t N, T* __restrict__ x, T* __restrict__ older) {
  const int64_t i = gidx();
  if (i >= N) return;
  const T v = x[i];
  x[i] = T(2) * v - older[i];
  older[i] = v;
}

// Rows of N values copied in one pass, dst[j][i] = src[j][i] for j < nrows (the adjoint
// recompute's record of the fields that do not depend on the potential: three phase fields, the
// previous step's phase fields and velocity, rho_e and the previous rho_e)
constexpr int kMaxRows = 12;
template <class T>
struct RowCopy {
  const T* src[kMaxRows];
  T* dst[kMaxRows];
  int nrows;
};
template <class T>
__global__ __launch_bounds__(kBlock) void k_copy_rows(int64_t N, RowCopy<T> rc) {
  const int64_t i = gidx();
  if (i >= N) return;
  T v[kMaxRows];
#pragma unroll
  for (int j = 0; j < kMaxRows; ++j)
    if (j < rc.nrows) v[j] = rc.src[j][i];
#pragma unroll
  for (int j = 0; j < kMaxRows; ++j)
    if (j < rc.nrows) rc.dst[j][i] = v[j];
}

// dst = src when *gate != 0 (a copy queued behind a solve, done only once it has stopped)
template <class T>
__global__ __launch_bounds__(kBlock) void k_copy_gated(const int* __restrict__ gate, int64_t N,
                                                         const T* __restrict__ src, T* __restrict__ dst) {
  if (*gate == 0) return;
  const int64_t i = gidx();
  if (i < N) dst[i] = src[i];
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_zero(int64_t N, T* __restrict__ x) {
  const int64_t i = gidx();
  if (i < N) x[i] = T(0);
}

// T -> double copy (read-out)
template <class T>
__global__ __launch_bounds__(kBlock) void k_to_double(int64_t N, const T* __restrict__ a, double* __restrict__ out) {
  const int64_t i = gidx();
  if (i < N) out[i] = (double)a[i];
}

// T -> double copy times a factor (the pressure cs^2 drho), rounded as the host does it
template <class T>
__global__ __launch_bounds__(kBlock) void k_to_double_scaled(int64_t N, const T* __restrict__ a, double scale,
                                                             double* __restrict__ out) {
  const int64_t i = gidx();
  if (i < N) {
    const double v = (double)a[i];
    out[i] = v * scale;
  }
}

}  // namespace ehd
