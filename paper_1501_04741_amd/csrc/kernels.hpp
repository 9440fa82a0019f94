// gfx950 kernels of the adjoint lattice-Boltzmann hot path.
//
// Data layout (HBM): a state is row-blocked.  Row r = y + ny*z holds Qt = Q + QS
// runs of nx values, one per population, each starting on a 128-byte line:
// population j of node (x, r) lives at (r*Qt + j)*pitch + x, with pitch = nx
// rounded up to 128 bytes (the padding is never touched).  A block that
// updates row r therefore writes one contiguous Qt*pitch run and pulls from at
// most 9 neighbour rows, instead of touching 2*Qt planes N values apart (fewer
// DRAM pages open at once; this measured ~15% faster than plane-major SoA on
// the 256x128x128 D3Q19 lattice).  Unaligned runs cost a third of the
// bandwidth (nx = 450 against 448 measured 0.46 against 0.68 of peak), hence the
// pitch.  The workspace's node arrays (design field, gradient, moments) use the
// same pitch, i = x + pitch*r; the compact index n = x + nx*r addresses every
// array exchanged through the ABI (plane-major exports, design in, gradient out).  Stored flow populations are
// shifted by their lattice weight (f~_j = f_j - w_j) so that FP32 keeps the
// small deviations from rest at full relative precision; the scalar is stored
// as is.  The primal buffers hold POST-collision states h^k; the pre-collision
// state of step k+1 is pulled, f^{k+1}_j(x) = h^k_j(x - e_j) (Section 2.1).
//
// Launch geometry (node kernels): block = BX threads along x, grid =
// (ceil(nx/BX), ny, nz).  The hot kernels (primal, adjoint, one-shot) may also
// stack R rows in a block (blockDim.y = R) when a row is narrower than the
// block they aim for; a wave never straddles two rows.  y and z are
// wave-uniform, so wall rows are decided per wave and every x-shift in the pull
// stays inside the row the wave's block owns: each fetched cache line of a
// source row is consumed by one block.
//
// Each node is owned by exactly one thread; there are no atomics, and every
// reduction runs in a fixed order, so results are bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"

namespace lbmk {

enum : int { INTERIOR = 0, WALL = 1, INLET = 2, OUTLET = 3 };
enum : int { G_POWER = 0, G_RAMP = 1 };
enum : int { S_ADIABATIC = 0, S_DIRICHLET = 1 };
enum : int { IN_VELOCITY = 0, IN_PRESSURE = 1 };
// Kernel variants (template mask V): forced MRT interior collision; scalar
// diffusivity blended with the design field.
enum : int { kVarMRT = 1, kVarVD = 2 };

// Per-context parameters, passed by value to every kernel.
template <typename Real>
struct Params {
  int nx, ny, nz, periodic;
  int N;                    // nodes (compact count, nx*ny*nz)
  int pitch;                // padded row length of the workspace arrays (multiple of 128 bytes)
  int Np;                   // pitch*ny*nz (Qt*Np < 2^31 is enforced on the host)
  int scalar_wall, split_axis, switch_fn;
  int theta_int;            // POWER with integer theta: theta, else -1
  Real om, oms;             // 1/tau, 1/tau_s
  Real u_in, rho_out;
  Real s_wall, s_in_lo, s_in_hi;
  Real sw_param;            // theta (POWER) or q (RAMP)
  int inlet_mode;           // IN_VELOCITY (u_in) or IN_PRESSURE (rho_in, limited to u_cap)
  Real drho_in;             // rho_in - 1 (pressure inlet; the state is stored shifted)
  Real u_cap;               // pressure inlet velocity limit (0: none)
  double rho_in;            // pressure inlet density, for the objective sums
  double c_dp, c_hf, c_var, c_mix;  // objective weights
  Real mrt_k[19];           // MRT: (1 - rate_k) / |U row k|^2 (interior collision U^T diag(mrt_k) U)
  Real taus_f, taus_s;      // scalar relaxation time of fluid (w = 1) and solid (w = 0), blended variant
  int plate_x0, plate_x1;   // heating plate: y = 0 wall nodes with plate_x0 <= x < plate_x1 (none if equal)
  Real s_plate;             // scalar value the plate holds
};

template <typename P>
__device__ __forceinline__ int node_class(const P& p, int x, int y, int z, bool is3d) {
  if (p.periodic) return INTERIOR;
  if (y == 0 || y == p.ny - 1) return WALL;
  if (is3d && (z == 0 || z == p.nz - 1)) return WALL;
  if (x == 0) return INLET;
  if (x == p.nx - 1) return OUTLET;
  return INTERIOR;
}

// Wrapped neighbour coordinates for s in {-1, 0, +1}: X[s+1] = (x+s) mod nx,
// Yr[s+1] = (y+s) mod ny, Zr[s+1] = ny*((z+s) mod nz); a row index is Yr + Zr.
// y and z are block-uniform, so the row parts live in scalar registers.
struct Nbr {
  int nx, pitch;
  int X[3], Yr[3], Zr[3];
};

template <typename P>
__device__ __forceinline__ Nbr make_nbr(const P& p, int x, int y, int z) {
  Nbr b;
  b.nx = p.nx;
  b.pitch = p.pitch;
  b.X[0] = (x == 0) ? p.nx - 1 : x - 1;
  b.X[1] = x;
  b.X[2] = (x == p.nx - 1) ? 0 : x + 1;
  b.Yr[0] = (y == 0) ? p.ny - 1 : y - 1;
  b.Yr[1] = y;
  b.Yr[2] = (y == p.ny - 1) ? 0 : y + 1;
  b.Zr[0] = ((z == 0) ? p.nz - 1 : z - 1) * p.ny;
  b.Zr[1] = z * p.ny;
  b.Zr[2] = ((z == p.nz - 1) ? 0 : z + 1) * p.ny;
  return b;
}

// Node index of the pull source x - e (streaming, Section 2.1) ...
__device__ __forceinline__ int pull_node(const Nbr& b, int ex, int ey, int ez) {
  return b.X[1 - ex] + b.nx * (b.Yr[1 - ey] + b.Zr[1 - ez]);
}
// ... and of x + e (reverse streaming S^{-1}, Lemma 1).
__device__ __forceinline__ int push_node(const Nbr& b, int ex, int ey, int ez) {
  return b.X[1 + ex] + b.nx * (b.Yr[1 + ey] + b.Zr[1 + ez]);
}
__device__ __forceinline__ int own_node(const Nbr& b) { return b.X[1] + b.nx * (b.Yr[1] + b.Zr[1]); }
// Index of the node in the workspace's padded node arrays (w, grad, moments).
__device__ __forceinline__ int own_inode(const Nbr& b) { return b.X[1] + b.pitch * (b.Yr[1] + b.Zr[1]); }

// State addresses in the row-blocked layout (population j, QT populations per node).
template <int QT>
__device__ __forceinline__ int pull_addr(const Nbr& b, int j, int ex, int ey, int ez) {
  return ((b.Yr[1 - ey] + b.Zr[1 - ez]) * QT + j) * b.pitch + b.X[1 - ex];
}
template <int QT>
__device__ __forceinline__ int push_addr(const Nbr& b, int j, int ex, int ey, int ez) {
  return ((b.Yr[1 + ey] + b.Zr[1 + ez]) * QT + j) * b.pitch + b.X[1 + ex];
}
template <int QT>
__device__ __forceinline__ int own_addr(const Nbr& b, int j) {
  return ((b.Yr[1] + b.Zr[1]) * QT + j) * b.pitch + b.X[1];
}

// Position of the calling thread in the hot kernels' launch geometry: blocks
// of blockDim.x = 64k threads along x (a multiple of the wave) and blockDim.y
// rows, grid (ceil(nx / blockDim.x), ceil(ny / blockDim.y), nz).  A wave never
// straddles two rows, so y is wave-uniform and is kept in a scalar register.
// Returns false for the padding lanes and rows.
template <typename P>
__device__ __forceinline__ bool hot_pos(const P& p, int& x, int& y, int& z) {
  x = blockIdx.x * blockDim.x + threadIdx.x;
  y = __builtin_amdgcn_readfirstlane((int)(blockIdx.y * blockDim.y + threadIdx.y));
  z = blockIdx.z;
  return x < p.nx && y < p.ny;
}

// Streaming stores: non-temporal when the state is too large to be re-read
// from the last-level cache by the next launch.
template <bool NT, typename Real>
__device__ __forceinline__ void put(Real* p, Real v) {
  if constexpr (NT) {
    __builtin_nontemporal_store(v, p);
  } else {
    *p = v;
  }
}
// Streaming loads, for populations read once per step (cotangent, recorded
// moments, and the primal state in the kernels listed at load_state).  Only
// accesses that are not shifted along x take the hint: a load shifted by one
// site spans one cache line more than its wave's 256 bytes, and that line is
// also read by the neighbouring wave; without the hint the second read hits the
// L2, with it the line is fetched from HBM twice.  Measured on the 256x128x128
// D3Q19 FP32 channel: adjoint 0.743 of peak without hints, 0.761 with every
// cotangent load hinted (HBM traffic 1.065x the algorithmic bytes), 0.792 with
// the unshifted ones only; in-place primal with every load hinted 0.819 ->
// 0.657.  The adjoint's recorded moments take the hint too (in-place adjoint
// 0.819 -> 0.829); its design value does not (0.829 -> 0.818).  The hint is a
// template argument and the shifted and unshifted loads sit in separate loops:
// a run-time flag, even one that folds to a constant after unrolling, lets the
// compiler merge the hinted and plain load of the same address and drop the hint.
template <bool NT, typename Real>
__device__ __forceinline__ Real get(const Real* p) {
  if constexpr (NT) {
    return __builtin_nontemporal_load(p);
  } else {
    return *p;
  }
}

template <typename Real, typename P>
__device__ __forceinline__ Real inlet_value(const P& p, int y, int z) {
  if (p.split_axis == 1) return (y < p.ny / 2) ? p.s_in_lo : p.s_in_hi;
  if (p.split_axis == 2) return (z < p.nz / 2) ? p.s_in_lo : p.s_in_hi;
  return p.s_in_lo;
}

// Density offset and normal velocity of an inlet node from the shifted sums
// s0 = sum_{e_x=0} f~ and sm = sum_{e_x=-1} f~ of the populations that reached
// x = 0 from inside (their unshifted P = s0 + 2 sm + 1 equals rho (1 - u_x) by
// mass and x-momentum of the rebuilt state, Zou-He).  Velocity form: u = u_in.
// Pressure form: rho = rho_in and up = (rho_in - 1 - s0 - 2 sm) / rho_in; when
// u_cap > 0 and up exceeds it, the node takes the velocity form at u_cap (the
// two forms agree at up = u_cap).  up is what the adjoint needs to know which
// form ran, so the recorded primal keeps it.
template <typename Real>
__device__ __forceinline__ bool inlet_state(const Params<Real>& p, Real s0, Real sm, Real& u, Real& drho, Real& up) {
  if (p.inlet_mode == IN_PRESSURE) {
    up = (p.drho_in - (s0 + Real(2) * sm)) / (Real(1) + p.drho_in);
    if (!(p.u_cap > Real(0) && up > p.u_cap)) {
      u = up;
      drho = p.drho_in;
      return true;  // pressure form
    }
    u = p.u_cap;
  } else {
    u = p.u_in;
    up = u;
  }
  drho = (s0 + Real(2) * sm + u) / (Real(1) - u);
  return false;  // velocity form
}

// Switching function G(w) and its derivative (Darcy/Brinkman, Section 3.2).
template <typename Real>
__device__ __forceinline__ void switch_fn(const Params<Real>& p, Real w, Real& G, Real& dG) {
  if (p.switch_fn == G_RAMP) {
    const Real q = p.sw_param;
    const Real d = w + q;
    G = (Real(1) + q) * w / d;
    dG = (Real(1) + q) * q / (d * d);
  } else if (p.theta_int >= 0) {
    Real r = Real(1), r1 = Real(1);
    for (int k = 0; k < p.theta_int; ++k) {
      r1 = r;
      r = r * w;
    }
    G = r;
    dG = p.theta_int > 0 ? Real(p.theta_int) * r1 : Real(0);
  } else {
    G = pow(w, p.sw_param);
    dG = p.sw_param * pow(w, p.sw_param - Real(1));
  }
}

// ------------------------------------------------------------------ loads
// In-place streaming (one buffer per state, the "AA" access pattern).  The
// ping-pong form (ACC_PP) keeps post-collision states and pulls.  In place, a
// buffer alternates between two phases: after an even number of steps slot j
// of node x holds the pre-collision f_j(x) (phase E); an even step reads its
// own slots and writes h_j(x) into its own slot opp(j) (phase O); an odd step
// reads f_j(x) = h_j(x - e_j) from slot opp(j) of x - e_j and writes h_j(x)
// into slot j of x + e_j (phase E again).  Each slot is read and written by
// one node only, so no step races.  The adjoint cotangent streams the other
// way (mu_j(x) = lambda_j(x + e_j)) and mirrors the pattern with e -> -e.
enum : int { ACC_PP = 0, ACC_EVEN = 1, ACC_ODD = 2 };

// NT: streaming hint on the loads that are not shifted along x (all of them in
// the even phase), as for the cotangent.  Which kernels take it was measured on
// the 256x128x128 D3Q19 FP32 channel: ping-pong primal 0.707 -> 0.728 of peak,
// ping-pong one-shot 0.739 -> 0.753, in-place one-shot (both phases) 0.707 ->
// 0.783, recorded in-place primal 0.822 -> 0.837 with the odd phase hinted
// alone: hinting its even phase too drops it to 0.776 on that 319 MB state,
// most of which the last-level cache keeps between the two phases, but lifts
// states beyond twice the cache (512x128x128: 0.659 -> 0.774; 512x256x128:
// 0.652 -> 0.733).  Unrecorded in-place steps take the hints (both phases) only
// beyond twice the cache as well.
template <int Q, int QS, typename Real, int ACC, bool NT = false>
__device__ __forceinline__ void load_state(const Real* a, const Nbr& b, Real (&f)[Q], Real (&g)[QS > 0 ? QS : 1]) {
  using L = Lat<Q>;
  using S = SLat<QS>;
  constexpr int QT = Q + QS;
  if constexpr (ACC == ACC_PP) {
#pragma unroll
    for (int j = 0; j < Q; ++j)
      if (L::ex(j) == 0) f[j] = get<NT>(a + pull_addr<QT>(b, j, L::ex(j), L::ey(j), L::ez(j)));
#pragma unroll
    for (int j = 0; j < Q; ++j)
      if (L::ex(j) != 0) f[j] = a[pull_addr<QT>(b, j, L::ex(j), L::ey(j), L::ez(j))];
#pragma unroll
    for (int i = 0; i < QS; ++i)
      if (S::ex(i) == 0) g[i] = get<NT>(a + pull_addr<QT>(b, Q + i, S::ex(i), S::ey(i), S::ez(i)));
#pragma unroll
    for (int i = 0; i < QS; ++i)
      if (S::ex(i) != 0) g[i] = a[pull_addr<QT>(b, Q + i, S::ex(i), S::ey(i), S::ez(i))];
  } else if constexpr (ACC == ACC_EVEN) {
#pragma unroll
    for (int j = 0; j < Q; ++j) f[j] = get<NT>(a + own_addr<QT>(b, j));
#pragma unroll
    for (int i = 0; i < QS; ++i) g[i] = get<NT>(a + own_addr<QT>(b, Q + i));
  } else {
#pragma unroll
    for (int j = 0; j < Q; ++j)
      if (L::ex(j) == 0) f[j] = get<NT>(a + pull_addr<QT>(b, L::opp(j), L::ex(j), L::ey(j), L::ez(j)));
#pragma unroll
    for (int j = 0; j < Q; ++j)
      if (L::ex(j) != 0) f[j] = a[pull_addr<QT>(b, L::opp(j), L::ex(j), L::ey(j), L::ez(j))];
#pragma unroll
    for (int i = 0; i < QS; ++i)
      if (S::ex(i) == 0) g[i] = get<NT>(a + pull_addr<QT>(b, Q + S::opp(i), S::ex(i), S::ey(i), S::ez(i)));
#pragma unroll
    for (int i = 0; i < QS; ++i)
      if (S::ex(i) != 0) g[i] = a[pull_addr<QT>(b, Q + S::opp(i), S::ex(i), S::ey(i), S::ez(i))];
  }
}

template <int Q, int QS, typename Real, bool NT, int ACC>
__device__ __forceinline__ void store_state(Real* a, const Nbr& b, const Real (&f)[Q], const Real (&g)[QS > 0 ? QS : 1]) {
  using L = Lat<Q>;
  using S = SLat<QS>;
  constexpr int QT = Q + QS;
  // In place the stores hit the addresses the loads used; an empty asm hides the
  // lane index so the compiler recomputes the store addresses instead of keeping
  // every load address live across the node update (measured: 92 -> 55 VGPRs and
  // 0.75 -> 0.81 of peak for the in-place primal; 186 -> 92 VGPRs and 0.784 ->
  // 0.799 for the in-place one-shot).  It emits no code.
  Nbr bb = b;
  if constexpr (ACC != ACC_PP) {
#pragma unroll
    for (int k = 0; k < 3; ++k) asm volatile("" : "+v"(bb.X[k]));
  }
  if constexpr (ACC == ACC_PP) {
#pragma unroll
    for (int j = 0; j < Q; ++j) put<NT>(a + own_addr<QT>(bb, j), f[j]);
#pragma unroll
    for (int i = 0; i < QS; ++i) put<NT>(a + own_addr<QT>(bb, Q + i), g[i]);
  } else if constexpr (ACC == ACC_EVEN) {
#pragma unroll
    for (int j = 0; j < Q; ++j) put<NT>(a + own_addr<QT>(bb, L::opp(j)), f[j]);
#pragma unroll
    for (int i = 0; i < QS; ++i) put<NT>(a + own_addr<QT>(bb, Q + S::opp(i)), g[i]);
  } else {
    // stores shifted along x share their end lines with the neighbouring wave's:
    // plain stores let the L2 merge the two halves (in-place primal 0.836 -> 0.839)
#pragma unroll
    for (int j = 0; j < Q; ++j)
      if (L::ex(j) == 0) put<NT>(a + push_addr<QT>(bb, j, L::ex(j), L::ey(j), L::ez(j)), f[j]);
#pragma unroll
    for (int j = 0; j < Q; ++j)
      if (L::ex(j) != 0) put<false>(a + push_addr<QT>(bb, j, L::ex(j), L::ey(j), L::ez(j)), f[j]);
#pragma unroll
    for (int i = 0; i < QS; ++i) put<NT>(a + push_addr<QT>(bb, Q + i, S::ex(i), S::ey(i), S::ez(i)), g[i]);
  }
}

// Cotangent of the post-collision populations, mu_j(x) = lambda_j(x + e_j),
// and the store of the new lambda(x), for the three access patterns.
template <int Q, int QS, typename Real, int ACC, bool NT>
__device__ __forceinline__ void load_cot(const Real* a, const Nbr& b, Real (&mu)[Q], Real (&nu)[QS > 0 ? QS : 1]) {
  using L = Lat<Q>;
  using S = SLat<QS>;
  constexpr int QT = Q + QS;
  if constexpr (ACC == ACC_PP) {
#pragma unroll
    for (int j = 0; j < Q; ++j)
      if (L::ex(j) == 0) mu[j] = get<NT>(a + push_addr<QT>(b, j, L::ex(j), L::ey(j), L::ez(j)));
#pragma unroll
    for (int j = 0; j < Q; ++j)
      if (L::ex(j) != 0) mu[j] = a[push_addr<QT>(b, j, L::ex(j), L::ey(j), L::ez(j))];
#pragma unroll
    for (int i = 0; i < QS; ++i)
      if (S::ex(i) == 0) nu[i] = get<NT>(a + push_addr<QT>(b, Q + i, S::ex(i), S::ey(i), S::ez(i)));
#pragma unroll
    for (int i = 0; i < QS; ++i)
      if (S::ex(i) != 0) nu[i] = a[push_addr<QT>(b, Q + i, S::ex(i), S::ey(i), S::ez(i))];
  } else if constexpr (ACC == ACC_EVEN) {
#pragma unroll
    for (int j = 0; j < Q; ++j) mu[j] = get<NT>(a + own_addr<QT>(b, j));
#pragma unroll
    for (int i = 0; i < QS; ++i) nu[i] = get<NT>(a + own_addr<QT>(b, Q + i));
  } else {
#pragma unroll
    for (int j = 0; j < Q; ++j)
      if (L::ex(j) == 0) mu[j] = get<NT>(a + push_addr<QT>(b, L::opp(j), L::ex(j), L::ey(j), L::ez(j)));
#pragma unroll
    for (int j = 0; j < Q; ++j)
      if (L::ex(j) != 0) mu[j] = a[push_addr<QT>(b, L::opp(j), L::ex(j), L::ey(j), L::ez(j))];
#pragma unroll
    for (int i = 0; i < QS; ++i)
      if (S::ex(i) == 0) nu[i] = get<NT>(a + push_addr<QT>(b, Q + S::opp(i), S::ex(i), S::ey(i), S::ez(i)));
#pragma unroll
    for (int i = 0; i < QS; ++i)
      if (S::ex(i) != 0) nu[i] = a[push_addr<QT>(b, Q + S::opp(i), S::ex(i), S::ey(i), S::ez(i))];
  }
}

template <int Q, int QS, typename Real, bool NT, int ACC>
__device__ __forceinline__ void store_cot(Real* a, const Nbr& b, const Real (&lf)[Q], const Real (&lg)[QS > 0 ? QS : 1]) {
  using L = Lat<Q>;
  using S = SLat<QS>;
  constexpr int QT = Q + QS;
  // In place the stores hit the addresses the loads used; an empty asm hides the
  // lane index so the compiler recomputes the store addresses instead of keeping
  // every load address live across the node update (measured: 92 -> 55 VGPRs and
  // 0.75 -> 0.81 of peak for the in-place primal; 186 -> 92 VGPRs and 0.784 ->
  // 0.799 for the in-place one-shot).  It emits no code.
  Nbr bb = b;
  if constexpr (ACC != ACC_PP) {
#pragma unroll
    for (int k = 0; k < 3; ++k) asm volatile("" : "+v"(bb.X[k]));
  }
  if constexpr (ACC == ACC_PP) {
#pragma unroll
    for (int j = 0; j < Q; ++j) put<NT>(a + own_addr<QT>(bb, j), lf[j]);
#pragma unroll
    for (int i = 0; i < QS; ++i) put<NT>(a + own_addr<QT>(bb, Q + i), lg[i]);
  } else if constexpr (ACC == ACC_EVEN) {
#pragma unroll
    for (int j = 0; j < Q; ++j) put<NT>(a + own_addr<QT>(bb, L::opp(j)), lf[j]);
#pragma unroll
    for (int i = 0; i < QS; ++i) put<NT>(a + own_addr<QT>(bb, Q + S::opp(i)), lg[i]);
  } else {
    // shifted stores plain, as for the state
#pragma unroll
    for (int j = 0; j < Q; ++j)
      if (L::ex(j) == 0) put<NT>(a + pull_addr<QT>(bb, j, L::ex(j), L::ey(j), L::ez(j)), lf[j]);
#pragma unroll
    for (int j = 0; j < Q; ++j)
      if (L::ex(j) != 0) put<false>(a + pull_addr<QT>(bb, j, L::ex(j), L::ey(j), L::ez(j)), lf[j]);
#pragma unroll
    for (int i = 0; i < QS; ++i) put<NT>(a + pull_addr<QT>(bb, Q + i, S::ex(i), S::ey(i), S::ez(i)), lg[i]);
  }
}

// ------------------------------------------------ x-shifts through LDS
// When a block spans whole rows (nx at most its width), the populations whose
// access is shifted along x (e_x != 0) are read and written line-aligned: for
// a load every thread reads the value at its own x of the source run into LDS
// and, after a barrier, takes the one at x - e_x (the shift wraps inside the
// row, as the periodic pull does); for a store it writes its result at x + e_x
// of the LDS run and, after a barrier, stores the value at its own x.  Every
// global access is then a whole-wave, line-aligned run and no cache line is
// shared between waves.  lds holds bt values per shifted population (one run
// per block row: the calling thread's row starts at seg, its position in the
// row is its x); act is false for padding lanes and rows, which skip every
// global access but take part in every barrier.
template <int Q, int QS>
struct Shifted {
  __host__ __device__ static constexpr int flow_slot(int j) {
    int n = 0;
    for (int k = 0; k < j; ++k) n += Lat<Q>::ex(k) != 0;
    return n;
  }
  __host__ __device__ static constexpr int scalar_slot(int i) {
    int n = flow_slot(Q);
    for (int k = 0; k < i; ++k) n += SLat<QS>::ex(k) != 0;
    return n;
  }
  __host__ __device__ static constexpr int count() { return scalar_slot(QS); }
};

// Largest block of the single-context hot kernels: a row of up to four waves
// (nx <= 256) is one block, so that its x-shifts can be staged in LDS.  Rows
// of up to eight waves as one 512-thread block (staged as well) measured slower
// on the 450-wide mixing duct: primal 0.789 -> 0.764, in-place one-shot
// 0.876 -> 0.832 of HBM peak.
constexpr int kHotThreads = 256;

// Staging runs of the single-context hot kernels, in dynamic LDS sized by the
// launch (shifted populations x block threads, twice for the one-shot).
extern __shared__ __align__(16) unsigned char lx_smem[];
template <typename Real>
__device__ __forceinline__ Real* lx_lds() {
  return reinterpret_cast<Real*>(lx_smem);
}

// Staging layout of the single-context hot kernels (blockDim.y rows of
// blockDim.x threads): the calling thread's row segment and the run stride.
__device__ __forceinline__ int lx_seg() { return threadIdx.y * blockDim.x; }
__device__ __forceinline__ int lx_span() { return blockDim.x * blockDim.y; }

// Row r(dy, dz) = Yr[1 + dy] + Zr[1 + dz]; address of slot jj's run in it.
template <int QT>
__device__ __forceinline__ int run_addr(const Nbr& b, int jj, int dy, int dz) {
  return ((b.Yr[1 + dy] + b.Zr[1 + dz]) * QT + jj) * b.pitch;
}

// Loads of a pulled (ping-pong, odd in-place phase) state with the x-shifted
// populations staged through LDS; the others as load_state.
// NTS: streaming hint on the staged (now aligned) loads.  It pays for the
// ping-pong pull (256x128x128 D3Q19 FP32: 0.732 -> 0.752 of HBM peak) but not
// in place, where the last-level cache keeps part of the state between the
// two phases (0.89 plain against 0.78 hinted); for states far beyond the cache
// the in-place adjoint takes it (8 x 128x96x96 batched: 0.79 -> 0.81) and the
// in-place primal does not (FP64 256x128x128: 0.768 -> 0.738 with it).
template <int Q, int QS, typename Real, int ACC, bool NT, bool NTS>
__device__ __forceinline__ void load_state_lx(const Real* a, const Nbr& b, Real (&f)[Q], Real (&g)[QS > 0 ? QS : 1],
                                              Real* lds, int seg, int bt, bool act) {
  static_assert(ACC != ACC_EVEN, "the even phase has no shifted access");
  using L = Lat<Q>;
  using S = SLat<QS>;
  using H = Shifted<Q, QS>;
  constexpr int QT = Q + QS;
  constexpr bool odd = (ACC == ACC_ODD);
#pragma unroll
  for (int j = 0; j < Q; ++j)
    if (L::ex(j) == 0)
      f[j] = act ? get<NT>(a + pull_addr<QT>(b, odd ? L::opp(j) : j, L::ex(j), L::ey(j), L::ez(j))) : Real(0);
#pragma unroll
  for (int i = 0; i < QS; ++i)
    if (S::ex(i) == 0)
      g[i] = act ? get<NT>(a + pull_addr<QT>(b, Q + (odd ? S::opp(i) : i), S::ex(i), S::ey(i), S::ez(i))) : Real(0);
  if (act) {
#pragma unroll
    for (int j = 0; j < Q; ++j)
      if (L::ex(j) != 0)
        lds[H::flow_slot(j) * bt + seg + b.X[1]] =
            get<NTS>(a + run_addr<QT>(b, odd ? L::opp(j) : j, -L::ey(j), -L::ez(j)) + b.X[1]);
#pragma unroll
    for (int i = 0; i < QS; ++i)
      if (S::ex(i) != 0)
        lds[H::scalar_slot(i) * bt + seg + b.X[1]] =
            get<NTS>(a + run_addr<QT>(b, Q + (odd ? S::opp(i) : i), -S::ey(i), -S::ez(i)) + b.X[1]);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < Q; ++j)
    if (L::ex(j) != 0) f[j] = act ? lds[H::flow_slot(j) * bt + seg + b.X[1 - L::ex(j)]] : Real(0);
#pragma unroll
  for (int i = 0; i < QS; ++i)
    if (S::ex(i) != 0) g[i] = act ? lds[H::scalar_slot(i) * bt + seg + b.X[1 - S::ex(i)]] : Real(0);
}

// Stores of the odd in-place phase (pushed to x + e_j) with the x-shifted
// populations staged through LDS.  The first barrier keeps the staging of the
// loads intact until every thread has read it.
// NTS: streaming stores for the staged populations.
template <int Q, int QS, typename Real, bool NT, bool NTS>
__device__ __forceinline__ void store_state_lx(Real* a, const Nbr& b, const Real (&f)[Q],
                                               const Real (&g)[QS > 0 ? QS : 1], Real* lds, int seg, int bt,
    bool act) {
  using L = Lat<Q>;
  using S = SLat<QS>;
  using H = Shifted<Q, QS>;
  constexpr int QT = Q + QS;
  __syncthreads();
  if (act) {
#pragma unroll
    for (int j = 0; j < Q; ++j)
      if (L::ex(j) != 0) lds[H::flow_slot(j) * bt + seg + b.X[1 + L::ex(j)]] = f[j];
#pragma unroll
    for (int i = 0; i < QS; ++i)
      if (S::ex(i) != 0) lds[H::scalar_slot(i) * bt + seg + b.X[1 + S::ex(i)]] = g[i];
  }
  __syncthreads();
  if (!act) return;
  Nbr bb = b;  // addresses recomputed (see store_state)
#pragma unroll
  for (int k = 0; k < 3; ++k) asm volatile("" : "+v"(bb.X[k]));
#pragma unroll
  for (int j = 0; j < Q; ++j)
    if (L::ex(j) == 0) put<NT>(a + push_addr<QT>(bb, j, L::ex(j), L::ey(j), L::ez(j)), f[j]);
#pragma unroll
  for (int i = 0; i < QS; ++i)
    if (S::ex(i) == 0) put<NT>(a + push_addr<QT>(bb, Q + i, S::ex(i), S::ey(i), S::ez(i)), g[i]);
#pragma unroll
  for (int j = 0; j < Q; ++j)
    if (L::ex(j) != 0)
      put<NTS>(a + run_addr<QT>(bb, j, L::ey(j), L::ez(j)) + bb.X[1], lds[H::flow_slot(j) * bt + seg + bb.X[1]]);
#pragma unroll
  for (int i = 0; i < QS; ++i)
    if (S::ex(i) != 0)
      put<NTS>(a + run_addr<QT>(bb, Q + i, S::ey(i), S::ez(i)) + bb.X[1], lds[H::scalar_slot(i) * bt + seg + bb.X[1]]);
}

// Cotangent loads (mu_j(x) = lambda_j(x + e_j): ping-pong, or the odd in-place
// pattern) with the x-shifted populations staged through LDS; the others as
// load_cot.  NTS as for load_state_lx.
template <int Q, int QS, typename Real, int ACC, bool NT, bool NTS>
__device__ __forceinline__ void load_cot_lx(const Real* a, const Nbr& b, Real (&mu)[Q], Real (&nu)[QS > 0 ? QS : 1],
                                            Real* lds, int seg, int bt, bool act) {
  static_assert(ACC != ACC_EVEN, "the even pattern has no shifted access");
  using L = Lat<Q>;
  using S = SLat<QS>;
  using H = Shifted<Q, QS>;
  constexpr int QT = Q + QS;
  constexpr bool odd = (ACC == ACC_ODD);
#pragma unroll
  for (int j = 0; j < Q; ++j)
    if (L::ex(j) == 0)
      mu[j] = act ? get<NT>(a + push_addr<QT>(b, odd ? L::opp(j) : j, L::ex(j), L::ey(j), L::ez(j))) : Real(0);
#pragma unroll
  for (int i = 0; i < QS; ++i)
    if (S::ex(i) == 0)
      nu[i] = act ? get<NT>(a + push_addr<QT>(b, Q + (odd ? S::opp(i) : i), S::ex(i), S::ey(i), S::ez(i))) : Real(0);
  if (act) {
#pragma unroll
    for (int j = 0; j < Q; ++j)
      if (L::ex(j) != 0)
        lds[H::flow_slot(j) * bt + seg + b.X[1]] =
            get<NTS>(a + run_addr<QT>(b, odd ? L::opp(j) : j, L::ey(j), L::ez(j)) + b.X[1]);
#pragma unroll
    for (int i = 0; i < QS; ++i)
      if (S::ex(i) != 0)
        lds[H::scalar_slot(i) * bt + seg + b.X[1]] =
            get<NTS>(a + run_addr<QT>(b, Q + (odd ? S::opp(i) : i), S::ey(i), S::ez(i)) + b.X[1]);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < Q; ++j)
    if (L::ex(j) != 0) mu[j] = act ? lds[H::flow_slot(j) * bt + seg + b.X[1 + L::ex(j)]] : Real(0);
#pragma unroll
  for (int i = 0; i < QS; ++i)
    if (S::ex(i) != 0) nu[i] = act ? lds[H::scalar_slot(i) * bt + seg + b.X[1 + S::ex(i)]] : Real(0);
}

// Cotangent stores of the odd in-place pattern (lambda_j(x) to slot j of
// x - e_j) with the x-shifted populations staged through LDS.
template <int Q, int QS, typename Real, bool NT, bool NTS>
__device__ __forceinline__ void store_cot_lx(Real* a, const Nbr& b, const Real (&lf)[Q],
                                             const Real (&lg)[QS > 0 ? QS : 1], Real* lds, int seg, int bt,
    bool act) {
  using L = Lat<Q>;
  using S = SLat<QS>;
  using H = Shifted<Q, QS>;
  constexpr int QT = Q + QS;
  __syncthreads();
  if (act) {
#pragma unroll
    for (int j = 0; j < Q; ++j)
      if (L::ex(j) != 0) lds[H::flow_slot(j) * bt + seg + b.X[1 - L::ex(j)]] = lf[j];
#pragma unroll
    for (int i = 0; i < QS; ++i)
      if (S::ex(i) != 0) lds[H::scalar_slot(i) * bt + seg + b.X[1 - S::ex(i)]] = lg[i];
  }
  __syncthreads();
  if (!act) return;
  Nbr bb = b;  // addresses recomputed (see store_state)
#pragma unroll
  for (int k = 0; k < 3; ++k) asm volatile("" : "+v"(bb.X[k]));
#pragma unroll
  for (int j = 0; j < Q; ++j)
    if (L::ex(j) == 0) put<NT>(a + pull_addr<QT>(bb, j, L::ex(j), L::ey(j), L::ez(j)), lf[j]);
#pragma unroll
  for (int i = 0; i < QS; ++i)
    if (S::ex(i) == 0) put<NT>(a + pull_addr<QT>(bb, Q + i, S::ex(i), S::ey(i), S::ez(i)), lg[i]);
#pragma unroll
  for (int j = 0; j < Q; ++j)
    if (L::ex(j) != 0)
      put<NTS>(a + run_addr<QT>(bb, j, -L::ey(j), -L::ez(j)) + bb.X[1], lds[H::flow_slot(j) * bt + seg + bb.X[1]]);
#pragma unroll
  for (int i = 0; i < QS; ++i)
    if (S::ex(i) != 0)
      put<NTS>(a + run_addr<QT>(bb, Q + i, -S::ey(i), -S::ez(i)) + bb.X[1],
               lds[H::scalar_slot(i) * bt + seg + bb.X[1]]);
}

// Pre-collision state of a node for the inspection and objective kernels: the
// access pattern of the buffer is a run-time argument there.
template <int Q, int QS, typename Real>
__device__ __forceinline__ void load_state_rt(const Real* a, const Nbr& b, int acc, Real (&f)[Q],
                                              Real (&g)[QS > 0 ? QS : 1]) {
  if (acc == ACC_EVEN) load_state<Q, QS, Real, ACC_EVEN>(a, b, f, g);
  else if (acc == ACC_ODD) load_state<Q, QS, Real, ACC_ODD>(a, b, f, g);
  else load_state<Q, QS, Real, ACC_PP>(a, b, f, g);
}

// ------------------------------------------------------- node operators
// All operators map the shifted pre-collision populations f~ (and scalar g)
// of one node to its shifted post-collision values in place.

// Interior: h = E(rho, G u) + (1 - omega)(f - E(rho, u))   (Section 3.1 with
// T = omega I, Section 3.2 for u_post = G(w) u_pre); scalar BGK toward the
// linear equilibrium at u_post.
// MRT relaxation map K = U^{-1} diag(1 - rate) U = U^T diag(mrt_k) U applied to
// a population vector (D3Q19; K is symmetric because U's rows are orthogonal).
template <typename Real>
__device__ __forceinline__ void mrt_apply(const Params<Real>& p, const Real (&d)[19], Real (&out)[19]) {
  Real m[19];
#pragma unroll
  for (int k = 0; k < 19; ++k) {
    Real s = 0;
#pragma unroll
    for (int j = 0; j < 19; ++j) {
      const int c = Mrt19::u(k, j);
      if (c == 1) s += d[j];
      else if (c == -1) s -= d[j];
      else if (c != 0) s += Real(c) * d[j];
    }
    m[k] = s * p.mrt_k[k];
  }
#pragma unroll
  for (int j = 0; j < 19; ++j) {
    Real s = 0;
#pragma unroll
    for (int k = 0; k < 19; ++k) {
      const int c = Mrt19::u(k, j);
      if (c == 1) s += m[k];
      else if (c == -1) s -= m[k];
      else if (c != 0) s += Real(c) * m[k];
    }
    out[j] = s;
  }
}

template <int Q, int QS, typename Real, int V = 0>
__device__ __forceinline__ void collide_interior(const Params<Real>& p, Real wn, Real (&f)[Q],
                                                 Real (&g)[QS > 0 ? QS : 1]) {
  using L = Lat<Q>;
  using S = SLat<QS>;
  constexpr bool MRT = (V & kVarMRT) != 0;
  constexpr bool VD = (V & kVarVD) != 0;
  Real drho = 0, mx = 0, my = 0, mz = 0;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    drho += f[j];
    if (L::ex(j)) mx += Real(L::ex(j)) * f[j];
    if (L::ey(j)) my += Real(L::ey(j)) * f[j];
    if (L::ez(j)) mz += Real(L::ez(j)) * f[j];
  }
  const Real rho = Real(1) + drho;
  const Real inv = Real(1) / rho;
  const Real ux = mx * inv, uy = my * inv, uz = mz * inv;
  Real G, dG;
  switch_fn(p, wn, G, dG);
  const Real usq = ux * ux + uy * uy + uz * uz;
  const Real G2 = G * G;
  if constexpr (MRT) {
    // FMRT (Section 3.1): h = E(rho, G u) + U^{-1}(I - T)U (f - E(rho, u))
    static_assert(Q == 19, "MRT is D3Q19 only");
    Real d[19];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const Real eu = Real(L::ex(j)) * ux + Real(L::ey(j)) * uy + Real(L::ez(j)) * uz;
      const Real Pu = Real(3) * eu + Real(4.5) * eu * eu - Real(1.5) * usq;
      d[j] = f[j] - Real(L::w(j)) * (drho + rho * Pu);  // shifted f minus shifted E(rho, u)
    }
    Real r[19];
    mrt_apply<Real>(p, d, r);
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const Real eu = Real(L::ex(j)) * ux + Real(L::ey(j)) * uy + Real(L::ez(j)) * uz;
      const Real Pv = G * Real(3) * eu + G2 * (Real(4.5) * eu * eu - Real(1.5) * usq);
      f[j] = Real(L::w(j)) * (drho + rho * Pv) + r[j];
    }
  } else {
    const Real om1 = Real(1) - p.om;
    const Real a0 = p.om * drho;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const Real eu = Real(L::ex(j)) * ux + Real(L::ey(j)) * uy + Real(L::ez(j)) * uz;
      // P(u) = 3 e.u + 4.5 (e.u)^2 - 1.5 u^2 (c_s^2 = 1/3), P(Gu) = G P1 + G^2 P2
      const Real P1 = Real(3) * eu;
      const Real P2 = Real(4.5) * eu * eu - Real(1.5) * usq;
      const Real Pu = P1 + P2;
      const Real Pv = G * P1 + G2 * P2;
      f[j] = om1 * f[j] + Real(L::w(j)) * (a0 + rho * (Pv - om1 * Pu));
    }
  }
  if constexpr (QS > 0) {
    Real T = 0;
#pragma unroll
    for (int i = 0; i < QS; ++i) T += g[i];
    const Real vx = G * ux, vy = G * uy, vz = G * uz;
    // blended diffusivity: tau_s(w) = w tau_fluid + (1 - w) tau_solid (Section 3.2)
    const Real oms = VD ? Real(1) / (wn * p.taus_f + (Real(1) - wn) * p.taus_s) : p.oms;
    const Real oms1 = Real(1) - oms;
    const Real ic2 = Real(1.0 / S::c2());
    // The rest population's equilibrium is T minus the others', so the
    // equilibria sum to T whatever the rounding of the weights: in FP32, 1/3 +
    // 4 (1/6) rounds to 1 + 3e-8, a bias that every step would add to the
    // conserved scalar (measured: a temperature drift of 4.7e-4 over 20000
    // steps of the 512x256 exchanger).
    Real E[QS], Es = 0;
#pragma unroll
    for (int i = 1; i < QS; ++i) {
      const Real ev = Real(S::ex(i)) * vx + Real(S::ey(i)) * vy + Real(S::ez(i)) * vz;
      E[i] = Real(S::w(i)) * T * (Real(1) + ev * ic2);
      Es += E[i];
    }
    E[0] = T - Es;
#pragma unroll
    for (int i = 0; i < QS; ++i) g[i] = oms1 * g[i] + oms * E[i];
  }
}

// Scalar condition of a wall node: Dirichlet at the heating plate (the stretch
// plate_x0 <= x < plate_x1 of the y = 0 wall, every z: the exchanger of Section
// 4), or at s_wall when the walls are Dirichlet; otherwise adiabatic (false).
template <typename Real>
__device__ __forceinline__ bool wall_dirichlet(const Params<Real>& p, int x, int y, Real& value) {
  if (y == 0 && x >= p.plate_x0 && x < p.plate_x1) {
    value = p.s_plate;
    return true;
  }
  value = p.s_wall;
  return p.scalar_wall == S_DIRICHLET;
}

// Wall: full-way bounce-back h_j = f_opp(j); scalar bounce-back (adiabatic)
// or equilibrium at the wall value with u = 0 (Dirichlet, see wall_dirichlet).
template <int Q, int QS, typename Real>
__device__ __forceinline__ void collide_wall(const Params<Real>& p, int x, int y, Real (&f)[Q],
                                             Real (&g)[QS > 0 ? QS : 1]) {
  using L = Lat<Q>;
  using S = SLat<QS>;
  Real t[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) t[j] = f[L::opp(j)];
#pragma unroll
  for (int j = 0; j < Q; ++j) f[j] = t[j];
  if constexpr (QS > 0) {
    Real tw;
    if (wall_dirichlet(p, x, y, tw)) {
#pragma unroll
      for (int i = 0; i < QS; ++i) g[i] = Real(S::w(i)) * tw;
    } else {
      Real s[QS];
#pragma unroll
      for (int i = 0; i < QS; ++i) s[i] = g[S::opp(i)];
#pragma unroll
      for (int i = 0; i < QS; ++i) g[i] = s[i];
    }
  }
}

// Inlet (x = 0): Zou-He, velocity u = (u_in, 0, 0) or pressure rho_in with
// its velocity limit (see inlet_state); the e_x = +1 populations are rebuilt
// from their opposites with the transverse correction
// N_t = 1/2 sum_{e_x=0} f_k e_kt, then BGK at E(rho, u).  The scalar's single
// unknown (+x) population is set so that sum g = T_in.
template <int Q, int QS, typename Real>
__device__ __forceinline__ void collide_inlet(const Params<Real>& p, int y, int z, Real (&f)[Q],
                                              Real (&g)[QS > 0 ? QS : 1]) {
  using L = Lat<Q>;
  using S = SLat<QS>;
  Real s0 = 0, sm = 0, Ny = 0, Nz = 0;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    if (L::ex(j) == 0) {
      s0 += f[j];
      if (L::ey(j)) Ny += Real(0.5 * L::ey(j)) * f[j];
      if (L::ez(j)) Nz += Real(0.5 * L::ez(j)) * f[j];
    } else if (L::ex(j) == -1) {
      sm += f[j];
    }
  }
  Real u, drho, up;
  inlet_state<Real>(p, s0, sm, u, drho, up);
  const Real rho = Real(1) + drho;
  const Real usq = u * u;
  Real fs[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    if (L::ex(j) == 1) {
      fs[j] = f[L::opp(j)] + Real(6.0 * L::w(j)) * rho * u - Real(L::ey(j)) * Ny - Real(L::ez(j)) * Nz;
    } else {
      fs[j] = f[j];
    }
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const Real eu = Real(L::ex(j)) * u;
    const Real E = Real(L::w(j)) * (drho + rho * (Real(3) * eu + Real(4.5) * eu * eu - Real(1.5) * usq));
    f[j] = fs[j] + p.om * (E - fs[j]);
  }
  if constexpr (QS > 0) {
    const Real T = inlet_value<Real>(p, y, z);
    Real rest = 0;
#pragma unroll
    for (int i = 0; i < QS; ++i)
      if (i != kPX) rest += g[i];
    g[kPX] = T - rest;
    const Real ic2 = Real(1.0 / S::c2());
#pragma unroll
    for (int i = 0; i < QS; ++i) {
      const Real E = Real(S::w(i)) * T * (Real(1) + Real(S::ex(i)) * u * ic2);
      g[i] = g[i] + p.oms * (E - g[i]);
    }
  }
}

// Outlet (x = nx-1): Zou-He density rho_out, u = (u_x, 0, 0); the e_x = -1
// populations are rebuilt, then BGK.  Scalar outflow: the unknown (-x)
// population takes its equilibrium value at the reconstructed T*.
template <int Q, int QS, typename Real>
__device__ __forceinline__ void collide_outlet(const Params<Real>& p, Real (&f)[Q], Real (&g)[QS > 0 ? QS : 1]) {
  using L = Lat<Q>;
  using S = SLat<QS>;
  Real s0 = 0, sp = 0, Ny = 0, Nz = 0;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    if (L::ex(j) == 0) {
      s0 += f[j];
      if (L::ey(j)) Ny += Real(0.5 * L::ey(j)) * f[j];
      if (L::ez(j)) Nz += Real(0.5 * L::ez(j)) * f[j];
    } else if (L::ex(j) == 1) {
      sp += f[j];
    }
  }
  const Real rho = p.rho_out;
  const Real drho = rho - Real(1);
  const Real ux = (s0 + Real(2) * sp - drho) / rho;
  const Real usq = ux * ux;
  Real fs[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    if (L::ex(j) == -1) {
      fs[j] = f[L::opp(j)] - Real(6.0 * L::w(j)) * rho * ux - Real(L::ey(j)) * Ny - Real(L::ez(j)) * Nz;
    } else {
      fs[j] = f[j];
    }
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const Real eu = Real(L::ex(j)) * ux;
    const Real E = Real(L::w(j)) * (drho + rho * (Real(3) * eu + Real(4.5) * eu * eu - Real(1.5) * usq));
    f[j] = fs[j] + p.om * (E - fs[j]);
  }
  if constexpr (QS > 0) {
    const Real ic2 = Real(1.0 / S::c2());
    Real rest = 0;
#pragma unroll
    for (int i = 0; i < QS; ++i)
      if (i != kMX) rest += g[i];
    const Real a = Real(S::w(kMX)) * (Real(1) - ux * ic2);
    const Real T = rest / (Real(1) - a);
    g[kMX] = a * T;
#pragma unroll
    for (int i = 0; i < QS; ++i) {
      const Real E = Real(S::w(i)) * T * (Real(1) + Real(S::ex(i)) * ux * ic2);
      g[i] = g[i] + p.oms * (E - g[i]);
    }
  }
}

// Moments of a node's pre-collision state that its transposed Jacobian needs:
// interior nodes (rho, u, and the scalar T = sum g), outlet nodes (u_x of the
// Zou-He reconstruction and the scalar sum over the known populations),
// pressure-inlet nodes (the pressure-form velocity up and the inlet scalar
// value); walls and velocity inlets are affine and need none.  The primal step
// records them (Mom::N values per node per step, plane-major) so the adjoint
// step does not re-read the Qt populations.  The sums follow the operators'
// order exactly.
template <int Q, int QS, int V = 0>
struct Mom {
  static constexpr int D = Lat<Q>::D;
  static constexpr bool VD = (V & kVarVD) != 0;
  // values per node: rho, u and the scalar sum T, or (blended diffusivity) the
  // QS scalar populations themselves, whose non-equilibrium part the w-derivative needs
  static constexpr int N = D + 1 + (QS > 0 ? (VD ? QS : 1) : 0);
  static constexpr int T = D + 1;  // index of the (first) scalar value
};

template <typename Real>
__device__ __forceinline__ bool has_moments(const Params<Real>& p, int cls) {
  return cls == INTERIOR || cls == OUTLET || (cls == INLET && p.inlet_mode == IN_PRESSURE);
}

template <int Q, int QS, typename Real, int V = 0>
__device__ __forceinline__ void node_moments(const Params<Real>& p, int cls, int y, int z, const Real (&f)[Q],
                                             const Real (&g)[QS > 0 ? QS : 1], Real (&m)[Mom<Q, QS, V>::N]) {
  using L = Lat<Q>;
  using M = Mom<Q, QS, V>;
#pragma unroll
  for (int k = 0; k < M::N; ++k) m[k] = Real(0);
  if (cls == INTERIOR) {
    Real drho = 0, mx = 0, my = 0, mz = 0;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      drho += f[j];
      if (L::ex(j)) mx += Real(L::ex(j)) * f[j];
      if (L::ey(j)) my += Real(L::ey(j)) * f[j];
      if (L::ez(j)) mz += Real(L::ez(j)) * f[j];
    }
    const Real rho = Real(1) + drho;
    const Real inv = Real(1) / rho;
    m[0] = rho;
    m[1] = mx * inv;
    m[2] = my * inv;
    if constexpr (M::D == 3) m[3] = mz * inv;
    if constexpr (QS > 0) {
      if constexpr (M::VD) {
#pragma unroll
        for (int i = 0; i < QS; ++i) m[M::T + i] = g[i];
      } else {
        Real T = 0;
#pragma unroll
        for (int i = 0; i < QS; ++i) T += g[i];
        m[M::T] = T;
      }
    }
  } else if (cls == OUTLET) {
    Real s0 = 0, sp = 0;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      if (L::ex(j) == 0) s0 += f[j];
      else if (L::ex(j) == 1) sp += f[j];
    }
    const Real ro = p.rho_out;
    m[1] = (s0 + Real(2) * sp - (ro - Real(1))) / ro;
    if constexpr (QS > 0) {
      Real rest = 0;
#pragma unroll
      for (int i = 0; i < QS; ++i)
        if (i != kMX) rest += g[i];
      m[M::T] = rest;
    }
  } else if (cls == INLET && p.inlet_mode == IN_PRESSURE) {
    Real s0 = 0, sm = 0;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      if (L::ex(j) == 0) s0 += f[j];
      else if (L::ex(j) == -1) sm += f[j];
    }
    Real u, drho, up;
    inlet_state<Real>(p, s0, sm, u, drho, up);
    m[1] = up;
    if constexpr (QS > 0) m[M::T] = inlet_value<Real>(p, y, z);
  }
}

// One primal node update: pull, collide by node class, store (coalesced).
// With MOM, also records the node's pre-collision moments (see Mom).
// src and dst are the same buffer for the in-place patterns, so they carry no
// restrict qualifier here (the ping-pong kernels declare theirs).
// NTE: streaming hint on the even phase's loads as well (states far beyond the
// last-level cache; see load_state)
template <int Q, int QS, typename Real, bool NT, bool MOM, int V, int ACC = ACC_PP, bool NTE = false, bool LX = false>
__device__ __forceinline__ void primal_node(const Params<Real>& p, const Real* src, Real* dst,
                                            const Real* __restrict__ w, Real* __restrict__ mom, int x, int y,
                                            int z, Real* lds = nullptr, int seg = 0, int bt = 0, bool act = true) {
  constexpr bool is3d = (Q == 19);
  const Nbr b = make_nbr(p, x, y, z);
  const int n = own_inode(b);  // workspace node arrays
  Real f[Q], g[QS > 0 ? QS : 1];
  if constexpr (LX)
    load_state_lx<Q, QS, Real, ACC, NT, NT && ACC == ACC_PP>(src, b, f, g, lds, seg, bt, act);
  else
    load_state<Q, QS, Real, ACC, NT && (ACC != ACC_EVEN || NTE)>(src, b, f, g);
  // padding lanes (LX only) take the wall operator: a permutation, no memory access
  const int cls = act ? node_class(p, x, y, z, is3d) : WALL;
  if constexpr (MOM) {
    if (has_moments(p, cls)) {  // the only classes whose transposes read them
      Real m[Mom<Q, QS, V>::N];
      node_moments<Q, QS, Real, V>(p, cls, y, z, f, g, m);
      // streaming stores whatever the state size: a moment set is read once, by the
      // adjoint, after the rest of the run has passed through the cache
#pragma unroll
      for (int k = 0; k < Mom<Q, QS, V>::N; ++k) put<true>(mom + (size_t)k * p.Np + n, m[k]);
    }
  }
  if (cls == INTERIOR) {
    collide_interior<Q, QS, Real, V>(p, w[n], f, g);
  } else if (cls == WALL) {
    collide_wall<Q, QS, Real>(p, x, y, f, g);
  } else if (cls == INLET) {
    collide_inlet<Q, QS, Real>(p, y, z, f, g);
  } else {
    collide_outlet<Q, QS, Real>(p, f, g);
  }
  if constexpr (LX && ACC == ACC_ODD)
    store_state_lx<Q, QS, Real, NT, false>(dst, b, f, g, lds, seg, bt, act);
  else if (act)
    store_state<Q, QS, Real, NT, ACC>(dst, b, f, g);
}

// LX: the block spans whole rows and the x-shifted populations go through LDS
// (see load_state_lx); no thread leaves before the barriers.
template <int Q, int QS, typename Real, bool NT, bool MOM, int V, bool LX = false>
__global__ __launch_bounds__(kHotThreads) void k_primal(Params<Real> p, const Real* __restrict__ src,
                                                Real* __restrict__ dst, const Real* __restrict__ w,
                                                Real* __restrict__ mom) {
  int x, y, z;
  const bool act = hot_pos(p, x, y, z);
  if constexpr (LX) {
    Real* lds = lx_lds<Real>();
    primal_node<Q, QS, Real, NT, MOM, V, ACC_PP, false, true>(p, src, dst, w, mom, x, y, z, lds, lx_seg(), lx_span(),
                                                              act);
  } else {
    if (!act) return;
    primal_node<Q, QS, Real, NT, MOM, V>(p, src, dst, w, mom, x, y, z);
  }
}

// One in-place step (even or odd phase); with MOM it also records the moments.
template <int Q, int QS, typename Real, bool NT, bool MOM, int V, int ACC, bool NTE = false, bool LX = false>
__global__ __launch_bounds__(kHotThreads) void k_primal_inplace(Params<Real> p, Real* a, const Real* __restrict__ w,
                                                        Real* __restrict__ mom) {
  int x, y, z;
  const bool act = hot_pos(p, x, y, z);
  if constexpr (LX) {
    static_assert(ACC == ACC_ODD, "only the odd phase has shifted access");
    Real* lds = lx_lds<Real>();
    primal_node<Q, QS, Real, NT, MOM, V, ACC, NTE, true>(p, a, a, w, mom, x, y, z, lds, lx_seg(), lx_span(), act);
  } else {
    if (!act) return;
    primal_node<Q, QS, Real, NT, MOM, V, ACC, NTE>(p, a, a, w, mom, x, y, z);
  }
}

// ------------------------------------------------------------ objective
// Boundary sums ("Globals") of the pre-collision state pulled from src, and
// J = c_dp*dp + c_hf*HF + c_var*Var + c_mix*Mix.  Stage 1: kObjBlocks blocks
// each reduce a fixed strided subset of the inlet/outlet nodes in LDS (fixed
// tree order) and write kNG partial sums; stage 2: one thread adds the partials
// in block order.  out[0..8] = sums (see lbm_objective), out[9] = J.
constexpr int kNG = 9;
constexpr int kObjThreads = 256;
constexpr int kObjBlocks = 64;

template <int Q, int QS, typename Real>
__global__ __launch_bounds__(kObjThreads) void k_objective_partial(Params<Real> p, const Real* __restrict__ src,
                                                                   double* __restrict__ part, int pattern) {
  using L = Lat<Q>;
  using S = SLat<QS>;
  constexpr bool is3d = (Q == 19);
  __shared__ double red[kNG][kObjThreads];
  double acc[kNG];
#pragma unroll
  for (int k = 0; k < kNG; ++k) acc[k] = 0.0;
  const int plane = p.ny * p.nz;
  if (!p.periodic) {
    for (int k = blockIdx.x * kObjThreads + threadIdx.x; k < 2 * plane; k += kObjBlocks * kObjThreads) {
      const int side = k / plane;
      const int r = k - side * plane;
      const int y = r % p.ny, z = r / p.ny;
      const int x = side ? p.nx - 1 : 0;
      if (node_class(p, x, y, z, is3d) == WALL) continue;
      const Nbr b = make_nbr(p, x, y, z);
      Real f[Q], g[QS > 0 ? QS : 1];
      load_state_rt<Q, QS, Real>(src, b, pattern, f, g);
      double s0 = 0, sk = 0;
      Real s0r = 0, skr = 0;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        if (L::ex(j) == 0) {
          s0 += (double)f[j];
          s0r += f[j];
        } else if (L::ex(j) == (side ? 1 : -1)) {
          sk += (double)f[j];
          skr += f[j];
        }
      }
      if (side == 0) {
        Real u, drho, up;  // which inlet form runs is decided exactly as in the step
        const bool pressure = inlet_state<Real>(p, s0r, skr, u, drho, up);
        acc[0] += pressure ? p.rho_in : (1.0 + s0 + 2.0 * sk) / (1.0 - (double)u);
        acc[1] += 1.0;
      } else {
        const double ro = (double)p.rho_out;
        const double ux = (1.0 + s0 + 2.0 * sk) / ro - 1.0;
        acc[2] += ro;
        acc[3] += 1.0;
        acc[7] += ux;
        if constexpr (QS > 0) {
          double rest = 0;
#pragma unroll
          for (int i = 0; i < QS; ++i)
            if (i != kMX) rest += (double)g[i];
          const double a = S::w(kMX) * (1.0 - ux / S::c2());
          const double T = rest / (1.0 - a);
          acc[4] += ux * T;
          acc[5] += T;
          acc[6] += T * T;
          acc[8] += ux * T * T;
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kNG; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = kObjThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int k = 0; k < kNG; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x < kNG) part[blockIdx.x * kNG + threadIdx.x] = red[threadIdx.x][0];
}

template <int Q, int QS, typename Real>
__global__ __launch_bounds__(64) void k_objective_final(Params<Real> p, const double* __restrict__ part,
                                                        double* __restrict__ out) {
  using L = Lat<Q>;
  if (threadIdx.x != 0) return;
  double G[kNG];
#pragma unroll
  for (int k = 0; k < kNG; ++k) G[k] = 0.0;
  for (int b = 0; b < kObjBlocks; ++b) {
#pragma unroll
    for (int k = 0; k < kNG; ++k) G[k] += part[b * kNG + k];
  }
  double J = 0;
  if (!p.periodic && G[1] > 0 && G[3] > 0) {
    const double dp = L::cs2() * (G[0] / G[1] - G[2] / G[3]);
    const double mean = G[5] / G[3];
    J = p.c_dp * dp + p.c_hf * G[4] + p.c_var * (G[6] / G[3] - mean * mean) + p.c_mix * (G[7] - G[8]);
  }
#pragma unroll
  for (int k = 0; k < kNG; ++k) out[k] = G[k];
  out[kNG] = J;
}

// ------------------------------------------------------------ adjoint seed
// dJ/df and dJ/dg of one node's pre-collision state (zero except at inlet and
// outlet nodes); glob holds the boundary sums of the current state.
template <int Q, int QS, typename Real>
__device__ __forceinline__ void seed_values(const Params<Real>& p, int cls, const Real (&f)[Q],
                                            const Real (&g)[QS > 0 ? QS : 1], const double* __restrict__ glob,
                                            double (&lf)[Q], double (&lg)[QS > 0 ? QS : 1]) {
  using L = Lat<Q>;
  using S = SLat<QS>;
#pragma unroll
  for (int j = 0; j < Q; ++j) lf[j] = 0.0;
#pragma unroll
  for (int i = 0; i < (QS > 0 ? QS : 1); ++i) lg[i] = 0.0;
  if (cls == INLET && glob[1] > 0) {
    // inlet rho: P / (1 - u) in the velocity form, the constant rho_in in the pressure form
    Real s0 = 0, sm = 0;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      if (L::ex(j) == 0) s0 += f[j];
      else if (L::ex(j) == -1) sm += f[j];
    }
    Real u, drho, up;
    const bool pressure = inlet_state<Real>(p, s0, sm, u, drho, up);
    const double dG0 = p.c_dp * L::cs2() / glob[1];
    const double c = pressure ? 0.0 : dG0 / (1.0 - (double)u);
#pragma unroll
    for (int j = 0; j < Q; ++j) lf[j] = (L::ex(j) == 0) ? c : (L::ex(j) == -1 ? 2.0 * c : 0.0);
  }
  if constexpr (QS > 0) {
    if (cls == OUTLET && glob[3] > 0) {
      const double G3 = glob[3];
      const double A4 = p.c_hf, A5 = -2.0 * p.c_var * glob[5] / (G3 * G3), A6 = p.c_var / G3;
      double s0 = 0, sp = 0, rest = 0;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        if (L::ex(j) == 0) s0 += (double)f[j];
        else if (L::ex(j) == 1) sp += (double)f[j];
      }
#pragma unroll
      for (int i = 0; i < QS; ++i)
        if (i != kMX) rest += (double)g[i];
      const double ro = (double)p.rho_out;
      const double ux = (1.0 + s0 + 2.0 * sp) / ro - 1.0;
      const double a = S::w(kMX) * (1.0 - ux / S::c2());
      const double T = rest / (1.0 - a);
      const double Am = p.c_mix;
      const double dT = A4 * ux + A5 + 2.0 * A6 * T - 2.0 * Am * ux * T;  // dJ/dT*
      const double dux = A4 * T + Am * (1.0 - T * T) + dT * (-T * S::w(kMX) / (S::c2() * (1.0 - a)));
#pragma unroll
      for (int j = 0; j < Q; ++j) lf[j] = (L::ex(j) == 0) ? dux / ro : (L::ex(j) == 1 ? 2.0 * dux / ro : 0.0);
#pragma unroll
      for (int i = 0; i < QS; ++i) lg[i] = (i == kMX) ? 0.0 : dT / (1.0 - a);
    }
  }
}

// lambda^N = dJ/df^N: non-zero only at inlet/outlet nodes.  Uses the sums
// written by the objective kernel (glob[0..7]).
template <int Q, int QS, typename Real>
__device__ __forceinline__ void seed_node(const Params<Real>& p, const Real* __restrict__ src,
                                          const double* __restrict__ glob, Real* __restrict__ lam, int x, int y,
                                          int z, int pattern, int inplace_out, double scale) {
  using L = Lat<Q>;
  using S = SLat<QS>;
  constexpr bool is3d = (Q == 19);
  constexpr int QT = Q + QS;
  const Nbr b = make_nbr(p, x, y, z);
  const int cls = node_class(p, x, y, z, is3d);
  Real f[Q], g[QS > 0 ? QS : 1];
  if ((QS > 0 && cls == OUTLET) || (cls == INLET && p.inlet_mode == IN_PRESSURE)) {
    load_state_rt<Q, QS, Real>(src, b, pattern, f, g);
  } else {
#pragma unroll
    for (int j = 0; j < Q; ++j) f[j] = Real(0);
#pragma unroll
    for (int i = 0; i < (QS > 0 ? QS : 1); ++i) g[i] = Real(0);
  }
  double lf[Q], lg[QS > 0 ? QS : 1];
  seed_values<Q, QS, Real>(p, cls, f, g, glob, lf, lg);
  // in place, lambda^N enters in the layout the first (odd-pattern) adjoint step
  // reads: lambda_j(x) in slot opp(j) of x.  scale: 1, or 1/W for an objective
  // averaged over the last W states
#pragma unroll
  for (int j = 0; j < Q; ++j) lam[own_addr<QT>(b, inplace_out ? L::opp(j) : j)] = (Real)(lf[j] * scale);
#pragma unroll
  for (int i = 0; i < QS; ++i) lam[own_addr<QT>(b, Q + (inplace_out ? S::opp(i) : i))] = (Real)(lg[i] * scale);
}

template <int Q, int QS, typename Real>
__global__ __launch_bounds__(256) void k_seed(Params<Real> p, const Real* __restrict__ src,
                                              const double* __restrict__ glob, Real* __restrict__ lam, int pattern,
                                              int inplace_out, double scale) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= p.nx) return;
  seed_node<Q, QS, Real>(p, src, glob, lam, x, blockIdx.y, blockIdx.z, pattern, inplace_out, scale);
}

// ------------------------------------------- time-averaged objective window
// With J = (1/W) sum of the objective over the states f^{N-W+1} .. f^N, each
// window state is captured after the step that produces it: its inlet and
// outlet columns (pre-collision, as pulled; bnd layout [side][Qt][row], row =
// y + ny z) and, through the objective kernels, its boundary sums and objective.
// The adjoint adds (1/W) dJ/df^n of every window state n < N to lambda^n.
template <int Q, int QS, typename Real>
__global__ __launch_bounds__(256) void k_capture_columns(Params<Real> p, const Real* __restrict__ src, int pattern,
                                                         Real* __restrict__ bnd) {
  constexpr int QT = Q + QS;
  const int plane = p.ny * p.nz;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 2 * plane) return;
  const int side = k / plane, r = k - side * plane;
  const int y = r % p.ny, z = r / p.ny;
  const Nbr b = make_nbr(p, side ? p.nx - 1 : 0, y, z);
  Real f[Q], g[QS > 0 ? QS : 1];
  load_state_rt<Q, QS, Real>(src, b, pattern, f, g);
  Real* o = bnd + (size_t)side * QT * plane + r;
#pragma unroll
  for (int j = 0; j < Q; ++j) o[(size_t)j * plane] = f[j];
#pragma unroll
  for (int i = 0; i < QS; ++i) o[(size_t)(Q + i) * plane] = g[i];
}

// lambda^n += scale * dJ/df^n at the inlet and outlet nodes, from the captured
// columns of f^n and its boundary sums glob; lambda^n in the cotangent layout
// pattern (ACC_PP: slot j of x; ACC_ODD: slot opp(j) of x; ACC_EVEN: slot j of
// x - e_j), as the adjoint step left it.
template <int Q, int QS, typename Real>
__global__ __launch_bounds__(256) void k_window_seed(Params<Real> p, const Real* __restrict__ bnd,
                                                     const double* __restrict__ glob, Real* __restrict__ lam,
                                                     int pattern, double scale) {
  using L = Lat<Q>;
  using S = SLat<QS>;
  constexpr bool is3d = (Q == 19);
  constexpr int QT = Q + QS;
  const int plane = p.ny * p.nz;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 2 * plane) return;
  const int side = k / plane, r = k - side * plane;
  const int y = r % p.ny, z = r / p.ny;
  const int x = side ? p.nx - 1 : 0;
  const int cls = node_class(p, x, y, z, is3d);
  if (cls != INLET && cls != OUTLET) return;
  const Nbr b = make_nbr(p, x, y, z);
  const Real* o = bnd + (size_t)side * QT * plane + r;
  Real f[Q], g[QS > 0 ? QS : 1];
#pragma unroll
  for (int j = 0; j < Q; ++j) f[j] = o[(size_t)j * plane];
#pragma unroll
  for (int i = 0; i < (QS > 0 ? QS : 1); ++i) g[i] = QS > 0 ? o[(size_t)(Q + i) * plane] : Real(0);
  double lf[Q], lg[QS > 0 ? QS : 1];
  seed_values<Q, QS, Real>(p, cls, f, g, glob, lf, lg);
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const int a = pattern == ACC_EVEN ? pull_addr<QT>(b, j, L::ex(j), L::ey(j), L::ez(j))
                                      : own_addr<QT>(b, pattern == ACC_ODD ? L::opp(j) : j);
    lam[a] += (Real)(lf[j] * scale);
  }
#pragma unroll
  for (int i = 0; i < QS; ++i) {
    const int a = pattern == ACC_EVEN ? pull_addr<QT>(b, Q + i, S::ex(i), S::ey(i), S::ez(i))
                                      : own_addr<QT>(b, Q + (pattern == ACC_ODD ? S::opp(i) : i));
    lam[a] += (Real)(lg[i] * scale);
  }
}

// J of the window: glob[kNG] = (1/W) sum of the window's objectives (each slot of
// win holds kNG sums and J); glob[0..kNG) keep the final state's sums.
__global__ void k_window_mean(const double* __restrict__ win, int W, double* __restrict__ glob) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double J = 0.0;
  for (int s = 0; s < W; ++s) J += win[(size_t)s * (kNG + 1) + kNG];
  glob[kNG] = J / (double)W;
}

// ------------------------------------------------------------ adjoint step
// Vector-Jacobian product of one node operator: given the moments m of the
// node's pre-collision state (see Mom), its design value wn and the cotangents
// (mu, nu) of its post-collision populations, returns lambda =
// (dW/d(f,g))^T (mu, nu) and gw = (dW/dw)^T (mu, nu) (zero except at interior
// nodes).  Wall and velocity-inlet operators are affine in (f, g): their
// products do not read m.  Hand-derived from the operators above.
template <int Q, int QS, typename Real, int V = 0>
__device__ __forceinline__ void adjoint_vjp(const Params<Real>& p, int cls, int x, int y,
                                            const Real (&m)[Mom<Q, QS, V>::N],
                                            Real wn, const Real (&mu)[Q], const Real (&nu)[QS > 0 ? QS : 1],
                                            Real (&lf)[Q], Real (&lg)[QS > 0 ? QS : 1], Real& gw) {
  using L = Lat<Q>;
  using S = SLat<QS>;
  using M = Mom<Q, QS, V>;
  constexpr bool MRT = (V & kVarMRT) != 0;
  constexpr bool VD = (V & kVarVD) != 0;
  gw = Real(0);
  const Real om1 = Real(1) - p.om;
  const Real oms1 = Real(1) - p.oms;
  if (cls == WALL) {
#pragma unroll
    for (int j = 0; j < Q; ++j) lf[j] = mu[L::opp(j)];
    Real tw;
    const bool dir = wall_dirichlet(p, x, y, tw);  // Dirichlet: g' does not depend on g
#pragma unroll
    for (int i = 0; i < QS; ++i) lg[i] = dir ? Real(0) : nu[S::opp(i)];
  } else if (cls == INLET) {
    // Velocity form (u_in, or u_cap where the pressure form was limited):
    // h = (1-omega) f* + omega E(rho, u) is affine in f.  Pressure form: rho is
    // fixed and u = (rho_in - P) / rho_in, so the product runs through u; which
    // form ran is read from the recorded pressure-form velocity m[1].
    bool pressure = false;
    Real u = p.u_in;
    if (p.inlet_mode == IN_PRESSURE) {
      const Real up = m[1];
      pressure = !(p.u_cap > Real(0) && up > p.u_cap);
      u = pressure ? up : p.u_cap;
    }
    if (!pressure) {
      const Real usq = u * u;
      Real B = 0, drho = 0, dNy = 0, dNz = 0;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const Real eu = Real(L::ex(j)) * u;
        B += mu[j] * Real(L::w(j)) * (Real(1) + Real(3) * eu + Real(4.5) * eu * eu - Real(1.5) * usq);
        if (L::ex(j) == 1) {
          drho += om1 * mu[j] * Real(6.0 * L::w(j)) * u;
          if (L::ey(j)) dNy -= om1 * mu[j] * Real(L::ey(j));
          if (L::ez(j)) dNz -= om1 * mu[j] * Real(L::ez(j));
        }
      }
      drho += p.om * B;
      const Real c = drho / (Real(1) - u);
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        Real v = 0;
        if (L::ex(k) == 0) v = om1 * mu[k] + c + Real(0.5) * (Real(L::ey(k)) * dNy + Real(L::ez(k)) * dNz);
        if (L::ex(k) == -1) v = om1 * (mu[k] + mu[L::opp(k)]) + Real(2) * c;
        lf[k] = v;
      }
    } else {
      const Real ro = Real(1) + p.drho_in;
      Real dux = 0, dNy = 0, dNz = 0;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const Real ex = Real(L::ex(j));
        dux += p.om * ro * mu[j] * Real(L::w(j)) * (Real(3) * ex + Real(9) * ex * ex * u - Real(3) * u);
        if (L::ex(j) == 1) {
          dux += om1 * mu[j] * Real(6.0 * L::w(j)) * ro;
          if (L::ey(j)) dNy -= om1 * mu[j] * Real(L::ey(j));
          if (L::ez(j)) dNz -= om1 * mu[j] * Real(L::ez(j));
        }
      }
      if constexpr (QS > 0) {
        // the scalar equilibrium at the fixed inlet value T_in (m[T]) moves with u
        Real N1x = 0;
#pragma unroll
        for (int i = 0; i < QS; ++i)
          if (S::ex(i)) N1x += Real(S::ex(i)) * nu[i] * Real(S::w(i));
        dux += p.oms * m[M::T] * N1x * Real(1.0 / S::c2());
      }
      const Real c = -dux / ro;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        Real v = 0;
        if (L::ex(k) == 0) v = om1 * mu[k] + c + Real(0.5) * (Real(L::ey(k)) * dNy + Real(L::ez(k)) * dNz);
        if (L::ex(k) == -1) v = om1 * (mu[k] + mu[L::opp(k)]) + Real(2) * c;
        lf[k] = v;
      }
    }
    if constexpr (QS > 0) {
#pragma unroll
      for (int i = 0; i < QS; ++i) lg[i] = (i == kPX) ? Real(0) : oms1 * (nu[i] - nu[kPX]);
    }
  } else {
    if (cls == INTERIOR) {
      const Real rho = m[0];
      const Real inv = Real(1) / rho;
      const Real ux = m[1], uy = m[2];
      Real uz = Real(0);
      if constexpr (M::D == 3) uz = m[3];
      const Real usq = ux * ux + uy * uy + uz * uz;
      Real G, dG;
      switch_fn(p, wn, G, dG);
      const Real G2 = G * G;
      // cotangent moments M0 = sum mu w, M1 = sum mu w e, P = sum mu w (e.u) e; M0 is
      // taken as mu_0 + sum_{j>0} w_j (mu_j - mu_0), which is exact for a uniform
      // cotangent however the weights round (the rounded weights sum to 1 + 1.5e-8
      // in FP32, and the plain sum would grow a uniform cotangent by that each step)
      Real M0 = mu[0], M1x = 0, M1y = 0, M1z = 0, Px = 0, Py = 0, Pz = 0;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const Real a = mu[j] * Real(L::w(j));
        const Real eu = Real(L::ex(j)) * ux + Real(L::ey(j)) * uy + Real(L::ez(j)) * uz;
        const Real be = a * eu;
        if (j > 0) M0 += Real(L::w(j)) * (mu[j] - mu[0]);
        if (L::ex(j)) { M1x += Real(L::ex(j)) * a; Px += Real(L::ex(j)) * be; }
        if (L::ey(j)) { M1y += Real(L::ey(j)) * a; Py += Real(L::ey(j)) * be; }
        if (L::ez(j)) { M1z += Real(L::ez(j)) * a; Pz += Real(L::ez(j)) * be; }
      }
      const Real Mu = M1x * ux + M1y * uy + M1z * uz;
      const Real Pu = Px * ux + Py * uy + Pz * uz;
      Real dL_drho, dux, duy, duz;
      Real kap[Q];  // MRT: the relaxed cotangent K mu (K symmetric); BGK uses (1 - omega) mu
      if constexpr (MRT) {
        // h = E(rho, G u) + K (f - E(rho, u)):  lambda = K mu + (dE(rho,Gu)/df)^T mu - (dE(rho,u)/df)^T K mu
        mrt_apply<Real>(p, mu, kap);
        Real K0 = kap[0], K1x = 0, K1y = 0, K1z = 0, KPx = 0, KPy = 0, KPz = 0;
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          const Real a = kap[j] * Real(L::w(j));
          const Real eu = Real(L::ex(j)) * ux + Real(L::ey(j)) * uy + Real(L::ez(j)) * uz;
          const Real be = a * eu;
          if (j > 0) K0 += Real(L::w(j)) * (kap[j] - kap[0]);  // as M0
          if (L::ex(j)) { K1x += Real(L::ex(j)) * a; KPx += Real(L::ex(j)) * be; }
          if (L::ey(j)) { K1y += Real(L::ey(j)) * a; KPy += Real(L::ey(j)) * be; }
          if (L::ez(j)) { K1z += Real(L::ez(j)) * a; KPz += Real(L::ez(j)) * be; }
        }
        const Real Ku = K1x * ux + K1y * uy + K1z * uz;
        const Real KPu = KPx * ux + KPy * uy + KPz * uz;
        dL_drho = (M0 + Real(3) * G * Mu + Real(4.5) * G2 * Pu - Real(1.5) * G2 * M0 * usq) -
                  (K0 + Real(3) * Ku + Real(4.5) * KPu - Real(1.5) * K0 * usq);
        const Real g1 = Real(3) * G, g2 = Real(9) * G2, g3 = Real(3) * G2 * M0, k3 = Real(3) * K0;
        dux = rho * ((g1 * M1x + g2 * Px - g3 * ux) - (Real(3) * K1x + Real(9) * KPx - k3 * ux));
        duy = rho * ((g1 * M1y + g2 * Py - g3 * uy) - (Real(3) * K1y + Real(9) * KPy - k3 * uy));
        duz = rho * ((g1 * M1z + g2 * Pz - g3 * uz) - (Real(3) * K1z + Real(9) * KPz - k3 * uz));
      } else {
        // d/drho at fixed u of A(rho, G u) - (1-omega) A(rho, u), A = sum mu_j E_j
        dL_drho = M0 * (Real(1) - om1) + Real(3) * (G - om1) * Mu + Real(4.5) * (G2 - om1) * Pu -
                  Real(1.5) * (G2 - om1) * M0 * usq;
        const Real c1 = Real(3) * (G - om1), c2 = Real(9) * (G2 - om1), c3 = Real(3) * (G2 - om1) * M0;
        dux = rho * (c1 * M1x + c2 * Px - c3 * ux);
        duy = rho * (c1 * M1y + c2 * Py - c3 * uy);
        duz = rho * (c1 * M1z + c2 * Pz - c3 * uz);
      }
      Real dLdG = rho * (Real(3) * Mu + Real(9) * G * Pu - Real(3) * G * M0 * usq);
      Real gws = 0;  // blended diffusivity: d omega_s / dw times the scalar's non-equilibrium product
      if constexpr (QS > 0) {
        Real T;
        if constexpr (VD) {
          T = 0;
#pragma unroll
          for (int i = 0; i < QS; ++i) T += m[M::T + i];
        } else {
          T = m[M::T];
        }
        // N0 = sum nu w as nu_0 + sum_{i>0} w_i (nu_i - nu_0), the transpose of the
        // primal's rest equilibrium taken by difference
        Real N0 = nu[0], N1x = 0, N1y = 0, N1z = 0;
#pragma unroll
        for (int i = 0; i < QS; ++i) {
          const Real a = nu[i] * Real(S::w(i));
          if (i > 0) N0 += Real(S::w(i)) * (nu[i] - nu[0]);
          if (S::ex(i)) N1x += Real(S::ex(i)) * a;
          if (S::ey(i)) N1y += Real(S::ey(i)) * a;
          if (S::ez(i)) N1z += Real(S::ez(i)) * a;
        }
        const Real ic2 = Real(1.0 / S::c2());
        const Real N1u = N1x * ux + N1y * uy + N1z * uz;
        Real oms = p.oms;
        if constexpr (VD) {
          // g' = g + omega(w) (E^s - g), omega(w) = 1 / (w tau_f + (1 - w) tau_s):
          // the w-derivative adds omega'(w) sum_i nu_i (E^s_i - g_i)
          const Real tw = wn * p.taus_f + (Real(1) - wn) * p.taus_s;
          oms = Real(1) / tw;
          Real nug = 0;
#pragma unroll
          for (int i = 0; i < QS; ++i) nug += nu[i] * m[M::T + i];
          gws = -(p.taus_f - p.taus_s) * oms * oms * (T * (N0 + G * N1u * ic2) - nug);
        }
        const Real k = oms * T * G * ic2;
        dux += k * N1x;
        duy += k * N1y;
        duz += k * N1z;
        dLdG += oms * T * N1u * ic2;
        const Real dT = oms * (N0 + G * N1u * ic2);
        const Real oms1w = Real(1) - oms;
#pragma unroll
        for (int i = 0; i < QS; ++i) lg[i] = oms1w * nu[i] + dT;
      }
      const Real dmx = dux * inv, dmy = duy * inv, dmz = duz * inv;
      const Real drt = dL_drho - (dux * ux + duy * uy + duz * uz) * inv;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        Real v;
        if constexpr (MRT) v = kap[k] + drt;
        else v = om1 * mu[k] + drt;
        if (L::ex(k)) v += Real(L::ex(k)) * dmx;
        if (L::ey(k)) v += Real(L::ey(k)) * dmy;
        if (L::ez(k)) v += Real(L::ez(k)) * dmz;
        lf[k] = v;
      }
      gw = dG * dLdG + gws;
    } else {  // OUTLET
      const Real ro = p.rho_out;
      const Real ux = m[1];
      Real dux = 0, dNy = 0, dNz = 0;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const Real ex = Real(L::ex(j));
        dux += p.om * ro * mu[j] * Real(L::w(j)) * (Real(3) * ex + Real(9) * ex * ex * ux - Real(3) * ux);
        if (L::ex(j) == -1) {
          dux -= om1 * mu[j] * Real(6.0 * L::w(j)) * ro;
          if (L::ey(j)) dNy -= om1 * mu[j] * Real(L::ey(j));
          if (L::ez(j)) dNz -= om1 * mu[j] * Real(L::ez(j));
        }
      }
      if constexpr (QS > 0) {
        const Real ic2 = Real(1.0 / S::c2());
        const Real rest = m[M::T];
        Real N0 = 0, N1x = 0;
#pragma unroll
        for (int i = 0; i < QS; ++i) {
          const Real a = nu[i] * Real(S::w(i));
          N0 += a;
          if (S::ex(i)) N1x += Real(S::ex(i)) * a;
        }
        const Real a = Real(S::w(kMX)) * (Real(1) - ux * ic2);
        const Real inv1a = Real(1) / (Real(1) - a);
        const Real T = rest * inv1a;
        const Real dT = oms1 * nu[kMX] * a + p.oms * (N0 + N1x * ux * ic2);
        const Real da = oms1 * nu[kMX] * T + dT * T * inv1a;
        const Real dS = dT * inv1a;
        dux += p.oms * T * N1x * ic2 - da * Real(S::w(kMX)) * ic2;
#pragma unroll
        for (int i = 0; i < QS; ++i) lg[i] = (i == kMX) ? Real(0) : oms1 * nu[i] + dS;
      }
      const Real c = dux / ro;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        Real v = 0;
        if (L::ex(k) == 0) v = om1 * mu[k] + c + Real(0.5) * (Real(L::ey(k)) * dNy + Real(L::ez(k)) * dNz);
        if (L::ex(k) == 1) v = om1 * (mu[k] + mu[L::opp(k)]) + Real(2) * c;
        lf[k] = v;
      }
    }
  }
}

// lambda^n(x) = (dW^x/df)^T(f^n(x)) mu(x),  mu_j(x) = lambda^{n+1}_j(x + e_j)
// grad(x)    += (dW^x/dw)^T mu(x)            (interior nodes only)
// The vector-Jacobian products below are hand-derived from the operators above.
// lam_in and lam_out are the same buffer in place (ACC_EVEN / ACC_ODD).  NTE:
// the even phase's cotangent loads take the streaming hint as well; as for the
// primal, that pays only for states far beyond the last-level cache (60
// recorded steps, in-place adjoint at 256x128x128: 0.829 with it, 0.847
// without, the 2000-step evaluation unchanged; at 512x128x128: 0.813 with it,
// 0.660 without).
template <int Q, int QS, typename Real, bool NT, int V, int ACC = ACC_PP, bool NTE = false, bool LX = false>
__device__ __forceinline__ void adjoint_node(const Params<Real>& p, const Real* __restrict__ mom,
                                             const Real* lam_in, Real* lam_out, const Real* __restrict__ w,
                                             Real* __restrict__ grad, int x, int y, int z, Real* lds = nullptr,
                                             int seg = 0, int bt = 0, bool act = true) {
  constexpr bool is3d = (Q == 19);
  constexpr int QSA = QS > 0 ? QS : 1;
  const Nbr b = make_nbr(p, x, y, z);
  const int n = own_inode(b);  // workspace node arrays
  Real mu[Q], nu[QSA];
  if constexpr (LX)
    load_cot_lx<Q, QS, Real, ACC, NT, NT && (ACC == ACC_PP || NTE)>(lam_in, b, mu, nu, lds, seg, bt, act);
  else
    load_cot<Q, QS, Real, ACC, NT && (ACC != ACC_EVEN || NTE)>(lam_in, b, mu, nu);
  // padding lanes (LX only) take the wall transpose: a permutation, no memory access
  const int cls = act ? node_class(p, x, y, z, is3d) : WALL;
  Real m[Mom<Q, QS, V>::N], lf[Q], lg[QSA], gw;
#pragma unroll
  for (int k = 0; k < Mom<Q, QS, V>::N; ++k) m[k] = Real(0);
  if (has_moments(p, cls)) {
#pragma unroll
    // read once: streaming hint whatever the state size, so that the moments do not
    // evict a cotangent state the last-level cache could hold between steps
    for (int k = 0; k < Mom<Q, QS, V>::N; ++k) m[k] = get<true>(mom + (size_t)k * p.Np + n);
  }
  const Real wn = (cls == INTERIOR) ? w[n] : Real(1);
  adjoint_vjp<Q, QS, Real, V>(p, cls, x, y, m, wn, mu, nu, lf, lg, gw);
  if (cls == INTERIOR) grad[n] += gw;
  if constexpr (LX && ACC == ACC_ODD)
    store_cot_lx<Q, QS, Real, NT, NT && NTE>(lam_out, b, lf, lg, lds, seg, bt, act);
  else if (act)
    store_cot<Q, QS, Real, NT, ACC>(lam_out, b, lf, lg);
}

// LX as for k_primal.
template <int Q, int QS, typename Real, bool NT, int V, bool LX = false>
__global__ __launch_bounds__(kHotThreads) void k_adjoint(Params<Real> p, const Real* __restrict__ mom,
                                                 const Real* __restrict__ lam_in, Real* __restrict__ lam_out,
                                                 const Real* __restrict__ w, Real* __restrict__ grad) {
  int x, y, z;
  const bool act = hot_pos(p, x, y, z);
  if constexpr (LX) {
    Real* lds = lx_lds<Real>();
    adjoint_node<Q, QS, Real, NT, V, ACC_PP, false, true>(p, mom, lam_in, lam_out, w, grad, x, y, z, lds, lx_seg(),
                                                          lx_span(), act);
  } else {
    if (!act) return;
    adjoint_node<Q, QS, Real, NT, V>(p, mom, lam_in, lam_out, w, grad, x, y, z);
  }
}

// One in-place adjoint step (even or odd pattern of the cotangent buffer l).
template <int Q, int QS, typename Real, bool NT, int V, int ACC, bool NTE = false, bool LX = false>
__global__ __launch_bounds__(kHotThreads) void k_adjoint_inplace(Params<Real> p, const Real* __restrict__ mom, Real* l,
                                                         const Real* __restrict__ w, Real* __restrict__ grad) {
  int x, y, z;
  const bool act = hot_pos(p, x, y, z);
  if constexpr (LX) {
    static_assert(ACC == ACC_ODD, "only the odd pattern has shifted access");
    Real* lds = lx_lds<Real>();
    adjoint_node<Q, QS, Real, NT, V, ACC, NTE, true>(p, mom, l, l, w, grad, x, y, z, lds, lx_seg(), lx_span(), act);
  } else {
    if (!act) return;
    adjoint_node<Q, QS, Real, NT, V, ACC, NTE>(p, mom, l, l, w, grad, x, y, z);
  }
}


// ------------------------------------------------------ inspection kernels
// Macroscopic fields of the pulled pre-collision state (double outputs).
template <int Q, int QS, typename Real>
__global__ __launch_bounds__(256) void k_fields(Params<Real> p, const Real* __restrict__ src,
                                                double* __restrict__ rho, double* __restrict__ u,
                                                double* __restrict__ s, int acc) {
  using L = Lat<Q>;
  using S = SLat<QS>;
  constexpr bool is3d = (Q == 19);
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= p.nx) return;
  const int y = blockIdx.y, z = blockIdx.z;
  const Nbr b = make_nbr(p, x, y, z);
  const int n = own_node(b);
  Real f[Q], g[QS > 0 ? QS : 1];
  load_state_rt<Q, QS, Real>(src, b, acc, f, g);
  const int cls = node_class(p, x, y, z, is3d);
  double dr = 0, mx = 0, my = 0, mz = 0, T = 0;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    dr += (double)f[j];
    mx += L::ex(j) * (double)f[j];
    my += L::ey(j) * (double)f[j];
    mz += L::ez(j) * (double)f[j];
  }
#pragma unroll
  for (int i = 0; i < QS; ++i) T += (double)g[i];
  double r = 1.0 + dr, ox = 0, oy = 0, oz = 0;
  if (cls == INTERIOR) {
    ox = mx / r;
    oy = my / r;
    oz = mz / r;
  } else if (cls == WALL) {
    Real tw;
    if (QS > 0 && wall_dirichlet(p, x, y, tw)) T = (double)tw;
  } else {
    double s0 = 0, sk = 0;
    Real s0r = 0, skr = 0;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      if (L::ex(j) == 0) {
        s0 += (double)f[j];
        s0r += f[j];
      } else if (L::ex(j) == (cls == INLET ? -1 : 1)) {
        sk += (double)f[j];
        skr += f[j];
      }
    }
    if (cls == INLET) {
      Real uu, drho, up;
      if (inlet_state<Real>(p, s0r, skr, uu, drho, up)) {
        r = p.rho_in;
        ox = (p.rho_in - 1.0 - s0 - 2.0 * sk) / p.rho_in;
      } else {
        r = (1.0 + s0 + 2.0 * sk) / (1.0 - (double)uu);
        ox = (double)uu;
      }
      if (QS > 0) T = (double)inlet_value<Real>(p, y, z);
    } else {
      r = (double)p.rho_out;
      ox = (1.0 + s0 + 2.0 * sk) / r - 1.0;
      if constexpr (QS > 0) {
        double rest = 0;
#pragma unroll
        for (int i = 0; i < QS; ++i)
          if (i != kMX) rest += (double)g[i];
        const double a = S::w(kMX) * (1.0 - ox / S::c2());
        T = rest / (1.0 - a);
      }
    }
  }
  rho[n] = r;
  u[n] = ox;
  u[(size_t)p.N + n] = oy;
  u[(size_t)2 * p.N + n] = oz;
  if (s) s[n] = T;
}

// Pre-collision state f^t (un-shifted, double) pulled from src.
template <int Q, int QS, typename Real>
__global__ __launch_bounds__(256) void k_get_state(Params<Real> p, const Real* __restrict__ src,
                                                   double* __restrict__ fo, double* __restrict__ go, int acc) {
  using L = Lat<Q>;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= p.nx) return;
  const Nbr b = make_nbr(p, x, blockIdx.y, blockIdx.z);
  const int n = own_node(b);
  Real f[Q], g[QS > 0 ? QS : 1];
  load_state_rt<Q, QS, Real>(src, b, acc, f, g);
#pragma unroll
  for (int j = 0; j < Q; ++j) fo[(size_t)j * p.N + n] = (double)f[j] + L::w(j);
  if (go) {
#pragma unroll
    for (int i = 0; i < QS; ++i) go[(size_t)i * p.N + n] = (double)g[i];
  }
}

// Ping-pong: the stored post-collision buffer h^{-1} with S h^{-1} = f0,
// h_j(x) = f0_j(x + e_j).  In place (phase E): slot j of x holds f0_j(x).
template <int Q, int QS, typename Real>
__global__ __launch_bounds__(256) void k_set_state(Params<Real> p, const double* __restrict__ f0,
                                                   const double* __restrict__ g0, Real* __restrict__ dst, int acc) {
  using L = Lat<Q>;
  using S = SLat<QS>;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= p.nx) return;
  constexpr int QT = Q + QS;
  const Nbr b = make_nbr(p, x, blockIdx.y, blockIdx.z);
  if (acc != ACC_PP) {
    const int n = own_node(b);
#pragma unroll
    for (int j = 0; j < Q; ++j) dst[own_addr<QT>(b, j)] = (Real)(f0[(size_t)j * p.N + n] - L::w(j));
#pragma unroll
    for (int i = 0; i < QS; ++i) dst[own_addr<QT>(b, Q + i)] = g0 ? (Real)g0[(size_t)i * p.N + n] : Real(0);
    return;
  }
#pragma unroll
  for (int j = 0; j < Q; ++j)
    dst[own_addr<QT>(b, j)] = (Real)(f0[(size_t)j * p.N + push_node(b, L::ex(j), L::ey(j), L::ez(j))] - L::w(j));
#pragma unroll
  for (int i = 0; i < QS; ++i)
    dst[own_addr<QT>(b, Q + i)] = g0 ? (Real)g0[(size_t)i * p.N + push_node(b, S::ex(i), S::ey(i), S::ez(i))] : Real(0);
}

// Node classes and pull-source map.
template <int Q, int QS, typename Real>
__global__ __launch_bounds__(256) void k_maps(Params<Real> p, uint8_t* __restrict__ mask, int64_t* __restrict__ src) {
  using L = Lat<Q>;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= p.nx) return;
  const Nbr b = make_nbr(p, x, blockIdx.y, blockIdx.z);
  const int n = own_node(b);
  if (mask) mask[n] = (uint8_t)node_class(p, x, (int)blockIdx.y, (int)blockIdx.z, Q == 19);
  if (src) {
#pragma unroll
    for (int j = 0; j < Q; ++j) src[(size_t)j * p.N + n] = pull_node(b, L::ex(j), L::ey(j), L::ez(j));
  }
}

// Adjoint state lambda(x) (row-blocked, context precision) to plane-major
// doubles.  Ping-pong: slot j of x.  In place, phase E: slot j of x - e_j
// (the buffer holds mu_j(x) = lambda_j(x + e_j) at slot j of x); phase O:
// slot opp(j) of x.
template <int Q, int QS, typename Real>
__global__ __launch_bounds__(256) void k_get_adjoint(Params<Real> p, const Real* __restrict__ lam,
                                                     double* __restrict__ lf, double* __restrict__ lg, int acc) {
  using L = Lat<Q>;
  using S = SLat<QS>;
  constexpr int QT = Q + QS;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= p.nx) return;
  const Nbr b = make_nbr(p, x, blockIdx.y, blockIdx.z);
  const int n = own_node(b);
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const int a = acc == ACC_EVEN ? pull_addr<QT>(b, j, L::ex(j), L::ey(j), L::ez(j))
                                  : (acc == ACC_ODD ? own_addr<QT>(b, L::opp(j)) : own_addr<QT>(b, j));
    lf[(size_t)j * p.N + n] = (double)lam[a];
  }
  if (lg) {
#pragma unroll
    for (int i = 0; i < QS; ++i) {
      const int a = acc == ACC_EVEN ? pull_addr<QT>(b, Q + i, S::ex(i), S::ey(i), S::ez(i))
                                    : (acc == ACC_ODD ? own_addr<QT>(b, Q + S::opp(i)) : own_addr<QT>(b, Q + i));
      lg[(size_t)i * p.N + n] = (double)lam[a];
    }
  }
}

// ----------------------------------------------------------- one-shot step
// One iteration of the one-shot descent (Section 3.3, eq. gradient:update),
// fused for one node: the primal state f^n is pulled once and used by
//   lambda^{n+1}(x) = (dW/df)^T(f^n(x)) mu(x) + dJ/df(f^n(x))   (eq. adjoint:iteration)
//   g(x)            = (dW/dw)^T(f^n(x)) mu(x)                   (eq. adjoint:derivative)
//   h^n(x)          = W(f^n(x), w(x))                           (eq. normal:iteration)
//   w(x)           <- clip(w + zeta (g + c_pen (1 - 2w)), 0, 1) (interior nodes; eq. P)
// with mu_j(x) = lambda^n_j(x + e_j).  Each node owns its w, so the in-place
// update races with nothing.
// prim_in/prim_out and lam_in/lam_out are the same buffers in place, hence no
// restrict on them here (the ping-pong kernel declares it).
// LX: x-shifted populations of both states through LDS (lds holds the
// primal's staging runs, then the cotangent's).
template <int Q, int QS, typename Real, bool NT, int V, int ACC, bool LX = false>
__device__ __forceinline__ void oneshot_node(const Params<Real>& p, const Real* prim_in, Real* prim_out,
                                             const Real* lam_in, Real* lam_out, Real* __restrict__ w,
                                             Real* __restrict__ grad, const double* __restrict__ glob, Real zeta,
                                             Real c_pen, int x, int y, int z, Real* lds = nullptr,
                                             int seg = 0, int bt = 0, bool act = true) {
  constexpr bool is3d = (Q == 19);
  constexpr int QSA = QS > 0 ? QS : 1;
  const int kRuns = Shifted<Q, QS>::count() * bt;  // the cotangent's runs follow the primal's
  const Nbr b = make_nbr(p, x, y, z);
  const int n = own_inode(b);  // workspace node arrays
  // padding lanes (LX only) take the wall operators: permutations, no memory access
  const int cls = act ? node_class(p, x, y, z, is3d) : WALL;
  Real f[Q], g[QSA], mu[Q], nu[QSA];
  if constexpr (LX) {
    load_state_lx<Q, QS, Real, ACC, NT, NT && ACC == ACC_PP>(prim_in, b, f, g, lds, seg, bt, act);
    load_cot_lx<Q, QS, Real, ACC, NT, NT && ACC == ACC_PP>(lam_in, b, mu, nu, lds + kRuns, seg, bt, act);
  } else {
    load_state<Q, QS, Real, ACC, NT>(prim_in, b, f, g);
    load_cot<Q, QS, Real, ACC, NT>(lam_in, b, mu, nu);
  }
  const Real wn = (cls == INTERIOR) ? w[n] : Real(1);
  Real m[Mom<Q, QS, V>::N], lf[Q], lg[QSA], gw;
  node_moments<Q, QS, Real, V>(p, cls, y, z, f, g, m);
  adjoint_vjp<Q, QS, Real, V>(p, cls, x, y, m, wn, mu, nu, lf, lg, gw);
  if (cls == INLET || cls == OUTLET) {
    double sf[Q], sg[QSA];
    seed_values<Q, QS, Real>(p, cls, f, g, glob, sf, sg);
#pragma unroll
    for (int j = 0; j < Q; ++j) lf[j] += (Real)sf[j];
#pragma unroll
    for (int i = 0; i < QS; ++i) lg[i] += (Real)sg[i];
  }
  if (cls == INTERIOR) {
    collide_interior<Q, QS, Real, V>(p, wn, f, g);
  } else if (cls == WALL) {
    collide_wall<Q, QS, Real>(p, x, y, f, g);
  } else if (cls == INLET) {
    collide_inlet<Q, QS, Real>(p, y, z, f, g);
  } else {
    collide_outlet<Q, QS, Real>(p, f, g);
  }
  if constexpr (LX && ACC == ACC_ODD) {
    store_state_lx<Q, QS, Real, NT, false>(prim_out, b, f, g, lds, seg, bt, act);
    store_cot_lx<Q, QS, Real, NT, false>(lam_out, b, lf, lg, lds + kRuns, seg, bt, act);
  } else if (act) {
    store_state<Q, QS, Real, NT, ACC>(prim_out, b, f, g);
    store_cot<Q, QS, Real, NT, ACC>(lam_out, b, lf, lg);
  }
  if (!act) return;
  grad[n] = gw;
  if (cls == INTERIOR) {
    const Real v = wn + zeta * (gw + c_pen * (Real(1) - Real(2) * wn));
    w[n] = v < Real(0) ? Real(0) : (v > Real(1) ? Real(1) : v);
  }
}

template <int Q, int QS, typename Real, bool NT, int V, bool LX = false>
__global__ __launch_bounds__(kHotThreads) void k_oneshot(Params<Real> p, const Real* __restrict__ prim_in,
                                                 Real* __restrict__ prim_out, const Real* __restrict__ lam_in,
                                                 Real* __restrict__ lam_out, Real* __restrict__ w,
                                                 Real* __restrict__ grad, const double* __restrict__ glob, Real zeta,
                                                 Real c_pen) {
  int x, y, z;
  const bool act = hot_pos(p, x, y, z);
  if constexpr (LX) {
    Real* lds = lx_lds<Real>();
    oneshot_node<Q, QS, Real, NT, V, ACC_PP, true>(p, prim_in, prim_out, lam_in, lam_out, w, grad, glob, zeta, c_pen,
                                                   x, y, z, lds, lx_seg(), lx_span(), act);
  } else {
    if (!act) return;
    oneshot_node<Q, QS, Real, NT, V, ACC_PP>(p, prim_in, prim_out, lam_in, lam_out, w, grad, glob, zeta, c_pen, x,
                                             y, z);
  }
}

// One in-place one-shot iteration (even or odd phase): a is the primal buffer,
// l the adjoint buffer, each read and rewritten in place.
template <int Q, int QS, typename Real, bool NT, int V, int ACC, bool LX = false>
__global__ __launch_bounds__(kHotThreads) void k_oneshot_inplace(Params<Real> p, Real* a, Real* l, Real* __restrict__ w,
                                                         Real* __restrict__ grad, const double* __restrict__ glob,
                                                         Real zeta, Real c_pen) {
  int x, y, z;
  const bool act = hot_pos(p, x, y, z);
  if constexpr (LX) {
    static_assert(ACC == ACC_ODD, "only the odd phase has shifted access");
    Real* lds = lx_lds<Real>();
    oneshot_node<Q, QS, Real, NT, V, ACC, true>(p, a, a, l, l, w, grad, glob, zeta, c_pen, x, y, z, lds, lx_seg(),
                                                lx_span(), act);
  } else {
    if (!act) return;
    oneshot_node<Q, QS, Real, NT, V, ACC>(p, a, a, l, l, w, grad, glob, zeta, c_pen, x, y, z);
  }
}

// --------------------------------------------------------- batched launches
// One launch advances many contexts of the same (Q, QS, Real) by one step.
// A row part is kw consecutive waves (64 x-nodes each) of one row, kw chosen per
// launch as the widest of 4, 3, 2, 1 waves that divides every context's waves
// per row (so no part straddles two rows and none holds more idle lanes than
// the row's padding to whole waves); a block holds rpb parts (several rows only
// when every row is one part); block b belongs to the context k with
// start[k] <= b < start[k+1].  The per-node code is the same device function
// as in the single-context kernels, so results are bitwise identical to them.
constexpr int kBatchMax = 32;
constexpr int kWave = 64;

// Per-context constants, stored once in the context's own workspace.
template <typename Real>
struct BatchStatic {
  Params<Real> p;
  int waves;  // waves per row: ceil(nx / 64)
};

// Per-launch arguments, passed by value (about 1.2 KB for kBatchMax = 32).
template <typename Real>
struct BatchArgs {
  int n;
  int kw;   // waves per row part (64 kw threads), dividing every context's waves per row
  int rpb;  // row parts per block (blockDim.x = 64 kw rpb); > 1 only when every row is one part
  int nt;   // streaming stores and hints: the states the launch touches exceed the last-level cache
  int nte;  // in place: the even phase's loads take the hint too (states far beyond the cache)
  int lx;   // every member's row is one row part: x-shifted populations through LDS
  int start[kBatchMax + 1];
  const BatchStatic<Real>* st[kBatchMax];
  const Real* a[kBatchMax];  // primal: source state; adjoint: moments of f^n
  const Real* b[kBatchMax];  // adjoint: lambda^{n+1} (in place: the cotangent buffer)
  Real* c[kBatchMax];        // primal: destination (in place: = a); adjoint: lambda^n (in place: = b)
  Real* m[kBatchMax];        // primal: where to record moments (all set or all null)
  const Real* w[kBatchMax];  // design field
  Real* g[kBatchMax];        // adjoint: gradient accumulator
};

static_assert(sizeof(BatchArgs<double>) <= 4096, "batched launch arguments exceed the kernel-argument limit");



// Stores a context's batch descriptor (passed by value, so the upload is a
// stream-ordered launch with no host-side staging).
template <typename Real>
__global__ void k_write_desc(BatchStatic<Real> h, BatchStatic<Real>* __restrict__ d) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *d = h;
}

// Node of the calling thread in local block lb of its context: with one row
// part per block (rpb = 1) block lb covers waves [kw bx, kw bx + kw) of row
// lb / (waves / kw); with rpb > 1 (every member's row is one block part) it
// covers rows rpb lb ... rpb lb + rpb - 1, one row per kw waves.
template <typename Real>
__device__ __forceinline__ bool batch_pos(const BatchArgs<Real>& A, const Params<Real>& p, int waves, int lb, int& x,
                                          int& y, int& z) {
  const int tw = kWave * A.kw;  // threads per row part
  int bx, row;
  if (A.rpb == 1) {
    const int gx = waves / A.kw;  // blocks per row
    bx = lb % gx;
    row = lb / gx;
  } else {
    bx = 0;
    row = __builtin_amdgcn_readfirstlane((int)(lb * A.rpb + threadIdx.x / tw));
  }
  x = bx * tw + (int)(threadIdx.x % tw);
  y = row % p.ny;
  z = row / p.ny;
  return x < p.nx && z < p.nz;
}

template <typename Real>
__device__ __forceinline__ int batch_find(const BatchArgs<Real>& A, int blk) {
  int k = 0;
  while (k + 1 < A.n && blk >= A.start[k + 1]) ++k;
  return k;
}

// NT (streaming stores and hints) and MOM (record the moments) are uniform over
// a launch, so they are template arguments: one code path per kernel keeps the
// register count of the single-context kernels.
// ACC: ping-pong (a = source, c = destination) or one in-place phase (a = c =
// the member's working buffer; members of other phases go in another launch).
// LX: every member's row is one block part; x-shifted populations through LDS
// (one run per row part of kw waves), no thread leaves before the barriers.
template <int Q, int QS, typename Real, int V, bool NT, bool MOM, int ACC, bool NTE = false, bool LX = false>
__global__ __launch_bounds__(256) void k_primal_batch(BatchArgs<Real> A) {
  const int blk = blockIdx.x;
  const int k = batch_find(A, blk);
  // local copy taken before any store: scalar loads, kept in registers (read
  // through the pointer they were reloaded after every store)
  const Params<Real> p = A.st[k]->p;
  const int waves = A.st[k]->waves;
  int x, y, z;
  const bool act = batch_pos(A, p, waves, blk - A.start[k], x, y, z);
  if constexpr (LX) {
    __shared__ Real lds[Shifted<Q, QS>::count() * 256];
    const int tw = kWave * A.kw;
    primal_node<Q, QS, Real, NT, MOM, V, ACC, NTE, true>(p, A.a[k], A.c[k], A.w[k], MOM ? A.m[k] : nullptr, x, y, z,
                                                         lds, (int)(threadIdx.x / tw) * tw, (int)blockDim.x, act);
  } else {
    if (!act) return;
    primal_node<Q, QS, Real, NT, MOM, V, ACC, NTE>(p, A.a[k], A.c[k], A.w[k], MOM ? A.m[k] : nullptr, x, y, z);
  }
}

// ACC: ping-pong (b = lambda^{n+1}, c = lambda^n) or one in-place pattern (b = c).
template <int Q, int QS, typename Real, int V, bool NT, int ACC, bool NTE = false, bool LX = false>
__global__ __launch_bounds__(256) void k_adjoint_batch(BatchArgs<Real> A) {
  const int blk = blockIdx.x;
  const int k = batch_find(A, blk);
  // local copy taken before any store: scalar loads, kept in registers (read
  // through the pointer they were reloaded after every store)
  const Params<Real> p = A.st[k]->p;
  const int waves = A.st[k]->waves;
  int x, y, z;
  const bool act = batch_pos(A, p, waves, blk - A.start[k], x, y, z);
  if constexpr (LX) {
    __shared__ Real lds[Shifted<Q, QS>::count() * 256];
    const int tw = kWave * A.kw;
    adjoint_node<Q, QS, Real, NT, V, ACC, NTE, true>(p, A.a[k], A.b[k], A.c[k], A.w[k], A.g[k], x, y, z, lds,
                                                     (int)(threadIdx.x / tw) * tw, (int)blockDim.x, act);
  } else {
    if (!act) return;
    adjoint_node<Q, QS, Real, NT, V, ACC, NTE>(p, A.a[k], A.b[k], A.c[k], A.w[k], A.g[k], x, y, z);
  }
}

// ------------------------------------------------------- small helpers
template <typename T>
__global__ __launch_bounds__(256) void k_fill(T* __restrict__ a, size_t n, T v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    a[i] = v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy(const T* __restrict__ a, T* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// Node array between the compact ABI index n = x + nx*r and the workspace's
// padded index i = x + pitch*r (node launch geometry).
template <typename Real>
__global__ __launch_bounds__(256) void k_node_in(Params<Real> p, const Real* __restrict__ a, Real* __restrict__ b) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= p.nx) return;
  const int r = blockIdx.y + p.ny * blockIdx.z;
  b[x + p.pitch * r] = a[x + p.nx * r];
}

// Gradient export with the penalty term: b = a + c_pen (1 - 2w) at interior
// nodes (the derivative of P = sum w (1 - w), eq. P), a elsewhere (zero: the
// design acts at interior nodes only); workspace layout in, compact out.
template <typename Real>
__global__ __launch_bounds__(256) void k_grad_penalty(Params<Real> p, const Real* __restrict__ a,
                                                      const Real* __restrict__ w, Real c_pen, Real* __restrict__ b) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= p.nx) return;
  const int r = blockIdx.y + p.ny * blockIdx.z;
  const int i = x + p.pitch * r;
  Real v = a[i];
  if (node_class(p, x, blockIdx.y, blockIdx.z, p.nz > 1) == INTERIOR) v += c_pen * (Real(1) - Real(2) * w[i]);
  b[x + p.nx * r] = v;
}

template <typename Real>
__global__ __launch_bounds__(256) void k_node_out(Params<Real> p, const Real* __restrict__ a, Real* __restrict__ b) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= p.nx) return;
  const int r = blockIdx.y + p.ny * blockIdx.z;
  b[x + p.nx * r] = a[x + p.pitch * r];
}


}  // namespace lbmk
