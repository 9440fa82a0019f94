// Host side of the adjoint lattice-Boltzmann library: context, workspace
// carving, checkpoint plan, launch dispatch and the C ABI of lbm_adj.h.
//
// The library never allocates device memory: every buffer below is a slice of
// the caller's workspace.  Workspace layout (each slice 256-byte aligned):
//   w        N x Real      design field (copied in by lbm_set_design)
//   grad     N x Real      dJ/dw accumulator (one-shot: last estimate)
//   glob     boundary sums + J of the last objective evaluation, objective partials
//   desc     this context's batch descriptor (constants for batched launches)
//   lam[2]   2 states      adjoint ping-pong (in place: one state)
//   pp[2]    2 states      primal ping-pong
//   ckpt[S]  S states      checkpoints h^{sC-1}, s = 0..S-1 (ckpt[0] = h^{-1})
//   mom[C]   C moment sets the moments of f^k for the C steps k of one segment
// A "state" is Qt x N values of the context precision; a "moment set" is
// Mom::N x N values (rho, u and the scalar value: what the transposed
// Jacobians read), so the trajectory the adjoint needs costs 4-5 values per
// node and step instead of Qt.
//
// Trajectory bookkeeping (step k computes h^k from h^{k-1}, k = 0..N-1): a
// recorded step writes the moments of f^k to mom[k % C] and h^k to
// ckpt[(k+1)/C] when (k+1) % C == 0 (while slots are left), else to a primal
// ping-pong buffer.  The adjoint step n reads mom[n % C]; when segment
// s = n / C is not the one held in mom, it is recomputed from ckpt[s] (C
// primal steps through the ping-pong buffers).  With C = N (store-all) no
// step is ever recomputed.
//
// In-place plan (one primal working buffer and one adjoint buffer, each read
// and rewritten by every step in the alternating even/odd access patterns):
// store-all keeps the state in ckpt[0] and never recomputes.  With C < N the
// working buffer is a slot of its own; before recorded step k with k % C == 0
// it is copied to ckpt[k / C] (in the buffer layout of phase k), and segment s
// is recomputed in place inside ckpt[s] itself, which the backward sweep needs
// no more once the segment's moments are rebuilt (segments are reversed in
// decreasing order, each once).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/lbm_adj.h"
#include "kernels.hpp"

using namespace lbmk;

namespace {

constexpr uint64_t kAlign = 256;
constexpr uint64_t kDescBytes = 1024;  // >= sizeof(BatchStatic<double>)
// Streaming stores bypass the caches when two primal states (what one step
// reads and writes) exceed the 256 MB last-level cache; below that, plain
// stores let the next step re-read the state from that cache.
constexpr uint64_t kLastLevelCacheBytes = 256ull << 20;
// glob region: kGlobSlots doubles of results, then the objective partial sums.
constexpr int kGlobSlots = 16;
constexpr uint64_t kGlobBytes = (kGlobSlots + kObjBlocks * kNG) * sizeof(double);

uint64_t align_up(uint64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Row length of the workspace arrays: nx rounded up to whole 128-byte lines.
int64_t row_pitch(int32_t nx, int32_t precision) {
  const int64_t per_line = 128 / (precision == LBM_FP32 ? 4 : 8);
  return ((int64_t)nx + per_line - 1) / per_line * per_line;
}

struct Plan {
  int Q = 0, QS = 0, QT = 0;
  int64_t N = 0;             // nodes
  int64_t pitch = 0, Np = 0; // padded row length, pitch*ny*nz
  uint64_t rs = 0;           // bytes per value
  uint64_t state_bytes = 0;  // aligned
  uint64_t mom_bytes = 0;    // aligned, one moment set
  uint64_t node_bytes = 0;   // aligned Np x Real
  int64_t C = 1, S = 1;      // checkpoint interval and slots
  bool inplace = false;      // one primal working buffer and one adjoint buffer, streamed in place
  int64_t W = 1;             // states averaged by the objective (the last W of the horizon)
  uint64_t cols_bytes = 0;   // inlet + outlet columns of one state (aligned)
  uint64_t win_bytes = 0;    // W > 1: W x (sums + J), then W x columns
  uint64_t total = 0;
};

}  // namespace

// Descriptor of one context in a batched launch (see kernels below).
struct BatchDesc;

struct lbm_ctx {
  lbm_config cfg;
  Plan plan;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  uint64_t ws_bytes = 0;
  // carved buffers
  void* w = nullptr;
  void* grad = nullptr;
  double* glob = nullptr;
  void* desc = nullptr;
  void* lam[2] = {nullptr, nullptr};
  void* pp[2] = {nullptr, nullptr};
  char* ckpt = nullptr;
  char* mom = nullptr;
  void* work = nullptr;   // in place: the primal working buffer (ckpt[0] when store-all)
  char* win = nullptr;    // W > 1: window slots (sums + J, then inlet/outlet columns), W of them
  int64_t win_count = 0;  // window states captured since the run started at t = 0
  // time bookkeeping
  int64_t t = 0;          // primal time: current state is h^{t-1}
  int64_t rec_len = 0;    // recorded steps (trajectory h^{-1}..h^{rec_len-1})
  bool rec_open = true;   // recording can be continued
  void* cur = nullptr;    // buffer holding h^{t-1}
  bool design_set = false;
  bool adj_started = false;
  int64_t t_adj = -1;     // adjoint time (lambda^{t_adj} in lam[lam_cur])
  int lam_cur = 0;
  int64_t mom_seg = -1;   // trajectory segment whose moments mom holds
  bool os_active = false; // one-shot iteration running (adjoint state in lam[lam_cur])
  bool state_lost = false; // a new design arrived after an adjoint had started: the primal
                           // buffers may hold recomputed states, so c->cur is not h^{t-1}
  int static_dev = -1;     // device whose static workspace this context uses (-1: caller's)
  std::string err;
};

namespace {

// Named range on the profiler's marker timeline (rocprofv3 --marker-trace):
// forward segments, recomputed segments, adjoint segments and one-shot runs
// show up as spans around their kernel launches (host-side enqueue time).
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

lbm_status fail(lbm_ctx* c, lbm_status s, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
lbm_status fail(lbm_ctx* c, lbm_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

lbm_status check_config(const lbm_config* c, std::string* why) {
  auto bad = [&](const char* m) {
    if (why) *why = m;
    return LBM_EINVAL;
  };
  if (!c) return bad("config is NULL");
  if (c->struct_size != sizeof(lbm_config)) return bad("struct_size does not match sizeof(lbm_config)");
  if (c->flow != LBM_D2Q9 && c->flow != LBM_D3Q19) return bad("flow must be LBM_D2Q9 or LBM_D3Q19");
  if (c->scalar != LBM_SCALAR_NONE && !((c->flow == LBM_D2Q9 && c->scalar == LBM_D2Q5) ||
                                        (c->flow == LBM_D3Q19 && c->scalar == LBM_D3Q7)))
    return bad("scalar lattice must be none, D2Q5 with D2Q9, or D3Q7 with D3Q19");
  if (c->precision != LBM_FP32 && c->precision != LBM_FP64) return bad("precision must be LBM_FP32 or LBM_FP64");
  if (c->nx < 3 || c->ny < 3 || c->nz < 1) return bad("nx, ny must be >= 3 and nz >= 1");
  if (c->flow == LBM_D2Q9 && c->nz != 1) return bad("D2Q9 needs nz = 1");
  if (c->flow == LBM_D3Q19 && c->nz < 3) return bad("D3Q19 needs nz >= 3");
  if (c->ny > 65535 || c->nz > 65535) return bad("ny and nz must be <= 65535");
  if (!(c->tau > 0.5) || (c->scalar && !(c->tau_s > 0.5))) return bad("relaxation times must exceed 1/2");
  if (!(std::fabs(c->u_in) < 1.0) || !(c->rho_out > 0.0)) return bad("need |u_in| < 1 and rho_out > 0");
  if (c->scalar_wall != LBM_WALL_ADIABATIC && c->scalar_wall != LBM_WALL_DIRICHLET) return bad("bad scalar_wall");
  if (c->s_split_axis < 0 || c->s_split_axis > 2) return bad("bad s_split_axis");
  if (c->switch_fn != LBM_G_POWER && c->switch_fn != LBM_G_RAMP) return bad("bad switch_fn");
  if (c->switch_fn == LBM_G_RAMP && !(c->switch_param > 0.0)) return bad("RAMP needs q > 0");
  if (c->switch_fn == LBM_G_POWER && !(c->switch_param >= 0.0)) return bad("POWER needs theta >= 0");
  if (c->reserved0 != 0) return bad("reserved0 must be 0");
  if (c->n_avg < 0) return bad("n_avg must be >= 0");
  if (c->n_avg > 1 && c->n_avg > c->nsteps)
    return bad("n_avg > 1 averages the last n_avg states of the horizon: needs nsteps >= n_avg");
  if (c->inlet != LBM_INLET_VELOCITY && c->inlet != LBM_INLET_PRESSURE) return bad("bad inlet");
  if (c->collision != LBM_COLL_BGK && c->collision != LBM_COLL_MRT) return bad("bad collision");
  if (c->collision == LBM_COLL_MRT) {
    if (c->flow != LBM_D3Q19) return bad("MRT collision is D3Q19 only");
    for (int k = 0; k < 5; ++k)
      if (!(c->mrt_rates[k] > 0.0 && c->mrt_rates[k] < 2.0)) return bad("MRT rates must lie in (0, 2)");
  }
  if (c->reserved2 != 0) return bad("reserved2 must be 0");
  if (c->tau_s_solid != 0.0 && !(c->tau_s_solid > 0.5)) return bad("tau_s_solid must be 0 or exceed 1/2");
  if (c->inplace != 0 && c->inplace != 1) return bad("inplace must be 0 or 1");
  if (c->reserved3 != 0) return bad("reserved3 must be 0");
  if (c->plate_x0 < 0 || c->plate_x1 < c->plate_x0 || c->plate_x1 > c->nx)
    return bad("heating plate needs 0 <= plate_x0 <= plate_x1 <= nx");
  if (c->inlet == LBM_INLET_PRESSURE && !(c->rho_in > 0.0 && c->u_cap >= 0.0 && c->u_cap < 1.0))
    return bad("pressure inlet needs rho_in > 0 and 0 <= u_cap < 1");
  if (c->nsteps < 0 || c->checkpoint_interval < 0) return bad("nsteps and checkpoint_interval must be >= 0");
  const int64_t Np = row_pitch(c->nx, c->precision) * c->ny * c->nz;
  const int QT = c->flow + c->scalar;
  if ((int64_t)QT * Np >= (int64_t(1) << 31)) return bad("lattice too large: Qt*N (rows padded) must be < 2^31");
  return LBM_OK;
}

// Workspace of a plan with checkpoint interval C and S checkpoint slots (N steps).
// Ping-pong: 2 adjoint + 2 primal states besides the checkpoints.  In place: one
// adjoint state, plus the working buffer unless C >= N (store-all: the state stays
// in ckpt[0]).
uint64_t plan_total(const Plan& p, int64_t C, int64_t S, int64_t N) {
  uint64_t t = 2 * p.node_bytes + align_up(kGlobBytes) + align_up(kDescBytes) + p.win_bytes;
  const uint64_t extra = p.inplace ? (C >= N ? 1 : 2) : 4;
  t += (uint64_t)(extra + S) * p.state_bytes + (uint64_t)C * p.mom_bytes;
  return t;
}

// Values per node in one moment set (must equal Mom<Q,QS>::N of the kernels).
// Blended (design-dependent) scalar diffusivity in use.
bool blended_diffusivity(const lbm_config* c) {
  return c->scalar != 0 && c->tau_s_solid != 0.0 && c->tau_s_solid != c->tau_s;
}

int mom_values(const lbm_config* c) {
  return (c->flow == LBM_D3Q19 ? 3 : 2) + 1 + (c->scalar ? (blended_diffusivity(c) ? c->scalar : 1) : 0);
}

lbm_status make_plan(const lbm_config* c, Plan* p, std::string* why) {
  lbm_status s = check_config(c, why);
  if (s != LBM_OK) return s;
  p->Q = c->flow;
  p->QS = c->scalar;
  p->QT = p->Q + p->QS;
  p->N = (int64_t)c->nx * c->ny * c->nz;
  p->pitch = row_pitch(c->nx, c->precision);
  p->Np = p->pitch * c->ny * c->nz;
  p->rs = (c->precision == LBM_FP32) ? 4 : 8;
  p->state_bytes = align_up((uint64_t)p->QT * p->Np * p->rs);
  p->mom_bytes = align_up((uint64_t)mom_values(c) * p->Np * p->rs);
  p->node_bytes = align_up((uint64_t)p->Np * p->rs);
  p->inplace = c->inplace != 0;
  p->W = c->n_avg > 1 ? c->n_avg : 1;
  p->win_bytes = 0;
  p->cols_bytes = align_up((uint64_t)2 * p->QT * c->ny * c->nz * p->rs);  // inlet + outlet columns
  if (p->W > 1) p->win_bytes = align_up((uint64_t)p->W * (kNG + 1) * sizeof(double)) + (uint64_t)p->W * p->cols_bytes;
  const int64_t Nst = std::max<int64_t>(c->nsteps, 1);
  if (p->inplace && c->nsteps == 0) {
    // unrecorded runs and the one-shot iteration only: the state and one adjoint buffer
    p->C = 0;
    p->S = 1;
    p->total = 2 * p->node_bytes + align_up(kGlobBytes) + align_up(kDescBytes) + 2 * p->state_bytes + p->win_bytes;
    return LBM_OK;
  }
  int64_t C;
  if (c->checkpoint_interval > 0) {
    C = std::min<int64_t>(c->checkpoint_interval, Nst);
  } else if (c->hbm_budget_bytes == 0 && p->inplace) {
    C = Nst;  // in place without a budget: every step's moments (no recompute)
  } else if (c->hbm_budget_bytes == 0) {
    // smallest workspace: minimise S*state + C*moments
    C = 1;
    uint64_t best = plan_total(*p, 1, Nst, Nst);
    for (int64_t cc = 2; cc <= Nst; ++cc) {
      const uint64_t t = plan_total(*p, cc, (Nst + cc - 1) / cc, Nst);
      if (t < best) {
        best = t;
        C = cc;
      }
    }
  } else {
    // largest C (fewest recomputed steps) whose workspace fits the budget
    C = 0;
    for (int64_t cc = Nst; cc >= 1; --cc) {
      const int64_t S = (Nst + cc - 1) / cc;
      if (plan_total(*p, cc, S, Nst) <= c->hbm_budget_bytes) {
        C = cc;
        break;
      }
    }
    if (C == 0) {
      if (why) *why = "no checkpoint interval fits hbm_budget_bytes";
      return LBM_ENOMEM;
    }
  }
  p->C = C;
  p->S = (Nst + C - 1) / C;
  p->total = plan_total(*p, p->C, p->S, Nst);
  return LBM_OK;
}

// ---------------------------------------------------------------- launches
template <typename Real>
Params<Real> make_params(const lbm_config& c, int64_t N) {
  Params<Real> p;
  p.nx = c.nx;
  p.ny = c.ny;
  p.nz = c.nz;
  p.periodic = c.periodic ? 1 : 0;
  p.N = (int)N;
  p.pitch = (int)row_pitch(c.nx, c.precision);
  p.Np = p.pitch * c.ny * c.nz;
  p.scalar_wall = c.scalar_wall;
  p.split_axis = c.s_split_axis;
  p.switch_fn = c.switch_fn;
  const double th = c.switch_param;
  p.theta_int = (c.switch_fn == LBM_G_POWER && th == std::floor(th) && th <= 16) ? (int)th : -1;
  p.om = (Real)(1.0 / c.tau);
  p.oms = (Real)(c.scalar ? 1.0 / c.tau_s : 0.0);
  p.u_in = (Real)c.u_in;
  p.rho_out = (Real)c.rho_out;
  p.s_wall = (Real)c.s_wall;
  p.s_in_lo = (Real)c.s_in_lo;
  p.s_in_hi = (Real)c.s_in_hi;
  p.sw_param = (Real)c.switch_param;
  p.inlet_mode = (c.inlet == LBM_INLET_PRESSURE) ? IN_PRESSURE : IN_VELOCITY;
  p.drho_in = (Real)(c.rho_in - 1.0);
  p.u_cap = (Real)c.u_cap;
  p.rho_in = c.rho_in;
  p.c_dp = c.c_dp;
  p.c_hf = c.c_hf;
  p.c_var = c.c_var;
  p.c_mix = c.c_mix;
  p.taus_f = (Real)c.tau_s;
  p.taus_s = (Real)(c.tau_s_solid != 0.0 ? c.tau_s_solid : c.tau_s);
  p.plate_x0 = c.periodic ? 0 : c.plate_x0;
  p.plate_x1 = c.periodic ? 0 : c.plate_x1;
  p.s_plate = (Real)c.s_plate;
  // MRT row scales (1 - rate) / |row|^2; rows of group 0 relax at 1/tau
  for (int k = 0; k < 19; ++k) {
    const int gr = Mrt19::group(k);
    const double rate = (gr == 0) ? 1.0 / c.tau : c.mrt_rates[gr - 1];
    p.mrt_k[k] = (Real)((1.0 - rate) / Mrt19::norm2(k));
  }
  return p;
}

struct Geo {
  dim3 grid, block;
};

// One thread per node of an x row, rows padded to whole waves; the block is the
// widest run of at most four waves that divides the row's waves, so no block
// holds more idle lanes than that padding (nx = 384: 2 x 192 threads instead of
// 2 x 256, where a quarter of the lanes idled).
Geo node_geometry(const lbm_config& c) {
  const int waves = (c.nx + 63) / 64;
  int k = 4;
  while (waves % k) --k;
  Geo g;
  g.block = dim3(64 * k, 1, 1);
  g.grid = dim3(waves / k, c.ny, c.nz);
  return g;
}

// Waves per block the hot kernels (primal, adjoint, one-shot) and batched
// launches aim for when a row is narrower (their kernels are bounded to 256
// threads).  Measured on D3Q19 FP32: 96x48x48 recorded in place 0.43 -> 0.48 of
// HBM peak (one 128-thread row per block against two rows per block); no change
// at 128x192x192, 192x96x96 or 256x128x128.
constexpr int kHotWaves = 4;

// x-shifted populations through LDS (kernels' LX variants): when one block
// part spans a whole row, i.e. nx <= 256.  Measured on the 256x128x128 D3Q19
// FP32 channel (fraction of HBM peak): recorded in-place primal 0.839 -> 0.892,
// in-place adjoint 0.846 -> 0.903, ping-pong primal 0.732 -> 0.752, ping-pong
// adjoint 0.798 -> 0.807; FP64 and the one-shot unchanged.  The MRT kernels
// (87-90 registers, five waves per SIMD) lose at the barriers (adjoint 0.80 ->
// 0.75, primal 0.79 -> 0.77) and keep the plain access.
bool lx_rows(const lbm_config& c) { return c.nx <= kHotThreads && c.collision != LBM_COLL_MRT; }

// Launch geometry of the hot kernels: a row of up to kHotThreads / 64 waves
// (nx <= 256) is one block (its x-shifts are then staged in LDS), and when a
// row is narrower than kHotWaves waves, R consecutive rows share a block
// (blockDim.y = R) so that it holds about that many; wider rows as
// node_geometry.
Geo hot_geometry(const lbm_config& c) {
  Geo g = node_geometry(c);
  const int waves = (c.nx + 63) / 64;
  if (waves * 64 <= kHotThreads) {
    const int R = std::max(1, kHotWaves / waves);
    g.block = dim3(64 * waves, R, 1);
    g.grid = dim3(1, (c.ny + R - 1) / R, c.nz);
  }
  return g;
}

dim3 flat_grid(size_t n) {
  size_t b = (n + 255) / 256;
  return dim3((unsigned)std::min<size_t>(std::max<size_t>(b, 1), 65536), 1, 1);
}

lbm_status launch_check(lbm_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, LBM_EHIP, "%s: %s", what, hipGetErrorString(e));
  return LBM_OK;
}

// Waves per x row of a context (rows padded to whole waves).
int batch_waves(const lbm_ctx* c) { return (c->cfg.nx + 63) / 64; }

// Waves per block of a batched launch: the widest of 4, 3, 2, 1 that divides
// every member's waves per row (as in the single-context launch geometry, which
// measured 0.737 of HBM peak with one-wave blocks against 0.835 with four).
int batch_block_waves(lbm_ctx* const* cs, int n) {
  for (int kw = 4; kw > 1; --kw) {
    bool all = true;
    for (int k = 0; k < n && all; ++k) all = batch_waves(cs[k]) % kw == 0;
    if (all) return kw;
  }
  return 1;
}

// Row parts per block of a batched launch: several rows per block only when
// every member's row is a single part of kw waves.
int batch_rows_per_block(lbm_ctx* const* cs, int n, int kw) {
  for (int k = 0; k < n; ++k)
    if (batch_waves(cs[k]) != kw) return 1;
  return std::max(1, kHotWaves / kw);
}

// x-shifted populations through LDS in a batched launch: when every member's
// row is a single row part (as lx_rows for one context).
int batch_lx(lbm_ctx* const* cs, int n, int kw) {
  for (int k = 0; k < n; ++k)
    if (batch_waves(cs[k]) != kw) return 0;
  return 1;
}

// Streaming stores and hints in a batched ping-pong launch: decided on the
// states the launch touches together (a source and a destination per member),
// not per member: eight 90 MB states are far beyond the cache although each
// member's pair alone fits.
int batch_nt(lbm_ctx* const* cs, int n) {
  uint64_t bytes = 0;
  for (int k = 0; k < n; ++k) bytes += 2 * cs[k]->plan.state_bytes;
  return bytes > kLastLevelCacheBytes ? 1 : 0;
}

// The same for an in-place launch (one buffer per member, read and rewritten),
// with the single-context rule: recorded and adjoint steps stream once the
// buffers exceed the cache; unrecorded steps stream in the odd phase only
// between one and two caches (4 x 128x96x96 D3Q19 FP32, 0.36 GB together: 0.69 ->
// 0.80 of HBM peak; 5 x: 0.67 -> 0.74) and in both phases beyond; the even
// phase's loads take the hint too beyond twice the cache (8 x 128x96x96 recorded,
// 0.72 GB together: primal 0.64, adjoint 0.66 of HBM peak without it).
void batch_nt_inplace(lbm_ctx* const* cs, int n, bool unrecorded, bool odd, int* nt, int* nte) {
  uint64_t bytes = 0;
  for (int k = 0; k < n; ++k) bytes += cs[k]->plan.state_bytes;
  const bool far = bytes > 2 * kLastLevelCacheBytes;
  const bool over = bytes > kLastLevelCacheBytes;
  *nt = (unrecorded ? far || (odd && over) : over) ? 1 : 0;
  *nte = far ? 1 : 0;
}

// Window of the time-averaged objective: slot s holds state f^{N-W+1+s}.
double* win_glob(lbm_ctx* c, int64_t s) { return (double*)c->win + s * (kNG + 1); }
void* win_cols(lbm_ctx* c, int64_t s) {
  return c->win + align_up((uint64_t)c->plan.W * (kNG + 1) * sizeof(double)) + (uint64_t)s * c->plan.cols_bytes;
}

// Typed operations on one context.
template <int Q, int QS, typename Real, int V = 0>
struct Ops {
  using RealT = Real;
  static constexpr int kQ = Q, kQS = QS;
  static Params<Real> P(lbm_ctx* c) { return make_params<Real>(c->cfg, c->plan.N); }
  static int batch_blocks(lbm_ctx* c, int kw, int rpb) {
    const int rows = c->cfg.ny * c->cfg.nz;
    return rpb == 1 ? batch_waves(c) / kw * rows : (rows + rpb - 1) / rpb;
  }
  // batched steps in access pattern acc (ping-pong, or one in-place phase)
  template <bool NTV, bool MOMV>
  static void primal_batch_acc(hipStream_t st, const BatchArgs<Real>& A, dim3 g, dim3 b, int acc) {
    constexpr bool kLx = !(V & kVarMRT);  // the MRT kernels keep the plain access (see lx_rows)
    if (acc == ACC_EVEN && NTV && A.nte)
      hipLaunchKernelGGL((k_primal_batch<Q, QS, Real, V, NTV, MOMV, ACC_EVEN, true>), g, b, 0, st, A);
    else if (acc == ACC_EVEN) hipLaunchKernelGGL((k_primal_batch<Q, QS, Real, V, NTV, MOMV, ACC_EVEN>), g, b, 0, st, A);
    else if (acc == ACC_ODD && A.lx)
      hipLaunchKernelGGL((k_primal_batch<Q, QS, Real, V, NTV, MOMV, ACC_ODD, false, kLx>), g, b, 0, st, A);
    else if (acc == ACC_ODD) hipLaunchKernelGGL((k_primal_batch<Q, QS, Real, V, NTV, MOMV, ACC_ODD>), g, b, 0, st, A);
    else if (A.lx) hipLaunchKernelGGL((k_primal_batch<Q, QS, Real, V, NTV, MOMV, ACC_PP, false, kLx>), g, b, 0, st, A);
    else hipLaunchKernelGGL((k_primal_batch<Q, QS, Real, V, NTV, MOMV, ACC_PP>), g, b, 0, st, A);
  }
  static void primal_batch(hipStream_t st, const BatchArgs<Real>& A, int blocks, int acc = ACC_PP) {
    const dim3 g(blocks), b(kWave * A.kw * A.rpb);
    const bool mom = A.m[0] != nullptr;  // every member records, or none
    if (A.nt) {
      if (mom) primal_batch_acc<true, true>(st, A, g, b, acc);
      else primal_batch_acc<true, false>(st, A, g, b, acc);
    } else {
      if (mom) primal_batch_acc<false, true>(st, A, g, b, acc);
      else primal_batch_acc<false, false>(st, A, g, b, acc);
    }
  }
  template <bool NTV>
  static void adjoint_batch_acc(hipStream_t st, const BatchArgs<Real>& A, dim3 g, dim3 b, int acc) {
    constexpr bool kLx = !(V & kVarMRT);  // the MRT kernels keep the plain access (see lx_rows)
    if (acc == ACC_EVEN && NTV && A.nte)
      hipLaunchKernelGGL((k_adjoint_batch<Q, QS, Real, V, NTV, ACC_EVEN, true>), g, b, 0, st, A);
    else if (acc == ACC_EVEN) hipLaunchKernelGGL((k_adjoint_batch<Q, QS, Real, V, NTV, ACC_EVEN>), g, b, 0, st, A);
    else if (acc == ACC_ODD && A.lx && A.nte)
      hipLaunchKernelGGL((k_adjoint_batch<Q, QS, Real, V, NTV, ACC_ODD, true, kLx>), g, b, 0, st, A);
    else if (acc == ACC_ODD && A.lx)
      hipLaunchKernelGGL((k_adjoint_batch<Q, QS, Real, V, NTV, ACC_ODD, false, kLx>), g, b, 0, st, A);
    else if (acc == ACC_ODD) hipLaunchKernelGGL((k_adjoint_batch<Q, QS, Real, V, NTV, ACC_ODD>), g, b, 0, st, A);
    else if (A.lx) hipLaunchKernelGGL((k_adjoint_batch<Q, QS, Real, V, NTV, ACC_PP, false, kLx>), g, b, 0, st, A);
    else hipLaunchKernelGGL((k_adjoint_batch<Q, QS, Real, V, NTV, ACC_PP>), g, b, 0, st, A);
  }
  static void adjoint_batch(hipStream_t st, const BatchArgs<Real>& A, int blocks, int acc = ACC_PP) {
    const dim3 g(blocks), b(kWave * A.kw * A.rpb);
    if (A.nt) adjoint_batch_acc<true>(st, A, g, b, acc);
    else adjoint_batch_acc<false>(st, A, g, b, acc);
  }

  // streaming stores (and cotangent loads) when the state buffers a launch touches exceed the
  // last-level cache: ping-pong primal and adjoint 2, in-place primal 1, one-shot 4 (2 in place)
  static bool nt(lbm_ctx* c, int buffers) { return buffers * c->plan.state_bytes > kLastLevelCacheBytes; }
  // dynamic LDS of an LX launch: the staging runs of `states` states, one value per thread each
  static size_t lx_bytes(const Geo& g, int states) {
    return (size_t)states * Shifted<Q, QS>::count() * g.block.x * g.block.y * sizeof(Real);
  }
  // LX variant for this context and launch: rows that fit a block, and staging
  // within 64 KB of LDS per block (the FP64 one-shot of D3Q19 + D3Q7 on 512-wide
  // blocks would need 96 KB and keeps the plain access)
  static bool lx(lbm_ctx* c, const Geo& g, int states) {
    return lx_rows(c->cfg) && lx_bytes(g, states) <= 65536;
  }
  // access pattern of the current state buffer: ping-pong, or the in-place phase of step t
  static int acc(lbm_ctx* c) { return c->plan.inplace ? ((c->t % 2 == 0) ? ACC_EVEN : ACC_ODD) : ACC_PP; }
  // One in-place step from the current phase; records the moments when mom != null.
  // Streaming stores and hints: a recorded step takes them once its state exceeds
  // the last-level cache (plain stores: 0.819 -> 0.748 of peak, D3Q19 FP32
  // 256x128x128), its even phase's loads only beyond twice the cache.  An
  // unrecorded step stores plainly up to the cache size (NT stores in the odd
  // phase cost 0.76 -> 0.73 at 128x96x96 and 0.88 -> 0.86 at 192x128x128); between
  // one and two caches its odd (staged) phase takes NT stores and the even phase
  // stays plain (0.787 -> 0.860 at 256x128x128; NT stores in both phases 0.741,
  // with the even-phase load hint 0.839); beyond twice the cache it takes NT
  // stores and hinted loads in both phases (0.662 -> 0.750 at 512x256x128, 0.668 ->
  // 0.815 at 512x128x128; a plain even phase there 0.66 and 0.67).
  static void primal_inplace(lbm_ctx* c, void* buf, int64_t t, void* mom) {
    Geo g = hot_geometry(c->cfg);
    Real* a = (Real*)buf;
    const Real* w = (const Real*)c->w;
    Real* m = (Real*)mom;
    const bool even = (t % 2 == 0);
    const bool lx = Ops::lx(c, g, 1);
#define LBM_PI(NTV, MOMV, ACCV)                                                                                    \
  do {                                                                                                             \
    if (ACCV == ACC_ODD && lx)                                                                                     \
      hipLaunchKernelGGL((k_primal_inplace<Q, QS, Real, NTV, MOMV, V, ACC_ODD, false, true>), g.grid, g.block,     \
                         lx_bytes(g, 1), c->stream, P(c), a, w, m);                                                \
    else                                                                                                           \
      hipLaunchKernelGGL((k_primal_inplace<Q, QS, Real, NTV, MOMV, V, ACCV>), g.grid, g.block, 0, c->stream, P(c), \
                         a, w, m);                                                                                 \
  } while (0)
    if (m && nt(c, 1)) {
      // the even phase's loads take the streaming hint too once the state is far beyond the cache
      if (even && c->plan.state_bytes > 2 * kLastLevelCacheBytes)
        hipLaunchKernelGGL((k_primal_inplace<Q, QS, Real, true, true, V, ACC_EVEN, true>), g.grid, g.block, 0,
                           c->stream, P(c), a, w, m);
      else if (even) LBM_PI(true, true, ACC_EVEN);
      else LBM_PI(true, true, ACC_ODD);
    } else if (m) {
      if (even) LBM_PI(false, true, ACC_EVEN);
      else LBM_PI(false, true, ACC_ODD);
    } else if (c->plan.state_bytes > 2 * kLastLevelCacheBytes) {
      // unrecorded, state far beyond the cache: streaming stores and hinted loads in both phases
      if (even)
        hipLaunchKernelGGL((k_primal_inplace<Q, QS, Real, true, false, V, ACC_EVEN, true>), g.grid, g.block, 0,
                           c->stream, P(c), a, w, m);
      else LBM_PI(true, false, ACC_ODD);
    } else if (nt(c, 1)) {
      // unrecorded, state between one and two caches: streaming stores in the odd phase only
      if (even) LBM_PI(false, false, ACC_EVEN);
      else LBM_PI(true, false, ACC_ODD);
    } else {
      if (even) LBM_PI(false, false, ACC_EVEN);
      else LBM_PI(false, false, ACC_ODD);
    }
#undef LBM_PI
  }
  static void oneshot_inplace(lbm_ctx* c, double zeta, double pen) {
    Geo g = hot_geometry(c->cfg);
    Real* a = (Real*)c->cur;
    Real* l = (Real*)c->lam[0];
    Real* w = (Real*)c->w;
    Real* gr = (Real*)c->grad;
    const double* gl = (const double*)c->glob;
    const bool even = (c->t % 2 == 0);
    const bool lx = Ops::lx(c, g, 2);
#define LBM_OS_INPLACE(NTV, ACCV)                                                                                 \
  do {                                                                                                            \
    if (ACCV == ACC_ODD && lx)                                                                                    \
      hipLaunchKernelGGL((k_oneshot_inplace<Q, QS, Real, NTV, V, ACC_ODD, true>), g.grid, g.block, lx_bytes(g, 2),  \
                         c->stream, P(c), a, l, w, gr, gl, (Real)zeta, (Real)pen);                                \
    else                                                                                                          \
      hipLaunchKernelGGL((k_oneshot_inplace<Q, QS, Real, NTV, V, ACCV>), g.grid, g.block, 0, c->stream, P(c), a, l, \
                         w, gr, gl, (Real)zeta, (Real)pen);                                                       \
  } while (0)
    if (nt(c, 2)) {
      if (even) LBM_OS_INPLACE(true, ACC_EVEN);
      else LBM_OS_INPLACE(true, ACC_ODD);
    } else {
      if (even) LBM_OS_INPLACE(false, ACC_EVEN);
      else LBM_OS_INPLACE(false, ACC_ODD);
    }
#undef LBM_OS_INPLACE
  }
  static lbm_status write_static(lbm_ctx* c) {
    static_assert(sizeof(BatchStatic<Real>) <= kDescBytes, "descriptor region too small");
    BatchStatic<Real> h;
    h.p = P(c);
    h.waves = batch_waves(c);
    hipLaunchKernelGGL((k_write_desc<Real>), dim3(1), dim3(64), 0, c->stream, h, (BatchStatic<Real>*)c->desc);
    return launch_check(c, "descriptor upload");
  }
  static_assert(Mom<Q, QS, V>::N == (Q == 19 ? 3 : 2) + 1 + (QS > 0 ? ((V & kVarVD) ? QS : 1) : 0),
                "moment count mismatch");
  // One primal step; records the moments of the pulled state when mom != null.
  static void primal(lbm_ctx* c, const void* src, void* dst, void* mom = nullptr) {
    Geo g = hot_geometry(c->cfg);
    const Real* s = (const Real*)src;
    Real* d = (Real*)dst;
    const Real* w = (const Real*)c->w;
    Real* m = (Real*)mom;
#define LBM_PP(NTV, MOMV)                                                                                     \
  do {                                                                                                        \
    if (Ops::lx(c, g, 1))                                                                                     \
      hipLaunchKernelGGL((k_primal<Q, QS, Real, NTV, MOMV, V, true>), g.grid, g.block, lx_bytes(g, 1), c->stream,  \
                         P(c), s, d, w, m);                                                                   \
    else                                                                                                      \
      hipLaunchKernelGGL((k_primal<Q, QS, Real, NTV, MOMV, V>), g.grid, g.block, 0, c->stream, P(c), s, d, w, m); \
  } while (0)
    if (nt(c, 2)) {
      if (m) LBM_PP(true, true);
      else LBM_PP(true, false);
    } else {
      if (m) LBM_PP(false, true);
      else LBM_PP(false, false);
    }
#undef LBM_PP
  }
  static void objective(lbm_ctx* c, const void* src, double* out) {
    double* part = c->glob + kGlobSlots;
    hipLaunchKernelGGL((k_objective_partial<Q, QS, Real>), dim3(kObjBlocks), dim3(kObjThreads), 0, c->stream, P(c),
                       (const Real*)src, part, acc(c));
    hipLaunchKernelGGL((k_objective_final<Q, QS, Real>), dim3(1), dim3(64), 0, c->stream, P(c),
                       (const double*)part, out);
  }
  static void seed(lbm_ctx* c, const void* src, void* lam) {
    Geo g = node_geometry(c->cfg);
    hipLaunchKernelGGL((k_seed<Q, QS, Real>), g.grid, g.block, 0, c->stream, P(c), (const Real*)src,
                       (const double*)c->glob, (Real*)lam, acc(c), c->plan.inplace ? 1 : 0,
                       1.0 / (double)c->plan.W);
  }
  // Window state s: its boundary sums and objective, and its inlet/outlet columns.
  static void capture(lbm_ctx* c, const void* src, int64_t s) {
    objective(c, src, win_glob(c, s));
    const int n = 2 * c->cfg.ny * c->cfg.nz;
    hipLaunchKernelGGL((k_capture_columns<Q, QS, Real>), dim3((n + 255) / 256), dim3(256), 0, c->stream, P(c),
                       (const Real*)src, acc(c), (Real*)win_cols(c, s));
  }
  // lambda^n += (1/W) dJ/df^n of window state s, lambda^n in layout pattern.
  static void window_seed(lbm_ctx* c, int64_t s, void* lam, int pattern) {
    const int n = 2 * c->cfg.ny * c->cfg.nz;
    hipLaunchKernelGGL((k_window_seed<Q, QS, Real>), dim3((n + 255) / 256), dim3(256), 0, c->stream, P(c),
                       (const Real*)win_cols(c, s), (const double*)win_glob(c, s), (Real*)lam, pattern,
                       1.0 / (double)c->plan.W);
  }
  // One in-place adjoint step: the cotangent buffer is in the odd-pattern layout
  // after an even number of adjoint steps (the seed writes that layout).
  static void adjoint_inplace(lbm_ctx* c, const void* mom, int64_t steps_done) {
    Geo g = hot_geometry(c->cfg);
    const Real* m = (const Real*)mom;
    Real* l = (Real*)c->lam[0];
    const Real* w = (const Real*)c->w;
    Real* gr = (Real*)c->grad;
    const bool odd = (steps_done % 2 == 0);
    const bool lx = Ops::lx(c, g, 1);
    const bool far = c->plan.state_bytes > 2 * kLastLevelCacheBytes;  // streaming hints on the staged accesses
#define LBM_AI(NTV, ACCV)                                                                                         \
  do {                                                                                                            \
    if (ACCV == ACC_ODD && lx && far)                                                                             \
      hipLaunchKernelGGL((k_adjoint_inplace<Q, QS, Real, NTV, V, ACC_ODD, true, true>), g.grid, g.block,          \
                         lx_bytes(g, 1), c->stream, P(c), m, l, w, gr);                                           \
    else if (ACCV == ACC_ODD && lx)                                                                               \
      hipLaunchKernelGGL((k_adjoint_inplace<Q, QS, Real, NTV, V, ACC_ODD, false, true>), g.grid, g.block,         \
                         lx_bytes(g, 1), c->stream, P(c), m, l, w, gr);                                           \
    else                                                                                                          \
      hipLaunchKernelGGL((k_adjoint_inplace<Q, QS, Real, NTV, V, ACCV>), g.grid, g.block, 0, c->stream, P(c), m, l, \
                         w, gr);                                                                                  \
  } while (0)
    // streaming stores and hints whatever the state size: the adjoint also streams a moment set per
    // step, and a cotangent state that fits the last-level cache gains nothing from staying there
    // (192x96x96 D3Q19 FP32, 134 MB: 0.769 -> 0.836 of HBM peak; 128x96x96: 0.738 -> 0.771)
    if (odd) LBM_AI(true, ACC_ODD);
    else if (c->plan.state_bytes > 2 * kLastLevelCacheBytes)  // even-phase hint far beyond the cache
      hipLaunchKernelGGL((k_adjoint_inplace<Q, QS, Real, true, V, ACC_EVEN, true>), g.grid, g.block, 0, c->stream,
                         P(c), m, l, w, gr);
    else LBM_AI(true, ACC_EVEN);
#undef LBM_AI
  }
  static void adjoint(lbm_ctx* c, const void* mom, const void* lin, void* lout) {
    Geo g = hot_geometry(c->cfg);
    const Real *m = (const Real*)mom, *li = (const Real*)lin, *w = (const Real*)c->w;
    Real *lo = (Real*)lout, *gr = (Real*)c->grad;
    const bool lx = Ops::lx(c, g, 1);
    // streaming whatever the state size, as the in-place adjoint
    if (lx)
      hipLaunchKernelGGL((k_adjoint<Q, QS, Real, true, V, true>), g.grid, g.block, lx_bytes(g, 1), c->stream, P(c), m,
                         li, lo, w, gr);
    else
      hipLaunchKernelGGL((k_adjoint<Q, QS, Real, true, V>), g.grid, g.block, 0, c->stream, P(c), m, li, lo, w, gr);
  }
  static void oneshot(lbm_ctx* c, const void* src, void* dst, const void* lin, void* lout, double zeta,
                      double pen) {
    Geo g = hot_geometry(c->cfg);
    const Real *s = (const Real*)src, *li = (const Real*)lin;
    Real *d = (Real*)dst, *lo = (Real*)lout, *w = (Real*)c->w, *gr = (Real*)c->grad;
    const double* gl = (const double*)c->glob;
    const bool lx = Ops::lx(c, g, 2);
#define LBM_OS(NTV, LXV)                                                                                   \
  hipLaunchKernelGGL((k_oneshot<Q, QS, Real, NTV, V, LXV>), g.grid, g.block, LXV ? lx_bytes(g, 2) : 0, c->stream, \
                     P(c), s, d, li, lo, w, gr, gl, (Real)zeta, (Real)pen)
    if (nt(c, 4)) {
      if (lx) LBM_OS(true, true);
      else LBM_OS(true, false);
    } else {
      if (lx) LBM_OS(false, true);
      else LBM_OS(false, false);
    }
#undef LBM_OS
  }
  static void get_adjoint(lbm_ctx* c, const void* lam, double* lf, double* lg, int pattern) {
    Geo g = node_geometry(c->cfg);
    hipLaunchKernelGGL((k_get_adjoint<Q, QS, Real>), g.grid, g.block, 0, c->stream, P(c), (const Real*)lam, lf, lg,
                       pattern);
  }
  static void fields(lbm_ctx* c, const void* src, double* rho, double* u, double* s) {
    Geo g = node_geometry(c->cfg);
    hipLaunchKernelGGL((k_fields<Q, QS, Real>), g.grid, g.block, 0, c->stream, P(c), (const Real*)src, rho, u, s,
                       acc(c));
  }
  static void get_state(lbm_ctx* c, const void* src, double* f, double* gg) {
    Geo g = node_geometry(c->cfg);
    hipLaunchKernelGGL((k_get_state<Q, QS, Real>), g.grid, g.block, 0, c->stream, P(c), (const Real*)src, f, gg,
                       acc(c));
  }
  static void set_state(lbm_ctx* c, const double* f, const double* gg, void* dst) {
    Geo g = node_geometry(c->cfg);
    hipLaunchKernelGGL((k_set_state<Q, QS, Real>), g.grid, g.block, 0, c->stream, P(c), f, gg, (Real*)dst,
                       c->plan.inplace ? ACC_EVEN : ACC_PP);
  }
  static void maps(lbm_ctx* c, uint8_t* mask, int64_t* src) {
    Geo g = node_geometry(c->cfg);
    hipLaunchKernelGGL((k_maps<Q, QS, Real>), g.grid, g.block, 0, c->stream, P(c), mask, src);
  }
  static void fill(lbm_ctx* c, void* a, size_t n) {
    hipLaunchKernelGGL((k_fill<Real>), flat_grid(n), dim3(256), 0, c->stream, (Real*)a, n, Real(0));
  }
  static void copy(lbm_ctx* c, const void* a, void* b, size_t n) {
    hipLaunchKernelGGL((k_copy<Real>), flat_grid(n), dim3(256), 0, c->stream, (const Real*)a, (Real*)b, n);
  }
  // node array: compact ABI layout -> padded workspace layout, and back
  static void node_in(lbm_ctx* c, const void* a, void* b) {
    Geo g = node_geometry(c->cfg);
    hipLaunchKernelGGL((k_node_in<Real>), g.grid, g.block, 0, c->stream, P(c), (const Real*)a, (Real*)b);
  }
  static void grad_penalty(lbm_ctx* c, double pen, void* b) {
    Geo g = node_geometry(c->cfg);
    hipLaunchKernelGGL((k_grad_penalty<Real>), g.grid, g.block, 0, c->stream, P(c), (const Real*)c->grad,
                       (const Real*)c->w, (Real)pen, (Real*)b);
  }
  static void node_out(lbm_ctx* c, const void* a, void* b) {
    Geo g = node_geometry(c->cfg);
    hipLaunchKernelGGL((k_node_out<Real>), g.grid, g.block, 0, c->stream, P(c), (const Real*)a, (Real*)b);
  }
};

// Calls F::template run<Ops<...>>(args) for the context's lattice/precision.
template <template <class> class F, class... A>
lbm_status dispatch(lbm_ctx* c, A&&... a) {
  const lbm_config& k = c->cfg;
  const bool f32 = k.precision == LBM_FP32;
  const bool mrt = k.collision == LBM_COLL_MRT;
  const bool vd = blended_diffusivity(&k);
  if (k.flow == 9 && k.scalar == 0) return f32 ? F<Ops<9, 0, float>>::run(c, a...) : F<Ops<9, 0, double>>::run(c, a...);
  if (k.flow == 9 && k.scalar == 5) {
    if (vd) return f32 ? F<Ops<9, 5, float, kVarVD>>::run(c, a...) : F<Ops<9, 5, double, kVarVD>>::run(c, a...);
    return f32 ? F<Ops<9, 5, float>>::run(c, a...) : F<Ops<9, 5, double>>::run(c, a...);
  }
  if (k.flow == 19 && k.scalar == 0) {
    if (mrt)
      return f32 ? F<Ops<19, 0, float, kVarMRT>>::run(c, a...) : F<Ops<19, 0, double, kVarMRT>>::run(c, a...);
    return f32 ? F<Ops<19, 0, float>>::run(c, a...) : F<Ops<19, 0, double>>::run(c, a...);
  }
  if (mrt && vd) {
    constexpr int V = kVarMRT | kVarVD;
    return f32 ? F<Ops<19, 7, float, V>>::run(c, a...) : F<Ops<19, 7, double, V>>::run(c, a...);
  }
  if (mrt) return f32 ? F<Ops<19, 7, float, kVarMRT>>::run(c, a...) : F<Ops<19, 7, double, kVarMRT>>::run(c, a...);
  if (vd) return f32 ? F<Ops<19, 7, float, kVarVD>>::run(c, a...) : F<Ops<19, 7, double, kVarVD>>::run(c, a...);
  return f32 ? F<Ops<19, 7, float>>::run(c, a...) : F<Ops<19, 7, double>>::run(c, a...);
}

void* ckpt_slot(lbm_ctx* c, int64_t s) { return c->ckpt + (uint64_t)s * c->plan.state_bytes; }
// Moment set of step k (slot k mod C).
void* mom_slot(lbm_ctx* c, int64_t k) { return c->mom + (uint64_t)(k % c->plan.C) * c->plan.mom_bytes; }
// Trajectory segment holding the horizon's last step (0 in a store-all plan).
int64_t last_segment(lbm_ctx* c) { return c->cfg.nsteps > 0 ? (c->cfg.nsteps - 1) / c->plan.C : 0; }
void* other_pp(lbm_ctx* c, const void* cur) { return (cur == c->pp[0]) ? c->pp[1] : c->pp[0]; }

// Destination of h^k while recording: a checkpoint slot or a ping-pong buffer.
void* rec_dst(lbm_ctx* c, int64_t k) {
  const int64_t C = c->plan.C;
  const int64_t s = (k + 1) / C, i = (k + 1) % C;
  if (i == 0 && s < c->plan.S) return ckpt_slot(c, s);
  return other_pp(c, c->cur);
}

// Time-averaged objective: capture the state just produced (time t) when it is
// the next state of the window [N - W + 1, N] of a run that started at t = 0.
template <class O>
void capture_window(lbm_ctx* c) {
  const int64_t W = c->plan.W, first = c->cfg.nsteps - W + 1;
  if (W > 1 && c->t >= first && c->t - first == c->win_count) {
    O::capture(c, c->cur, c->win_count);
    ++c->win_count;
  }
}

// Whole window captured and the run at its end: the objective is the window mean.
bool window_complete(const lbm_ctx* c) {
  return c->plan.W > 1 && c->win_count == c->plan.W && c->t == c->cfg.nsteps;
}

template <class O>
struct RunPrimal {
  static lbm_status run(lbm_ctx* c, int64_t nsteps, int record) {
    // A recorded run keeps the moments of the horizon's last segment only (all of
    // them in a store-all plan): the backward recomputes every earlier segment
    // from its checkpoint before it reads that segment's moments.
    const int64_t keep_from = last_segment(c) * c->plan.C;
    if (c->plan.inplace) {
      const bool ckpts = record && c->work != ckpt_slot(c, 0);  // checkpointed plan (C < N)
      for (int64_t i = 0; i < nsteps; ++i) {
        if (ckpts && c->t % c->plan.C == 0)  // the state at t = sC, in its phase's layout
          O::copy(c, c->work, ckpt_slot(c, c->t / c->plan.C), (size_t)c->plan.QT * c->plan.Np);
        O::primal_inplace(c, c->work, c->t, record && c->t >= keep_from ? mom_slot(c, c->t) : nullptr);
        ++c->t;
        capture_window<O>(c);
      }
      return launch_check(c, "in-place primal step");
    }
    for (int64_t i = 0; i < nsteps; ++i) {
      void* src = c->cur;
      void* dst = record ? rec_dst(c, c->t) : other_pp(c, c->cur);
      O::primal(c, src, dst, record && c->t >= keep_from ? mom_slot(c, c->t) : nullptr);
      c->cur = dst;
      ++c->t;
      capture_window<O>(c);
    }
    return launch_check(c, "primal step");
  }
};

template <class O>
struct RunObjective {
  static lbm_status run(lbm_ctx* c, double* J_dev) {
    O::objective(c, c->cur, c->glob);
    if (window_complete(c))
      hipLaunchKernelGGL(k_window_mean, dim3(1), dim3(64), 0, c->stream, (const double*)c->win, (int)c->plan.W,
                         c->glob);
    if (J_dev) {
      hipError_t e = hipMemcpyAsync(J_dev, c->glob + kNG, sizeof(double), hipMemcpyDeviceToDevice, c->stream);
      if (e != hipSuccess) return fail(c, LBM_EHIP, "objective copy: %s", hipGetErrorString(e));
    }
    return launch_check(c, "objective");
  }
};

// Recompute segment s from its checkpoint: steps k = sC .. min(sC + C, N) - 1,
// recording their moments (the states themselves go through the ping-pong).
template <class O>
void recompute_segment(lbm_ctx* c, int64_t s) {
  Range r("lbm recompute segment");
  const int64_t C = c->plan.C;
  const int64_t end = std::min<int64_t>(s * C + C, c->rec_len);
  const void* src = ckpt_slot(c, s);
  for (int64_t k = s * C; k < end; ++k) {
    void* dst = other_pp(c, src);
    O::primal(c, src, dst, mom_slot(c, k));
    src = dst;
  }
  c->mom_seg = s;
}

// In-place plan: recompute segment s inside its own checkpoint slot (its last
// use), recording the moments of steps sC .. min(sC + C, N) - 1; step k runs in
// the access pattern of its phase k mod 2, the layout the slot was saved in.
template <class O>
void recompute_segment_inplace(lbm_ctx* c, int64_t s) {
  Range r("lbm recompute segment (in place)");
  const int64_t C = c->plan.C;
  const int64_t end = std::min<int64_t>(s * C + C, c->rec_len);
  void* buf = ckpt_slot(c, s);
  for (int64_t k = s * C; k < end; ++k) O::primal_inplace(c, buf, k, mom_slot(c, k));
  c->mom_seg = s;
}

// Seeds lambda^N = dJ/df^N and zeroes the gradient (first adjoint call).
template <class O>
void start_adjoint(lbm_ctx* c) {
  const int64_t C = c->plan.C;
  O::objective(c, c->cur, c->glob);
  O::seed(c, c->cur, c->lam[0]);
  O::fill(c, c->grad, (size_t)c->plan.Np);
  c->lam_cur = 0;
  c->t_adj = c->rec_len;
  // the recorded run's moments are held when it ended in the horizon's last segment
  // (a batched run records every step, so this can miss a segment it holds: that
  // segment is then recomputed, with the same result)
  const int64_t s = c->rec_len > 0 ? (c->rec_len - 1) / C : -1;
  c->mom_seg = s == last_segment(c) ? s : -1;
  c->adj_started = true;
}

template <class O>
struct RunAdjoint {
  static lbm_status run(lbm_ctx* c, int64_t nsteps) {
    const int64_t C = c->plan.C;
    // window states n < N whose objective terms enter lambda^n (none unless W > 1)
    const int64_t first = c->plan.W > 1 ? c->cfg.nsteps - c->plan.W + 1 : INT64_MAX;
    if (!c->adj_started) start_adjoint<O>(c);
    if (c->plan.inplace) {  // store-all never recomputes; C < N recomputes each segment in place
      for (int64_t i = 0; i < nsteps; ++i) {
        const int64_t n = c->t_adj - 1;
        const int64_t s = n / C;
        if (s != c->mom_seg) recompute_segment_inplace<O>(c, s);
        O::adjoint_inplace(c, mom_slot(c, n), c->rec_len - c->t_adj);
        --c->t_adj;
        if (n >= first)  // lambda^n now in the layout of its step count
          O::window_seed(c, n - first, c->lam[0], ((c->rec_len - c->t_adj) % 2 == 0) ? ACC_ODD : ACC_EVEN);
      }
      return launch_check(c, "in-place adjoint step");
    }
    for (int64_t i = 0; i < nsteps; ++i) {
      const int64_t n = c->t_adj - 1;
      const int64_t s = n / C;
      if (s != c->mom_seg) recompute_segment<O>(c, s);
      O::adjoint(c, mom_slot(c, n), c->lam[c->lam_cur], c->lam[1 - c->lam_cur]);
      c->lam_cur ^= 1;
      --c->t_adj;
      if (n >= first) O::window_seed(c, n - first, c->lam[c->lam_cur], ACC_PP);
    }
    return launch_check(c, "adjoint step");
  }
};

// The buffer that holds the state at t = 0: the in-place working buffer, or
// checkpoint slot 0 (ping-pong: the first checkpoint itself).
void* initial_buffer(lbm_ctx* c) { return c->plan.inplace ? c->work : ckpt_slot(c, 0); }

template <class O>
struct RunReset {
  static lbm_status run(lbm_ctx* c) {
    O::fill(c, initial_buffer(c), (size_t)c->plan.QT * c->plan.Np);
    return launch_check(c, "reset");
  }
};

template <class O>
struct RunSetState {
  static lbm_status run(lbm_ctx* c, const double* f, const double* g) {
    O::set_state(c, f, g, initial_buffer(c));
    return launch_check(c, "set_state");
  }
};

template <class O>
struct RunGradient {
  static lbm_status run(lbm_ctx* c, void* out) {
    O::node_out(c, c->grad, out);
    return launch_check(c, "gradient");
  }
};

template <class O>
struct RunGradientPenalty {
  static lbm_status run(lbm_ctx* c, double pen, void* out) {
    O::grad_penalty(c, pen, out);
    return launch_check(c, "gradient_penalty");
  }
};

template <class O>
struct RunFields {
  static lbm_status run(lbm_ctx* c, double* rho, double* u, double* s) {
    O::fields(c, c->cur, rho, u, s);
    return launch_check(c, "fields");
  }
};

template <class O>
struct RunGetState {
  static lbm_status run(lbm_ctx* c, double* f, double* g) {
    O::get_state(c, c->cur, f, g);
    return launch_check(c, "get_state");
  }
};

template <class O>
struct RunGetAdjoint {
  static lbm_status run(lbm_ctx* c, double* lf, double* lg) {
    // the one-shot's in-place buffer follows the primal's phase; the unsteady adjoint's
    // alternates from the seed's layout (odd pattern after an even number of steps)
    int pattern = c->adj_started ? ACC_PP : O::acc(c);
    if (c->plan.inplace && c->adj_started) pattern = ((c->rec_len - c->t_adj) % 2 == 0) ? ACC_ODD : ACC_EVEN;
    O::get_adjoint(c, c->lam[c->lam_cur], lf, c->plan.QS ? lg : nullptr, pattern);
    return launch_check(c, "get_adjoint");
  }
};

template <class O>
struct RunMaps {
  static lbm_status run(lbm_ctx* c, uint8_t* mask, int64_t* src) {
    O::maps(c, mask, src);
    return launch_check(c, "export_maps");
  }
};

template <class O>
struct RunSetDesign {
  static lbm_status run(lbm_ctx* c, const void* w) {
    O::node_in(c, w, c->w);
    return launch_check(c, "set_design");
  }
};

// One-shot iterations: each is [objective sums of f^n when the seed depends
// on them] + one fused k_oneshot launch.  The first call zeroes lambda.
template <class O>
struct RunOneshot {
  static lbm_status run(lbm_ctx* c, int64_t nsteps, double zeta, double pen) {
    if (!c->os_active) {
      O::fill(c, c->lam[0], (size_t)c->plan.QT * c->plan.Np);
      c->lam_cur = 0;
      O::objective(c, c->cur, c->glob);
      c->os_active = true;
      c->rec_open = false;
    }
    // the variance term's source depends on the current outlet mean: refresh the sums every iteration
    const bool state_dependent_seed = (c->cfg.c_var != 0.0);
    for (int64_t i = 0; i < nsteps; ++i) {
      if (state_dependent_seed) O::objective(c, c->cur, c->glob);
      if (c->plan.inplace) {
        O::oneshot_inplace(c, zeta, pen);
        ++c->t;
        continue;
      }
      void* dst = (c->cur == c->pp[0]) ? c->pp[1] : c->pp[0];
      O::oneshot(c, c->cur, dst, c->lam[c->lam_cur], c->lam[1 - c->lam_cur], zeta, pen);
      c->cur = dst;
      c->lam_cur ^= 1;
      ++c->t;
    }
    return launch_check(c, "one-shot step");
  }
};

template <class O>
struct RunGetDesign {
  static lbm_status run(lbm_ctx* c, void* out) {
    O::node_out(c, c->w, out);
    return launch_check(c, "get_design");
  }
};

template <class O>
struct RunWriteStatic {
  static lbm_status run(lbm_ctx* c) { return O::write_static(c); }
};

// Batched primal steps: one launch per step covers every context.
template <class O>
struct RunPrimalBatch {
  // In place: per step, the checkpoint copies of members at t = sC (checkpointed
  // plans), then one launch per phase among the members (two when their
  // parities differ), each member's buffer read and rewritten in place.
  static lbm_status run_inplace(lbm_ctx* c0, lbm_ctx* const* cs, int n, int64_t nsteps, int record) {
    using Real = typename O::RealT;
    BatchArgs<Real> A;
    std::memset(&A, 0, sizeof A);
    for (int64_t i = 0; i < nsteps; ++i) {
      for (int k = 0; k < n; ++k) {
        lbm_ctx* c = cs[k];
        const bool ckpts = record && c->work != ckpt_slot(c, 0);  // checkpointed plan (C < N)
        if (ckpts && c->t % c->plan.C == 0)
          O::copy(c, c->work, ckpt_slot(c, c->t / c->plan.C), (size_t)c->plan.QT * c->plan.Np);
      }
      for (int phase = 0; phase < 2; ++phase) {
        lbm_ctx* mem[kBatchMax];
        int nm = 0;
        for (int k = 0; k < n; ++k)
          if (cs[k]->t % 2 == phase) mem[nm++] = cs[k];
        if (nm == 0) continue;
        A.n = nm;
        A.kw = batch_block_waves(mem, nm);
        A.rpb = batch_rows_per_block(mem, nm, A.kw);
        A.lx = batch_lx(mem, nm, A.kw);
        batch_nt_inplace(mem, nm, !record, phase == 1, &A.nt, &A.nte);
        int total = 0;
        for (int k = 0; k < nm; ++k) {
          lbm_ctx* c = mem[k];
          A.start[k] = total;
          A.st[k] = (const BatchStatic<Real>*)c->desc;
          A.w[k] = (const Real*)c->w;
          A.g[k] = (Real*)c->grad;
          A.a[k] = (const Real*)c->work;
          A.b[k] = nullptr;
          A.c[k] = (Real*)c->work;
          A.m[k] = record ? (Real*)mom_slot(c, c->t) : nullptr;
          total += O::batch_blocks(c, A.kw, A.rpb);
        }
        A.start[nm] = total;
        O::primal_batch(c0->stream, A, total, phase == 0 ? ACC_EVEN : ACC_ODD);
      }
      for (int k = 0; k < n; ++k) ++cs[k]->t;
    }
    return launch_check(c0, "batched in-place primal step");
  }

  static lbm_status run(lbm_ctx* c0, lbm_ctx* const* cs, int n, int64_t nsteps, int record) {
    using Real = typename O::RealT;
    if (c0->plan.inplace) return run_inplace(c0, cs, n, nsteps, record);
    BatchArgs<Real> A;
    std::memset(&A, 0, sizeof A);
    A.n = n;
    A.kw = batch_block_waves(cs, n);
    A.rpb = batch_rows_per_block(cs, n, A.kw);
    A.lx = batch_lx(cs, n, A.kw);
    A.nt = batch_nt(cs, n);
    for (int64_t i = 0; i < nsteps; ++i) {
      int total = 0;
      for (int k = 0; k < n; ++k) {
        lbm_ctx* c = cs[k];
        void* dst = record ? rec_dst(c, c->t) : other_pp(c, c->cur);
        A.start[k] = total;
        A.st[k] = (const BatchStatic<Real>*)c->desc;
        A.w[k] = (const Real*)c->w;
        A.g[k] = (Real*)c->grad;
        A.a[k] = (const Real*)c->cur;
        A.b[k] = nullptr;
        A.c[k] = (Real*)dst;
        A.m[k] = record ? (Real*)mom_slot(c, c->t) : nullptr;
        total += O::batch_blocks(c, A.kw, A.rpb);
        c->cur = dst;
        ++c->t;
      }
      A.start[n] = total;
      O::primal_batch(c0->stream, A, total);
    }
    return launch_check(c0, "batched primal step");
  }
};

// Batched adjoint steps.  Contexts that still have to be seeded are seeded
// first; before each reverse step, the contexts whose next step lies in a
// segment whose moments are not held recompute it, batched together.
template <class O>
struct RunAdjointBatch {
  // In place: members whose next step lies in a segment whose moments are not
  // held recompute it inside its checkpoint (single-context launches); then one
  // launch per cotangent pattern among the members.
  static lbm_status run_inplace(lbm_ctx* c0, lbm_ctx* const* cs, int n, int64_t nsteps) {
    using Real = typename O::RealT;
    BatchArgs<Real> A;
    std::memset(&A, 0, sizeof A);
    for (int64_t i = 0; i < nsteps; ++i) {
      for (int k = 0; k < n; ++k) {
        lbm_ctx* c = cs[k];
        const int64_t s = (c->t_adj - 1) / c->plan.C;
        if (s != c->mom_seg) recompute_segment_inplace<O>(c, s);
      }
      for (int odd = 0; odd < 2; ++odd) {
        lbm_ctx* mem[kBatchMax];
        int nm = 0;
        for (int k = 0; k < n; ++k)  // the cotangent is in the odd-pattern layout after an even step count
          if (((cs[k]->rec_len - cs[k]->t_adj) % 2 == 0) == (odd == 1)) mem[nm++] = cs[k];
        if (nm == 0) continue;
        A.n = nm;
        A.kw = batch_block_waves(mem, nm);
        A.rpb = batch_rows_per_block(mem, nm, A.kw);
        A.lx = batch_lx(mem, nm, A.kw);
        batch_nt_inplace(mem, nm, false, false, &A.nt, &A.nte);
        A.nt = 1;  // the adjoint streams whatever the state size (see Ops::adjoint_inplace)
        int total = 0;
        for (int k = 0; k < nm; ++k) {
          lbm_ctx* c = mem[k];
          A.start[k] = total;
          A.st[k] = (const BatchStatic<Real>*)c->desc;
          A.w[k] = (const Real*)c->w;
          A.g[k] = (Real*)c->grad;
          A.a[k] = (const Real*)mom_slot(c, c->t_adj - 1);
          A.m[k] = nullptr;
          A.b[k] = (const Real*)c->lam[0];
          A.c[k] = (Real*)c->lam[0];
          total += O::batch_blocks(c, A.kw, A.rpb);
        }
        A.start[nm] = total;
        O::adjoint_batch(c0->stream, A, total, odd ? ACC_ODD : ACC_EVEN);
      }
      for (int k = 0; k < n; ++k) --cs[k]->t_adj;
    }
    return launch_check(c0, "batched in-place adjoint step");
  }

  static lbm_status run(lbm_ctx* c0, lbm_ctx* const* cs, int n, int64_t nsteps) {
    using Real = typename O::RealT;
    for (int k = 0; k < n; ++k)
      if (!cs[k]->adj_started) start_adjoint<O>(cs[k]);
    if (c0->plan.inplace) return run_inplace(c0, cs, n, nsteps);
    BatchArgs<Real> A;
    std::memset(&A, 0, sizeof A);
    for (int64_t i = 0; i < nsteps; ++i) {
      // segment recomputes
      lbm_ctx* need[kBatchMax];
      int64_t first[kBatchMax], last[kBatchMax], seg[kBatchMax];
      const void* src[kBatchMax];
      int nn = 0;
      int64_t longest = 0;
      for (int k = 0; k < n; ++k) {
        lbm_ctx* c = cs[k];
        const int64_t C = c->plan.C;
        const int64_t s = (c->t_adj - 1) / C;
        if (s == c->mom_seg) continue;
        need[nn] = c;
        seg[nn] = s;
        first[nn] = s * C;
        last[nn] = std::min<int64_t>(s * C + C, c->rec_len) - 1;
        src[nn] = ckpt_slot(c, s);
        longest = std::max<int64_t>(longest, last[nn] - first[nn] + 1);
        ++nn;
      }
      for (int64_t r = 0; r < longest; ++r) {
        lbm_ctx* mem[kBatchMax];  // the contexts with a recompute step r left
        int nm = 0;
        for (int q = 0; q < nn; ++q)
          if (first[q] + r <= last[q]) mem[nm++] = need[q];
        A.kw = batch_block_waves(mem, nm);
        A.rpb = batch_rows_per_block(mem, nm, A.kw);
        A.lx = batch_lx(mem, nm, A.kw);
        A.nt = batch_nt(mem, nm);
        int m = 0, total = 0;
        for (int q = 0; q < nn; ++q) {
          const int64_t kk = first[q] + r;
          if (kk > last[q]) continue;
          lbm_ctx* c = need[q];
          void* dst = other_pp(c, src[q]);
          A.start[m] = total;
          A.st[m] = (const BatchStatic<Real>*)c->desc;
          A.w[m] = (const Real*)c->w;
          A.g[m] = (Real*)c->grad;
          A.a[m] = (const Real*)src[q];
          A.b[m] = nullptr;
          A.c[m] = (Real*)dst;
          A.m[m] = (Real*)mom_slot(c, kk);
          total += O::batch_blocks(c, A.kw, A.rpb);
          src[q] = dst;
          ++m;
        }
        A.n = m;
        A.start[m] = total;
        O::primal_batch(c0->stream, A, total);
      }
      for (int q = 0; q < nn; ++q) need[q]->mom_seg = seg[q];
      // one reverse step for every context
      int total = 0;
      A.n = n;
      A.kw = batch_block_waves(cs, n);
      A.rpb = batch_rows_per_block(cs, n, A.kw);
      A.lx = batch_lx(cs, n, A.kw);
      A.nt = 1;  // the adjoint streams whatever the state size (see Ops::adjoint_inplace)
      for (int k = 0; k < n; ++k) {
        lbm_ctx* c = cs[k];
        const int64_t nstep = c->t_adj - 1;
        A.start[k] = total;
        A.st[k] = (const BatchStatic<Real>*)c->desc;
        A.w[k] = (const Real*)c->w;
        A.g[k] = (Real*)c->grad;
        A.a[k] = (const Real*)mom_slot(c, nstep);
        A.m[k] = nullptr;
        A.b[k] = (const Real*)c->lam[c->lam_cur];
        A.c[k] = (Real*)c->lam[1 - c->lam_cur];
        total += O::batch_blocks(c, A.kw, A.rpb);
        c->lam_cur ^= 1;
        --c->t_adj;
      }
      A.start[n] = total;
      O::adjoint_batch(c0->stream, A, total);
    }
    return launch_check(c0, "batched adjoint step");
  }
};

// Checks shared by every batched call: same lattice/precision/stream, distinct.
lbm_status check_batch(lbm_ctx* const* cs, int32_t n) {
  if (!cs || n < 1 || n > kBatchMax) return LBM_EINVAL;
  for (int k = 0; k < n; ++k) {
    if (!cs[k]) return LBM_EINVAL;
    for (int q = 0; q < k; ++q)
      if (cs[q] == cs[k]) return fail(cs[0], LBM_EINVAL, "batch: context %d appears twice", k);
    if (cs[k]->plan.inplace != cs[0]->plan.inplace)
      return fail(cs[0], LBM_EINVAL, "batch: context %d %s in place, context 0 %s", k,
                  cs[k]->plan.inplace ? "streams" : "does not stream", cs[0]->plan.inplace ? "does" : "does not");
    if (cs[k]->plan.W > 1) return fail(cs[0], LBM_EINVAL, "batch: context %d averages its objective", k);
    const lbm_config &a = cs[0]->cfg, &b = cs[k]->cfg;
    if (a.flow != b.flow || a.scalar != b.scalar || a.precision != b.precision)
      return fail(cs[0], LBM_EINVAL, "batch: context %d has another lattice or precision", k);
    if (cs[k]->stream != cs[0]->stream) return fail(cs[0], LBM_EINVAL, "batch: context %d uses another stream", k);
  }
  return LBM_OK;
}

void reset_times(lbm_ctx* c) {
  c->t = 0;
  c->rec_len = 0;
  c->rec_open = true;
  c->cur = initial_buffer(c);
  c->adj_started = false;
  c->t_adj = -1;
  c->lam_cur = 0;
  c->mom_seg = -1;
  c->os_active = false;
  c->state_lost = false;
  c->win_count = 0;
}

lbm_status sync_check(lbm_ctx* c, const char* what) {
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(c, LBM_EHIP, "%s: %s", what, hipGetErrorString(e));
  return LBM_OK;
}

// ------------------------------------------------- static device workspace
// For callers that cannot allocate device memory (code under HIP graph
// capture, allocation-free serving loops): lbm_create_static carves the
// context from this file-scope array instead of a caller's workspace.  Each
// device holds its own copy until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns for the current device (the
// array's name in host code is a host-side stand-in, not a device address).
constexpr uint64_t kStaticWorkspaceBytes = 128ull << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

struct StaticSlot {
  void* ptr = nullptr;  // device address of scratch on this device
  bool busy = false;    // a static context is alive on this device
};
std::mutex g_static_mu;
StaticSlot g_static[kMaxDevices];

}  // namespace

// ================================================================= C ABI
extern "C" {

lbm_status lbm_required_bytes(const lbm_config* cfg, uint64_t* bytes_out) {
  if (!bytes_out) return LBM_EINVAL;
  Plan p;
  lbm_status s = make_plan(cfg, &p, nullptr);
  if (s != LBM_OK) return s;
  *bytes_out = p.total;
  return LBM_OK;
}

lbm_status lbm_create(const lbm_config* cfg, void* hip_stream, void* workspace_dev, uint64_t workspace_bytes,
                      lbm_ctx** ctx_out) {
  if (!ctx_out) return LBM_EINVAL;
  *ctx_out = nullptr;
  Plan p;
  std::string why;
  lbm_status s = make_plan(cfg, &p, &why);
  if (s != LBM_OK) {
    fprintf(stderr, "lbm_create: %s\n", why.c_str());
    return s;
  }
  if (!workspace_dev || ((uintptr_t)workspace_dev % kAlign) != 0) return LBM_EINVAL;
  if (workspace_bytes < p.total) return LBM_ENOMEM;
  lbm_ctx* c = new lbm_ctx();
  c->cfg = *cfg;
  c->plan = p;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)workspace_dev;
  c->ws_bytes = workspace_bytes;
  char* q = c->ws;
  c->w = q;
  q += p.node_bytes;
  c->grad = q;
  q += p.node_bytes;
  c->glob = (double*)q;
  q += align_up(kGlobBytes);
  c->desc = q;
  q += align_up(kDescBytes);
  if (p.inplace) {
    c->lam[0] = c->lam[1] = q;  // one adjoint buffer, rewritten in place
    q += p.state_bytes;
    c->pp[0] = c->pp[1] = nullptr;
    if (cfg->nsteps > 0 && p.C < cfg->nsteps) {  // checkpointed: a working buffer of its own
      c->work = q;
      q += p.state_bytes;
    }
  } else {
    for (int i = 0; i < 2; ++i) {
      c->lam[i] = q;
      q += p.state_bytes;
    }
    for (int i = 0; i < 2; ++i) {
      c->pp[i] = q;
      q += p.state_bytes;
    }
  }
  c->ckpt = q;
  q += (uint64_t)p.S * p.state_bytes;
  c->mom = q;
  q += (uint64_t)p.C * p.mom_bytes;
  if (p.W > 1) {
    c->win = q;
    q += p.win_bytes;
  }
  if (p.inplace && !c->work) c->work = c->ckpt;  // store-all / unrecorded: the state lives in ckpt[0]
  reset_times(c);
  s = dispatch<RunReset>(c);
  if (s == LBM_OK) s = dispatch<RunWriteStatic>(c);
  if (s != LBM_OK) {
    delete c;
    return s;
  }
  *ctx_out = c;
  return LBM_OK;
}

lbm_status lbm_create_static(const lbm_config* cfg, void* hip_stream, lbm_ctx** ctx_out) {
  if (!ctx_out) return LBM_EINVAL;
  *ctx_out = nullptr;
  uint64_t need = 0;
  lbm_status s = lbm_required_bytes(cfg, &need);
  if (s != LBM_OK) return s;
  if (need > kStaticWorkspaceBytes) {
    fprintf(stderr, "lbm_create_static: the configuration needs %llu bytes, the static workspace holds %llu\n",
            (unsigned long long)need, (unsigned long long)kStaticWorkspaceBytes);
    return LBM_ENOMEM;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LBM_EHIP;
  std::lock_guard<std::mutex> lock(g_static_mu);
  StaticSlot& slot = g_static[dev];
  if (!slot.ptr) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      fprintf(stderr, "lbm_create_static: hipGetSymbolAddress: %s\n", hipGetErrorString(e));
      return LBM_EHIP;
    }
    slot.ptr = ptr;
  }
  if (slot.busy) {
    fprintf(stderr, "lbm_create_static: another static context is alive on device %d\n", dev);
    return LBM_ESTATE;
  }
  s = lbm_create(cfg, hip_stream, slot.ptr, kStaticWorkspaceBytes, ctx_out);
  if (s != LBM_OK) return s;
  slot.busy = true;
  (*ctx_out)->static_dev = dev;
  return LBM_OK;
}

uint64_t lbm_static_workspace_bytes(void) { return kStaticWorkspaceBytes; }

lbm_status lbm_destroy(lbm_ctx* ctx) {
  if (!ctx) return LBM_EINVAL;
  if (ctx->static_dev >= 0) {
    // the next static context on this device reuses the array: let this
    // context's queued work finish first (unless its stream is being captured)
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(ctx->stream, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone)
      (void)hipStreamSynchronize(ctx->stream);
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static[ctx->static_dev].busy = false;
  }
  delete ctx;
  return LBM_OK;
}

lbm_status lbm_set_design(lbm_ctx* c, const void* w_dev) {
  if (!c) return LBM_EINVAL;
  if (!w_dev) return fail(c, LBM_EINVAL, "set_design: NULL design field");
  lbm_status s = dispatch<RunSetDesign>(c, w_dev);
  if (s != LBM_OK) return s;
  c->design_set = true;
  // a recorded trajectory or adjoint of another design is no longer valid; once an
  // adjoint has run, recomputed segments may have overwritten the buffer that held
  // the primal state, so calls that read it wait for lbm_reset / lbm_set_state
  if (c->adj_started) c->state_lost = true;
  if (c->rec_len > 0 || c->adj_started) {
    c->rec_len = 0;
    c->rec_open = false;
    c->adj_started = false;
    c->t_adj = -1;
  }
  return LBM_OK;
}

lbm_status lbm_reset(lbm_ctx* c) {
  if (!c) return LBM_EINVAL;
  reset_times(c);
  return dispatch<RunReset>(c);
}

lbm_status lbm_set_state(lbm_ctx* c, const double* f_dev, const double* g_dev) {
  if (!c) return LBM_EINVAL;
  if (!f_dev) return fail(c, LBM_EINVAL, "set_state: NULL f");
  reset_times(c);
  return dispatch<RunSetState>(c, f_dev, g_dev);
}

lbm_status lbm_primal_steps(lbm_ctx* c, int64_t nsteps, int32_t record) {
  if (!c) return LBM_EINVAL;
  if (nsteps < 0) return fail(c, LBM_EINVAL, "primal_steps: negative count");
  if (!c->design_set) return fail(c, LBM_ESTATE, "primal_steps: no design field set");
  if (c->adj_started) return fail(c, LBM_ESTATE, "primal_steps: adjoint started; call lbm_reset first");
  if (c->state_lost) return fail(c, LBM_ESTATE, "primal_steps: primal state consumed by an adjoint; call lbm_reset");
  if (record && c->os_active) return fail(c, LBM_ESTATE, "primal_steps: one-shot running; call lbm_reset first");
  if (record && c->plan.inplace && c->cfg.nsteps == 0)
    return fail(c, LBM_ESTATE, "primal_steps: an in-place context with no horizon does not record");
  if (record) {
    if (!(c->rec_open && c->t == c->rec_len))
      return fail(c, LBM_ESTATE, "primal_steps: recording must start at t = 0 or continue a recorded run");
    if (c->t + nsteps > c->cfg.nsteps)
      return fail(c, LBM_EINVAL, "primal_steps: recorded run of %lld steps exceeds the horizon %lld",
                  (long long)(c->t + nsteps), (long long)c->cfg.nsteps);
  }
  if (nsteps == 0) return LBM_OK;
  Range r(record ? "lbm_primal_steps (recorded)" : "lbm_primal_steps");
  lbm_status s = dispatch<RunPrimal>(c, nsteps, (int)(record != 0));
  if (record) {
    c->rec_len = c->t;
  } else {
    c->rec_open = false;
  }
  return s;
}

lbm_status lbm_objective_async(lbm_ctx* c, double* J_dev) {
  if (!c) return LBM_EINVAL;
  if (c->adj_started || c->state_lost) return fail(c, LBM_ESTATE, "objective: primal state consumed by the adjoint");
  return dispatch<RunObjective>(c, J_dev);
}

lbm_status lbm_objective(lbm_ctx* c, double* J_host, double* globals_host) {
  if (!c) return LBM_EINVAL;
  if (c->adj_started || c->state_lost) return fail(c, LBM_ESTATE, "objective: primal state consumed by the adjoint");
  lbm_status s = dispatch<RunObjective>(c, (double*)nullptr);
  if (s != LBM_OK) return s;
  double h[kNG + 1];
  hipError_t e = hipMemcpyAsync(h, c->glob, sizeof h, hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return fail(c, LBM_EHIP, "objective: %s", hipGetErrorString(e));
  s = sync_check(c, "objective");
  if (s != LBM_OK) return s;
  if (J_host) *J_host = h[kNG];
  if (globals_host) std::memcpy(globals_host, h, kNG * sizeof(double));
  if (!std::isfinite(h[kNG])) return fail(c, LBM_ENONFINITE, "objective is not finite");
  return LBM_OK;
}

lbm_status lbm_adjoint_steps(lbm_ctx* c, int64_t nsteps) {
  if (!c) return LBM_EINVAL;
  if (nsteps < 0) return fail(c, LBM_EINVAL, "adjoint_steps: negative count");
  if (c->os_active) return fail(c, LBM_ESTATE, "adjoint_steps: one-shot running; call lbm_reset first");
  if (c->plan.inplace && c->cfg.nsteps == 0)
    return fail(c, LBM_ESTATE, "adjoint_steps: an in-place context with no horizon keeps no trajectory");
  if (!c->adj_started) {
    if (!c->design_set) return fail(c, LBM_ESTATE, "adjoint_steps: no design field set");
    if (!(c->rec_open && c->t == c->rec_len))
      return fail(c, LBM_ESTATE, "adjoint_steps: needs a recorded run ending at the current time");
    if (nsteps > c->rec_len) return fail(c, LBM_EINVAL, "adjoint_steps: more steps than recorded");
    if (c->plan.W > 1 && !window_complete(c))
      return fail(c, LBM_ESTATE, "adjoint_steps: the time-averaged objective needs a recorded run to the horizon");
  } else if (nsteps > c->t_adj) {
    return fail(c, LBM_EINVAL, "adjoint_steps: only %lld steps remain", (long long)c->t_adj);
  }
  Range r("lbm_adjoint_steps");
  return dispatch<RunAdjoint>(c, nsteps);
}

lbm_status lbm_gradient(lbm_ctx* c, void* grad_dev) {
  if (!c) return LBM_EINVAL;
  if (!grad_dev) return fail(c, LBM_EINVAL, "gradient: NULL output");
  if (!(c->adj_started && c->t_adj == 0) && !c->os_active)
    return fail(c, LBM_ESTATE, "gradient: adjoint has not reached t = 0 and no one-shot iteration ran");
  return dispatch<RunGradient>(c, grad_dev);
}

lbm_status lbm_gradient_penalty(lbm_ctx* c, double penalty, void* grad_dev) {
  if (!c) return LBM_EINVAL;
  if (!grad_dev) return fail(c, LBM_EINVAL, "gradient_penalty: NULL output");
  if (!std::isfinite(penalty)) return fail(c, LBM_EINVAL, "gradient_penalty: non-finite weight");
  if (!(c->adj_started && c->t_adj == 0) && !c->os_active)
    return fail(c, LBM_ESTATE, "gradient_penalty: adjoint has not reached t = 0 and no one-shot iteration ran");
  return dispatch<RunGradientPenalty>(c, penalty, grad_dev);
}

lbm_status lbm_fields(lbm_ctx* c, double* rho_dev, double* u_dev, double* s_dev) {
  if (!c) return LBM_EINVAL;
  if (!rho_dev || !u_dev) return fail(c, LBM_EINVAL, "fields: NULL output");
  if (c->adj_started || c->state_lost) return fail(c, LBM_ESTATE, "fields: primal state consumed by the adjoint");
  return dispatch<RunFields>(c, rho_dev, u_dev, s_dev);
}

lbm_status lbm_get_state(lbm_ctx* c, double* f_dev, double* g_dev) {
  if (!c) return LBM_EINVAL;
  if (!f_dev) return fail(c, LBM_EINVAL, "get_state: NULL output");
  if (c->adj_started || c->state_lost)
    return fail(c, LBM_ESTATE, "get_state: primal state consumed by the adjoint");
  return dispatch<RunGetState>(c, f_dev, g_dev);
}

lbm_status lbm_get_adjoint(lbm_ctx* c, double* lf_dev, double* lg_dev) {
  if (!c) return LBM_EINVAL;
  if (!lf_dev) return fail(c, LBM_EINVAL, "get_adjoint: NULL output");
  if (!c->adj_started && !c->os_active) return fail(c, LBM_ESTATE, "get_adjoint: no adjoint state");
  return dispatch<RunGetAdjoint>(c, lf_dev, lg_dev);
}

lbm_status lbm_export_maps(lbm_ctx* c, uint8_t* mask_dev, int64_t* src_dev) {
  if (!c) return LBM_EINVAL;
  return dispatch<RunMaps>(c, mask_dev, src_dev);
}

lbm_status lbm_oneshot_steps(lbm_ctx* c, int64_t nsteps, double zeta, double penalty) {
  if (!c) return LBM_EINVAL;
  if (nsteps < 0) return fail(c, LBM_EINVAL, "oneshot_steps: negative count");
  if (!std::isfinite(zeta) || !std::isfinite(penalty)) return fail(c, LBM_EINVAL, "oneshot_steps: non-finite step");
  if (!c->design_set) return fail(c, LBM_ESTATE, "oneshot_steps: no design field set");
  if (c->adj_started || c->state_lost)
    return fail(c, LBM_ESTATE, "oneshot_steps: unsteady adjoint started; call lbm_reset first");
  Range r("lbm_oneshot_steps");
  return dispatch<RunOneshot>(c, nsteps, zeta, penalty);
}

lbm_status lbm_get_design(lbm_ctx* c, void* w_dev) {
  if (!c) return LBM_EINVAL;
  if (!w_dev) return fail(c, LBM_EINVAL, "get_design: NULL output");
  if (!c->design_set) return fail(c, LBM_ESTATE, "get_design: no design field set");
  return dispatch<RunGetDesign>(c, w_dev);
}

lbm_status lbm_times(const lbm_ctx* c, int64_t* t, int64_t* recorded, int64_t* t_adj) {
  if (!c) return LBM_EINVAL;
  if (t) *t = c->t;
  if (recorded) *recorded = c->rec_len;
  if (t_adj) *t_adj = c->adj_started ? c->t_adj : -1;
  return LBM_OK;
}

lbm_status lbm_plan(const lbm_ctx* c, int64_t* interval, int64_t* n_checkpoints, int64_t* n_moment_sets,
                    uint64_t* state_bytes) {
  if (!c) return LBM_EINVAL;
  if (interval) *interval = c->plan.C;
  if (n_checkpoints) *n_checkpoints = c->plan.S;
  if (n_moment_sets) *n_moment_sets = c->plan.C;
  if (state_bytes) *state_bytes = c->plan.state_bytes;
  return LBM_OK;
}

lbm_status lbm_primal_steps_batch(lbm_ctx* const* ctxs, int32_t n, int64_t nsteps, int32_t record) {
  lbm_status s = check_batch(ctxs, n);
  if (s != LBM_OK) return s;
  lbm_ctx* c0 = ctxs[0];
  if (nsteps < 0) return fail(c0, LBM_EINVAL, "primal_steps_batch: negative count");
  for (int k = 0; k < n; ++k) {
    lbm_ctx* c = ctxs[k];
    if (!c->design_set) return fail(c0, LBM_ESTATE, "primal_steps_batch: context %d has no design", k);
    if (c->adj_started || c->state_lost)
      return fail(c0, LBM_ESTATE, "primal_steps_batch: context %d is in its adjoint", k);
    if (record && !(c->rec_open && c->t == c->rec_len))
      return fail(c0, LBM_ESTATE, "primal_steps_batch: context %d cannot continue recording", k);
    if (record && c->t + nsteps > c->cfg.nsteps)
      return fail(c0, LBM_EINVAL, "primal_steps_batch: context %d would exceed its horizon", k);
  }
  if (nsteps == 0) return LBM_OK;
  Range r("lbm_primal_steps_batch");
  s = dispatch<RunPrimalBatch>(c0, ctxs, (int)n, nsteps, (int)(record != 0));
  for (int k = 0; k < n; ++k) {
    if (record) ctxs[k]->rec_len = ctxs[k]->t;
    else ctxs[k]->rec_open = false;
  }
  return s;
}

lbm_status lbm_adjoint_steps_batch(lbm_ctx* const* ctxs, int32_t n, int64_t nsteps) {
  lbm_status s = check_batch(ctxs, n);
  if (s != LBM_OK) return s;
  lbm_ctx* c0 = ctxs[0];
  if (nsteps < 0) return fail(c0, LBM_EINVAL, "adjoint_steps_batch: negative count");
  for (int k = 0; k < n; ++k) {
    lbm_ctx* c = ctxs[k];
    if (!c->adj_started) {
      if (!c->design_set) return fail(c0, LBM_ESTATE, "adjoint_steps_batch: context %d has no design", k);
      if (!(c->rec_open && c->t == c->rec_len))
        return fail(c0, LBM_ESTATE, "adjoint_steps_batch: context %d has no complete recorded run", k);
      if (nsteps > c->rec_len) return fail(c0, LBM_EINVAL, "adjoint_steps_batch: context %d: too many steps", k);
    } else if (nsteps > c->t_adj) {
      return fail(c0, LBM_EINVAL, "adjoint_steps_batch: context %d: only %lld steps remain", k,
                  (long long)c->t_adj);
    }
  }
  if (nsteps == 0) {
    // still seed, so that a zero-step call behaves like the single-context form
    return dispatch<RunAdjointBatch>(c0, ctxs, (int)n, (int64_t)0);
  }
  Range r("lbm_adjoint_steps_batch");
  return dispatch<RunAdjointBatch>(c0, ctxs, (int)n, nsteps);
}

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

const char* lbm_status_string(lbm_status s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "workspace too small";
    case LBM_EHIP: return "HIP error";
    case LBM_ESTATE: return "invalid state";
    case LBM_ENONFINITE: return "non-finite objective";
  }
  return "unknown status";
}

}  // extern "C"
