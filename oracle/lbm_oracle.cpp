// Plain FP64 CPU oracle for the adjoint lattice-Boltzmann hot path.
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference
// that the GPU library is checked against.  Only the test suite, the smoke check
// and the CPU-baseline leg of the benchmark may load it.  It shares no source,
// header, table or helper with the GPU library and must never be used as a
// fallback for it.
//
// What it computes, and where the paper defines it:
//  * the lattice L, the state f : L -> R^M and the periodic streaming
//    (Sf)_j(x+e_j) = f_j(x)                         -- Section 2.1
//  * one step of the local scheme f^{n+1}_j(x+e_j) = W^x_j(f^n(x), w)
//                                                   -- Section 2.1, eq. (normal:iteration)
//  * node operators W^x: interior BGK (eq. SRT) or, in 3D, the forced
//    multiple-relaxation-time collision (Section 3.1, the FMRT form with
//    d'Humieres' D3Q19 moment basis) with the exact-difference forcing carrying
//    the Darcy/Brinkman velocity switch u_post = G(w) u_pre of Section 3.2
//    (inlet/outlet nodes collide by BGK after their Zou-He reconstruction);
//    the scalar diffusivity interpolates linearly between fluid and solid,
//    alpha(w) = w alpha_fluid + (1-w) alpha_solid (Section 3.2), i.e.
//    tau_s(w) = w tau_s + (1-w) tau_s_solid at interior nodes; Zou-He inlet/outlet and bounce-back
//    walls (Section 3, node classes); a passive scalar on the first 5/7
//    velocities relaxed by BGK (Section 3, heat-transfer lattice)
//  * objective F = sum over nodes of node functions (eq. objective:function),
//    here through a few boundary sums ("Globals", Section 3.4); optionally
//    averaged over the last n_avg states of the run
//  * the discrete adjoint of the unsteady N-step map: reverse streaming
//    (Lemma 1, S^{-1}) followed by the transposed local Jacobian
//    (eq. adjoint:operator), and the gradient sum_j v_j dW_j/dw
//    (eq. adjoint:derivative), accumulated over every step.
//
// Every local derivative is taken by COMPLEX STEP: the node operator is a
// template on its scalar type, and evaluating it on std::complex<double> with an
// imaginary perturbation i*h (h = 1e-30) returns Im(W)/h = dW exactly to
// rounding, with no hand-derived formula.  The GPU library uses hand-derived
// vector-Jacobian products instead, so the two share no derivative algebra.
//
// Readings of the paper that this file encodes (the paper is silent or
// self-contradictory on them):
//  * switching function G: POWER G(w) = w^theta (theta = 3), or RAMP
//    G(w) = (1+q) w / (w+q); both satisfy G(0)=0, G(1)=1.
//  * Brinkman forcing acts at interior nodes only; boundary nodes ignore w.
//  * inlet: Zou-He velocity plug u = (u_in,0,0) at x = 0, or Zou-He pressure
//    (density rho_in, u = (u_x,0,0)) whose velocity is limited to u_cap: a node
//    whose pressure-form velocity would exceed u_cap takes the velocity form at
//    u_cap instead (the setup of Section 4 states the limit, not how it acts);
//    outlet: Zou-He density rho_out at x = nx-1 with zero transverse velocity;
//    the transverse momentum correction N_t = 1/2 sum_{e_x=0} f_k e_kt
//    (Hecht-Harting form in 3D).
//  * walls: rows y in {0, ny-1} (and z in {0, nz-1} in 3D) use full-way
//    bounce-back; wall rows win over inlet/outlet at corners.
//  * scalar: D2Q5 weights (1/3, 1/6 x4), c^2 = 1/3; D3Q7 weights (1/4, 1/8 x6),
//    c^2 = 1/4; equilibrium linear in u; advected by G(w) u; inlet fixes T by
//    the single unknown population; outlet takes the unknown population at its
//    equilibrium value; walls adiabatic (bounce-back) or Dirichlet (equilibrium
//    at T_wall, u = 0).
//  * heat exchanger (Section 4): its D x D heating plate at the bottom of the
//    duct is the stretch plate_x0 <= x < plate_x1 of the y = 0 wall, across the
//    whole width; those wall nodes hold the scalar at s_plate (Dirichlet) while
//    the rest of the walls stay as configured.
//  * the objective is evaluated on the pre-collision state after N steps,
//    reconstructed at the inlet/outlet exactly as the node operators do.
#include <complex>
#include <cstdint>
#include <cstring>
#include <cmath>
#include <utility>
#include <vector>
#include <omp.h>

namespace {

using cplx = std::complex<double>;
constexpr double kCsH = 1e-30;   // complex-step size

// ---------------------------------------------------------------- lattices
// D3Q19 velocities in the paper's order e_1..e_19 (Section 3), 0-based here.
const int kE19[19][3] = {
    {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, 1, 0}, {1, -1, 0}, {-1, -1, 0}, {1, 0, 1},  {-1, 0, 1}, {1, 0, -1},
    {-1, 0, -1}, {0, 1, 1}, {0, -1, 1}, {0, 1, -1}, {0, -1, -1}};

struct Lattice {
  int q = 0;
  int e[19][3] = {};
  double wt[19] = {};
  int opp[19] = {};
  double cs2 = 0;  // squared lattice sound speed of the equilibrium
};

// Builds one of the four lattices.  The 2D velocity set is the z = 0 subset
// of the D3Q19 list kept in the same order; the scalar lattices are its first
// 5 (2D) or 7 (3D) members.
Lattice make_lattice(int q) {
  Lattice L;
  L.q = q;
  if (q == 19 || q == 7) {
    for (int j = 0; j < q; ++j)
      for (int a = 0; a < 3; ++a) L.e[j][a] = kE19[j][a];
  } else {  // 9 or 5: z = 0 subset in paper order
    int k = 0;
    for (int j = 0; j < 19 && k < q; ++j)
      if (kE19[j][2] == 0) {
        for (int a = 0; a < 3; ++a) L.e[k][a] = kE19[j][a];
        ++k;
      }
  }
  for (int j = 0; j < q; ++j) {
    int n2 = L.e[j][0] * L.e[j][0] + L.e[j][1] * L.e[j][1] + L.e[j][2] * L.e[j][2];
    double w = 0;
    if (q == 19) w = (n2 == 0) ? 1.0 / 3 : (n2 == 1) ? 1.0 / 18 : 1.0 / 36;
    if (q == 9) w = (n2 == 0) ? 4.0 / 9 : (n2 == 1) ? 1.0 / 9 : 1.0 / 36;
    if (q == 7) w = (n2 == 0) ? 1.0 / 4 : 1.0 / 8;
    if (q == 5) w = (n2 == 0) ? 1.0 / 3 : 1.0 / 6;
    L.wt[j] = w;
    for (int k = 0; k < q; ++k)
      if (L.e[k][0] == -L.e[j][0] && L.e[k][1] == -L.e[j][1] && L.e[k][2] == -L.e[j][2])
        L.opp[j] = k;
  }
  L.cs2 = (q == 7) ? 0.25 : 1.0 / 3;
  return L;
}

// ---------------------------------------------------------------- config
enum { INTERIOR = 0, WALL = 1, INLET = 2, OUTLET = 3 };
enum { G_POWER = 0, G_RAMP = 1 };
enum { S_ADIABATIC = 0, S_DIRICHLET = 1 };
enum { IN_VELOCITY = 0, IN_PRESSURE = 1 };
enum { COLL_BGK = 0, COLL_MRT = 1 };

}  // namespace

extern "C" {
// Mirrored field by field in oracle/__init__.py.
struct lbmo_cfg {
  int32_t flow_q;        // 9 (D2Q9) or 19 (D3Q19)
  int32_t scalar_q;      // 0 (none), 5 (D2Q5) or 7 (D3Q7)
  int32_t nx, ny, nz;    // nz = 1 in 2D
  int32_t periodic;      // 1: every node interior (no walls, no inlet/outlet)
  double tau, tau_s;     // flow and scalar relaxation times, omega = 1/tau
  double u_in, rho_out;  // inlet velocity, outlet density
  int32_t scalar_wall;   // 0 adiabatic, 1 Dirichlet
  int32_t s_split_axis;  // inlet scalar: 0 uniform s_in_lo, 1 split on y, 2 split on z
  double s_wall, s_in_lo, s_in_hi;
  int32_t switch_fn;     // 0 POWER, 1 RAMP
  int32_t reserved;
  double switch_param;   // theta (POWER) or q (RAMP)
  double c_dp, c_hf, c_var;  // J = c_dp*dp + c_hf*HF + c_var*Var + c_mix*Mix
  int32_t inlet_mode;    // 0 velocity (u_in), 1 pressure (rho_in, velocity capped at u_cap)
  int32_t reserved2;
  double rho_in;         // inlet density of the pressure form
  double u_cap;          // pressure form: largest inlet velocity (0: no limit)
  double c_mix;          // weight of the mixing flux sum_outlet u_x (1 - T^2)
  int32_t collision;     // 0 BGK, 1 MRT (D3Q19 only)
  int32_t reserved3;
  double mrt_s[5];       // MRT rates of the moments e, eps, q, pi, m (viscous moments relax at 1/tau)
  double tau_s_solid;    // scalar relaxation time at w = 0 (0: tau_s everywhere)
  int32_t plate_x0, plate_x1;  // heating plate: the bottom-wall (y = 0) nodes with
                               // plate_x0 <= x < plate_x1, every z (none when equal)
  double s_plate;        // scalar value the plate imposes (Dirichlet)
  int32_t n_avg;         // objective = mean over the last n_avg states (<= 1: the final state)
  int32_t reserved4;
};
}

namespace {

struct Model {
  lbmo_cfg c;
  Lattice F, S;        // flow and scalar lattices (S.q == 0 when absent)
  int64_t n = 0;       // number of nodes
  int qt = 0;          // flow + scalar populations per node
  // MRT: K = U^{-1} (I - T) U, the map of the non-equilibrium part
  double K[19][19] = {};
};

// d'Humieres' D3Q19 moment basis (the matrix the paper cites for its 3D MRT),
// each row a polynomial in the velocity c: density; energy 19|c|^2 - 30;
// energy square (21|c|^4 - 53|c|^2 + 24)/2; momentum c_a and energy flux
// (5|c|^2 - 9) c_a for a = x, y, z; stresses 3c_x^2 - |c|^2 and c_y^2 - c_z^2
// with their fourth-order partners (3|c|^2 - 5) times each; off-diagonal
// stresses c_x c_y, c_y c_z, c_x c_z; third-order moments (c_y^2 - c_z^2) c_x,
// (c_z^2 - c_x^2) c_y, (c_x^2 - c_y^2) c_z.  rate[k] is the relaxation rate of
// row k: the viscous stresses (and the conserved rows, whose non-equilibrium
// part is zero) relax at omega = 1/tau, the others at the configured rates.
void mrt_basis(const Lattice& L, const lbmo_cfg& c, double U[19][19], double rate[19]) {
  for (int j = 0; j < 19; ++j) {
    const double x = L.e[j][0], y = L.e[j][1], z = L.e[j][2];
    const double c2 = x * x + y * y + z * z;
    const double row[19] = {1.0,
                            19 * c2 - 30,
                            (21 * c2 * c2 - 53 * c2 + 24) / 2,
                            x, (5 * c2 - 9) * x,
                            y, (5 * c2 - 9) * y,
                            z, (5 * c2 - 9) * z,
                            3 * x * x - c2, (3 * c2 - 5) * (3 * x * x - c2),
                            y * y - z * z, (3 * c2 - 5) * (y * y - z * z),
                            x * y, y * z, x * z,
                            (y * y - z * z) * x, (z * z - x * x) * y, (x * x - y * y) * z};
    for (int k = 0; k < 19; ++k) U[k][j] = row[k];
  }
  const double om = 1.0 / c.tau;
  const double* s = c.mrt_s;  // e, eps, q, pi, m
  const double r[19] = {om, s[0], s[1], om, s[2], om, s[2], om, s[2], om, s[3], om, s[3], om, om, om, s[4], s[4], s[4]};
  for (int k = 0; k < 19; ++k) rate[k] = r[k];
}

// K = U^{-1} diag(1 - rate) U, with U^{-1} from Gauss-Jordan elimination.
void mrt_matrix(const Lattice& L, const lbmo_cfg& c, double K[19][19]) {
  double U[19][19], rate[19], A[19][38];
  mrt_basis(L, c, U, rate);
  for (int i = 0; i < 19; ++i)
    for (int j = 0; j < 38; ++j) A[i][j] = (j < 19) ? U[i][j] : (j - 19 == i ? 1.0 : 0.0);
  for (int col = 0; col < 19; ++col) {
    int piv = col;
    for (int i = col + 1; i < 19; ++i)
      if (std::fabs(A[i][col]) > std::fabs(A[piv][col])) piv = i;
    for (int j = 0; j < 38; ++j) std::swap(A[col][j], A[piv][j]);
    const double d = A[col][col];
    for (int j = 0; j < 38; ++j) A[col][j] /= d;
    for (int i = 0; i < 19; ++i)
      if (i != col) {
        const double m = A[i][col];
        for (int j = 0; j < 38; ++j) A[i][j] -= m * A[col][j];
      }
  }
  for (int i = 0; i < 19; ++i)
    for (int j = 0; j < 19; ++j) {
      double v = 0;
      for (int k = 0; k < 19; ++k) v += A[i][19 + k] * (1.0 - rate[k]) * U[k][j];
      K[i][j] = v;
    }
}

bool make_model(const lbmo_cfg* c, Model* m) {
  if (!c) return false;
  if (c->flow_q != 9 && c->flow_q != 19) return false;
  if (c->flow_q == 9 && c->nz != 1) return false;
  if (c->flow_q == 19 && c->nz < (c->periodic ? 1 : 3)) return false;
  if (c->nx < 3 || c->ny < 3 || c->nz < 1) return false;
  if (c->scalar_q != 0 && !((c->flow_q == 9 && c->scalar_q == 5) || (c->flow_q == 19 && c->scalar_q == 7)))
    return false;
  if (c->inlet_mode != IN_VELOCITY && c->inlet_mode != IN_PRESSURE) return false;
  if (c->collision != COLL_BGK && c->collision != COLL_MRT) return false;
  if (c->collision == COLL_MRT && c->flow_q != 19) return false;
  if (c->tau_s_solid != 0.0 && !(c->tau_s_solid > 0.5)) return false;
  if (c->inlet_mode == IN_PRESSURE && !(c->rho_in > 0.0 && c->u_cap >= 0.0 && c->u_cap < 1.0)) return false;
  if (c->plate_x0 < 0 || c->plate_x1 < c->plate_x0 || c->plate_x1 > c->nx) return false;
  if (c->n_avg < 0) return false;
  m->c = *c;
  m->F = make_lattice(c->flow_q);
  m->S = Lattice();
  if (c->scalar_q) m->S = make_lattice(c->scalar_q);
  m->n = (int64_t)c->nx * c->ny * c->nz;
  m->qt = c->flow_q + c->scalar_q;
  if (c->collision == COLL_MRT) mrt_matrix(m->F, *c, m->K);
  return true;
}

// Node class (Section 3: interior, inlet/outlet, wall).
int node_class(const lbmo_cfg& c, int x, int y, int z) {
  if (c.periodic) return INTERIOR;
  bool wall = (y == 0 || y == c.ny - 1);
  if (c.flow_q == 19 && (z == 0 || z == c.nz - 1)) wall = true;
  if (wall) return WALL;
  if (x == 0) return INLET;
  if (x == c.nx - 1) return OUTLET;
  return INTERIOR;
}

// Heating plate (Section 4, heat exchanger): part of the bottom wall held at a
// fixed scalar value; the flow still bounces back there.
bool on_plate(const lbmo_cfg& c, int x, int y) { return y == 0 && x >= c.plate_x0 && x < c.plate_x1; }

inline int64_t node_index(const lbmo_cfg& c, int x, int y, int z) {
  return (int64_t)x + (int64_t)c.nx * ((int64_t)y + (int64_t)c.ny * z);
}
inline int wrap(int a, int n) { return ((a % n) + n) % n; }

// Inlet scalar value at transverse position (y, z).
double inlet_scalar(const lbmo_cfg& c, int y, int z) {
  if (c.s_split_axis == 1) return (y < c.ny / 2) ? c.s_in_lo : c.s_in_hi;
  if (c.s_split_axis == 2) return (z < c.nz / 2) ? c.s_in_lo : c.s_in_hi;
  return c.s_in_lo;
}

// Flow equilibrium, second order in u (BGK, eq. SRT).
template <class T>
T feq(const Lattice& L, int j, const T& rho, const T u[3]) {
  T eu = double(L.e[j][0]) * u[0] + double(L.e[j][1]) * u[1] + double(L.e[j][2]) * u[2];
  T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double c2 = L.cs2;
  return L.wt[j] * rho * (1.0 + eu / c2 + eu * eu / (2 * c2 * c2) - uu / (2 * c2));
}

// Scalar equilibrium, linear in u.
template <class T>
T seq(const Lattice& L, int i, const T& s, const T u[3]) {
  T eu = double(L.e[i][0]) * u[0] + double(L.e[i][1]) * u[1] + double(L.e[i][2]) * u[2];
  return L.wt[i] * s * (1.0 + eu / L.cs2);
}

// Switching function G(w) of the Darcy/Brinkman term (Section 3.2).
template <class T>
T switch_G(const lbmo_cfg& c, const T& w) {
  if (c.switch_fn == G_POWER) {
    double th = c.switch_param;
    int ith = (int)th;
    if ((double)ith == th && ith >= 0) {
      T r = T(1.0);
      for (int k = 0; k < ith; ++k) r = r * w;
      return r;
    }
    return std::pow(w, th);
  }
  double q = c.switch_param;
  return (1.0 + q) * w / (w + q);
}

// Index of the velocity (+1,0,0) and (-1,0,0) in a lattice (paper order: 1, 2).
constexpr int kPX = 1, kMX = 2;

inline double re(double a) { return a; }
inline double re(const cplx& a) { return a.real(); }

// Density and normal velocity of an inlet node from P = sum_{e_x=0} f +
// 2 sum_{e_x=-1} f, the part of the state that arrived from inside.  Mass and
// x-momentum of the rebuilt state tie them by P = rho (1 - u_x) (Zou-He).
// Velocity form: u_x = u_in, rho = P / (1 - u_in).  Pressure form: rho = rho_in,
// u_x = 1 - P / rho_in, unless u_cap > 0 and that exceeds u_cap: then the
// velocity form at u_cap (the two agree where u_x = u_cap, so rho and u_x are
// continuous in f).  The branch is decided on the real part.
template <class T>
void inlet_state(const lbmo_cfg& c, const T& P, T* rho, T* ux) {
  if (c.inlet_mode == IN_PRESSURE) {
    T up = 1.0 - P / c.rho_in;
    if (c.u_cap > 0.0 && re(up) > c.u_cap) {
      *ux = T(c.u_cap);
      *rho = P / (1.0 - c.u_cap);
    } else {
      *ux = up;
      *rho = T(c.rho_in);
    }
    return;
  }
  *ux = T(c.u_in);
  *rho = P / (1.0 - c.u_in);
}

// Local node operator W^x: pre-collision (f, g) at node x -> post-collision (h, gp).
template <class T>
void node_op(const Model& M, int cls, int x, int y, int z, const T* f, const T* g, const T& w, T* h, T* gp) {
  const Lattice& F = M.F;
  const Lattice& S = M.S;
  const lbmo_cfg& c = M.c;
  const double om = 1.0 / c.tau;
  const double oms = (S.q ? 1.0 / c.tau_s : 0.0);
  if (cls == INTERIOR) {
    T rho = T(0.0), m[3] = {T(0.0), T(0.0), T(0.0)};
    for (int j = 0; j < F.q; ++j) {
      rho += f[j];
      for (int a = 0; a < 3; ++a) m[a] += double(F.e[j][a]) * f[j];
    }
    T u[3], v[3];
    T G = switch_G(c, w);
    for (int a = 0; a < 3; ++a) {
      u[a] = m[a] / rho;
      v[a] = G * u[a];  // u_post = G(w) u_pre
    }
    // exact-difference form with T = omega I: h = E(rho,u_post) + (1-omega)(f - E(rho,u_pre))
    if (c.collision == COLL_MRT) {
      // FMRT: h = E(rho, u_post) + U^{-1}(I - T)U (f - E(rho, u_pre))
      T d[19];
      for (int j = 0; j < F.q; ++j) d[j] = f[j] - feq(F, j, rho, u);
      for (int j = 0; j < F.q; ++j) {
        T r = T(0.0);
        for (int k = 0; k < F.q; ++k) r += M.K[j][k] * d[k];
        h[j] = feq(F, j, rho, v) + r;
      }
    } else {
      for (int j = 0; j < F.q; ++j) h[j] = feq(F, j, rho, v) + (1.0 - om) * (f[j] - feq(F, j, rho, u));
    }
    if (S.q) {
      T s = T(0.0);
      for (int i = 0; i < S.q; ++i) s += g[i];
      if (c.tau_s_solid != 0.0) {
        // diffusivity interpolated between solid and fluid: tau_s(w) = w tau_s + (1 - w) tau_s_solid
        const T omw = 1.0 / (w * c.tau_s + (1.0 - w) * c.tau_s_solid);
        for (int i = 0; i < S.q; ++i) gp[i] = g[i] + omw * (seq(S, i, s, v) - g[i]);
      } else {
        for (int i = 0; i < S.q; ++i) gp[i] = g[i] + oms * (seq(S, i, s, v) - g[i]);
      }
    }
    return;
  }
  if (cls == WALL) {
    for (int j = 0; j < F.q; ++j) h[j] = f[F.opp[j]];
    if (S.q) {
      if (on_plate(c, x, y)) {
        for (int i = 0; i < S.q; ++i) gp[i] = T(S.wt[i] * c.s_plate);
      } else if (c.scalar_wall == S_DIRICHLET) {
        for (int i = 0; i < S.q; ++i) gp[i] = T(S.wt[i] * c.s_wall);
      } else {
        for (int i = 0; i < S.q; ++i) gp[i] = g[S.opp[i]];
      }
    }
    return;
  }
  // Inlet (x = 0, unknown populations have e_x = +1) or outlet (x = nx-1,
  // unknown populations have e_x = -1).
  const int sgn = (cls == INLET) ? +1 : -1;
  T s0 = T(0.0), sk = T(0.0);  // sums over e_x = 0 and over the known e_x = -sgn
  T Nt[3] = {T(0.0), T(0.0), T(0.0)};
  for (int j = 0; j < F.q; ++j) {
    int ex = F.e[j][0];
    if (ex == 0) {
      s0 += f[j];
      for (int a = 1; a < 3; ++a) Nt[a] += 0.5 * double(F.e[j][a]) * f[j];
    } else if (ex == -sgn) {
      sk += f[j];
    }
  }
  T rho, u[3] = {T(0.0), T(0.0), T(0.0)};
  if (cls == INLET) {
    inlet_state(c, s0 + 2.0 * sk, &rho, &u[0]);
  } else {
    rho = T(c.rho_out);
    u[0] = -1.0 + (s0 + 2.0 * sk) / c.rho_out;
  }
  T fs[19];
  for (int j = 0; j < F.q; ++j) {
    if (F.e[j][0] == sgn) {
      T eu = double(F.e[j][0]) * u[0];
      T corr = double(F.e[j][1]) * Nt[1] + double(F.e[j][2]) * Nt[2];
      fs[j] = f[F.opp[j]] + 2.0 * F.wt[j] * rho * eu / F.cs2 - corr;
    } else {
      fs[j] = f[j];
    }
  }
  // BGK after the reconstruction, whatever the interior collision (the paper
  // gives FMRT for interior nodes and Zou-He for the inlet/outlet; MRT there
  // lets the third-order moments of the rebuilt state ring when their rate
  // nears 2)
  for (int j = 0; j < F.q; ++j) h[j] = fs[j] + om * (feq(F, j, rho, u) - fs[j]);
  if (!S.q) return;
  T gs[7];
  for (int i = 0; i < S.q; ++i) gs[i] = g[i];
  T sT;
  if (cls == INLET) {
    sT = T(inlet_scalar(c, y, z));
    T rest = T(0.0);
    for (int i = 0; i < S.q; ++i)
      if (i != kPX) rest += g[i];
    gs[kPX] = sT - rest;
  } else {
    T rest = T(0.0);
    for (int i = 0; i < S.q; ++i)
      if (i != kMX) rest += g[i];
    T a = S.wt[kMX] * (1.0 - u[0] / S.cs2);
    sT = rest / (1.0 - a);
    gs[kMX] = a * sT;
  }
  for (int i = 0; i < S.q; ++i) gp[i] = gs[i] + oms * (seq(S, i, sT, u) - gs[i]);
}

// Boundary sums contributed by one node's pre-collision state (the
// "Globals" of Section 3.4):
//  G0 sum inlet rho, G1 inlet count, G2 sum outlet rho, G3 outlet count,
//  G4 sum outlet u_x*T, G5 sum outlet T, G6 sum outlet T^2, G7 sum outlet u_x,
//  G8 sum outlet u_x*T^2.
constexpr int kNG = 9;
template <class T>
void node_globals(const Model& M, int cls, const T* f, const T* g, T* G) {
  for (int k = 0; k < kNG; ++k) G[k] = T(0.0);
  const Lattice& F = M.F;
  const Lattice& S = M.S;
  const lbmo_cfg& c = M.c;
  if (cls != INLET && cls != OUTLET) return;
  const int sgn = (cls == INLET) ? +1 : -1;
  T s0 = T(0.0), sk = T(0.0);
  for (int j = 0; j < F.q; ++j) {
    if (F.e[j][0] == 0) s0 += f[j];
    else if (F.e[j][0] == -sgn) sk += f[j];
  }
  if (cls == INLET) {
    T ux;
    inlet_state(c, s0 + 2.0 * sk, &G[0], &ux);
    G[1] = T(1.0);
    return;
  }
  T ux = -1.0 + (s0 + 2.0 * sk) / c.rho_out;
  G[2] = T(c.rho_out);
  G[3] = T(1.0);
  G[7] = ux;
  if (S.q) {
    T rest = T(0.0);
    for (int i = 0; i < S.q; ++i)
      if (i != kMX) rest += g[i];
    T a = S.wt[kMX] * (1.0 - ux / S.cs2);
    T sT = rest / (1.0 - a);
    G[4] = ux * sT;
    G[5] = sT;
    G[6] = sT * sT;
    G[8] = ux * sT * sT;
  }
}

// Objective from the boundary sums.
template <class T>
T objective_from_globals(const Model& M, const T* G) {
  const lbmo_cfg& c = M.c;
  T J = T(0.0);
  if (c.c_dp != 0.0) {
    T dp = M.F.cs2 * (G[0] / G[1] - G[2] / G[3]);  // p = c_s^2 rho
    J += c.c_dp * dp;
  }
  if (c.c_hf != 0.0) J += c.c_hf * G[4];
  if (c.c_var != 0.0) {
    T mean = G[5] / G[3];
    J += c.c_var * (G[6] / G[3] - mean * mean);
  }
  // mixing flux of the outlet, sum u_x (1 - T)(1 + T)  (eq. mixing:obj)
  if (c.c_mix != 0.0) J += c.c_mix * (G[7] - G[8]);
  return J;
}

// ------------------------------------------------------------ whole lattice
// State arrays are structure-of-arrays: population j of node n at j*N + n.
template <class T>
struct State {
  std::vector<T> f, g;
  void resize(const Model& M) {
    f.assign((size_t)M.F.q * M.n, T(0.0));
    g.assign((size_t)M.S.q * M.n, T(0.0));
  }
};

template <class T>
void init_state(const Model& M, const double* f0, const double* g0, State<T>& st) {
  st.resize(M);
  for (int j = 0; j < M.F.q; ++j)
    for (int64_t n = 0; n < M.n; ++n) st.f[j * M.n + n] = T(f0 ? f0[j * M.n + n] : M.F.wt[j]);
  for (int i = 0; i < M.S.q; ++i)
    for (int64_t n = 0; n < M.n; ++n) st.g[i * M.n + n] = T(g0 ? g0[i * M.n + n] : 0.0);
}

// One step of eq. (normal:iteration): collide at x, then stream to x + e_j.
template <class T, class TW>
void step(const Model& M, const TW* w, const State<T>& cur, State<T>& nxt) {
  const lbmo_cfg& c = M.c;
  const int Q = M.F.q, Qs = M.S.q;
  const int64_t N = M.n;
#pragma omp parallel for schedule(static) collapse(2)
  for (int z = 0; z < c.nz; ++z)
    for (int y = 0; y < c.ny; ++y)
      for (int x = 0; x < c.nx; ++x) {
        int64_t n = node_index(c, x, y, z);
        T f[19], g[7], h[19], gp[7];
        for (int j = 0; j < Q; ++j) f[j] = cur.f[j * N + n];
        for (int i = 0; i < Qs; ++i) g[i] = cur.g[i * N + n];
        T wn = T(w[n]);
        node_op(M, node_class(c, x, y, z), x, y, z, f, g, wn, h, gp);
        for (int j = 0; j < Q; ++j) {
          int64_t d = node_index(c, wrap(x + M.F.e[j][0], c.nx), wrap(y + M.F.e[j][1], c.ny),
                                 wrap(z + M.F.e[j][2], c.nz));
          nxt.f[j * N + d] = h[j];
        }
        for (int i = 0; i < Qs; ++i) {
          int64_t d = node_index(c, wrap(x + M.S.e[i][0], c.nx), wrap(y + M.S.e[i][1], c.ny),
                                 wrap(z + M.S.e[i][2], c.nz));
          nxt.g[i * N + d] = gp[i];
        }
      }
}

template <class T>
void globals_of(const Model& M, const State<T>& st, T* G) {
  const lbmo_cfg& c = M.c;
  for (int k = 0; k < kNG; ++k) G[k] = T(0.0);
  // serial, fixed order
  for (int z = 0; z < c.nz; ++z)
    for (int y = 0; y < c.ny; ++y)
      for (int x = 0; x < c.nx; ++x) {
        int cls = node_class(c, x, y, z);
        if (cls != INLET && cls != OUTLET) continue;
        int64_t n = node_index(c, x, y, z);
        T f[19], g[7], Gn[kNG];
        for (int j = 0; j < M.F.q; ++j) f[j] = st.f[j * M.n + n];
        for (int i = 0; i < M.S.q; ++i) g[i] = st.g[i * M.n + n];
        node_globals(M, cls, f, g, Gn);
        for (int k = 0; k < kNG; ++k) G[k] += Gn[k];
      }
}

template <class T>
T objective_of(const Model& M, const State<T>& st, T* Gout) {
  T G[kNG];
  globals_of(M, st, G);
  if (Gout)
    for (int k = 0; k < kNG; ++k) Gout[k] = G[k];
  if (M.c.periodic) return T(0.0);  // no boundary: no objective
  return objective_from_globals(M, G);
}

// Length W of the averaging window of the unsteady objective: J is the mean of
// the node-sum objective over the states f^{N-W+1} .. f^N (W = 1: f^N alone).
int64_t window(const lbmo_cfg& c) { return c.n_avg > 1 ? c.n_avg : 1; }

// dJ/df^N at every node, by the chain rule J = Phi(G), G = sum_x phi(f(x)):
// dPhi/dG by complex step on Phi, dphi/df_k(x) by complex step on phi.
void objective_seed(const Model& M, const State<double>& st, double* J, State<double>& lam) {
  const lbmo_cfg& c = M.c;
  lam.resize(M);
  double G[kNG];
  double Jv = objective_of(M, st, G);
  if (J) *J = Jv;
  if (c.periodic) return;
  double dPhi[kNG];
  for (int k = 0; k < kNG; ++k) {
    cplx Gc[kNG];
    for (int l = 0; l < kNG; ++l) Gc[l] = cplx(G[l], 0.0);
    Gc[k] += cplx(0.0, kCsH);
    dPhi[k] = std::imag(objective_from_globals(M, Gc)) / kCsH;
  }
  const int Q = M.F.q, Qs = M.S.q;
#pragma omp parallel for schedule(static) collapse(2)
  for (int z = 0; z < c.nz; ++z)
    for (int y = 0; y < c.ny; ++y)
      for (int x = 0; x < c.nx; ++x) {
        int cls = node_class(c, x, y, z);
        if (cls != INLET && cls != OUTLET) continue;
        int64_t n = node_index(c, x, y, z);
        for (int k = 0; k < Q + Qs; ++k) {
          cplx f[19], g[7], Gn[kNG];
          for (int j = 0; j < Q; ++j) f[j] = st.f[j * M.n + n];
          for (int i = 0; i < Qs; ++i) g[i] = st.g[i * M.n + n];
          if (k < Q) f[k] += cplx(0.0, kCsH);
          else g[k - Q] += cplx(0.0, kCsH);
          node_globals(M, cls, f, g, Gn);
          double d = 0;
          for (int l = 0; l < kNG; ++l) d += dPhi[l] * (std::imag(Gn[l]) / kCsH);
          if (k < Q) lam.f[k * M.n + n] = d;
          else lam.g[(k - Q) * M.n + n] = d;
        }
      }
}

// One adjoint step (transposed eq. normal:iteration):
//   v_j(x) = lam^{n+1}_j(x + e_j)                         (S^{-1}, Lemma 1)
//   lam^n_k(x) = sum_j v_j(x) dW_j/df_k (f^n(x))         (eq. adjoint:operator)
//   gw(x)     += sum_j v_j(x) dW_j/dw  (f^n(x))          (eq. adjoint:derivative)
// Each column of the local Jacobian is one complex-step evaluation of W^x.
void adjoint_step(const Model& M, const double* w, const State<double>& fn, const State<double>& lam_next,
                  State<double>& lam, double* gw) {
  const lbmo_cfg& c = M.c;
  const int Q = M.F.q, Qs = M.S.q;
  const int64_t N = M.n;
  lam.resize(M);
#pragma omp parallel for schedule(static) collapse(2)
  for (int z = 0; z < c.nz; ++z)
    for (int y = 0; y < c.ny; ++y)
      for (int x = 0; x < c.nx; ++x) {
        int64_t n = node_index(c, x, y, z);
        int cls = node_class(c, x, y, z);
        double v[19], vs[7];
        for (int j = 0; j < Q; ++j) {
          int64_t d = node_index(c, wrap(x + M.F.e[j][0], c.nx), wrap(y + M.F.e[j][1], c.ny),
                                 wrap(z + M.F.e[j][2], c.nz));
          v[j] = lam_next.f[j * N + d];
        }
        for (int i = 0; i < Qs; ++i) {
          int64_t d = node_index(c, wrap(x + M.S.e[i][0], c.nx), wrap(y + M.S.e[i][1], c.ny),
                                 wrap(z + M.S.e[i][2], c.nz));
          vs[i] = lam_next.g[i * N + d];
        }
        // columns k = 0..Q+Qs-1 for the state, k = Q+Qs for w
        for (int k = 0; k <= Q + Qs; ++k) {
          cplx f[19], g[7], h[19], gp[7];
          for (int j = 0; j < Q; ++j) f[j] = fn.f[j * N + n];
          for (int i = 0; i < Qs; ++i) g[i] = fn.g[i * N + n];
          cplx wc(w[n], 0.0);
          if (k < Q) f[k] += cplx(0.0, kCsH);
          else if (k < Q + Qs) g[k - Q] += cplx(0.0, kCsH);
          else wc += cplx(0.0, kCsH);
          node_op(M, cls, x, y, z, f, g, wc, h, gp);
          double acc = 0;
          for (int j = 0; j < Q; ++j) acc += v[j] * (std::imag(h[j]) / kCsH);
          for (int i = 0; i < Qs; ++i) acc += vs[i] * (std::imag(gp[i]) / kCsH);
          if (k < Q) lam.f[k * N + n] = acc;
          else if (k < Q + Qs) lam.g[(k - Q) * N + n] = acc;
          else gw[n] += acc;
        }
      }
}

int threads_used() { return omp_get_max_threads(); }

}  // namespace

// ================================================================ C ABI
extern "C" {

int lbmo_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
  return threads_used();
}

// Lattice tables: e (3 ints per velocity), weights, opposite index, c^2.
int lbmo_lattice(int q, int32_t* e, double* wt, int32_t* opp, double* cs2) {
  if (q != 5 && q != 7 && q != 9 && q != 19) return -1;
  Lattice L = make_lattice(q);
  for (int j = 0; j < q; ++j) {
    for (int a = 0; a < 3; ++a) e[3 * j + a] = L.e[j][a];
    wt[j] = L.wt[j];
    opp[j] = L.opp[j];
  }
  *cs2 = L.cs2;
  return 0;
}

// The MRT moment basis U (19 x 19, row k = moment k), the rates of its rows
// and K = U^{-1}(I - T)U for a D3Q19 configuration.
int lbmo_mrt(const lbmo_cfg* cfg, double* U, double* rate, double* K) {
  Model M;
  if (!make_model(cfg, &M) || M.F.q != 19) return -1;
  double Ub[19][19], r[19], Kb[19][19];
  mrt_basis(M.F, M.c, Ub, r);
  mrt_matrix(M.F, M.c, Kb);
  for (int i = 0; i < 19; ++i) {
    rate[i] = r[i];
    for (int j = 0; j < 19; ++j) {
      U[19 * i + j] = Ub[i][j];
      K[19 * i + j] = Kb[i][j];
    }
  }
  return 0;
}

int lbmo_mask(const lbmo_cfg* cfg, uint8_t* mask) {
  Model M;
  if (!make_model(cfg, &M)) return -1;
  const lbmo_cfg& c = M.c;
  for (int z = 0; z < c.nz; ++z)
    for (int y = 0; y < c.ny; ++y)
      for (int x = 0; x < c.nx; ++x) mask[node_index(c, x, y, z)] = (uint8_t)node_class(c, x, y, z);
  return 0;
}

// Pull-source map: src[j*N + n] = index of node (x - e_j) mod L.
int lbmo_src_map(const lbmo_cfg* cfg, int64_t* src) {
  Model M;
  if (!make_model(cfg, &M)) return -1;
  const lbmo_cfg& c = M.c;
  for (int j = 0; j < M.F.q; ++j)
    for (int z = 0; z < c.nz; ++z)
      for (int y = 0; y < c.ny; ++y)
        for (int x = 0; x < c.nx; ++x)
          src[j * M.n + node_index(c, x, y, z)] = node_index(
              c, wrap(x - M.F.e[j][0], c.nx), wrap(y - M.F.e[j][1], c.ny), wrap(z - M.F.e[j][2], c.nz));
  return 0;
}

// One node operator evaluation (class taken from the position).
int lbmo_node_op(const lbmo_cfg* cfg, int x, int y, int z, const double* f, const double* g, double w,
                 double* h, double* gp) {
  Model M;
  if (!make_model(cfg, &M)) return -1;
  double gdummy[7] = {0}, gpd[7];
  node_op<double>(M, node_class(M.c, x, y, z), x, y, z, f, g ? g : gdummy, w, h, gp ? gp : gpd);
  return 0;
}

// Primal run: N steps from f0/g0 (NULL: rest state f = w_j, g = 0).
// Outputs the pre-collision state after N steps, the boundary sums and J.
int lbmo_primal(const lbmo_cfg* cfg, const double* w, const double* f0, const double* g0, int64_t nsteps,
                double* fN, double* gN, double* globals, double* J) {
  Model M;
  if (!make_model(cfg, &M) || nsteps < 0) return -1;
  const int64_t W = window(M.c);
  if (W > 1 && nsteps < W) return -1;  // the window reaches back before f^1
  State<double> a, b;
  init_state(M, f0, g0, a);
  b.resize(M);
  double Jsum = 0.0;  // objectives of the window's states before the last
  for (int64_t s = 0; s < nsteps; ++s) {
    step(M, w, a, b);
    std::swap(a, b);
    if (W > 1 && s + 1 >= nsteps - W + 1 && s + 1 < nsteps) Jsum += objective_of(M, a, (double*)nullptr);
  }
  if (fN) std::memcpy(fN, a.f.data(), sizeof(double) * a.f.size());
  if (gN && M.S.q) std::memcpy(gN, a.g.data(), sizeof(double) * a.g.size());
  double G[kNG];
  double Jv = objective_of(M, a, G);
  if (globals)
    for (int k = 0; k < kNG; ++k) globals[k] = G[k];
  if (J) *J = (W > 1) ? (Jsum + Jv) / (double)W : Jv;
  return 0;
}

// Directional derivative dJ/dw . dw by complex step through the whole run
// (the tangent model of eq. normal:tangent, evaluated exactly).
int lbmo_directional(const lbmo_cfg* cfg, const double* w, const double* dw, int64_t nsteps, double* J,
                     double* dJ) {
  Model M;
  if (!make_model(cfg, &M) || nsteps < 0) return -1;
  std::vector<cplx> wc(M.n);
  for (int64_t n = 0; n < M.n; ++n) wc[n] = cplx(w[n], kCsH * dw[n]);
  const int64_t W = window(M.c);
  if (W > 1 && nsteps < W) return -1;
  State<cplx> a, b;
  init_state(M, nullptr, nullptr, a);
  b.resize(M);
  cplx Jsum(0.0, 0.0);
  for (int64_t s = 0; s < nsteps; ++s) {
    step(M, wc.data(), a, b);
    std::swap(a, b);
    if (W > 1 && s + 1 >= nsteps - W + 1 && s + 1 < nsteps) Jsum += objective_of<cplx>(M, a, nullptr);
  }
  cplx Jc = objective_of<cplx>(M, a, nullptr);
  if (W > 1) Jc = (Jsum + Jc) / (double)W;
  if (J) *J = std::real(Jc);
  if (dJ) *dJ = std::imag(Jc) / kCsH;
  return 0;
}

// Unsteady discrete adjoint: J after N steps and dJ/dw at every node.
// The trajectory f^0..f^{N-1} is kept as checkpoints every C = ceil(sqrt(N))
// steps and recomputed segment by segment (identical values to storing all).
int lbmo_adjoint(const lbmo_cfg* cfg, const double* w, const double* f0, const double* g0, int64_t nsteps,
                 double* J, double* grad, double* lam_f0, double* lam_g0) {
  Model M;
  if (!make_model(cfg, &M) || nsteps < 0) return -1;
  const int64_t N = nsteps;
  int64_t C = 1;
  while (C * C < N) ++C;
  const int64_t W = window(M.c);
  if (W > 1 && N < W) return -1;
  std::vector<State<double>> ckpt;
  State<double> cur, nxt;
  init_state(M, f0, g0, cur);
  nxt.resize(M);
  double Jsum = 0.0;
  for (int64_t s = 0; s < N; ++s) {
    if (s % C == 0) ckpt.push_back(cur);
    step(M, w, cur, nxt);
    std::swap(cur, nxt);
    if (W > 1 && s + 1 >= N - W + 1 && s + 1 < N) Jsum += objective_of(M, cur, (double*)nullptr);
  }
  State<double> lam, lam_prev, src;
  double JN = 0.0;
  objective_seed(M, cur, &JN, lam);  // lam^N = dJ/df^N
  if (J) *J = (W > 1) ? (Jsum + JN) / (double)W : JN;
  // averaged objective: every state of the window contributes (1/W) dPhi/df^n
  auto scale = [&](State<double>& st) {
    for (double& v : st.f) v /= (double)W;
    for (double& v : st.g) v /= (double)W;
  };
  if (W > 1) scale(lam);
  std::vector<double> gw(M.n, 0.0);
  std::vector<State<double>> seg;
  for (int64_t k = (int64_t)ckpt.size() - 1; k >= 0; --k) {
    int64_t n0 = k * C, n1 = std::min(N, n0 + C);
    seg.assign(1, ckpt[k]);
    for (int64_t s = n0 + 1; s < n1; ++s) {
      State<double> t;
      t.resize(M);
      step(M, w, seg.back(), t);
      seg.push_back(std::move(t));
    }
    for (int64_t s = n1 - 1; s >= n0; --s) {
      adjoint_step(M, w, seg[s - n0], lam, lam_prev, gw.data());
      std::swap(lam, lam_prev);
      if (W > 1 && s >= N - W + 1) {  // lam^s += (1/W) dPhi/df^s
        objective_seed(M, seg[s - n0], nullptr, src);
        scale(src);
        for (size_t i = 0; i < lam.f.size(); ++i) lam.f[i] += src.f[i];
        for (size_t i = 0; i < lam.g.size(); ++i) lam.g[i] += src.g[i];
      }
    }
  }
  if (grad) std::memcpy(grad, gw.data(), sizeof(double) * M.n);
  if (lam_f0) std::memcpy(lam_f0, lam.f.data(), sizeof(double) * lam.f.size());
  if (lam_g0 && M.S.q) std::memcpy(lam_g0, lam.g.data(), sizeof(double) * lam.g.size());
  return 0;
}

// Macroscopic fields of a pre-collision state, reconstructed at the
// inlet/outlet the way the node operators reconstruct them.
//   interior: rho = sum f, u = m / rho, T = sum g
//   wall:     rho = sum f, u = 0, T = sum g (adiabatic) or T_wall (Dirichlet)
//   inlet:    Zou-He rho and u = (u_x,0,0) of the inlet form, T = inlet value
//   outlet:   rho_out, u = (u_x,0,0), T = reconstructed outflow value
int lbmo_fields(const lbmo_cfg* cfg, const double* fs, const double* gs, double* rho, double* u, double* T) {
  Model M;
  if (!make_model(cfg, &M)) return -1;
  const lbmo_cfg& c = M.c;
  const int Q = M.F.q, Qs = M.S.q;
  for (int z = 0; z < c.nz; ++z)
    for (int y = 0; y < c.ny; ++y)
      for (int x = 0; x < c.nx; ++x) {
        int64_t n = node_index(c, x, y, z);
        int cls = node_class(c, x, y, z);
        double f[19], g[7] = {0};
        for (int j = 0; j < Q; ++j) f[j] = fs[j * M.n + n];
        for (int i = 0; i < Qs; ++i) g[i] = gs[i * M.n + n];
        double r = 0, m[3] = {0, 0, 0}, s = 0;
        for (int j = 0; j < Q; ++j) {
          r += f[j];
          for (int a = 0; a < 3; ++a) m[a] += M.F.e[j][a] * f[j];
        }
        for (int i = 0; i < Qs; ++i) s += g[i];
        double uo[3] = {0, 0, 0};
        if (cls == INTERIOR) {
          for (int a = 0; a < 3; ++a) uo[a] = m[a] / r;
        } else if (cls == WALL) {
          if (Qs && on_plate(c, x, y)) s = c.s_plate;
          else if (Qs && c.scalar_wall == S_DIRICHLET) s = c.s_wall;
        } else {
          double G[kNG];
          node_globals<double>(M, cls, f, g, G);
          if (cls == INLET) {
            double s0 = 0, sk = 0;
            for (int j = 0; j < Q; ++j)
              if (M.F.e[j][0] == 0) s0 += f[j];
              else if (M.F.e[j][0] == -1) sk += f[j];
            inlet_state(c, s0 + 2.0 * sk, &r, &uo[0]);
            if (Qs) s = inlet_scalar(c, y, z);
          } else {
            r = c.rho_out;
            uo[0] = G[7];
            if (Qs) s = G[5];
          }
        }
        rho[n] = r;
        for (int a = 0; a < 3; ++a) u[a * M.n + n] = uo[a];
        if (T) T[n] = s;
      }
  return 0;
}

// Single step, real arithmetic (pre-collision in, pre-collision out).
int lbmo_step(const lbmo_cfg* cfg, const double* w, const double* f, const double* g, double* fn, double* gn) {
  Model M;
  if (!make_model(cfg, &M)) return -1;
  State<double> a, b;
  init_state(M, f, g, a);
  b.resize(M);
  step(M, w, a, b);
  std::memcpy(fn, b.f.data(), sizeof(double) * b.f.size());
  if (gn && M.S.q) std::memcpy(gn, b.g.data(), sizeof(double) * b.g.size());
  return 0;
}

// Tangent of one step by complex step: d(step)(f,g,w)[df,dg,dw].
int lbmo_step_tangent(const lbmo_cfg* cfg, const double* w, const double* f, const double* g, const double* df,
                      const double* dg, const double* dw, double* dfn, double* dgn) {
  Model M;
  if (!make_model(cfg, &M)) return -1;
  State<cplx> a, b;
  a.resize(M);
  b.resize(M);
  for (size_t k = 0; k < a.f.size(); ++k) a.f[k] = cplx(f[k], kCsH * df[k]);
  for (size_t k = 0; k < a.g.size(); ++k) a.g[k] = cplx(g[k], kCsH * dg[k]);
  std::vector<cplx> wc(M.n);
  for (int64_t n = 0; n < M.n; ++n) wc[n] = cplx(w[n], kCsH * dw[n]);
  step(M, wc.data(), a, b);
  for (size_t k = 0; k < b.f.size(); ++k) dfn[k] = std::imag(b.f[k]) / kCsH;
  if (dgn)
    for (size_t k = 0; k < b.g.size(); ++k) dgn[k] = std::imag(b.g[k]) / kCsH;
  return 0;
}

// Transposed step: given the cotangent of the next state, the cotangent of
// the current state and the w-cotangent of this step.
int lbmo_step_adjoint(const lbmo_cfg* cfg, const double* w, const double* f, const double* g, const double* lf,
                      const double* lg, double* lf_out, double* lg_out, double* gw_out) {
  Model M;
  if (!make_model(cfg, &M)) return -1;
  State<double> st, ln, lo;
  init_state(M, f, g, st);
  ln.resize(M);
  std::memcpy(ln.f.data(), lf, sizeof(double) * ln.f.size());
  if (M.S.q) std::memcpy(ln.g.data(), lg, sizeof(double) * ln.g.size());
  std::vector<double> gw(M.n, 0.0);
  adjoint_step(M, w, st, ln, lo, gw.data());
  std::memcpy(lf_out, lo.f.data(), sizeof(double) * lo.f.size());
  if (lg_out && M.S.q) std::memcpy(lg_out, lo.g.data(), sizeof(double) * lo.g.size());
  std::memcpy(gw_out, gw.data(), sizeof(double) * M.n);
  return 0;
}

// J and dJ/df, dJ/dg of a pre-collision state.
int lbmo_objective_seed(const lbmo_cfg* cfg, const double* f, const double* g, double* J, double* lam_f,
                        double* lam_g) {
  Model M;
  if (!make_model(cfg, &M)) return -1;
  State<double> st, lam;
  init_state(M, f, g, st);
  objective_seed(M, st, J, lam);
  std::memcpy(lam_f, lam.f.data(), sizeof(double) * lam.f.size());
  if (lam_g && M.S.q) std::memcpy(lam_g, lam.g.data(), sizeof(double) * lam.g.size());
  return 0;
}

// One-shot descent (Section 3.3, eq. gradient:update).  Iteration n, on the
// current pre-collision state f^n, adjoint lam^n and design w^n:
//   s        = dJ/df (f^n)                                   (objective source)
//   lam^{n+1}= (dW/df)^T(f^n) S^{-1} lam^n + s               (eq. adjoint:iteration)
//   g^n      = (dW/dw)^T(f^n) S^{-1} lam^n                   (eq. adjoint:derivative)
//   f^{n+1}  = S W(f^n, w^n)                                 (eq. normal:iteration)
//   w^{n+1}  = clip(w^n + zeta (g^n + c_pen (1 - 2 w^n)), 0, 1) at interior nodes
// where c_pen weighs the penalty P = sum w(1-w) (eq. P).  lam^0 = 0 unless given.
// w is updated in place; outputs: final state, adjoint, last g and last J.
int lbmo_oneshot(const lbmo_cfg* cfg, double* w, const double* f0, const double* g0, int64_t iters, double zeta,
                 double c_pen, double* fN, double* gN, double* lam_f, double* lam_g, double* g_last, double* J_last) {
  Model M;
  if (!make_model(cfg, &M) || iters < 0) return -1;
  const lbmo_cfg& c = M.c;
  State<double> cur, nxt, lam, lam_new, seed;
  init_state(M, f0, g0, cur);
  nxt.resize(M);
  lam.resize(M);
  std::vector<double> gw(M.n, 0.0);
  double J = 0.0;
  for (int64_t it = 0; it < iters; ++it) {
    objective_seed(M, cur, &J, seed);
    std::fill(gw.begin(), gw.end(), 0.0);
    adjoint_step(M, w, cur, lam, lam_new, gw.data());
    for (size_t k = 0; k < lam_new.f.size(); ++k) lam_new.f[k] += seed.f[k];
    for (size_t k = 0; k < lam_new.g.size(); ++k) lam_new.g[k] += seed.g[k];
    step(M, w, cur, nxt);
    std::swap(cur, nxt);
    std::swap(lam, lam_new);
    for (int z = 0; z < c.nz; ++z)
      for (int y = 0; y < c.ny; ++y)
        for (int x = 0; x < c.nx; ++x) {
          if (node_class(c, x, y, z) != INTERIOR) continue;
          const int64_t n = node_index(c, x, y, z);
          double v = w[n] + zeta * (gw[n] + c_pen * (1.0 - 2.0 * w[n]));
          w[n] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
        }
  }
  if (fN) std::memcpy(fN, cur.f.data(), sizeof(double) * cur.f.size());
  if (gN && M.S.q) std::memcpy(gN, cur.g.data(), sizeof(double) * cur.g.size());
  if (lam_f) std::memcpy(lam_f, lam.f.data(), sizeof(double) * lam.f.size());
  if (lam_g && M.S.q) std::memcpy(lam_g, lam.g.data(), sizeof(double) * lam.g.size());
  if (g_last) std::memcpy(g_last, gw.data(), sizeof(double) * M.n);
  if (J_last) *J_last = J;
  return 0;
}

}  // extern "C"
