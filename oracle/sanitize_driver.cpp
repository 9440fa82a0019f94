// Driver that runs every entry point of the FP64 oracle on small lattices, for a
// build of the oracle with AddressSanitizer and UndefinedBehaviorSanitizer.
//
// TEST INFRASTRUCTURE ONLY (tests/test_oracle_sanitizers.py compiles it together
// with lbm_oracle.cpp into one host executable).  It covers the node classes and
// options of the oracle: D2Q9 + D2Q5 and D3Q19 + D3Q7, periodic boxes, velocity
// and pressure inlets, Dirichlet and adiabatic walls with a heating plate, MRT
// collision, blended diffusivity and the time-averaged objective.  Exit status 0 when every call succeeded and
// returned finite results; any sanitizer report aborts the run.
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

extern "C" {
// Field-for-field copy of the oracle's configuration record.
struct lbmo_cfg {
  int32_t flow_q, scalar_q, nx, ny, nz, periodic;
  double tau, tau_s, u_in, rho_out;
  int32_t scalar_wall, s_split_axis;
  double s_wall, s_in_lo, s_in_hi;
  int32_t switch_fn, reserved;
  double switch_param, c_dp, c_hf, c_var;
  int32_t inlet_mode, reserved2;
  double rho_in, u_cap, c_mix;
  int32_t collision, reserved3;
  double mrt_s[5];
  double tau_s_solid;
  int32_t plate_x0, plate_x1;
  double s_plate;
  int32_t n_avg, reserved4;
};
int lbmo_threads(int n);
int lbmo_lattice(int q, int32_t* e, double* wt, int32_t* opp, double* cs2);
int lbmo_mrt(const lbmo_cfg* cfg, double* U, double* rate, double* K);
int lbmo_mask(const lbmo_cfg* cfg, uint8_t* mask);
int lbmo_src_map(const lbmo_cfg* cfg, int64_t* src);
int lbmo_node_op(const lbmo_cfg* cfg, int x, int y, int z, const double* f, const double* g, double w, double* h,
                 double* gp);
int lbmo_primal(const lbmo_cfg* cfg, const double* w, const double* f0, const double* g0, int64_t nsteps, double* fN,
                double* gN, double* G, double* J);
int lbmo_directional(const lbmo_cfg* cfg, const double* w, const double* dw, int64_t nsteps, double* J, double* dJ);
int lbmo_adjoint(const lbmo_cfg* cfg, const double* w, const double* f0, const double* g0, int64_t nsteps, double* J,
                 double* grad, double* lam_f0, double* lam_g0);
int lbmo_fields(const lbmo_cfg* cfg, const double* fs, const double* gs, double* rho, double* u, double* T);
int lbmo_step(const lbmo_cfg* cfg, const double* w, const double* f, const double* g, double* fn, double* gn);
int lbmo_step_tangent(const lbmo_cfg* cfg, const double* w, const double* f, const double* g, const double* df,
                      const double* dg, const double* dw, double* dfn, double* dgn);
int lbmo_step_adjoint(const lbmo_cfg* cfg, const double* w, const double* f, const double* g, const double* lf,
                      const double* lg, double* lfo, double* lgo, double* gw);
int lbmo_objective_seed(const lbmo_cfg* cfg, const double* f, const double* g, double* J, double* lam_f,
                        double* lam_g);
int lbmo_oneshot(const lbmo_cfg* cfg, double* w, const double* f0, const double* g0, int64_t iters, double zeta,
                 double c_pen, double* fN, double* gN, double* lam_f, double* lam_g, double* g_last, double* J_last);
}

namespace {

int failures = 0;

void check(bool ok, const char* what, int ci) {
  if (!ok) {
    std::fprintf(stderr, "case %d: %s failed\n", ci, what);
    ++failures;
  }
}

bool finite(const std::vector<double>& v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

lbmo_cfg base(int flow, int scalar, int nx, int ny, int nz) {
  lbmo_cfg c;
  std::memset(&c, 0, sizeof c);
  c.flow_q = flow;
  c.scalar_q = scalar;
  c.nx = nx;
  c.ny = ny;
  c.nz = nz;
  c.tau = 0.8;
  c.tau_s = 0.6;
  c.u_in = 0.02;
  c.rho_out = 1.0;
  c.s_wall = 1.0;
  c.s_in_lo = 0.0;
  c.s_in_hi = 1.0;
  c.switch_fn = 1;
  c.switch_param = 0.05;
  c.c_dp = 0.1;
  c.c_hf = scalar ? 1.0 : 0.0;
  c.c_var = scalar ? 0.5 : 0.0;
  c.rho_in = 1.02;
  c.mrt_s[0] = 1.19;
  c.mrt_s[1] = 1.4;
  c.mrt_s[2] = 1.2;
  c.mrt_s[3] = 1.4;
  c.mrt_s[4] = 1.98;
  c.s_plate = 1.0;
  return c;
}

void run_case(const lbmo_cfg& c, int ci) {
  const int64_t n = (int64_t)c.nx * c.ny * c.nz;
  const int Q = c.flow_q, Qs = c.scalar_q, Qg = Qs ? Qs : 1;
  std::vector<double> w(n), dw(n), f0(Q * n), g0(Qg * n, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    w[i] = 0.5 + 0.4 * std::sin(0.37 * (double)i);
    dw[i] = std::cos(0.11 * (double)i);
  }
  std::vector<uint8_t> mask(n);
  std::vector<int64_t> src(Q * n);
  check(lbmo_mask(&c, mask.data()) == 0, "mask", ci);
  check(lbmo_src_map(&c, src.data()) == 0, "src_map", ci);
  for (int64_t i = 0; i < Q * n; ++i) check(src[i] >= 0 && src[i] < n, "src range", ci);
  std::vector<double> fN(Q * n), gN(Qg * n), G(9), grad(n), lf(Q * n), lg(Qg * n);
  double J = 0, dJ = 0;
  check(lbmo_primal(&c, w.data(), nullptr, nullptr, 12, fN.data(), gN.data(), G.data(), &J) == 0, "primal", ci);
  check(finite(fN) && std::isfinite(J), "primal finite", ci);
  check(lbmo_directional(&c, w.data(), dw.data(), 9, &J, &dJ) == 0 && std::isfinite(dJ), "directional", ci);
  check(lbmo_adjoint(&c, w.data(), nullptr, nullptr, 9, &J, grad.data(), lf.data(), lg.data()) == 0, "adjoint", ci);
  check(finite(grad) && finite(lf), "adjoint finite", ci);
  std::vector<double> rho(n), u(3 * n), T(n);
  check(lbmo_fields(&c, fN.data(), gN.data(), rho.data(), u.data(), T.data()) == 0 && finite(u), "fields", ci);
  std::vector<double> fn(Q * n), gn(Qg * n), dfn(Q * n), dgn(Qg * n), lfo(Q * n), lgo(Qg * n), gw(n);
  check(lbmo_step(&c, w.data(), fN.data(), gN.data(), fn.data(), gn.data()) == 0, "step", ci);
  check(lbmo_step_tangent(&c, w.data(), fN.data(), gN.data(), lf.data(), lg.data(), dw.data(), dfn.data(),
                          dgn.data()) == 0 && finite(dfn), "step_tangent", ci);
  check(lbmo_step_adjoint(&c, w.data(), fN.data(), gN.data(), lf.data(), lg.data(), lfo.data(), lgo.data(),
                          gw.data()) == 0 && finite(lfo), "step_adjoint", ci);
  check(lbmo_objective_seed(&c, fN.data(), gN.data(), &J, lf.data(), lg.data()) == 0 && finite(lf), "seed", ci);
  std::vector<double> ws(w), gl(n);
  double Jl = 0;
  check(lbmo_oneshot(&c, ws.data(), nullptr, nullptr, 7, 0.5, 0.01, fN.data(), gN.data(), lf.data(), lg.data(),
                     gl.data(), &Jl) == 0 && finite(ws) && finite(gl), "oneshot", ci);
  std::vector<double> h(Q), gp(Qg);
  check(lbmo_node_op(&c, 0, 1, c.nz > 1 ? 1 : 0, fN.data(), gN.data(), 0.7, h.data(), gp.data()) == 0, "node_op",
        ci);
}

}  // namespace

int main() {
  lbmo_threads(2);
  for (int q : {5, 7, 9, 19}) {
    int32_t e[3 * 19], opp[19];
    double wt[19], cs2;
    check(lbmo_lattice(q, e, wt, opp, &cs2) == 0, "lattice", q);
  }
  std::vector<lbmo_cfg> cases;
  cases.push_back(base(9, 0, 12, 6, 1));
  lbmo_cfg c = base(9, 5, 14, 7, 1);
  c.scalar_wall = 1;
  c.s_split_axis = 1;
  c.n_avg = 4;
  cases.push_back(c);
  c = base(19, 7, 9, 6, 5);
  c.s_split_axis = 2;
  c.plate_x0 = 3;
  c.plate_x1 = 6;
  c.tau_s_solid = 2.0;
  cases.push_back(c);
  c = base(19, 7, 8, 6, 5);
  c.collision = 1;
  c.inlet_mode = 1;
  c.u_cap = 0.01;
  c.c_mix = 1.0;
  cases.push_back(c);
  c = base(19, 0, 6, 5, 4);
  c.periodic = 1;
  cases.push_back(c);
  for (size_t i = 0; i < cases.size(); ++i) run_case(cases[i], (int)i);
  lbmo_cfg bad = base(9, 0, 2, 6, 1);  // rejected configurations return an error
  double J;
  check(lbmo_primal(&bad, nullptr, nullptr, nullptr, 1, nullptr, nullptr, nullptr, &J) != 0, "reject", -1);
  double U[361], r[19], K[361];
  check(lbmo_mrt(&cases[3], U, r, K) == 0, "mrt", 3);
  std::printf("sanitized oracle run: %d failures\n", failures);
  return failures ? 1 : 0;
}
