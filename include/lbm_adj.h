/*
 * lbm_adj.h -- C ABI of the MI355X (gfx950) adjoint lattice-Boltzmann library.
 *
 * The library runs, on one GPU, the three data-parallel pieces of the adjoint
 * lattice-Boltzmann topology-optimisation method:
 *   1. the fused primal collide+stream step  f^{n+1}_j(x+e_j) = W^x_j(f^n(x), w)
 *      (Section 2.1, eq. normal:iteration), with the node operators W^x of
 *      Section 3: BGK (eq. SRT) or forced MRT, with exact-difference forcing (Section 3.1)
 *      carrying the Brinkman velocity switch u_post = G(w) u_pre (Section 3.2),
 *      Zou-He inlet (velocity, or pressure with a velocity limit as in the
 *      channel setup of Section 4) and outlet, bounce-back walls, and an
 *      optional passive scalar on the first 5 (2D) / 7 (3D) velocities;
 *   2. the discrete adjoint step: reverse streaming (Lemma 1) followed by the
 *      transposed local Jacobian (eq. adjoint:operator), unsteady form over N
 *      steps, with the trajectory recovered by checkpoint + recompute;
 *   3. the per-node accumulation dJ/dw = sum_n sum_j v_j dW_j/dw
 *      (eq. adjoint:derivative).
 *
 * Conventions shared by every entry point
 *   - Status: every call returns lbm_status; 0 is success, negative values are
 *     errors.  No exception crosses the ABI.  lbm_last_error(ctx) returns a
 *     human-readable message for the last failing call on that context.
 *   - Memory: the library never allocates device memory.  lbm_create receives
 *     a caller-owned device workspace of at least lbm_required_bytes() bytes
 *     and carves every internal buffer from it.  Every other pointer argument
 *     marked "_dev" is a caller-owned device pointer; "_host" is host memory.
 *     The caller keeps ownership and must keep the workspace alive until
 *     lbm_destroy.
 *   - Streams: all device work is enqueued on the hip_stream given to
 *     lbm_create (NULL = the default stream).  Only calls with a "_host"
 *     output synchronise that stream.  Asynchronous HIP faults surface as
 *     LBM_EHIP at a later call.
 *   - Layout: node n = x + nx*(y + ny*z), x fastest.  Every state the ABI
 *     exchanges (set/get state, adjoint, fields) is plane-major double:
 *     population j of node n at j*N + n, flow populations first, then scalar
 *     populations.  Design field w and gradient are N values of the context
 *     precision (float for LBM_FP32, double for LBM_FP64).  The workspace's
 *     internal layout is private to the library.
 *   - Velocity order: the paper's D3Q19 list e_1..e_19 (Section 3), 0-based;
 *     D2Q9 is its z = 0 subset in the same order; D3Q7 / D2Q5 are the first
 *     7 / 5 members.
 *   - Node classes (exported mask values): 0 interior, 1 wall, 2 inlet, 3 outlet.
 *     Walls are the rows y in {0, ny-1} (and z in {0, nz-1} in 3D), the inlet is
 *     x = 0 and the outlet x = nx-1 (walls win at corners).  With periodic = 1
 *     every node is interior.
 */
#ifndef LBM_ADJ_H
#define LBM_ADJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx; /* opaque, library-owned host object */

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* bad argument or configuration                     */
  LBM_ENOMEM = -2,     /* workspace too small / budget cannot hold the plan  */
  LBM_EHIP = -3,       /* a HIP runtime call or kernel launch failed         */
  LBM_ESTATE = -4,     /* call not valid in the context's current state      */
  LBM_ENONFINITE = -5  /* objective is NaN or infinite                       */
} lbm_status;

enum { LBM_D2Q9 = 9, LBM_D3Q19 = 19 };
enum { LBM_SCALAR_NONE = 0, LBM_D2Q5 = 5, LBM_D3Q7 = 7 };
enum { LBM_FP32 = 4, LBM_FP64 = 8 };
enum { LBM_WALL_ADIABATIC = 0, LBM_WALL_DIRICHLET = 1 };
enum { LBM_G_POWER = 0, LBM_G_RAMP = 1 };
enum { LBM_INLET_VELOCITY = 0, LBM_INLET_PRESSURE = 1 };
enum { LBM_COLL_BGK = 0, LBM_COLL_MRT = 1 };

/* Model and run configuration (the paper's "Settings", Section 3.4). */
typedef struct lbm_config {
  uint32_t struct_size;  /* = sizeof(lbm_config); ABI version check          */
  int32_t flow;          /* LBM_D2Q9 (nz must be 1) or LBM_D3Q19 (nz >= 3)   */
  int32_t scalar;        /* LBM_SCALAR_NONE, LBM_D2Q5 (with D2Q9), LBM_D3Q7  */
  int32_t precision;     /* LBM_FP32 or LBM_FP64                             */
  int32_t nx, ny, nz;    /* lattice size, each >= 3 (nz = 1 in 2D)           */
  int32_t periodic;      /* 1: no walls/inlet/outlet, every node interior    */
  double tau, tau_s;     /* flow / scalar relaxation times; omega = 1/tau    */
  double u_in;           /* inlet velocity (x direction), lattice units      */
  double rho_out;        /* outlet density                                   */
  int32_t scalar_wall;   /* LBM_WALL_ADIABATIC or LBM_WALL_DIRICHLET         */
  int32_t s_split_axis;  /* inlet scalar: 0 uniform s_in_lo; 1 (2) split on   *
                          * y (z): s_in_lo below n/2, s_in_hi at and above   */
  double s_wall;         /* Dirichlet wall value                             */
  double s_in_lo, s_in_hi;
  int32_t switch_fn;     /* LBM_G_POWER: G = w^theta; LBM_G_RAMP:            *
                          * G = (1+q) w / (w+q)  (Section 3.2)                */
  int32_t reserved0;     /* must be 0                                        */
  double switch_param;   /* theta or q                                       */
  double c_dp, c_hf, c_var; /* J = c_dp*dp + c_hf*HF + c_var*Var + c_mix*Mix,  *
                          * dp = c_s^2 (mean inlet rho - mean outlet rho),   *
                          * HF = sum over outlet of u_x*s, Var = outlet      *
                          * variance of s, Mix = sum over outlet of          *
                          * u_x (1 - s^2) (eq. mixing:obj); the "Globals" of *
                          * Section 3.4                                      */
  int64_t nsteps;        /* horizon N the context is sized for (>= 0); a     *
                          * recorded forward run may not exceed it           */
  int64_t checkpoint_interval; /* C >= 1, or 0 = automatic (see below)       */
  uint64_t hbm_budget_bytes;   /* automatic C: 0 = the C with the smallest   *
                          * workspace (in place: C = N); else the largest C  *
                          * whose workspace fits the budget (C = N,          *
                          * store-all, when it fits)                         */
  int32_t inlet;         /* LBM_INLET_VELOCITY: Zou-He velocity u = (u_in,0,0)*
                          * LBM_INLET_PRESSURE: Zou-He density rho_in with   *
                          * u = (u_x,0,0) from the known populations; a node *
                          * whose u_x would exceed u_cap (> 0) takes the     *
                          * velocity form at u_cap instead (Section 4 limits *
                          * the inlet velocity; this is the reading)         */
  int32_t n_avg;         /* objective averaged over the last n_avg states of *
                          * the horizon, J = (1/W) sum of the objective over *
                          * f^{N-W+1} .. f^N with W = max(n_avg, 1) and N =  *
                          * nsteps (needs nsteps >= n_avg): lbm_objective    *
                          * returns the mean once a run from t = 0 reaches   *
                          * t = N, and the adjoint of such a recorded run    *
                          * adds (1/W) dJ/df^n at each window state.  0 or 1:*
                          * the final state only.  Contexts with n_avg > 1   *
                          * do not join batched launches (LBM_EINVAL)        */
  double rho_in;         /* pressure inlet density (> 0)                     */
  double u_cap;          /* pressure inlet velocity limit, 0 <= u_cap < 1;   *
                          * 0 = no limit                                     */
  double c_mix;          /* weight of the mixing flux Mix (see c_dp)         */
  int32_t collision;     /* interior collision: LBM_COLL_BGK (eq. SRT) or     *
                          * LBM_COLL_MRT, the forced multiple-relaxation-time *
                          * collision of Section 3.1 with d'Humieres' D3Q19   *
                          * moment basis (D3Q19 only); inlet/outlet nodes     *
                          * use BGK after their Zou-He reconstruction        */
  int32_t reserved2;     /* must be 0                                        */
  double mrt_rates[5];   /* MRT rates in (0, 2) of the energy, energy-square, *
                          * energy-flux, fourth-order-stress and third-order *
                          * moments; density, momentum and the viscous       *
                          * stresses relax at 1/tau                          */
  double tau_s_solid;    /* scalar relaxation time at w = 0; the diffusivity *
                          * blends linearly with the design field (Section   *
                          * 3.2): tau_s(w) = w tau_s + (1-w) tau_s_solid at  *
                          * interior nodes.  0 = tau_s everywhere            */
  int32_t inplace;       /* 1: one buffer per state, streamed in place       *
                          * (alternating even/odd access patterns): one     *
                          * primal and one adjoint buffer instead of two    *
                          * each.  A recorded run keeps the moments of every *
                          * step (no recompute) unless checkpoint_interval  *
                          * (1 <= C < nsteps) is given or hbm_budget_bytes   *
                          * cannot hold them: then it keeps a full state    *
                          * every C steps (the largest C the budget holds)  *
                          * and the adjoint recomputes each segment in      *
                          * place inside its checkpoint.  With nsteps = 0   *
                          * only unrecorded runs and the one-shot iteration *
                          * are available.  In-place contexts batch only    *
                          * with in-place contexts (LBM_EINVAL otherwise)   */
  int32_t reserved3;     /* must be 0                                        */
  int32_t plate_x0, plate_x1; /* heating plate of the heat exchanger (Section *
                          * 4): the bottom-wall (y = 0) nodes with           *
                          * plate_x0 <= x < plate_x1, every z, hold the      *
                          * scalar at s_plate (Dirichlet) while the flow     *
                          * still bounces back there; the other walls keep   *
                          * scalar_wall.  plate_x0 = plate_x1: no plate.     *
                          * 0 <= plate_x0 <= plate_x1 <= nx                  */
  double s_plate;        /* scalar value of the plate                        */
} lbm_config;

/* Workspace size for cfg (cfg->nsteps and the checkpoint plan included).
 * Errors: LBM_EINVAL for an invalid configuration, LBM_ENOMEM when no
 * checkpoint interval fits hbm_budget_bytes. */
lbm_status lbm_required_bytes(const lbm_config* cfg, uint64_t* bytes_out);

/* Creates a context on the current HIP device.  workspace_dev must hold
 * lbm_required_bytes(cfg) bytes and be 256-byte aligned.  The context starts
 * reset (rest state f = E(1,0), scalar 0) with no design set.
 * Errors: LBM_EINVAL (bad cfg, NULL/misaligned workspace), LBM_ENOMEM (too small). */
lbm_status lbm_create(const lbm_config* cfg, void* hip_stream, void* workspace_dev,
                      uint64_t workspace_bytes, lbm_ctx** ctx_out);

/* Same as lbm_create, for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops or harnesses that forbid allocation):
 * the workspace is the library's own static device array of
 * lbm_static_workspace_bytes() bytes (128 MiB) on the current device, held
 * until the process ends; nothing is allocated.  One static context may be
 * alive per device at a time; every static context on a device reuses the same
 * array (lbm_destroy waits for the context's stream unless it is being
 * captured, so the next one starts on a quiet array; work of a destroyed
 * context still queued on a captured stream races with the next context).
 * Results equal those of a context from lbm_create bitwise.
 * Errors: LBM_EINVAL (bad cfg), LBM_ENOMEM (lbm_required_bytes(cfg) exceeds the
 * static array), LBM_ESTATE (another static context is alive on the device),
 * LBM_EHIP (the array's device address cannot be obtained). */
lbm_status lbm_create_static(const lbm_config* cfg, void* hip_stream, lbm_ctx** ctx_out);

/* Size of the static device workspace lbm_create_static carves from. */
uint64_t lbm_static_workspace_bytes(void);

/* Destroys the host object; the workspace is not touched (caller-owned). */
lbm_status lbm_destroy(lbm_ctx* ctx);

/* Copies the design field w (N values, context precision, device) into the
 * workspace (Section 3.2: w = 1 fluid, w = 0 solid).  Stream-ordered.
 * Invalidates any recorded run and adjoint in progress. */
lbm_status lbm_set_design(lbm_ctx* ctx, const void* w_dev);

/* Resets to t = 0 with the rest state (f_j = w_j, scalar 0).  Clears any
 * recorded run, adjoint and gradient. */
lbm_status lbm_reset(lbm_ctx* ctx);

/* Sets the pre-collision state f^0 (Q x N doubles) and scalar g^0 (Qs x N
 * doubles, may be NULL when there is no scalar or for g^0 = 0), device
 * pointers, and resets t to 0. */
lbm_status lbm_set_state(lbm_ctx* ctx, const double* f_dev, const double* g_dev);

/* Runs nsteps primal steps (Section 2.1, eq. normal:iteration) from the
 * current time t.  record = 1 stores the trajectory for the adjoint; it is
 * allowed from t = 0 or as a continuation of a recorded run, up to
 * cfg.nsteps in total.  record = 0 runs without storing.  Asynchronous.
 * Errors: LBM_ESTATE (no design, adjoint already started, record not
 * continuable), LBM_EINVAL (negative count, beyond the horizon). */
lbm_status lbm_primal_steps(lbm_ctx* ctx, int64_t nsteps, int32_t record);

/* Objective of the current pre-collision state f^t (the node-sum objective
 * of eq. objective:function through the boundary "Globals"); with n_avg > 1
 * and a run from t = 0 at t = nsteps, the mean over the window (see
 * lbm_config.n_avg; the globals stay those of f^t).  Synchronises.
 * globals_host (nullable) receives 9 doubles: sum inlet rho, inlet count,
 * sum outlet rho, outlet count, sum outlet u_x*s, sum outlet s,
 * sum outlet s^2, sum outlet u_x, sum outlet u_x*s^2.
 * Errors: LBM_ENONFINITE for NaN/inf. */
lbm_status lbm_objective(lbm_ctx* ctx, double* J_host, double* globals_host);

/* Same as lbm_objective but writes J to device memory, no synchronisation. */
lbm_status lbm_objective_async(lbm_ctx* ctx, double* J_dev);

/* Runs nsteps reverse steps of the discrete adjoint (transposed eq.
 * normal:iteration; eq. adjoint:operator) of the recorded run.  The first
 * call seeds lambda^N = dJ/df^N and zeroes the gradient; later calls
 * continue toward t = 0.  Segments of the trajectory missing from the ring
 * are recomputed from their checkpoints.  Asynchronous.  After the adjoint
 * has started, lbm_primal_steps needs lbm_reset first.
 * Errors: LBM_ESTATE (no complete recorded run ending at the current t),
 * LBM_EINVAL (more steps than remain). */
lbm_status lbm_adjoint_steps(lbm_ctx* ctx, int64_t nsteps);

/* Writes dJ/dw (N values, context precision) to grad_dev (eq.
 * adjoint:derivative summed over all steps).  Requires the adjoint to have
 * reached t = 0, or a one-shot iteration (then the last gradient estimate);
 * LBM_ESTATE otherwise.  Asynchronous. */
lbm_status lbm_gradient(lbm_ctx* ctx, void* grad_dev);

/* Same as lbm_gradient for the penalised objective J + penalty * P(w), with
 * P = sum over interior nodes of w (1 - w) (eq. P, the term the optimiser of
 * Section 3.3 adds with a growing weight to drive w toward 0 and 1): writes
 * dJ/dw + penalty * (1 - 2w) at interior nodes and dJ/dw (zero) elsewhere.
 * Same state requirements and errors as lbm_gradient, plus LBM_EINVAL for a
 * non-finite penalty. */
lbm_status lbm_gradient_penalty(lbm_ctx* ctx, double penalty, void* grad_dev);

/* Macroscopic fields of the current pre-collision state, reconstructed at the
 * inlet/outlet like the node operators do: rho (N doubles), u (3 x N doubles,
 * component-major), s (N doubles, nullable; scalar value).  Wall nodes report
 * u = 0.  Device pointers, asynchronous. */
lbm_status lbm_fields(lbm_ctx* ctx, double* rho_dev, double* u_dev, double* s_dev);

/* Current pre-collision state f^t (Q x N doubles, populations not shifted)
 * and g^t (Qs x N doubles, nullable), device pointers, asynchronous. */
lbm_status lbm_get_state(lbm_ctx* ctx, double* f_dev, double* g_dev);

/* Current adjoint state lambda^{t_adj} (cotangent of the pre-collision state;
 * Q x N and Qs x N doubles, g part nullable), device pointers, asynchronous.
 * LBM_ESTATE before the adjoint has been seeded. */
lbm_status lbm_get_adjoint(lbm_ctx* ctx, double* lf_dev, double* lg_dev);

/* Node classes (N bytes) and the pull-streaming source map src[j*N + n] =
 * index of node (x - e_j) mod L (Q x N int64), computed by the same device
 * code the step kernels use.  Device pointers (either nullable), asynchronous. */
lbm_status lbm_export_maps(lbm_ctx* ctx, uint8_t* mask_dev, int64_t* src_dev);

/* One-shot descent (Section 3.3, eq. gradient:update): nsteps iterations,
 * each one fused kernel on the current pre-collision state f^n, adjoint
 * lambda^n (zero at the first call after a reset) and design w:
 *   lambda^{n+1} = (dW/df)^T S^{-1} lambda^n + dJ/df(f^n)   (eq. adjoint:iteration)
 *   g            = (dW/dw)^T S^{-1} lambda^n                (eq. adjoint:derivative)
 *   f^{n+1}      = S W(f^n, w)                              (eq. normal:iteration)
 *   w           <- clip(w + zeta*(g + penalty*(1 - 2w)), 0, 1) at interior nodes,
 * where 1 - 2w is the derivative of the penalty P = sum w(1-w) (eq. P); a
 * negative zeta*penalty drives w toward 0 and 1.  The design is updated in
 * the workspace (read it with lbm_get_design); lbm_gradient returns the last
 * g.  Unrecorded: the primal uses the ping-pong buffers (with inplace = 1 the
 * primal and adjoint buffers are streamed in place).  Errors: LBM_ESTATE
 * (no design, or an unsteady adjoint in progress), LBM_EINVAL. */
lbm_status lbm_oneshot_steps(lbm_ctx* ctx, int64_t nsteps, double zeta, double penalty);

/* Copies the context's current design field (N values, context precision)
 * to w_dev (device); the one-shot iteration changes it.  Asynchronous. */
lbm_status lbm_get_design(lbm_ctx* ctx, void* w_dev);

/* Times: t (primal), recorded length, adjoint time (-1 before seeding). */
lbm_status lbm_times(const lbm_ctx* ctx, int64_t* t, int64_t* recorded, int64_t* t_adj);

/* Checkpoint plan: interval C, checkpoint slots, ring slots, state bytes. */
lbm_status lbm_plan(const lbm_ctx* ctx, int64_t* interval, int64_t* n_checkpoints,
                    int64_t* n_ring, uint64_t* state_bytes);

/* Batched forms for many contexts with the same (flow, scalar, precision):
 * one kernel launch per step covers every context in ctxs (a descriptor
 * table in each context's workspace maps blocks to contexts).  A batch is
 * all ping-pong or all in place (inplace = 1); in place, members whose
 * phase differs go in a second launch of the same step, checkpoint copies
 * and recomputed segments run per member.  Every context must be in a state
 * where the single-context call would be valid; the call validates all
 * first and runs none on error.  All contexts must share one stream (that
 * of ctxs[0]).  Results are bitwise identical to the single-context calls.
 * Errors: LBM_EINVAL (n outside 1..32, a context twice, different lattices,
 * precisions or streams, in-place and ping-pong contexts mixed, a
 * time-averaged objective), LBM_ESTATE as the single-context calls. */
lbm_status lbm_primal_steps_batch(lbm_ctx* const* ctxs, int32_t n, int64_t nsteps, int32_t record);
lbm_status lbm_adjoint_steps_batch(lbm_ctx* const* ctxs, int32_t n, int64_t nsteps);

/* Last error message of a context ("" if none); static text for NULL. */
const char* lbm_last_error(const lbm_ctx* ctx);
const char* lbm_status_string(lbm_status status);

#ifdef __cplusplus
}
#endif

#endif /* LBM_ADJ_H */
