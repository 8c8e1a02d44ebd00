/*
 * dg.h -- C ABI of the MI355X tensor-product nodal DG Vlasov-Poisson library.
 *
 * The library advances a phase-space distribution f on a rectilinear grid of
 * Legendre-Gauss-Lobatto (LGL) nodal elements with the weak-form DG
 * semi-discretisation of the (magnetised) Vlasov equation and a Fourier
 * spectral Poisson solve, inside Shu-Osher SSP-RK3 stages.
 *
 *   Problem (Sec. 4, eq. vlasov / eq. poisson): d_t f + F^j d_j f = 0 with
 *     1D2V, axes (x, u, v):  F = [u, -E - v B, u B]
 *     1D1V, axes (x, v):     F = [v, -E]
 *   and d_xx Phi = int f dv - 1, E = -d_x Phi.  B is omega_c / omega_p.
 *   Semi-discrete RHS (eq. weak, eq. decoupled, eq. numerical_flux): per
 *     element and per axis, J (Upsilon F + Xi_0 F*_L - Xi_1 F*_R) with upwind
 *     face fluxes F* (Sec. 3.1.1, App. A), J = 2 / element width.
 *   Poisson (Sec. 5.3, eq. spectral_transform, eq. electric_sol): Fourier
 *     coefficients c_p = T_p^{mj} (n_mj - 1) of the charge density through the
 *     LGL->Fourier connection tensor, E_mj = sum_{0<|p|<=pmax} -(i k_p)^-1 c_p
 *     e^{i k_p x_mj}.
 *   Time stepping (Sec. 6): SSP-RK3 of Shu and Osher, E recomputed from the
 *     argument of every stage.
 *
 * Conventions shared by every call:
 *   - State layout (Sec. 3.1): dense row-major [Nx, n, Nu, n, Nv, n] for 1D2V
 *     and [Nx, n, Nv, n] for 1D1V: element index then node index per axis.
 *     Element m of an axis spans [lo + m dx, lo + (m+1) dx]; node j sits at
 *     lo + (m + 1/2) dx + xi_j dx / 2 with xi_j the ascending LGL nodes.
 *   - Every array pointer passed to a compute call is a DEVICE pointer owned
 *     by the caller.  The library never allocates device memory: all scratch
 *     lives in the caller-provided workspace of dg_workspace_bytes() bytes.
 *   - Calls enqueue work on the context's stream and return without waiting,
 *     except dg_diagnostics and dg_rk_step with a non-NULL host_diag, which
 *     wait for completion.  Asynchronous device faults surface as
 *     DG_ERR_DEVICE at the next waiting call.
 *   - State storage is FP32 or FP64 (dg_config.storage); density, Fourier
 *     coefficients, E and all diagnostics are FP64.
 *   - Errors are reported by return code; dg_last_error() gives a message.
 *     The library never aborts the process.  One context per stream; a
 *     context is not thread safe.
 */
#ifndef DG_H
#define DG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_ctx dg_ctx;

typedef enum {
  DG_OK = 0,
  DG_ERR_INVALID = 1,     /* bad argument or configuration                     */
  DG_ERR_UNSUPPORTED = 2, /* valid in principle, not built (e.g. n outside 2..9) */
  DG_ERR_OOM = 3,         /* workspace smaller than dg_workspace_bytes()        */
  DG_ERR_DEVICE = 4,      /* HIP runtime error                                  */
  DG_ERR_CFL = 5,         /* dt above dg_dt_max()                               */
  DG_ERR_NONFINITE = 6    /* a logged step produced NaN/Inf                     */
} dg_status;

typedef enum { DG_F32 = 0, DG_F64 = 1 } dg_dtype;

/* Velocity-axis boundary: periodic wrap (App. A rolls every axis) or zero
 * inflow (the value beyond a velocity edge is 0).  x is always periodic.    */
typedef enum { DG_VBC_PERIODIC = 0, DG_VBC_ZERO_INFLOW = 1 } dg_vbc;

typedef struct {
  int32_t nv;        /* velocity dimensions: 1 (1D1V) or 2 (1D2V)               */
  int32_t n;         /* LGL nodes per element per axis, 2..9                     */
  int32_t nelem[3];  /* elements along x, u (v for 1D1V), v; nelem[2] unused if nv==1 */
  double lo[3];      /* axis lower bounds                                         */
  double hi[3];      /* axis upper bounds (x period L = hi[0] - lo[0])            */
  double omega_c;    /* B = omega_c/omega_p along z; must be 0 when nv == 1       */
  int32_t pmax;      /* Fourier modes kept, 0..2048; 0 selects nelem[0] (Sec. 5.3.1) */
  int32_t storage;   /* dg_dtype of f                                             */
  int32_t vbc;       /* dg_vbc                                                    */
  int32_t reserved;  /* must be 0                                                 */
} dg_config;

/* One diagnostics record (FP64).  mass = int f, field_energy = 1/2 int E^2 dx
 * by nodal LGL quadrature, kinetic_energy = 1/2 int |v|^2 f, l2sq = int f^2,
 * max_abs_E over the x nodes, finite = 1 if every reduced value is finite.   */
typedef struct {
  double t, mass, field_energy, kinetic_energy, l2sq, max_abs_E;
  int32_t finite, step;
} dg_diag;

/* Bytes of device workspace the caller must provide to dg_init for cfg
 * (0 if cfg is invalid).  Host-only; no device is touched.                  */
size_t dg_workspace_bytes(const dg_config* cfg);

/* Validate cfg, build the LGL operators (eq. num_flux_wow) and the
 * connection tensor (eq. spectral_transform) in FP64 on the host, upload them
 * into the workspace, and return a context bound to hip_stream (a
 * hipStream_t; NULL = the legacy default stream).  The workspace must stay
 * valid and untouched by the caller until dg_destroy.  *out is owned by the
 * library and released by dg_destroy.                                       */
dg_status dg_init(const dg_config* cfg, void* workspace, size_t workspace_bytes,
                  void* hip_stream, dg_ctx** out);

/* Release the context (waits for its outstanding work).  NULL is a no-op.   */
dg_status dg_destroy(dg_ctx* ctx);

/* rhs <- L(f): the weak-form semi-discrete right-hand side (eq. weak) for the
 * field E (Nx*n doubles at the x nodes, device).  E == NULL solves Poisson
 * from f first (as dg_poisson).  f and rhs have the state layout and dtype;
 * they must not overlap.                                                    */
dg_status dg_rhs(dg_ctx* ctx, const void* f, const double* E, void* rhs);

/* E <- field of f (Nx*n doubles, device).  If coeffs != NULL it receives the
 * Fourier coefficients c_p, p = 1..pmax, as 2*pmax doubles (re, im) of the
 * source n - 1 (eq. spectral_transform, eq. electric_sol).                  */
dg_status dg_poisson(dg_ctx* ctx, const void* f, double* E, double* coeffs);

/* Advance f in place by nsteps SSP-RK3 steps of size dt (Sec. 6), solving
 * Poisson at every stage.  Returns DG_ERR_CFL if dt > dg_dt_max(ctx, m) where
 * m is max|E| of the initial state.  If host_diag != NULL it receives nsteps
 * records (state after each step) and the call waits; DG_ERR_NONFINITE is
 * returned if any record is non-finite.  The context's time t advances by
 * nsteps*dt.  Steps are replayed from a captured HIP graph.                 */
dg_status dg_rk_step(dg_ctx* ctx, void* f, double dt, int32_t nsteps, dg_diag* host_diag);

/* Profiling form of dg_rk_step: the same nsteps steps, launched eagerly
 * (no graph) with a HIP event pair around every kernel group on the
 * library stream; waits.  host_ms receives 6*nsteps durations in ms, per
 * step [stage 1, field 1, stage 2, field 2, stage 3, field 3] where "stage k"
 * is the fused stage kernel and "field k" the density-reduce + Poisson
 * kernels that follow it.  Same CFL and finiteness checks as dg_rk_step.   */
dg_status dg_profile_step(dg_ctx* ctx, void* f, double dt, int32_t nsteps, double* host_ms);

/* Full diagnostics of state f (its own Poisson solve) into *host_out; waits. */
dg_status dg_diagnostics(dg_ctx* ctx, const void* f, dg_diag* host_out);

/* Largest stable SSP-RK3 step for a field bounded by max_abs_E:
 * C_n / sum_axes(max|speed_a| / dx_a), C_n the RK3 + upwind-DG stability
 * limit from the Bloch eigenvalues of the 1-D operator.  Host-only.         */
double dg_dt_max(const dg_ctx* ctx, double max_abs_E);

/* Node coordinates of one axis (0 = x, 1 = u or v, 2 = v): nelem*n doubles
 * into host memory, in state order.  Host-only.                             */
dg_status dg_node_coords(const dg_ctx* ctx, int32_t axis, double* host_out);

/* Message of the last error on ctx (or of the last failed dg_init when ctx
 * is NULL).  Never NULL.                                                    */
const char* dg_last_error(const dg_ctx* ctx);

/* ---------- batched runs (many independent, uneven runs in one launch) ---- */

typedef struct dg_batch dg_batch;

/* Bytes of device workspace for a batch of nruns configurations (FP32 storage,
 * any nv / n / sizes).  0 if any configuration is invalid or not FP32.      */
size_t dg_batch_workspace_bytes(const dg_config* cfgs, int32_t nruns);

/* Set up every run (as dg_init does) inside one workspace, build the (run,
 * tile) work list ordered by decreasing tile cost and split over the 8 XCDs,
 * and bind the batch to hip_stream.  cfgs is copied.                        */
dg_status dg_batch_init(const dg_config* cfgs, int32_t nruns, void* workspace, size_t workspace_bytes,
                        void* hip_stream, dg_batch** out);
dg_status dg_batch_destroy(dg_batch* b);

/* Advance every run r by nsteps SSP-RK3 steps of its own dt[r] (host array)
 * on its state f[r] (host array of device pointers), all runs' stages in ONE
 * persistent launch per RK stage followed by one batched field launch pair,
 * replayed from a captured HIP graph.  CFL and finiteness checks per run as
 * dg_rk_step.  host_diag: NULL or nruns*nsteps records, run-major
 * (record s of run r at host_diag[r*nsteps + s]); then the call waits.      */
dg_status dg_batch_rk_step(dg_batch* b, void* const* f, const double* dt, int32_t nsteps, dg_diag* host_diag);

/* Autotuner: time `reps` batched steps for each candidate persistent grid
 * (work-groups per CU from 1 to the occupancy limit) and work-list order,
 * keep the fastest for this batch, and return its mean step time in ms.
 * The states are advanced by the timed steps.                               */
dg_status dg_batch_tune(dg_batch* b, void* const* f, const double* dt, int32_t reps, double* best_ms);

/* Current persistent grid (work-groups) of the batched stage kernel.        */
int32_t dg_batch_grid(const dg_batch* b);

const char* dg_batch_last_error(const dg_batch* b);

/* ---------- host-only introspection of the FP64 setup (no device) -------- */

/* Reference-element operators for n nodes (eq. quad_weights, eq. minv,
 * eq. num_flux_wow): xi[n], w[n], ups[n*n] (row = output node), xi_face[n*2]
 * (columns: left, right face), dmat[n*n].  Any output may be NULL.          */
dg_status dg_basis(int32_t n, double* xi, double* w, double* ups, double* xi_face, double* dmat);

/* Connection tensor T_p^{mj} of eq. spectral_transform for an axis of nelem
 * equal elements on [lo, hi], p = 1..pmax: 2*pmax*nelem*n doubles, (re, im)
 * innermost, then j, then m, then p.                                         */
dg_status dg_connection_tensor(int32_t n, int32_t nelem, double lo, double hi, int32_t pmax, double* out);

/* RK3 + upwind-DG Courant number C_n (dt <= C_n dx / |a|).                  */
double dg_courant_number(int32_t n);

#ifdef __cplusplus
}
#endif
#endif /* DG_H */
