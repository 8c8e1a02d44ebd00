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
 *     and [Nx, n, Nv, n] for 1D1V: element index then node index per axis
 *     (1D2V may pad the v rows instead: DG_LAYOUT_VPAD below).
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
  DG_ERR_UNSUPPORTED = 2, /* valid in principle, not built (e.g. n outside 2..12) */
  DG_ERR_OOM = 3,         /* workspace smaller than dg_workspace_bytes()        */
  DG_ERR_DEVICE = 4,      /* HIP runtime error                                  */
  DG_ERR_CFL = 5,         /* dt above dg_dt_max()                               */
  DG_ERR_NONFINITE = 6    /* a logged step produced NaN/Inf                     */
} dg_status;

typedef enum { DG_F32 = 0, DG_F64 = 1 } dg_dtype;

/* Velocity-axis boundary: periodic wrap (App. A rolls every axis) or zero
 * inflow (the value beyond a velocity edge is 0).  x is always periodic.    */
typedef enum { DG_VBC_PERIODIC = 0, DG_VBC_ZERO_INFLOW = 1 } dg_vbc;

/* State layouts (dg_config.layout).
 *   DG_LAYOUT_DENSE: the dense row-major arrays described above.
 *   DG_LAYOUT_VPAD (1D2V only): the same order of rows, but each row of
 *     Nv*n v values (one x node, one u node) is stored as C = ceil(Nv / TV)
 *     chunks of 64 values, TV = floor(64 / n): chunk c holds the values of v
 *     elements [c TV, min(c TV + TV, Nv)) followed by unused slots, so every
 *     chunk starts on a 64-value boundary (256 bytes in FP32) and each
 *     64-lane load or store of the stage kernel covers whole aligned memory
 *     lines.  A row holds 64 C values and a state dg_state_elems() values.
 *     Unused slots never influence a result; dg_state_pack fills them with
 *     zeros and every call that writes a state writes zeros there (whole
 *     memory lines are cheaper to write than partial ones).  For n = 2, 4, 8
 *     and Nv a multiple of TV the two layouts coincide.
 * The learned-correction and projection calls accept only DG_LAYOUT_DENSE. */
typedef enum { DG_LAYOUT_DENSE = 0, DG_LAYOUT_VPAD = 1 } dg_layout;

typedef struct {
  int32_t nv;        /* velocity dimensions: 1 (1D1V) or 2 (1D2V)               */
  int32_t n;         /* LGL nodes per element per axis, 2..12                    */
  int32_t nelem[3];  /* elements along x, u (v for 1D1V), v; nelem[2] unused if nv==1 */
  double lo[3];      /* axis lower bounds                                         */
  double hi[3];      /* axis upper bounds (x period L = hi[0] - lo[0])            */
  double omega_c;    /* B = omega_c/omega_p along z; must be 0 when nv == 1       */
  int32_t pmax;      /* Fourier modes kept, 0..2048; 0 selects nelem[0] (Sec. 5.3.1) */
  int32_t storage;   /* dg_dtype of f                                             */
  int32_t vbc;       /* dg_vbc                                                    */
  int32_t layout;    /* dg_layout of every state array of the context            */
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

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: dg_rhs with
 * no context and no workspace.  rhs <- L(f) for the configuration cfg
 * (copied; checked as by dg_init), with the field E (Nx*n doubles, device) or,
 * if E == NULL, the field solved from f.  The call enqueues on hip_stream
 * (a hipStream_t; NULL = the legacy default stream) and returns without
 * waiting; it calls no hipMalloc / hipFree and copies nothing from the host.
 * Scratch (node tables and connection tensor, rebuilt by a device kernel on
 * every call, density and Fourier partials, E) lives in a library-owned
 * array of DG_RHS_STATIC_SCRATCH_BYTES bytes per GPU, held until the process
 * ends: configurations needing more are rejected with DG_ERR_OOM.  Every
 * call on a GPU uses that GPU's one array, so calls that overlap on one GPU
 * (concurrent streams or threads) race; calls on one stream are ordered.
 * Errors are read with dg_last_error(NULL).  Results equal dg_rhs's up to
 * the rounding of the device-built tables.                                 */
#define DG_RHS_STATIC_SCRATCH_BYTES ((size_t)8 << 20)
dg_status dg_rhs_static(const dg_config* cfg, const void* f, const double* E, void* rhs, void* hip_stream);

/* E <- field of f (Nx*n doubles, device).  If coeffs != NULL it receives the
 * Fourier coefficients c_p, p = 1..pmax, as 2*pmax doubles (re, im) of the
 * source n - 1 (eq. spectral_transform, eq. electric_sol).                  */
dg_status dg_poisson(dg_ctx* ctx, const void* f, double* E, double* coeffs);

/* Advance f in place by nsteps SSP-RK3 steps of size dt (Sec. 6), solving
 * Poisson at every stage.  Returns DG_ERR_CFL if dt > dg_dt_max(ctx, m) where
 * m is max|E| of the initial state.  If host_diag != NULL it receives nsteps
 * records (state after each step) and the call waits; DG_ERR_NONFINITE is
 * returned if any record is non-finite.  The context's time t advances by
 * nsteps*dt.  Pairs of steps are replayed from a captured HIP graph (an odd
 * last step is launched directly).                                         */
dg_status dg_rk_step(dg_ctx* ctx, void* f, double dt, int32_t nsteps, dg_diag* host_diag);

/* Profiling form of dg_rk_step: the same nsteps steps, launched eagerly
 * (no graph) with a HIP event pair around every kernel group on the
 * library stream; waits.  host_ms receives 6*nsteps durations in ms, per
 * step [stage 1, field 1, stage 2, field 2, stage 3, field 3] where "stage k"
 * is the fused stage kernel and "field k" the density-reduce + Poisson
 * kernels that follow it.  Same CFL and finiteness checks as dg_rk_step.   */
dg_status dg_profile_step(dg_ctx* ctx, void* f, double dt, int32_t nsteps, double* host_ms);

/* ---------- spectral tools on the x grid (Sec. 5.3) ---------------------- */

/* Fourier coefficients of arbitrary nodal data on the x grid through the
 * connection tensor (eq. spectral_transform): coeffs (device, 2*pmax
 * doubles, re/im) <- c_p = sum_mj T_p^{mj} g_mj for p = 1..pmax, g (device,
 * Nx*n doubles).  pmax is the context's (dg_config.pmax), which may exceed
 * Nx: the paper finds the transform accurate past the DFT Nyquist limit
 * (Sec. 5.3.1, errors figure).                                              */
dg_status dg_fourier(dg_ctx* ctx, const double* g, double* coeffs);

/* Global spectral filter along x (Sec. 5.3: a global filter for
 * anti-aliasing): every (u, v) node's x profile of f_in is replaced by its
 * truncated Fourier series c_0 + sum_{p=1..pmax} 2 Re(sigma_p c_p e^{i k_p x})
 * evaluated at the x nodes, c_p from the connection tensor; sigma (host,
 * pmax doubles) weights the modes (all ones: the projection onto the first
 * pmax modes; e.g. exp(-a (p / pmax)^s): an exponential filter).  f_in and
 * f_out are states of the context's layout and dtype, not overlapping.
 * The (Nx n) x (Nx n) filter matrix is built on the host in FP64 and applied
 * on the device in the storage precision; Nx n <= 4096 (DG_ERR_UNSUPPORTED
 * beyond).  Waits.                                                          */
dg_status dg_filter_x(dg_ctx* ctx, const double* sigma, const void* f_in, void* f_out);

/* delta-f storage (Sec. 2: the weak form is linear in f for a given field, so
 * L(f0 + g) = L(f0) + L(g)).  f0_host: an x-uniform background f0(u, v) as
 * host FP64 nodal values, dense [Nu*n][Nv*n] (1D2V) or [Nv*n] (1D1V), which
 * must be continuous across every velocity element face including the
 * periodic wrap (relative jump <= 1e-10; then its upwind face values do not
 * depend on the direction and L(f0) = -E(x) G_u(u, v) + G_b(u, v) exactly,
 * with G_u its weak u derivative and G_b its gyration -vB G_u + uB G_v, both
 * built once in FP64 on the host).  Afterwards every state the context is
 * given holds g = f - f0: dg_rhs returns L(f0 + g), dg_rk_step advances g,
 * dg_poisson and the diagnostics (mass, energies, L2 norm) are those of
 * f0 + g.  With FP32 storage this keeps the rounding of f0 out of every
 * stage.  NULL returns to whole-f states.  Needs periodic velocity
 * boundaries (DG_ERR_UNSUPPORTED otherwise); invalidates the cached step
 * graph; waits.  The learned-correction calls reject contexts with a
 * background.                                                               */
dg_status dg_set_background(dg_ctx* ctx, const double* f0_host);

/* Bandwidth references for the stage kernel (measurement only): `reps`
 * launches of a copy of state `in` into state `out` (context layout and
 * dtype, not overlapping) timed with HIP events on the context stream after
 * one warm-up launch; *host_ms receives the mean per launch; waits.
 * pattern 0: a plain streaming copy (16-byte accesses; the state's size
 * rounded down to 16 bytes); pattern 1 (1D2V): the stage kernel's own access
 * pattern -- its tiles, their order and store policy -- with no halos and no
 * arithmetic.  Each moves 2 * dg_state_elems() * sizeof(storage) bytes.
 * pattern 2: an empty kernel (in and out untouched): the time of one launch
 * that waits for the one before it on the stream, the floor under each of
 * the step's kernels.  pattern 3 (1D2V): pattern 1 with no more work-groups
 * resident per CU than the stage-1 kernel of this shape (unused LDS per
 * work-group); DG_ERR_DEVICE where that would take more than 64 KiB of LDS. */
dg_status dg_profile_copy(dg_ctx* ctx, const void* in, void* out, int32_t pattern, int32_t reps, double* host_ms);

/* Full diagnostics of state f (its own Poisson solve) into *host_out; waits.
 * The quantities are those the paper tracks over its runs (Sec. 6, energy
 * figure): mass, the domain-integrated field energy (the paper leaves its
 * definition open; taken as 1/2 int E^2 dx by nodal LGL quadrature), kinetic
 * energy and the L2 norm of f, with max |E|.                                */
dg_status dg_diagnostics(dg_ctx* ctx, const void* f, dg_diag* host_out);

/* Largest stable SSP-RK3 step for a field bounded by max_abs_E:
 * C_n / sum_axes(max|speed_a| / dx_a), C_n the RK3 + upwind-DG stability
 * limit from the Bloch eigenvalues of the 1-D operator (the paper defers its
 * CFL numbers to the DG literature, Sec. 6; this is the exact limit of the
 * scheme as implemented).  Host-only.                                       */
double dg_dt_max(const dg_ctx* ctx, double max_abs_E);

/* Node coordinates of one axis (0 = x, 1 = u or v, 2 = v): nelem*n doubles
 * into host memory, in state order.  Host-only.                             */
dg_status dg_node_coords(const dg_ctx* ctx, int32_t axis, double* host_out);

/* Message of the last error on ctx (or of the last failed dg_init when ctx
 * is NULL).  Never NULL.                                                    */
const char* dg_last_error(const dg_ctx* ctx);

/* Values (of the storage dtype) in one state array of ctx's layout: the DOF
 * count for DG_LAYOUT_DENSE, Nx n Nu n 64 C for DG_LAYOUT_VPAD.  Host-only.  */
size_t dg_state_elems(const dg_ctx* ctx);

/* Layout conversion on the context's stream (device arrays of the storage
 * dtype, not overlapping): dg_state_pack writes the dense array `dense` (DOF
 * values) into `state` (dg_state_elems() values, zeros in unused slots);
 * dg_state_unpack is its inverse.  For DG_LAYOUT_DENSE both are copies.    */
dg_status dg_state_pack(dg_ctx* ctx, const void* dense, void* state);
dg_status dg_state_unpack(dg_ctx* ctx, const void* state, void* dense);

/* ---------- batched runs (many independent, uneven runs in one launch) ---- */

typedef struct dg_batch dg_batch;

/* Bytes of device workspace for a batch of nruns configurations (FP32 storage,
 * any nv / n / sizes).  0 if any configuration is invalid or not FP32.      */
size_t dg_batch_workspace_bytes(const dg_config* cfgs, int32_t nruns);

/* Set up every run (as dg_init does) inside one workspace, group the runs by
 * kind (the 1D2V runs by n; all 1D1V runs, any n, form one kind, reported
 * as (n, nv) = (0, 1)), build each kind's (run, tile) work list ordered by
 * decreasing tile cost and split over the 8 XCDs, and bind the batch to
 * hip_stream.  cfgs is copied.                                              */
dg_status dg_batch_init(const dg_config* cfgs, int32_t nruns, void* workspace, size_t workspace_bytes,
                        void* hip_stream, dg_batch** out);
dg_status dg_batch_destroy(dg_batch* b);

/* Advance every run r by nsteps SSP-RK3 steps of its own dt[r] (host array)
 * on its state f[r] (host array of device pointers): per RK stage one
 * launch per kind present (persistent or one work-group per tile, as chosen
 * by dg_batch_tune or dg_batch_set_choice), covering all runs of that kind,
 * then one batched field launch pair for all runs, replayed from a captured
 * HIP graph.  CFL and finiteness checks per run as
 * dg_rk_step.  host_diag: NULL or nruns*nsteps records, run-major
 * (record s of run r at host_diag[r*nsteps + s]); then the call waits.      */
dg_status dg_batch_rk_step(dg_batch* b, void* const* f, const double* dt, int32_t nsteps, dg_diag* host_diag);

/* Autotuner: time `reps` batched steps per candidate and keep the fastest
 * for this batch: first the work-list order (cost-sorted or run-interleaved),
 * then, per kind (n, nv), its launch shape (a persistent grid of 1 to the
 * kind's occupancy limit work-groups per CU, or one work-group per tile),
 * one kind at a time, largest first, then the other list order once more.
 * The
 * per-kind grids are kept per (GPU arch, n, nv, FP32) for the life of the
 * process and start later batches.  Returns the
 * mean step time in ms of the choice; the states are advanced by the timed
 * steps.                                                                    */
dg_status dg_batch_tune(dg_batch* b, void* const* f, const double* dt, int32_t reps, double* best_ms);

/* Current persistent grid: work-groups of all kinds' stage launches summed.  */
int32_t dg_batch_grid(const dg_batch* b);

/* The current choices: returns the number of kinds K; if host_out != NULL it
 * receives 2 + 4 K ints: [concurrent kind launches (always 0: the form is
 * switched off), order (0 cost-sorted, 1 run-interleaved), then per kind n,
 * nv, work-groups per CU (0: one work-group per tile), grid].              */
int32_t dg_batch_choice(const dg_batch* b, int32_t* host_out);
/* Apply choices in the layout dg_batch_choice returns (nint = 2 + 4 K; the
 * kinds must be this batch's, in its order; the grid entries are ignored and
 * recomputed), e.g. a tuning saved from another process.  Concurrent kind
 * launches (first entry 1) return DG_ERR_UNSUPPORTED.  Waits.             */
dg_status dg_batch_set_choice(dg_batch* b, const int32_t* choice, int32_t nint);

const char* dg_batch_last_error(const dg_batch* b);

/* ---------- learned coarse-grid correction ----------------------------------
 * A per-element multilayer perceptron corrects the RHS of a coarse 1D2V grid.
 * Two input forms, told apart by the network's input width:
 *   7 n^3 + n  whole values: the element's n^3 nodal values, the six face
 *              neighbours' n^3 blocks (periodic) and E at its n x nodes; the
 *              correction is made mass-neutral per element;
 *   8 n^3 + n  fluctuations: the same blocks minus the x average of the
 *              state (per (u, v) node, LGL-weighted), E, then the element's
 *              own block of that x average; the correction's x average is
 *              removed (so the x-averaged distribution and the mass are not
 *              changed by it).
 * Features are normalised per column; the output is an n^3 RHS correction.
 * Layers are Linear with exact GELU after all but the last; matrix products
 * run on BF16 MFMA with FP32 accumulation, parameters are FP32 masters with
 * BF16 copies, training uses MSE and AdamW.  Fine-grid DG runs generate the
 * training data: f and RHS are L2-projected to the coarse grid and the target
 * is P RHS_fine(f) - RHS_coarse(P f) (minus its x average for fluctuations). */

typedef struct dg_nn dg_nn;

/* sizes[0..nlayers]: input width, hidden widths..., output width.  Buffers
 * for up to max_rows rows.                                                  */
size_t dg_nn_workspace_bytes(const int32_t* sizes, int32_t nlayers, int32_t max_rows);
dg_status dg_nn_init(const int32_t* sizes, int32_t nlayers, int32_t max_rows, void* workspace,
                     size_t workspace_bytes, void* hip_stream, dg_nn** out);
dg_status dg_nn_destroy(dg_nn* nn);
int64_t dg_nn_param_count(const dg_nn* nn);
/* Padded row stride (BF16 elements, multiple of 16) of the input rows X.   */
int32_t dg_nn_input_ld(const dg_nn* nn);
/* Host parameter vector: W_0 (in x out, row-major), b_0, W_1, b_1, ...     */
dg_status dg_nn_set_params(dg_nn* nn, const float* host_params);
dg_status dg_nn_get_params(dg_nn* nn, float* host_params);
/* Y (device, rows x out FP32) = network(X) for X (device, rows x input_ld
 * BF16); rows <= max_rows.  Networks of at most 8 layers with input width
 * <= 1024 and every layer width <= 128 run as one fused launch (every
 * layer's MFMA GEMM, bias and GELU per 16-row block, activations kept on
 * chip); others one GEMM launch per layer.  The corrected steps use the
 * same form.                                                               */
dg_status dg_nn_forward(dg_nn* nn, const uint16_t* X, int32_t rows, float* Y);
/* Inference form: on = 1 (default) the fused launch where the shape allows
 * it, 0 one GEMM launch per layer (the form training uses).  Returns
 * DG_ERR_UNSUPPORTED for on = 1 when the shape has no fused form, and then
 * changes nothing.                                                          */
dg_status dg_nn_set_fused(dg_nn* nn, int32_t on);
/* Forward + backward of the MSE loss mean((Y - T)^2) for targets T (device,
 * rows x out FP32); *loss receives the loss (host, waits); host_grads (may be
 * NULL) receives the gradient in the parameter-vector order.               */
dg_status dg_nn_loss_grad(dg_nn* nn, const uint16_t* X, const float* T, int32_t rows, double* loss, float* host_grads);
/* One AdamW step (beta1 0.9, beta2 0.999, eps 1e-8) with the gradients of
 * the last dg_nn_loss_grad; weight decay on weights only.                   */
dg_status dg_nn_adamw(dg_nn* nn, float lr, float weight_decay);

/* One-axis L2 projection matrix (host, FP64, row-major nc x r*nf) from the r
 * fine elements with nf LGL nodes inside one coarse element with nc nodes:
 * exact mass matrix and coupling integrals.  nc*r*nf <= 324.                */
dg_status dg_projection_matrix(int32_t nc, int32_t nf, int32_t r, double* out);
/* L2 projection of a fine state (1D1V or 1D2V; FP32 or FP64 storage as the
 * fine context says) onto a nested coarse grid with the same domain (fine
 * element counts multiples of the coarse ones), axis by axis with
 * dg_projection_matrix, FP64 arithmetic, result in the coarse context's
 * storage precision.
 * Uses the fine context's two stage buffers as scratch (each partial result
 * must fit one of them, else DG_ERR_UNSUPPORTED).  Enqueued on the fine
 * context's stream after both callers' streams; the coarse caller's stream
 * waits for it.                                                             */
dg_status dg_project(dg_ctx* fine, dg_ctx* coarse, const void* f_fine, void* f_coarse);
/* Network input rows of a coarse FP32 state f with field E (device, Nx*n):
 * (value - mean) * inv_std per feature (device arrays of the network's input
 * width), BF16, one row per element, element order (ix, iu, iv); the form
 * (whole / fluctuation) follows the network's input width.  Uses the coarse
 * context's stage buffers as scratch.                                       */
dg_status dg_nn_features(dg_ctx* coarse, const dg_nn* nn, const void* f, const double* E, const float* mean,
                         const float* inv_std, uint16_t* X);
/* Raw (FP32, unnormalised) feature rows, elements x (7 n^3 + n), or
 * elements x (8 n^3 + n) fluctuation features when fluct != 0.             */
dg_status dg_nn_features_raw(dg_ctx* coarse, const void* f, const double* E, int32_t fluct, float* out);
/* Element-major FP32 copy (elements x n^3) of scale * (x - sub) for coarse
 * state-layout arrays x and sub in the coarse context's storage precision
 * (sub may be NULL: scale * x), minus its x average when fluct != 0: the
 * training target (with an FP64 context the difference and the average are
 * taken in FP64).  Uses the coarse context's stage buffers as scratch.      */
dg_status dg_nn_to_elements(dg_ctx* coarse, const void* x, const void* sub, float scale, int32_t fluct, float* out);
/* Per-column sums and sums of squares (host FP64) of a device FP32 matrix.  */
dg_status dg_nn_column_stats(dg_nn* nn, const float* X, int64_t rows, int32_t cols, double* host_sum, double* host_sumsq);
/* nsteps SSP-RK3 steps of the coarse grid with RHS L(u) + out_scale * NN(u)
 * at every stage (whole-value networks: the correction made mass neutral per
 * element under the LGL product weights; fluctuation networks: its x average
 * removed), Poisson from each corrected stage state.  f: coarse FP32 state in
 * place.  host_diag as dg_rk_step.  The step is captured in a HIP graph once
 * per (context, f, dt, statistics, scale, diag) and replayed.              */
dg_status dg_nn_rk_step(dg_ctx* coarse, dg_nn* nn, const float* mean, const float* inv_std, float out_scale,
                        void* f, double dt, int32_t nsteps, dg_diag* host_diag);
const char* dg_nn_last_error(const dg_nn* nn);

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
