// C ABI of the DG Vlasov-Poisson library: configuration checks, workspace
// layout, host setup uploads, stage orchestration and HIP-graph replay of
// SSP-RK3 steps.  Every entry point is declared and documented in dg.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <atomic>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/dg.h"
#include "dg_host.h"
#include "dg_kernels.h"
#include "ctx.h"

using dgi::Layout;

namespace {

constexpr size_t kAlign = 256;
// Last-level (Infinity) cache of the GPU: stage outputs use non-temporal
// stores when a run's three state buffers do not fit in it.
constexpr size_t kLastLevelCache = size_t(256) << 20;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
// dg_filter_x keeps a dense (Nx n) x (Nx n) matrix in the workspace
constexpr size_t kMaxFilterNodes = 4096;

std::mutex g_err_mu;
std::string g_init_error = "no error";

const char* validate(const dg_config* c) {
  if (!c) return "cfg is NULL";
  if (c->nv != 1 && c->nv != 2) return "nv must be 1 or 2";
  if (c->n < 2) return "n must be >= 2";
  for (int a = 0; a <= c->nv; ++a) {
    if (c->nelem[a] < 1) return "nelem must be >= 1 on every axis";
    if (!(c->hi[a] > c->lo[a]) || !std::isfinite(c->lo[a]) || !std::isfinite(c->hi[a])) return "need lo < hi (finite) on every axis";
  }
  if (c->nv == 1 && c->omega_c != 0.0) return "omega_c must be 0 for 1D1V";
  if (!std::isfinite(c->omega_c)) return "omega_c must be finite";
  if (c->pmax < 0 || c->pmax > 2048) return "pmax must be in 0..2048";
  if (c->storage != DG_F32 && c->storage != DG_F64) return "storage must be DG_F32 or DG_F64";
  if (c->vbc != DG_VBC_PERIODIC && c->vbc != DG_VBC_ZERO_INFLOW) return "vbc must be DG_VBC_PERIODIC or DG_VBC_ZERO_INFLOW";
  if (c->layout != DG_LAYOUT_DENSE && c->layout != DG_LAYOUT_VPAD) return "layout must be DG_LAYOUT_DENSE or DG_LAYOUT_VPAD";
  if (c->layout == DG_LAYOUT_VPAD && c->nv != 2) return "DG_LAYOUT_VPAD needs nv == 2";
  return nullptr;
}

// Workspace layout.  Without stage buffers (the allocation-free entry point)
// B and C are not reserved and the diagnostics ring holds one record.
Layout make_layout(const dg_config* c, bool stage_buffers = true) {
  Layout L;
  L.n = c->n;
  L.naxes = 1 + c->nv;
  L.esize = c->storage == DG_F64 ? 8 : 4;
  L.Nx = c->nelem[0];
  L.Nu = c->nv == 2 ? c->nelem[1] : 1;
  L.Nv = c->nv == 2 ? c->nelem[2] : c->nelem[1];
  L.pmax = c->pmax > 0 ? c->pmax : c->nelem[0];
  L.dof = static_cast<size_t>(L.Nx) * L.n * L.Nv * L.n * (c->nv == 2 ? static_cast<size_t>(L.Nu) * L.n : 1);
  const int tv = dgk::tv_of(L.n);
  L.nvchunks = (L.Nv + tv - 1) / tv;
  L.ntiles_slab = L.Nu * L.nvchunks;
  L.ntiles = L.Nx * L.ntiles_slab;
  const bool vpad = c->layout == DG_LAYOUT_VPAD;
  L.cpitch = vpad ? dgk::kWave : tv * L.n;
  L.lpitch = vpad ? L.nvchunks * dgk::kWave : L.Nv * L.n;
  L.selems = vpad ? static_cast<size_t>(L.Nx) * L.n * L.Nu * L.n * L.lpitch : L.dof;
  const size_t nx = static_cast<size_t>(L.Nx) * L.n;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += align_up(bytes); return r; };
  L.off_B = take(stage_buffers ? L.selems * L.esize : 0);
  L.off_C = take(stage_buffers ? L.selems * L.esize : 0);
  L.off_part = take(nx * L.ntiles_slab * 8);
  L.off_mom = take(static_cast<size_t>(L.ntiles) * 4 * 8);
  L.off_dens = take(nx * 8);
  L.off_E = take(nx * 8);
  L.off_cpart = take(static_cast<size_t>(L.Nx) * L.pmax * 16);
  L.off_mpart = take(static_cast<size_t>(L.Nx) * 8);
  L.off_coef = take(static_cast<size_t>(L.pmax) * 16);
  L.off_ring = take(static_cast<size_t>(stage_buffers ? dgk::kRing : 1) * 64);
  L.off_last = take(64);
  L.off_ctr = take(sizeof(int));
  L.off_T = take(static_cast<size_t>(L.pmax) * nx * 16);
  L.off_z1 = take(nx * 16);
  L.off_wx = take(nx * 8);
  L.off_wu = take(static_cast<size_t>(L.Nu) * L.n * 8);
  L.off_wv = take(static_cast<size_t>(L.Nv) * L.n * 8);
  L.off_uc = take(static_cast<size_t>(L.Nu) * L.n * L.esize);
  L.off_vc = take(static_cast<size_t>(L.Nv) * L.n * L.esize);
  L.off_uc64 = take(static_cast<size_t>(L.Nu) * L.n * 8);
  L.off_vc64 = take(static_cast<size_t>(L.Nv) * L.n * 8);
  // background tables (dg_set_background): G_u and G_b in the state-row
  // layout (1D2V) or G_v (1D1V) in the storage precision, f0 in FP64
  const size_t vrows = c->nv == 2 ? static_cast<size_t>(L.Nu) * L.n : 1;
  L.off_bgu = take(stage_buffers ? vrows * L.lpitch * L.esize : 0);
  L.off_bgb = take(stage_buffers && c->nv == 2 ? vrows * L.lpitch * L.esize : 0);
  L.off_bg64 = take(stage_buffers ? vrows * L.Nv * L.n * 8 : 0);
  // x-filter matrix (dg_filter_x), for up to kMaxFilterNodes x nodes
  L.off_M = take(stage_buffers && nx <= kMaxFilterNodes ? nx * nx * L.esize : 0);
  L.total = o;
  return L;
}

const char* check_cfg(const dg_config* cfg, dg_status* st);

}  // namespace


namespace dgi {

dg_status fail(dg_ctx* c, dg_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

dg_status hip_fail(dg_ctx* c, hipError_t e, const char* what) {
  return fail(c, DG_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define DG_HIP(ctx, expr)                                   \
  do {                                                      \
    hipError_t e__ = (expr);                                \
    if (e__ != hipSuccess) return hip_fail(ctx, e__, #expr); \
  } while (0)

// Node coordinates / quadrature weights of an axis.
std::vector<double> axis_nodes(const dgh::Basis& b, int N, double lo, double hi) {
  std::vector<double> x(static_cast<size_t>(N) * b.n);
  const double dx = (hi - lo) / N;
  for (int m = 0; m < N; ++m)
    for (int j = 0; j < b.n; ++j) x[m * b.n + j] = lo + (m + 0.5) * dx + b.xi[j] * 0.5 * dx;
  return x;
}
std::vector<double> axis_weights(const dgh::Basis& b, int N, double lo, double hi) {
  std::vector<double> w(static_cast<size_t>(N) * b.n);
  const double dx = (hi - lo) / N;
  for (int m = 0; m < N; ++m)
    for (int j = 0; j < b.n; ++j) w[m * b.n + j] = b.w[j] * 0.5 * dx;
  return w;
}

// Stage coefficients in the storage precision.  A stage that reads u^n
// computes out = fin + c_un (u^n - fin) + c_dt L(fin), i.e. the convex
// combination c_un u^n + (1 - c_un) fin for the rounded c_un, so no rounded
// pair (c_un, c_in) has to sum to one (FP32 1/3 + 2/3 is 1 + 3e-8, which
// would grow the mass by that much every step).  c_dt is (1 - c_un) dt for
// the rounded c_un; c_in is stored as 1 - c_un.  Without u^n, c_in is 0 (RHS
// only) or 1 and is applied as given.
template <typename T>
void store_coefficients(double c_un, double c_in, double c_dt, T* cu, T* ci, T* cd) {
  *cu = static_cast<T>(c_un);
  if (c_un != 0.0 && c_in > 0.0) {
    const double in_rounded = 1.0 - static_cast<double>(*cu);
    *ci = static_cast<T>(in_rounded);
    *cd = static_cast<T>(c_dt / c_in * in_rounded);
    return;
  }
  *ci = static_cast<T>(c_in);
  *cd = static_cast<T>(c_dt);
}

template <typename T>
void fill_pack(const dg_ctx* c, dgk::StageArgs<T>* p, const void* fin, const void* fun, void* out,
               const double* E, double* partials, double c_un, double c_in, double c_dt) {
  const Layout& L = c->L;
  std::memset(static_cast<void*>(p), 0, sizeof(*p));
  auto& a = *p;
  a.fin = static_cast<const T*>(fin);
  a.fun = static_cast<const T*>(fun ? fun : fin);
  a.out = static_cast<T*>(out);
  a.E = E;
  a.ucoord = c->at<const T>(L.off_uc);
  a.vcoord = c->at<const T>(L.off_vc);
  a.wu = c->at<const double>(L.off_wu);
  a.wv = c->at<const double>(L.off_wv);
  a.wx = c->at<const double>(L.off_wx);
  a.uc64 = c->at<const double>(L.off_uc64);
  a.vc64 = c->at<const double>(L.off_vc64);
  a.partials = partials;
  if (c->bg) {
    a.bg_u = c->at<const T>(L.off_bgu);
    a.bg_b = c->cfg.nv == 2 ? c->at<const T>(L.off_bgb) : nullptr;
    a.bg64 = c->at<const double>(L.off_bg64);
  }
  a.hu = c->cfg.nv == 2 ? 0.5 * c->dx[1] : 1.0;
  a.Nx = L.Nx;
  a.Nu = L.Nu;
  a.Nv = L.Nv;
  a.nvchunks = L.nvchunks;
  a.cpitch = L.cpitch;
  a.lpitch = L.lpitch;
  a.nt_store = 3 * L.selems * L.esize > kLastLevelCache ? 1 : 0;
  a.zero_inflow = c->cfg.vbc == DG_VBC_ZERO_INFLOW ? 1 : 0;
  a.n1v = c->cfg.nv == 1 ? c->cfg.n : 0;
  a.Jx = static_cast<T>(2.0 / c->dx[0]);
  if (c->cfg.nv == 2) {
    a.Ju = static_cast<T>(2.0 / c->dx[1]);
    a.Jv = static_cast<T>(2.0 / c->dx[2]);
  } else {
    a.Ju = T(0);
    a.Jv = static_cast<T>(2.0 / c->dx[1]);
  }
  a.wc = static_cast<T>(c->cfg.omega_c);
  store_coefficients(c_un, c_in, c_dt, &a.c_un, &a.c_in, &a.c_dt);
}

// One fused stage kernel: out = c_un un + c_in fin + c_dt L(fin) (L with field E).
dg_status stage(dg_ctx* c, const void* fin, const void* fun, void* out, const double* E,
                double* partials, double c_un, double c_in, double c_dt, bool reverse, const float* corr,
                const float* corr_xm) {
  hipError_t e;
  if (corr) {
    // the corrected stage of the learned correction: FP32, 1D2V, dense rows, whole f
    if (c->f64() || c->cfg.nv != 2 || c->cfg.layout != DG_LAYOUT_DENSE || c->bg)
      return fail(c, DG_ERR_UNSUPPORTED, "corrected stage needs FP32 1D2V dense whole-f states");
    dgk::StageArgs<float> p;
    fill_pack(c, &p, fin, fun, out, E, partials, c_un, c_in, c_dt);
    p.reverse = reverse ? 1 : 0;
    p.corr = corr;
    p.corr_xm = corr_xm;
    e = dgk::launch_stage(c->cfg.nv, c->L.n, false, &p, c->L.ntiles, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "corrected stage kernel launch");
    return DG_OK;
  }
  if (c->f64()) {
    dgk::StageArgs<double> p;
    fill_pack(c, &p, fin, fun, out, E, partials, c_un, c_in, c_dt);
    p.reverse = reverse ? 1 : 0;
    e = dgk::launch_stage(c->cfg.nv, c->L.n, true, &p, c->L.ntiles, c->stream);
  } else {
    dgk::StageArgs<float> p;
    fill_pack(c, &p, fin, fun, out, E, partials, c_un, c_in, c_dt);
    p.reverse = reverse ? 1 : 0;
    e = dgk::launch_stage(c->cfg.nv, c->L.n, false, &p, c->L.ntiles, c->stream);
  }
  if (e != hipSuccess) return hip_fail(c, e, "stage kernel launch");
  return DG_OK;
}

dg_status density(dg_ctx* c, const void* f) {
  hipError_t e;
  double* part = c->at<double>(c->L.off_part);
  if (c->f64()) {
    dgk::StageArgs<double> p;
    fill_pack(c, &p, f, f, nullptr, nullptr, part, 0, 0, 0);
    e = dgk::launch_density(c->cfg.nv, c->L.n, true, &p, c->L.ntiles, c->stream);
  } else {
    dgk::StageArgs<float> p;
    fill_pack(c, &p, f, f, nullptr, nullptr, part, 0, 0, 0);
    e = dgk::launch_density(c->cfg.nv, c->L.n, false, &p, c->L.ntiles, c->stream);
  }
  if (e != hipSuccess) return hip_fail(c, e, "density kernel launch");
  return DG_OK;
}

dg_status moments(dg_ctx* c, const void* f) {
  hipError_t e;
  double* mom = c->at<double>(c->L.off_mom);
  if (c->f64()) {
    dgk::StageArgs<double> p;
    fill_pack(c, &p, f, f, nullptr, nullptr, nullptr, 0, 0, 0);
    e = dgk::launch_moments(c->cfg.nv, c->L.n, true, &p, mom, c->L.ntiles, c->stream);
  } else {
    dgk::StageArgs<float> p;
    fill_pack(c, &p, f, f, nullptr, nullptr, nullptr, 0, 0, 0);
    e = dgk::launch_moments(c->cfg.nv, c->L.n, false, &p, mom, c->L.ntiles, c->stream);
  }
  if (e != hipSuccess) return hip_fail(c, e, "moments kernel launch");
  e = dgk::launch_moments_reduce(mom, c->L.ntiles, c->at<double>(c->L.off_ring), c->at<int>(c->L.off_ctr), c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "moments reduce launch");
  return DG_OK;
}

void fill_field(const dg_ctx* c, dgk::FieldArgs* pa, double* E, double* coeffs, bool record) {
  const Layout& L = c->L;
  dgk::FieldArgs& a = *pa;
  a = dgk::FieldArgs{};
  a.partials = c->at<double>(L.off_part);
  a.ntiles = L.ntiles_slab;
  a.Nx = L.Nx;
  a.n = L.n;
  a.pmax = L.pmax;
  a.k1 = 2.0 * M_PI / (c->cfg.hi[0] - c->cfg.lo[0]);
  a.T = c->at<double>(L.off_T);
  a.z1 = c->at<double>(L.off_z1);
  a.wx = c->at<double>(L.off_wx);
  a.dens = c->at<double>(L.off_dens);
  a.cpart = c->at<double>(L.off_cpart);
  a.mpart = c->at<double>(L.off_mpart);
  a.E = E;
  a.coeffs = coeffs ? coeffs : c->at<double>(L.off_coef);
  a.ring = c->at<double>(L.off_ring);
  a.last = c->at<double>(L.off_last);
  a.counter = c->at<int>(L.off_ctr);
  a.record = record ? 1 : 0;
  a.mass0 = c->bg ? c->mass0 : 0.0;
}

dg_status field(dg_ctx* c, double* E, double* coeffs, bool record) {
  dgk::FieldArgs a;
  fill_field(c, &a, E, coeffs, record);
  hipError_t e = dgk::launch_field(a, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "field kernel launch");
  return DG_OK;
}

// Order the library stream after the caller's stream (enter) and the caller's
// stream after the library stream (leave).
dg_status enter(dg_ctx* c) {
  DG_HIP(c, hipEventRecord(c->ev_in, c->user));
  DG_HIP(c, hipStreamWaitEvent(c->stream, c->ev_in, 0));
  return DG_OK;
}
dg_status leave(dg_ctx* c) {
  DG_HIP(c, hipEventRecord(c->ev_out, c->stream));
  DG_HIP(c, hipStreamWaitEvent(c->user, c->ev_out, 0));
  return DG_OK;
}

#define DG_TRY(expr)                 \
  do {                               \
    dg_status s__ = (expr);          \
    if (s__ != DG_OK) return s__;    \
  } while (0)

// One SSP-RK3 step (Shu-Osher form) on f, with E already solved for f:
//   B = f + dt L(f);  C = 3/4 f + 1/4 (B + dt L(B));  f = 1/3 f + 2/3 (C + dt L(C)).
// Each stage's density partials feed the next stage's field solve; the last
// one gives the field of the new state (the next step's first stage).
// One SSP-RK3 step.  The stages alternate the direction in which they visit
// the tiles, so each starts with the tiles its predecessor wrote last; over a
// pair of steps (odd = false, then true) every hand-over alternates.
dg_status enqueue_step(dg_ctx* c, void* f, double dt, bool diag, bool odd) {
  void* B = c->ws + c->L.off_B;
  void* C = c->ws + c->L.off_C;
  double* E = c->at<double>(c->L.off_E);
  double* part = c->at<double>(c->L.off_part);
  DG_TRY(stage(c, f, nullptr, B, E, part, 0.0, 1.0, dt, odd));
  DG_TRY(field(c, E, nullptr, false));
  DG_TRY(stage(c, B, f, C, E, part, 0.75, 0.25, 0.25 * dt, !odd));
  DG_TRY(field(c, E, nullptr, false));
  DG_TRY(stage(c, C, f, f, E, part, 1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0 * dt, odd));
  DG_TRY(field(c, E, nullptr, diag));
  if (diag) DG_TRY(moments(c, f));
  return DG_OK;
}

dg_status build_graph(dg_ctx* c, void* f, double dt, bool diag) {
  if (c->gexec && c->g_f == f && c->g_dt == dt && c->g_diag == diag) return DG_OK;
  if (c->gexec) {
    drop_graph(c->stream, &c->gexec);
  }
  // the graph holds a pair of steps (the two tile-order patterns)
  DG_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  dg_status s = enqueue_step(c, f, dt, diag, false);
  if (s == DG_OK) s = enqueue_step(c, f, dt, diag, true);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (s != DG_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    c->gexec = nullptr;
    return hip_fail(c, e, "hipGraphInstantiate");
  }
  c->g_f = f;
  c->g_dt = dt;
  c->g_diag = diag;
  return DG_OK;
}

Layout scratch_layout(const dg_config* cfg) { return make_layout(cfg, false); }

const char* config_error(const dg_config* cfg, dg_status* st) { return check_cfg(cfg, st); }

dg_status global_fail(dg_status s, const std::string& msg) {
  std::lock_guard<std::mutex> lk(g_err_mu);
  g_init_error = msg;
  return s;
}

void copy_record(const double* r, double t, dg_diag* out) {
  out->t = t;
  out->mass = r[1];
  out->field_energy = r[2];
  out->kinetic_energy = r[3];
  out->l2sq = r[4];
  out->max_abs_E = r[5];
  out->finite = r[6] != 0.0 ? 1 : 0;
  out->step = static_cast<int32_t>(r[7]);
}

}  // namespace dgi

using namespace dgi;

namespace {

// dense <-> context layout (Layout::cpitch / lpitch), on the context stream
dg_status repack_state(dg_ctx* ctx, bool pack, const void* in, void* out) {
  if (!ctx) return DG_ERR_INVALID;
  if (!in || !out) return fail(ctx, DG_ERR_INVALID, pack ? "dg_state_pack: NULL array" : "dg_state_unpack: NULL array");
  const Layout& L = ctx->L;
  DG_TRY(enter(ctx));
  const hipError_t e = dgk::launch_repack(pack, L.esize == 8, in, out, L.selems / L.lpitch, L.lpitch, L.cpitch,
                                          dgk::tv_of(L.n) * L.n, L.Nv * L.n, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "layout conversion launch");
  return leave(ctx);
}

}  // namespace

extern "C" {

size_t dg_workspace_bytes(const dg_config* cfg) {
  dg_status st;
  if (check_cfg(cfg, &st)) return 0;
  return make_layout(cfg).total;
}

}  // extern "C"

namespace {

// Build a context on `ws`: FP64 host setup (basis, Courant number, tables)
// uploaded on `stream`.  If own_stream, the context creates its own
// non-blocking stream and ordering events (dg_init); otherwise it enqueues on
// `stream` directly (runs of a batch).  On failure *err holds the reason.
dg_status make_ctx(const dg_config* cfg, char* ws, hipStream_t user, bool own_stream, dg_ctx** out, std::string* err) {
  *out = nullptr;
  const Layout L = make_layout(cfg);
  dg_ctx* c = new (std::nothrow) dg_ctx();
  if (!c) { *err = "host allocation failed"; return DG_ERR_INVALID; }
  static std::atomic<uint64_t> next_id{1};
  c->cfg = *cfg;
  c->id = next_id.fetch_add(1);
  c->L = L;
  c->ws = ws;
  c->user = user;
  c->owns_stream = own_stream;
  try {
    c->basis = dgh::make_basis(cfg->n);
    c->courant = dgh::courant_number(cfg->n);
  } catch (const std::exception& ex) {
    delete c;
    *err = std::string("basis setup failed: ") + ex.what();
    return DG_ERR_INVALID;
  }
  for (int a = 0; a <= cfg->nv; ++a) c->dx[a] = (cfg->hi[a] - cfg->lo[a]) / cfg->nelem[a];

  auto cleanup = [&](hipError_t e, const char* what) {
    *err = std::string(what) + ": " + hipGetErrorString(e);
    if (c->owns_stream) {
      if (c->stream) (void)hipStreamDestroy(c->stream);
      if (c->ev_in) (void)hipEventDestroy(c->ev_in);
      if (c->ev_out) (void)hipEventDestroy(c->ev_out);
    }
    delete c;
    return DG_ERR_DEVICE;
  };
  hipError_t e;
  if (own_stream) {
    if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess) return cleanup(e, "hipStreamCreate");
    if ((e = hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming)) != hipSuccess) return cleanup(e, "hipEventCreate");
    if ((e = hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming)) != hipSuccess) return cleanup(e, "hipEventCreate");
  } else {
    c->stream = user;
  }

  // FP64 host tables.
  const int n = cfg->n;
  const int vax = cfg->nv == 2 ? 2 : 1;
  std::vector<double> wx = axis_weights(c->basis, L.Nx, cfg->lo[0], cfg->hi[0]);
  std::vector<double> wu = cfg->nv == 2 ? axis_weights(c->basis, L.Nu, cfg->lo[1], cfg->hi[1]) : std::vector<double>(n, 1.0);
  std::vector<double> wv = axis_weights(c->basis, L.Nv, cfg->lo[vax], cfg->hi[vax]);
  std::vector<double> uc = cfg->nv == 2 ? axis_nodes(c->basis, L.Nu, cfg->lo[1], cfg->hi[1]) : std::vector<double>(n, 0.0);
  std::vector<double> vc = axis_nodes(c->basis, L.Nv, cfg->lo[vax], cfg->hi[vax]);
  // connection tensor stored node-major ([m*n + j][p]) so lanes over p are contiguous
  auto Tp = dgh::connection_tensor(c->basis, L.Nx, cfg->lo[0], cfg->hi[0], L.pmax);
  const size_t nxn = static_cast<size_t>(L.Nx) * n;
  std::vector<std::complex<double>> T(Tp.size());
  for (int p = 0; p < L.pmax; ++p)
    for (size_t q = 0; q < nxn; ++q) T[q * L.pmax + p] = Tp[p * nxn + q];
  // e^{i k_1 x_mj}: first column of the synthesis recurrence
  std::vector<std::complex<double>> Z1(nxn);
  {
    std::vector<double> xn = axis_nodes(c->basis, L.Nx, cfg->lo[0], cfg->hi[0]);
    const double k1 = 2.0 * M_PI / (cfg->hi[0] - cfg->lo[0]);
    for (size_t q = 0; q < nxn; ++q) Z1[q] = std::polar(1.0, k1 * xn[q]);
  }
  std::vector<float> ucf(uc.begin(), uc.end()), vcf(vc.begin(), vc.end());
  auto up = [&](size_t off, const void* src, size_t bytes) {
    return hipMemcpyAsync(c->ws + off, src, bytes, hipMemcpyHostToDevice, c->stream);
  };
  if ((e = up(L.off_wx, wx.data(), wx.size() * 8)) != hipSuccess ||
      (e = up(L.off_wu, wu.data(), wu.size() * 8)) != hipSuccess ||
      (e = up(L.off_wv, wv.data(), wv.size() * 8)) != hipSuccess ||
      (e = up(L.off_T, T.data(), T.size() * 16)) != hipSuccess ||
      (e = up(L.off_z1, Z1.data(), Z1.size() * 16)) != hipSuccess ||
      (e = (c->f64() ? up(L.off_uc, uc.data(), uc.size() * 8) : up(L.off_uc, ucf.data(), ucf.size() * 4))) != hipSuccess ||
      (e = (c->f64() ? up(L.off_vc, vc.data(), vc.size() * 8) : up(L.off_vc, vcf.data(), vcf.size() * 4))) != hipSuccess ||
      (e = up(L.off_uc64, uc.data(), uc.size() * 8)) != hipSuccess ||
      (e = up(L.off_vc64, vc.data(), vc.size() * 8)) != hipSuccess)
    return cleanup(e, "upload of setup tables");
  if ((e = dgk::launch_reset_counter(c->at<int>(L.off_ctr), c->stream)) != hipSuccess) return cleanup(e, "counter reset");
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return cleanup(e, "hipStreamSynchronize");
  *out = c;
  return DG_OK;
}

// Configuration checks shared by dg_init and the batch.
const char* check_cfg(const dg_config* cfg, dg_status* st) {
  *st = DG_ERR_INVALID;
  if (const char* why = validate(cfg)) return why;
  *st = DG_ERR_UNSUPPORTED;
  if (cfg->n > dgk::kMaxN) return "n above 12 is not built";
  const Layout L = make_layout(cfg);
  if (L.ntiles <= 0 || static_cast<long long>(L.Nx) * L.ntiles_slab > 0x7fffffffLL) return "grid too large";
  // one x element must be addressable by a 31-bit buffer offset
  if (static_cast<double>(L.selems) / L.Nx * L.esize >= 2147483648.0) return "x element larger than 2 GiB";
  *st = DG_OK;
  return nullptr;
}

}  // namespace

extern "C" {

dg_status dg_init(const dg_config* cfg, void* workspace, size_t workspace_bytes, void* hip_stream, dg_ctx** out) {
  auto init_fail = [](dg_status s, const std::string& m) {
    std::lock_guard<std::mutex> lk(g_err_mu);
    g_init_error = m;
    return s;
  };
  if (!out) return init_fail(DG_ERR_INVALID, "out is NULL");
  *out = nullptr;
  dg_status st;
  if (const char* why = check_cfg(cfg, &st)) return init_fail(st, why);
  const Layout L = make_layout(cfg);
  if (!workspace) return init_fail(DG_ERR_INVALID, "workspace is NULL");
  if (workspace_bytes < L.total) return init_fail(DG_ERR_OOM, "workspace smaller than dg_workspace_bytes()");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return init_fail(DG_ERR_INVALID, "workspace must be 256-byte aligned");
  std::string err;
  st = make_ctx(cfg, static_cast<char*>(workspace), static_cast<hipStream_t>(hip_stream), true, out, &err);
  if (st != DG_OK) return init_fail(st, err);
  return DG_OK;
}

dg_status dg_destroy(dg_ctx* ctx) {
  if (!ctx) return DG_OK;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
  if (ctx->owns_stream) {
    (void)hipEventDestroy(ctx->ev_in);
    (void)hipEventDestroy(ctx->ev_out);
    (void)hipStreamDestroy(ctx->stream);
  }
  delete ctx;
  return e == hipSuccess ? DG_OK : DG_ERR_DEVICE;
}

dg_status dg_rhs(dg_ctx* ctx, const void* f, const double* E, void* rhs) {
  if (!ctx) return DG_ERR_INVALID;
  if (!f || !rhs) return fail(ctx, DG_ERR_INVALID, "dg_rhs: f and rhs must be non-NULL");
  if (f == rhs) return fail(ctx, DG_ERR_INVALID, "dg_rhs: f and rhs must not overlap");
  DG_TRY(enter(ctx));
  const double* Ef = E;
  if (!Ef) {
    double* Ews = ctx->at<double>(ctx->L.off_E);
    DG_TRY(density(ctx, f));
    DG_TRY(field(ctx, Ews, nullptr, false));
    Ef = Ews;
  }
  DG_TRY(stage(ctx, f, nullptr, rhs, Ef, nullptr, 0.0, 0.0, 1.0));
  return leave(ctx);
}

dg_status dg_poisson(dg_ctx* ctx, const void* f, double* E, double* coeffs) {
  if (!ctx) return DG_ERR_INVALID;
  if (!f || !E) return fail(ctx, DG_ERR_INVALID, "dg_poisson: f and E must be non-NULL");
  DG_TRY(enter(ctx));
  DG_TRY(density(ctx, f));
  DG_TRY(field(ctx, E, coeffs, false));
  return leave(ctx);
}

size_t dg_state_elems(const dg_ctx* ctx) { return ctx ? ctx->L.selems : 0; }

dg_status dg_state_pack(dg_ctx* ctx, const void* dense, void* state) { return repack_state(ctx, true, dense, state); }

dg_status dg_state_unpack(dg_ctx* ctx, const void* state, void* dense) { return repack_state(ctx, false, state, dense); }

double dg_dt_max(const dg_ctx* ctx, double max_abs_E) {
  if (!ctx) return 0.0;
  const dg_config& c = ctx->cfg;
  auto vmax = [&](int a) { return std::max(std::fabs(c.lo[a]), std::fabs(c.hi[a])); };
  double rate;
  if (c.nv == 1) {
    rate = vmax(1) / ctx->dx[0] + std::fabs(max_abs_E) / ctx->dx[1];
  } else {
    const double B = std::fabs(c.omega_c);
    rate = vmax(1) / ctx->dx[0] + (std::fabs(max_abs_E) + vmax(2) * B) / ctx->dx[1] + vmax(1) * B / ctx->dx[2];
  }
  return ctx->courant / rate;
}

}  // extern "C"

namespace dgi {
// Field of the initial state and the CFL check shared by the stepping calls.
dg_status begin_steps(dg_ctx* ctx, void* f, double dt, int32_t nsteps) {
  if (!f) return fail(ctx, DG_ERR_INVALID, "f is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, DG_ERR_INVALID, "dt must be positive and finite");
  if (nsteps < 0) return fail(ctx, DG_ERR_INVALID, "nsteps < 0");
  const Layout& L = ctx->L;
  DG_TRY(enter(ctx));
  DG_TRY(density(ctx, f));
  DG_TRY(field(ctx, ctx->at<double>(L.off_E), nullptr, false));
  double last[8];
  DG_HIP(ctx, hipMemcpyAsync(last, ctx->at<double>(L.off_last), sizeof(last), hipMemcpyDeviceToHost, ctx->stream));
  DG_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (!std::isfinite(last[5]) || last[6] == 0.0) {
    leave(ctx);
    return fail(ctx, DG_ERR_NONFINITE, "initial field is not finite");
  }
  const double dtm = dg_dt_max(ctx, last[5]);
  if (dt > dtm) {
    leave(ctx);
    char buf[160];
    std::snprintf(buf, sizeof(buf), "dt = %.6g exceeds the CFL bound %.6g", dt, dtm);
    return fail(ctx, DG_ERR_CFL, buf);
  }
  return DG_OK;
}
}  // namespace dgi

extern "C" {

dg_status dg_rk_step(dg_ctx* ctx, void* f, double dt, int32_t nsteps, dg_diag* host_diag) {
  if (!ctx) return DG_ERR_INVALID;
  if (nsteps == 0 && f && dt > 0.0) return DG_OK;
  DG_TRY(begin_steps(ctx, f, dt, nsteps));
  const Layout& L = ctx->L;
  const bool diag = host_diag != nullptr;
  if (nsteps >= 2) DG_TRY(build_graph(ctx, f, dt, diag));
  int done = 0;
  bool bad = false;
  while (done < nsteps) {
    const int chunk = std::min(nsteps - done, dgk::kRing);
    if (diag) {
      hipError_t e = dgk::launch_reset_counter(ctx->at<int>(L.off_ctr), ctx->stream);
      if (e != hipSuccess) return hip_fail(ctx, e, "counter reset");
    }
    int s = 0;
    for (; s + 2 <= chunk; s += 2) DG_HIP(ctx, hipGraphLaunch(ctx->gexec, ctx->stream));
    if (s < chunk) DG_TRY(enqueue_step(ctx, f, dt, diag, false));   // odd count: last step eagerly
    if (diag) {
      std::vector<double> ring(static_cast<size_t>(chunk) * 8);
      DG_HIP(ctx, hipMemcpyAsync(ring.data(), ctx->at<double>(L.off_ring), ring.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
      DG_HIP(ctx, hipStreamSynchronize(ctx->stream));
      for (int s = 0; s < chunk; ++s) {
        copy_record(&ring[static_cast<size_t>(s) * 8], ctx->t + (done + s + 1) * dt, &host_diag[done + s]);
        host_diag[done + s].step = done + s;
        if (!host_diag[done + s].finite) bad = true;
      }
    }
    done += chunk;
  }
  ctx->t += nsteps * dt;
  DG_TRY(leave(ctx));
  if (diag) DG_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (bad) return fail(ctx, DG_ERR_NONFINITE, "a step produced non-finite diagnostics");
  return DG_OK;
}

dg_status dg_profile_step(dg_ctx* ctx, void* f, double dt, int32_t nsteps, double* host_ms) {
  if (!ctx) return DG_ERR_INVALID;
  if (!host_ms) return fail(ctx, DG_ERR_INVALID, "host_ms is NULL");
  if (nsteps == 0 && f && dt > 0.0) return DG_OK;
  DG_TRY(begin_steps(ctx, f, dt, nsteps));
  const Layout& L = ctx->L;
  void* B = ctx->ws + L.off_B;
  void* C = ctx->ws + L.off_C;
  double* E = ctx->at<double>(L.off_E);
  double* part = ctx->at<double>(L.off_part);
  hipEvent_t ev[7] = {};
  for (auto& e : ev) DG_HIP(ctx, hipEventCreate(&e));
  dg_status st = DG_OK;
  for (int s = 0; s < nsteps && st == DG_OK; ++s) {
    const void* ins[3] = {f, B, C};
    void* outs[3] = {B, C, f};
    const double cu[3] = {0.0, 0.75, 1.0 / 3.0}, ci[3] = {1.0, 0.25, 2.0 / 3.0}, cd[3] = {dt, 0.25 * dt, 2.0 / 3.0 * dt};
    if (hipEventRecord(ev[0], ctx->stream) != hipSuccess) { st = fail(ctx, DG_ERR_DEVICE, "event record"); break; }
    for (int k = 0; k < 3 && st == DG_OK; ++k) {
      st = stage(ctx, ins[k], f, outs[k], E, part, cu[k], ci[k], cd[k], (k == 1) != (s % 2 == 1));   // as enqueue_step
      if (st == DG_OK && hipEventRecord(ev[2 * k + 1], ctx->stream) != hipSuccess) st = fail(ctx, DG_ERR_DEVICE, "event record");
      if (st == DG_OK) st = field(ctx, E, nullptr, false);
      if (st == DG_OK && hipEventRecord(ev[2 * k + 2], ctx->stream) != hipSuccess) st = fail(ctx, DG_ERR_DEVICE, "event record");
    }
    if (st != DG_OK) break;
    if (hipEventSynchronize(ev[6]) != hipSuccess) { st = fail(ctx, DG_ERR_DEVICE, "event synchronize"); break; }
    for (int q = 0; q < 6; ++q) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, ev[q], ev[q + 1]) != hipSuccess) { st = fail(ctx, DG_ERR_DEVICE, "event elapsed"); break; }
      host_ms[6 * s + q] = ms;
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (st != DG_OK) return st;
  ctx->t += nsteps * dt;
  return leave(ctx);
}

dg_status dg_diagnostics(dg_ctx* ctx, const void* f, dg_diag* host_out) {
  if (!ctx) return DG_ERR_INVALID;
  if (!f || !host_out) return fail(ctx, DG_ERR_INVALID, "dg_diagnostics: NULL argument");
  const Layout& L = ctx->L;
  DG_TRY(enter(ctx));
  hipError_t e = dgk::launch_reset_counter(ctx->at<int>(L.off_ctr), ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "counter reset");
  DG_TRY(density(ctx, f));
  DG_TRY(field(ctx, ctx->at<double>(L.off_E), nullptr, true));
  DG_TRY(moments(ctx, f));
  double rec[8];
  DG_HIP(ctx, hipMemcpyAsync(rec, ctx->at<double>(L.off_ring), sizeof(rec), hipMemcpyDeviceToHost, ctx->stream));
  DG_HIP(ctx, hipStreamSynchronize(ctx->stream));
  copy_record(rec, ctx->t, host_out);
  host_out->step = 0;
  DG_TRY(leave(ctx));
  return host_out->finite ? DG_OK : fail(ctx, DG_ERR_NONFINITE, "dg_diagnostics: non-finite moments");
}

dg_status dg_profile_copy(dg_ctx* ctx, const void* in, void* out, int32_t pattern, int32_t reps, double* host_ms) {
  if (!ctx) return DG_ERR_INVALID;
  if (!in || !out || !host_ms || reps < 1) return fail(ctx, DG_ERR_INVALID, "dg_profile_copy: bad argument");
  if (in == out) return fail(ctx, DG_ERR_INVALID, "dg_profile_copy: in and out must not overlap");
  if (pattern < 0 || pattern > 3) return fail(ctx, DG_ERR_INVALID, "dg_profile_copy: pattern must be 0..3");
  if ((pattern == 1 || pattern == 3) && ctx->cfg.nv != 2)
    return fail(ctx, DG_ERR_UNSUPPORTED, "dg_profile_copy: the tile pattern is 1D2V");
  const Layout& L = ctx->L;
  auto launch = [&]() -> hipError_t {
    if (pattern == 2) return dgk::launch_empty(ctx->stream);
    if (pattern == 0) return dgk::launch_linear_copy(in, out, L.selems * L.esize / 16 * 16, ctx->stream);
    if (ctx->f64()) {
      dgk::StageArgs<double> p;
      fill_pack(ctx, &p, in, in, out, nullptr, nullptr, 0, 0, 0);
      return dgk::launch_pattern_copy(2, L.n, true, &p, L.ntiles, pattern == 3, ctx->stream);
    }
    dgk::StageArgs<float> p;
    fill_pack(ctx, &p, in, in, out, nullptr, nullptr, 0, 0, 0);
    return dgk::launch_pattern_copy(2, L.n, false, &p, L.ntiles, pattern == 3, ctx->stream);
  };
  DG_TRY(enter(ctx));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  DG_HIP(ctx, hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  if (e == hipSuccess) e = launch();   // warm-up launch
  if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(ctx, e, "dg_profile_copy");
  *host_ms = ms / reps;
  return leave(ctx);
}

dg_status dg_fourier(dg_ctx* ctx, const double* g, double* coeffs) {
  if (!ctx) return DG_ERR_INVALID;
  if (!g || !coeffs) return fail(ctx, DG_ERR_INVALID, "dg_fourier: NULL argument");
  const Layout& L = ctx->L;
  DG_TRY(enter(ctx));
  hipError_t e = dgk::launch_fourier(ctx->at<double>(L.off_T), g, L.Nx * L.n, L.pmax, coeffs, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "fourier kernel launch");
  return leave(ctx);
}

dg_status dg_filter_x(dg_ctx* ctx, const double* sigma, const void* f_in, void* f_out) {
  if (!ctx) return DG_ERR_INVALID;
  if (!sigma || !f_in || !f_out) return fail(ctx, DG_ERR_INVALID, "dg_filter_x: NULL argument");
  if (f_in == f_out) return fail(ctx, DG_ERR_INVALID, "dg_filter_x: f_in and f_out must not overlap");
  const Layout& L = ctx->L;
  const dg_config& C = ctx->cfg;
  const int R = L.Nx * L.n, n = L.n;
  if (static_cast<size_t>(R) > kMaxFilterNodes)
    return fail(ctx, DG_ERR_UNSUPPORTED, "dg_filter_x: more than 4096 x nodes");
  for (int p = 0; p < L.pmax; ++p)
    if (!std::isfinite(sigma[p])) return fail(ctx, DG_ERR_INVALID, "dg_filter_x: sigma is not finite");
  // M[r][q] = T_0^q + sum_{p=1..pmax} 2 Re(sigma_p T_p^q e^{i k_p x_r}) (eq. spectral_transform,
  // then eq. fourier_series truncated at pmax with the weights sigma), T_0^{mj} = (dx/L) w_j / 2
  const auto T = dgh::connection_tensor(ctx->basis, L.Nx, C.lo[0], C.hi[0], L.pmax);
  const std::vector<double> xn = axis_nodes(ctx->basis, L.Nx, C.lo[0], C.hi[0]);
  const double Lx = C.hi[0] - C.lo[0], dx = Lx / L.Nx;
  std::vector<double> M(static_cast<size_t>(R) * R);
  for (int r = 0; r < R; ++r) {
    std::vector<std::complex<double>> z(L.pmax);
    for (int p = 1; p <= L.pmax; ++p) z[p - 1] = sigma[p - 1] * std::polar(1.0, 2.0 * M_PI * p / Lx * xn[r]);
    for (int q = 0; q < R; ++q) {
      double v = dx / Lx * ctx->basis.w[q % n] * 0.5;
      for (int p = 1; p <= L.pmax; ++p) v += 2.0 * (z[p - 1] * T[static_cast<size_t>(p - 1) * R + q]).real();
      M[static_cast<size_t>(r) * R + q] = v;
    }
  }
  DG_TRY(enter(ctx));
  if (ctx->f64()) {
    DG_HIP(ctx, hipMemcpyAsync(ctx->ws + L.off_M, M.data(), M.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  } else {
    std::vector<float> Mf(M.begin(), M.end());
    DG_HIP(ctx, hipMemcpyAsync(ctx->ws + L.off_M, Mf.data(), Mf.size() * 4, hipMemcpyHostToDevice, ctx->stream));
    DG_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  hipError_t e = dgk::launch_xfilter(ctx->f64(), f_in, f_out, ctx->ws + L.off_M, R, L.selems / R, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "x-filter kernel launch");
  DG_HIP(ctx, hipStreamSynchronize(ctx->stream));   // M is host memory of this call
  return leave(ctx);
}

dg_status dg_set_background(dg_ctx* ctx, const double* f0) {
  if (!ctx) return DG_ERR_INVALID;
  // a cached step graph holds the stage kernels of the previous mode
  if (ctx->gexec) {
    drop_graph(ctx->stream, &ctx->gexec);
  }
  if (!f0) {
    ctx->bg = false;
    ctx->mass0 = 0.0;
    return DG_OK;
  }
  ctx->bg = false;
  const dg_config& C = ctx->cfg;
  if (C.vbc != DG_VBC_PERIODIC) return fail(ctx, DG_ERR_UNSUPPORTED, "dg_set_background: needs periodic velocity boundaries");
  const Layout& L = ctx->L;
  const dgh::Basis& b = ctx->basis;
  const int n = L.n;
  const bool two = C.nv == 2;
  const int nu = two ? L.Nu * n : 1, nvn = L.Nv * n;
  auto F = [&](int p, int q) { return f0[static_cast<size_t>(p) * nvn + q]; };
  double fmax = 0.0;
  for (size_t i = 0; i < static_cast<size_t>(nu) * nvn; ++i) {
    if (!std::isfinite(f0[i])) return fail(ctx, DG_ERR_INVALID, "dg_set_background: f0 is not finite");
    fmax = std::max(fmax, std::fabs(f0[i]));
  }
  // continuity across every element face of both velocity axes (periodic
  // wrap included): then the upwind face value of f0 is the same from either
  // side and L(f0) is linear in E without a sign choice
  const double tol = 1e-10 * fmax;
  for (int p = 0; p < nu; ++p)
    for (int e = 0; e < L.Nv; ++e)
      if (std::fabs(F(p, e * n + n - 1) - F(p, ((e + 1) % L.Nv) * n)) > tol)
        return fail(ctx, DG_ERR_INVALID, "dg_set_background: f0 jumps across a v face");
  if (two)
    for (int q = 0; q < nvn; ++q)
      for (int e = 0; e < L.Nu; ++e)
        if (std::fabs(F(e * n + n - 1, q) - F(((e + 1) % L.Nu) * n, q)) > tol)
          return fail(ctx, DG_ERR_INVALID, "dg_set_background: f0 jumps across a u face");
  // G = J (Upsilon f0 + Xi_0 f0(left face) - Xi_1 f0(right face)) along an axis
  auto deriv = [&](int Ne, double J, auto get, auto put) {
    for (int e = 0; e < Ne; ++e)
      for (int j = 0; j < n; ++j) {
        double s = b.xi_face[j * 2 + 0] * get(e * n) - b.xi_face[j * 2 + 1] * get(e * n + n - 1);
        for (int k = 0; k < n; ++k) s += b.ups[j * n + k] * get(e * n + k);
        put(e * n + j, J * s);
      }
  };
  const int vax = two ? 2 : 1;
  std::vector<double> Gv(static_cast<size_t>(nu) * nvn), Gu(two ? static_cast<size_t>(nu) * nvn : 0);
  for (int p = 0; p < nu; ++p)
    deriv(L.Nv, 2.0 / ctx->dx[vax], [&](int q) { return F(p, q); },
          [&](int q, double g) { Gv[static_cast<size_t>(p) * nvn + q] = g; });
  if (two)
    for (int q = 0; q < nvn; ++q)
      deriv(L.Nu, 2.0 / ctx->dx[1], [&](int p) { return F(p, q); },
            [&](int p, double g) { Gu[static_cast<size_t>(p) * nvn + q] = g; });
  // tables in the storage precision: 1D2V G_u and G_b = -v B G_u + u B G_v
  // (the gyration of f0, cancelled in FP64) in the state's row layout;
  // 1D1V G_v (the whole L(f0) is -E G_v)
  const std::vector<double> uc = two ? axis_nodes(b, L.Nu, C.lo[1], C.hi[1]) : std::vector<double>(1, 0.0);
  const std::vector<double> vc = axis_nodes(b, L.Nv, C.lo[vax], C.hi[vax]);
  const int tv = dgk::tv_of(n);
  const size_t rowlen = two ? static_cast<size_t>(L.lpitch) : static_cast<size_t>(nvn);
  std::vector<double> tu(static_cast<size_t>(nu) * rowlen, 0.0), tb(two ? tu.size() : 0, 0.0);
  for (int p = 0; p < nu; ++p)
    for (int q = 0; q < nvn; ++q) {
      const int iv = q / n, c = iv / tv;
      const size_t pos = two ? static_cast<size_t>(c) * L.cpitch + (iv - c * tv) * n + q % n : q;
      const size_t i = static_cast<size_t>(p) * nvn + q;
      if (two) {
        tu[p * rowlen + pos] = Gu[i];
        tb[p * rowlen + pos] = -vc[q] * C.omega_c * Gu[i] + uc[p] * C.omega_c * Gv[i];
      } else {
        tu[pos] = Gv[i];
      }
    }
  // mass of f0 over the whole domain
  const std::vector<double> wu = two ? axis_weights(b, L.Nu, C.lo[1], C.hi[1]) : std::vector<double>(1, 1.0);
  const std::vector<double> wv = axis_weights(b, L.Nv, C.lo[vax], C.hi[vax]);
  double m0 = 0.0;
  for (int p = 0; p < nu; ++p)
    for (int q = 0; q < nvn; ++q) m0 += wu[p] * wv[q] * F(p, q);
  m0 *= C.hi[0] - C.lo[0];
  auto upload = [&](size_t off, const std::vector<double>& v) -> hipError_t {
    if (ctx->f64()) return hipMemcpyAsync(ctx->ws + off, v.data(), v.size() * 8, hipMemcpyHostToDevice, ctx->stream);
    std::vector<float> w(v.begin(), v.end());
    hipError_t e = hipMemcpyAsync(ctx->ws + off, w.data(), w.size() * 4, hipMemcpyHostToDevice, ctx->stream);
    return e == hipSuccess ? hipStreamSynchronize(ctx->stream) : e;   // w is released on return
  };
  DG_TRY(enter(ctx));
  DG_HIP(ctx, upload(L.off_bgu, tu));
  if (two) DG_HIP(ctx, upload(L.off_bgb, tb));
  DG_HIP(ctx, hipMemcpyAsync(ctx->ws + L.off_bg64, f0, static_cast<size_t>(nu) * nvn * 8, hipMemcpyHostToDevice, ctx->stream));
  DG_HIP(ctx, hipStreamSynchronize(ctx->stream));
  DG_TRY(leave(ctx));
  ctx->bg = true;
  ctx->mass0 = m0;
  return DG_OK;
}

dg_status dg_node_coords(const dg_ctx* ctx, int32_t axis, double* host_out) {
  if (!ctx || !host_out) return DG_ERR_INVALID;
  if (axis < 0 || axis > ctx->cfg.nv) return DG_ERR_INVALID;
  auto x = axis_nodes(ctx->basis, ctx->cfg.nelem[axis], ctx->cfg.lo[axis], ctx->cfg.hi[axis]);
  std::memcpy(host_out, x.data(), x.size() * sizeof(double));
  return DG_OK;
}

const char* dg_last_error(const dg_ctx* ctx) {
  if (ctx) return ctx->err.c_str();
  std::lock_guard<std::mutex> lk(g_err_mu);
  return g_init_error.c_str();
}

dg_status dg_basis(int32_t n, double* xi, double* w, double* ups, double* xi_face, double* dmat) {
  if (n < 2 || n > 64) return DG_ERR_INVALID;
  dgh::Basis b = dgh::make_basis(n);
  if (xi) std::memcpy(xi, b.xi.data(), n * sizeof(double));
  if (w) std::memcpy(w, b.w.data(), n * sizeof(double));
  if (ups) std::memcpy(ups, b.ups.data(), n * n * sizeof(double));
  if (xi_face) std::memcpy(xi_face, b.xi_face.data(), 2 * n * sizeof(double));
  if (dmat) std::memcpy(dmat, b.dmat.data(), n * n * sizeof(double));
  return DG_OK;
}

dg_status dg_connection_tensor(int32_t n, int32_t nelem, double lo, double hi, int32_t pmax, double* out) {
  if (n < 2 || n > 64 || nelem < 1 || !(hi > lo) || pmax < 1 || !out) return DG_ERR_INVALID;
  dgh::Basis b = dgh::make_basis(n);
  auto T = dgh::connection_tensor(b, nelem, lo, hi, pmax);
  std::memcpy(out, T.data(), T.size() * sizeof(std::complex<double>));
  return DG_OK;
}

double dg_courant_number(int32_t n) {
  if (n < 2 || n > 64) return 0.0;
  try {
    return dgh::courant_number(n);
  } catch (...) {
    return 0.0;
  }
}


}  // extern "C"

// ---------------------------------------------------------------------------
// Batches: every run keeps its own tables in a sub-workspace; the stage
// kernels of all runs share one persistent launch per RK stage.
// ---------------------------------------------------------------------------
namespace {
// Tuned work-groups per CU of the batched stage kernel, per (arch, n, nv,
// FP32 storage), kept for the life of the process: later batches on the same
// kind of GPU start from them.
std::mutex g_tune_mu;
std::map<std::string, int> g_tune_cache;
std::string tune_key(const std::string& arch, int n, int nv) {
  return arch + "/n" + std::to_string(n) + "/nv" + std::to_string(nv) + "/f32";
}
int tune_cache_get(const std::string& arch, int n, int nv, int fallback) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune_cache.find(tune_key(arch, n, nv));
  return it == g_tune_cache.end() ? fallback : it->second;
}
void tune_cache_put(const std::string& arch, int n, int nv, int wm) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[tune_key(arch, n, nv)] = wm;
}
}  // namespace

struct dg_batch {
  int nruns = 0;
  bool nt = false;   // the runs' buffers exceed the last-level cache: non-temporal stage stores and u^n loads
  std::vector<dg_ctx*> runs;
  std::vector<size_t> run_off;
  hipStream_t user = nullptr, stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  char* ws = nullptr;
  // device tables
  dgk::StageArgs<float>* d_args = nullptr;   // 3 * nruns
  int2* d_items = nullptr;
  int* d_xcd = nullptr;                       // 9 per kind
  dgk::FieldArgs* d_fa = nullptr;             // 3 * nruns (record flag differs)
  dgk::FieldArgs* d_fa0 = nullptr;            // nruns: the field of the current states (no record)
  double* d_last = nullptr;                   // 8 * nruns: their records, contiguous
  int2* d_xitems = nullptr;
  int nitems = 0, nxitems = 0, max_pmax = 0;
  // runs of one kind (n, nv): items [begin, begin + count) of the work list
  struct Group {
    int n, nv, begin, count, occ[2], grid;
    int wm;                                   // work-groups per CU of this kind's launch (capped by occupancy)
  };
  std::vector<Group> groups;
  int cus = 0;
  std::string arch;
  std::vector<int2> items_cost, items_rr;     // the two work-list orders
  int order = 0;                              // 0: cost-sorted, 1: run-interleaved
  hipGraphExec_t gexec = nullptr;
  std::vector<const void*> g_f;
  std::vector<double> g_dt;
  bool g_diag = false;
  std::string err = "no error";
};

namespace {

constexpr size_t kBatchTail = 1 << 16;

struct BatchLayout {
  std::vector<size_t> run_off;
  size_t args, items, xcd, fa, fa0, last, xitems, total;
};

BatchLayout batch_layout(const dg_config* cfgs, int nruns) {
  BatchLayout B;
  size_t o = 0;
  int ntiles = 0, nx = 0;
  for (int r = 0; r < nruns; ++r) {
    B.run_off.push_back(o);
    const Layout L = make_layout(&cfgs[r]);
    o += align_up(L.total);
    ntiles += L.ntiles;
    nx += L.Nx;
  }
  auto take = [&](size_t bytes) { size_t r = o; o += align_up(bytes); return r; };
  B.args = take(3 * nruns * sizeof(dgk::StageArgs<float>));
  B.items = take(static_cast<size_t>(ntiles) * sizeof(int2));
  B.xcd = take(9 * static_cast<size_t>(nruns) * sizeof(int));
  B.fa = take(3 * nruns * sizeof(dgk::FieldArgs));
  B.fa0 = take(nruns * sizeof(dgk::FieldArgs));
  B.last = take(8 * static_cast<size_t>(nruns) * sizeof(double));
  B.xitems = take(static_cast<size_t>(nx) * sizeof(int2));
  B.total = o;
  return B;
}

dg_status bfail(dg_batch* b, dg_status s, const std::string& m) {
  if (b) b->err = m;
  return s;
}

#define DGB_HIP(b, expr)                                                              \
  do {                                                                                \
    hipError_t e__ = (expr);                                                          \
    if (e__ != hipSuccess) return bfail(b, DG_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e__)); \
  } while (0)

// Split a work list into 8 contiguous ranges of roughly equal cost.
std::vector<int> xcd_split(const std::vector<int2>& items, const std::vector<double>& cost_of_run) {
  double total = 0.0;
  for (auto& it : items) total += cost_of_run[it.x];
  std::vector<int> begin(9, static_cast<int>(items.size()));
  begin[0] = 0;
  double acc = 0.0;
  int c = 1;
  for (size_t i = 0; i < items.size() && c < 8; ++i) {
    acc += cost_of_run[items[i].x];
    while (c < 8 && acc >= total * c / 8.0) begin[c++] = static_cast<int>(i + 1);
  }
  for (; c < 8; ++c) begin[c] = static_cast<int>(items.size());
  begin[8] = static_cast<int>(items.size());
  return begin;
}

// Work lists of the current order and their per-kind XCD splits; grids for
// the current work-groups-per-CU multiplier.
dg_status upload_items(dg_batch* b) {
  const std::vector<int2>& items = b->order == 0 ? b->items_cost : b->items_rr;
  std::vector<double> cost(b->nruns);
  for (int r = 0; r < b->nruns; ++r) {
    const Layout& L = b->runs[r]->L;
    cost[r] = static_cast<double>(L.dof) / L.ntiles;
  }
  std::vector<int> xcd;
  for (auto& g : b->groups) {
    std::vector<int2> part(items.begin() + g.begin, items.begin() + g.begin + g.count);
    std::vector<int> x = xcd_split(part, cost);
    xcd.insert(xcd.end(), x.begin(), x.end());
    const int occ = std::max(1, std::min(g.occ[0], g.occ[1]));
    // wm = 0: one work-group per tile (the hardware dispatcher balances the
    // CUs); else a persistent grid of wm work-groups per CU.  At least one
    // work-group per XCD range (8), else a range would be skipped.
    g.grid = g.wm == 0 ? std::max(8, g.count) : std::max(8, std::min(g.count, b->cus * std::min(g.wm, occ)));
  }
  DGB_HIP(b, hipMemcpyAsync(b->d_items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream));
  DGB_HIP(b, hipMemcpyAsync(b->d_xcd, xcd.data(), xcd.size() * sizeof(int), hipMemcpyHostToDevice, b->stream));
  DGB_HIP(b, hipStreamSynchronize(b->stream));
  return DG_OK;
}

// Per-stage argument tables for the current states and time steps.
dg_status upload_args(dg_batch* b, void* const* f, const double* dt) {
  std::vector<dgk::StageArgs<float>> args(3 * b->nruns);
  std::vector<dgk::FieldArgs> fa(3 * b->nruns);
  for (int r = 0; r < b->nruns; ++r) {
    dg_ctx* c = b->runs[r];
    void* B = c->ws + c->L.off_B;
    void* C = c->ws + c->L.off_C;
    double* E = c->at<double>(c->L.off_E);
    double* part = c->at<double>(c->L.off_part);
    const void* ins[3] = {f[r], B, C};
    void* outs[3] = {B, C, f[r]};
    const double cu[3] = {0.0, 0.75, 1.0 / 3.0}, ci[3] = {1.0, 0.25, 2.0 / 3.0};
    const double cd[3] = {dt[r], 0.25 * dt[r], 2.0 / 3.0 * dt[r]};
    for (int k = 0; k < 3; ++k) {
      fill_pack(c, &args[k * b->nruns + r], ins[k], f[r], outs[k], E, part, cu[k], ci[k], cd[k]);
      fill_field(c, &fa[k * b->nruns + r], E, nullptr, k == 2);
    }
  }
  // the batch's runs share the cache: the store policy follows their total
  size_t total = 0;
  for (int r = 0; r < b->nruns; ++r) total += 3 * b->runs[r]->L.selems * b->runs[r]->L.esize;
  b->nt = total > kLastLevelCache;
  for (auto& a : args) a.nt_store = b->nt ? 1 : 0;
  DGB_HIP(b, hipMemcpyAsync(b->d_args, args.data(), args.size() * sizeof(args[0]), hipMemcpyHostToDevice, b->stream));
  DGB_HIP(b, hipMemcpyAsync(b->d_fa, fa.data(), fa.size() * sizeof(fa[0]), hipMemcpyHostToDevice, b->stream));
  DGB_HIP(b, hipStreamSynchronize(b->stream));
  return DG_OK;
}

dg_status enqueue_batch_step(dg_batch* b, bool diag) {
  const size_t nk = b->groups.size();
  for (int k = 0; k < 3; ++k) {
    for (size_t q = 0; q < nk; ++q) {
      const auto& g = b->groups[q];
      DGB_HIP(b, dgk::launch_stage_batched(k > 0, b->nt, g.n, g.nv, b->d_args + k * b->nruns, b->d_items + g.begin,
                                           b->d_xcd + 9 * q, g.grid, b->stream));
    }
    DGB_HIP(b, dgk::launch_field_batched(b->d_fa + k * b->nruns, b->d_xitems, b->nxitems, b->nruns, b->max_pmax, b->stream));
  }
  if (diag) {
    for (int r = 0; r < b->nruns; ++r) {
      dg_ctx* c = b->runs[r];
      dg_status s = moments(c, b->g_f[r]);
      if (s != DG_OK) return bfail(b, s, c->err);
    }
  }
  return DG_OK;
}

dg_status build_batch_graph(dg_batch* b, void* const* f, const double* dt, bool diag) {
  bool same = b->gexec && b->g_diag == diag;
  for (int r = 0; same && r < b->nruns; ++r) same = b->g_f[r] == f[r] && b->g_dt[r] == dt[r];
  if (same) return DG_OK;
  drop_graph(b->stream, &b->gexec);
  b->g_f.assign(f, f + b->nruns);
  b->g_dt.assign(dt, dt + b->nruns);
  b->g_diag = diag;
  dg_status s = upload_args(b, f, dt);
  if (s != DG_OK) return s;
  DGB_HIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  s = enqueue_batch_step(b, diag);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (s != DG_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return bfail(b, DG_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->gexec = nullptr;
    return bfail(b, DG_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  return DG_OK;
}

// Field of every run's initial state and the per-run CFL check.
dg_status batch_begin(dg_batch* b, void* const* f, const double* dt) {
  DGB_HIP(b, hipEventRecord(b->ev_in, b->user));
  DGB_HIP(b, hipStreamWaitEvent(b->stream, b->ev_in, 0));
  for (int r = 0; r < b->nruns; ++r) {
    if (!f[r]) return bfail(b, DG_ERR_INVALID, "f[r] is NULL");
    if (!(dt[r] > 0.0) || !std::isfinite(dt[r])) return bfail(b, DG_ERR_INVALID, "dt[r] must be positive and finite");
  }
  // the field of the current states: density partials per run, then one
  // batched field launch pair and one read-back of all records
  for (int r = 0; r < b->nruns; ++r) {
    dg_ctx* c = b->runs[r];
    dg_status s = density(c, f[r]);
    if (s != DG_OK) return bfail(b, s, c->err);
  }
  DGB_HIP(b, dgk::launch_field_batched(b->d_fa0, b->d_xitems, b->nxitems, b->nruns, b->max_pmax, b->stream));
  std::vector<double> last(8 * b->nruns);
  DGB_HIP(b, hipMemcpyAsync(last.data(), b->d_last, last.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  DGB_HIP(b, hipStreamSynchronize(b->stream));
  for (int r = 0; r < b->nruns; ++r) {
    if (!std::isfinite(last[8 * r + 5]) || last[8 * r + 6] == 0.0) {
      char buf[96];
      std::snprintf(buf, sizeof(buf), "run %d: initial field is not finite", r);
      return bfail(b, DG_ERR_NONFINITE, buf);
    }
    const double dtm = dg_dt_max(b->runs[r], last[8 * r + 5]);
    if (dt[r] > dtm) {
      char buf[128];
      std::snprintf(buf, sizeof(buf), "run %d: dt = %.6g exceeds the CFL bound %.6g", r, dt[r], dtm);
      return bfail(b, DG_ERR_CFL, buf);
    }
  }
  return DG_OK;
}

dg_status batch_leave(dg_batch* b) {
  DGB_HIP(b, hipEventRecord(b->ev_out, b->stream));
  DGB_HIP(b, hipStreamWaitEvent(b->user, b->ev_out, 0));
  return DG_OK;
}

}  // namespace

extern "C" {

size_t dg_batch_workspace_bytes(const dg_config* cfgs, int32_t nruns) {
  if (!cfgs || nruns <= 0) return 0;
  for (int r = 0; r < nruns; ++r) {
    dg_status st;
    if (check_cfg(&cfgs[r], &st) || cfgs[r].storage != DG_F32) return 0;
  }
  return batch_layout(cfgs, nruns).total;
}

dg_status dg_batch_init(const dg_config* cfgs, int32_t nruns, void* workspace, size_t workspace_bytes,
                        void* hip_stream, dg_batch** out) {
  auto init_fail = [](dg_status s, const std::string& m) {
    std::lock_guard<std::mutex> lk(g_err_mu);
    g_init_error = m;
    return s;
  };
  if (!out) return init_fail(DG_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!cfgs || nruns <= 0) return init_fail(DG_ERR_INVALID, "need nruns >= 1 configurations");
  for (int r = 0; r < nruns; ++r) {
    dg_status st;
    if (const char* why = check_cfg(&cfgs[r], &st)) return init_fail(st, std::string("run ") + std::to_string(r) + ": " + why);
    if (cfgs[r].storage != DG_F32) return init_fail(DG_ERR_UNSUPPORTED, "batched runs use FP32 storage");
  }
  const BatchLayout BL = batch_layout(cfgs, nruns);
  if (!workspace) return init_fail(DG_ERR_INVALID, "workspace is NULL");
  if (workspace_bytes < BL.total) return init_fail(DG_ERR_OOM, "workspace smaller than dg_batch_workspace_bytes()");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return init_fail(DG_ERR_INVALID, "workspace must be 256-byte aligned");
  dg_batch* b = new (std::nothrow) dg_batch();
  if (!b) return init_fail(DG_ERR_INVALID, "host allocation failed");
  b->nruns = nruns;
  b->ws = static_cast<char*>(workspace);
  b->user = static_cast<hipStream_t>(hip_stream);
  b->run_off = BL.run_off;
  auto cleanup = [&](dg_status s, const std::string& m) {
    for (dg_ctx* c : b->runs) delete c;
    if (b->stream) (void)hipStreamDestroy(b->stream);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    delete b;
    return init_fail(s, m);
  };
  hipError_t e;
  if ((e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking)) != hipSuccess) return cleanup(DG_ERR_DEVICE, "hipStreamCreate");
  if ((e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming)) != hipSuccess) return cleanup(DG_ERR_DEVICE, "hipEventCreate");
  if ((e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming)) != hipSuccess) return cleanup(DG_ERR_DEVICE, "hipEventCreate");
  for (int r = 0; r < nruns; ++r) {
    dg_ctx* c = nullptr;
    std::string err;
    dg_status st = make_ctx(&cfgs[r], b->ws + BL.run_off[r], b->stream, false, &c, &err);
    if (st != DG_OK) return cleanup(st, "run " + std::to_string(r) + ": " + err);
    b->runs.push_back(c);
  }
  b->d_args = reinterpret_cast<dgk::StageArgs<float>*>(b->ws + BL.args);
  b->d_items = reinterpret_cast<int2*>(b->ws + BL.items);
  b->d_xcd = reinterpret_cast<int*>(b->ws + BL.xcd);
  b->d_fa = reinterpret_cast<dgk::FieldArgs*>(b->ws + BL.fa);
  b->d_xitems = reinterpret_cast<int2*>(b->ws + BL.xitems);
  b->d_fa0 = reinterpret_cast<dgk::FieldArgs*>(b->ws + BL.fa0);
  b->d_last = reinterpret_cast<double*>(b->ws + BL.last);
  int dev = 0;
  hipDeviceProp_t prop;
  if ((e = hipGetDevice(&dev)) != hipSuccess || (e = hipGetDeviceProperties(&prop, dev)) != hipSuccess)
    return cleanup(DG_ERR_DEVICE, std::string("device query: ") + hipGetErrorString(e));
  b->cus = prop.multiProcessorCount;
  b->arch = prop.gcnArchName;
  // Kinds: the 1D2V runs by n, in order of decreasing n, then all 1D1V runs
  // (any n) as one kind (code 1).  Within a kind: runs by decreasing tile
  // cost, tiles in order (cost-sorted), or the kind's runs' tiles interleaved
  // round-robin (run-interleaved).
  std::vector<int2> xitems;
  std::vector<int> kinds;
  for (int r = 0; r < nruns; ++r) {
    kinds.push_back(cfgs[r].nv == 2 ? 10 * cfgs[r].n + 2 : 1);
    for (int ix = 0; ix < b->runs[r]->L.Nx; ++ix) xitems.push_back(make_int2(r, ix));
    b->max_pmax = std::max(b->max_pmax, b->runs[r]->L.pmax);
  }
  std::vector<int> distinct(kinds);
  std::sort(distinct.begin(), distinct.end(), [](int p, int q) { return p > q; });
  distinct.erase(std::unique(distinct.begin(), distinct.end()), distinct.end());
  int maxocc = 1;
  for (int kd : distinct) {
    dg_batch::Group g{};
    g.n = kd == 1 ? 0 : kd / 10;   // the 1D1V kind is reported as (n, nv) = (0, 1)
    g.nv = kd == 1 ? 1 : 2;
    g.begin = static_cast<int>(b->items_cost.size());
    std::vector<int> byc;
    for (int r = 0; r < nruns; ++r)
      if (kinds[r] == kd) byc.push_back(r);
    std::stable_sort(byc.begin(), byc.end(), [&](int p, int q) {
      const Layout &A = b->runs[p]->L, &B = b->runs[q]->L;
      return static_cast<double>(A.dof) / A.ntiles > static_cast<double>(B.dof) / B.ntiles;
    });
    for (int r : byc)
      for (int t = 0; t < b->runs[r]->L.ntiles; ++t) b->items_cost.push_back(make_int2(r, t));
    std::vector<int> next(nruns, 0);
    bool any = true;
    while (any) {
      any = false;
      for (int r : byc)
        if (next[r] < b->runs[r]->L.ntiles) {
          b->items_rr.push_back(make_int2(r, next[r]++));
          any = true;
        }
    }
    g.count = static_cast<int>(b->items_cost.size()) - g.begin;
    g.occ[0] = dgk::batched_occupancy(false, g.n, g.nv);
    g.occ[1] = dgk::batched_occupancy(true, g.n, g.nv);
    maxocc = std::max(maxocc, std::min(g.occ[0], g.occ[1]));
    // a tuned choice for this (arch, n, nv, FP32) if one was made in this process
    g.wm = tune_cache_get(b->arch, g.n, g.nv, std::max(1, std::min(g.occ[0], g.occ[1])));
    b->groups.push_back(g);
  }
  (void)maxocc;
  b->nitems = static_cast<int>(b->items_cost.size());
  b->nxitems = static_cast<int>(xitems.size());
  if ((e = hipMemcpyAsync(b->d_xitems, xitems.data(), xitems.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream)) != hipSuccess)
    return cleanup(DG_ERR_DEVICE, std::string("table upload: ") + hipGetErrorString(e));
  // field of the current states (each call's first step needs it): one
  // batched launch pair, every run's record into one contiguous array
  std::vector<dgk::FieldArgs> fa0(nruns);
  for (int r = 0; r < nruns; ++r) {
    dg_ctx* c = b->runs[r];
    fill_field(c, &fa0[r], c->at<double>(c->L.off_E), nullptr, false);
    fa0[r].last = b->d_last + 8 * r;
  }
  if ((e = hipMemcpyAsync(b->d_fa0, fa0.data(), fa0.size() * sizeof(fa0[0]), hipMemcpyHostToDevice, b->stream)) != hipSuccess)
    return cleanup(DG_ERR_DEVICE, std::string("table upload: ") + hipGetErrorString(e));
  if (upload_items(b) != DG_OK) return cleanup(DG_ERR_DEVICE, b->err);
  *out = b;
  return DG_OK;
}

dg_status dg_batch_destroy(dg_batch* b) {
  if (!b) return DG_OK;
  hipError_t e = hipStreamSynchronize(b->stream);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  for (dg_ctx* c : b->runs) (void)dg_destroy(c);
  (void)hipEventDestroy(b->ev_in);
  (void)hipEventDestroy(b->ev_out);
  (void)hipStreamDestroy(b->stream);
  delete b;
  return e == hipSuccess ? DG_OK : DG_ERR_DEVICE;
}

dg_status dg_batch_rk_step(dg_batch* b, void* const* f, const double* dt, int32_t nsteps, dg_diag* host_diag) {
  if (!b) return DG_ERR_INVALID;
  if (!f || !dt) return bfail(b, DG_ERR_INVALID, "f and dt must be non-NULL");
  if (nsteps < 0) return bfail(b, DG_ERR_INVALID, "nsteps < 0");
  if (nsteps == 0) return DG_OK;
  dg_status s = batch_begin(b, f, dt);
  if (s != DG_OK) {
    batch_leave(b);
    return s;
  }
  const bool diag = host_diag != nullptr;
  s = build_batch_graph(b, f, dt, diag);
  if (s != DG_OK) return s;
  int done = 0;
  bool bad = false;
  while (done < nsteps) {
    const int chunk = std::min(nsteps - done, dgk::kRing);
    if (diag)
      for (dg_ctx* c : b->runs) DGB_HIP(b, dgk::launch_reset_counter(c->at<int>(c->L.off_ctr), b->stream));
    for (int k = 0; k < chunk; ++k) DGB_HIP(b, hipGraphLaunch(b->gexec, b->stream));
    if (diag) {
      std::vector<double> ring(static_cast<size_t>(chunk) * 8);
      for (int r = 0; r < b->nruns; ++r) {
        dg_ctx* c = b->runs[r];
        DGB_HIP(b, hipMemcpyAsync(ring.data(), c->at<double>(c->L.off_ring), ring.size() * 8, hipMemcpyDeviceToHost, b->stream));
        DGB_HIP(b, hipStreamSynchronize(b->stream));
        for (int k = 0; k < chunk; ++k) {
          dg_diag* d = &host_diag[static_cast<size_t>(r) * nsteps + done + k];
          copy_record(&ring[static_cast<size_t>(k) * 8], c->t + (done + k + 1) * dt[r], d);
          d->step = done + k;
          if (!d->finite) bad = true;
        }
      }
    }
    done += chunk;
  }
  for (int r = 0; r < b->nruns; ++r) b->runs[r]->t += nsteps * dt[r];
  s = batch_leave(b);
  if (s != DG_OK) return s;
  if (diag) DGB_HIP(b, hipStreamSynchronize(b->stream));
  if (bad) return bfail(b, DG_ERR_NONFINITE, "a step produced non-finite diagnostics");
  return DG_OK;
}

dg_status dg_batch_tune(dg_batch* b, void* const* f, const double* dt, int32_t reps, double* best_ms) {
  if (!b) return DG_ERR_INVALID;
  if (!f || !dt || reps < 1) return bfail(b, DG_ERR_INVALID, "need f, dt and reps >= 1");
  dg_status s = batch_begin(b, f, dt);
  if (s != DG_OK) {
    batch_leave(b);
    return s;
  }
  hipEvent_t e0, e1;
  DGB_HIP(b, hipEventCreate(&e0));
  DGB_HIP(b, hipEventCreate(&e1));
  // mean ms per step of the current choices (graph rebuilt, one warm-up replay)
  auto measure = [&](double* ms_out) -> dg_status {
    dg_status st = upload_items(b);
    if (st != DG_OK) return st;
    drop_graph(b->stream, &b->gexec);
    st = build_batch_graph(b, f, dt, false);
    if (st != DG_OK) return st;
    DGB_HIP(b, hipGraphLaunch(b->gexec, b->stream));
    DGB_HIP(b, hipEventRecord(e0, b->stream));
    for (int k = 0; k < reps; ++k) DGB_HIP(b, hipGraphLaunch(b->gexec, b->stream));
    DGB_HIP(b, hipEventRecord(e1, b->stream));
    DGB_HIP(b, hipEventSynchronize(e1));
    float ms = 0.0f;
    DGB_HIP(b, hipEventElapsedTime(&ms, e0, e1));
    for (int r = 0; r < b->nruns; ++r) b->runs[r]->t += (reps + 1) * dt[r];
    *ms_out = ms / reps;
    return DG_OK;
  };
  auto occ_of = [](const dg_batch::Group& g) { return std::max(1, std::min(g.occ[0], g.occ[1])); };
  // 1. list order, every kind at its occupancy limit
  for (auto& g : b->groups) g.wm = occ_of(g);
  double best = 1e300;
  int best_order = b->order;
  for (int order = 0; order < 2 && s == DG_OK; ++order) {
    b->order = order;
    double ms = 0.0;
    s = measure(&ms);
    if (s == DG_OK && ms < best) {
      best = ms;
      best_order = order;
    }
  }
  b->order = best_order;
  // 2. per kind (n, nv): its launch shape, one kind at a time with the others
  //    at their current best (coordinate descent, largest kinds first): a
  //    persistent grid of 1 .. occupancy work-groups per CU, or one
  //    work-group per tile (wm = 0)
  std::vector<size_t> byc(b->groups.size());
  for (size_t q = 0; q < byc.size(); ++q) byc[q] = q;
  std::stable_sort(byc.begin(), byc.end(), [&](size_t p, size_t q) { return b->groups[p].count > b->groups[q].count; });
  for (size_t q : byc) {
    if (s != DG_OK) break;
    auto& g = b->groups[q];
    int best_w = g.wm;
    std::vector<int> cand;
    for (int w = 1; w < occ_of(g); ++w) cand.push_back(w);
    cand.push_back(0);
    for (int w : cand) {
      if (s != DG_OK) break;
      g.wm = w;
      double ms = 0.0;
      s = measure(&ms);
      if (s == DG_OK && ms < best) {
        best = ms;
        best_w = w;
      }
    }
    g.wm = best_w;
  }
  // 3. the other list order once more, under the launch shapes chosen in 2
  if (s == DG_OK) {
    b->order = 1 - b->order;
    double ms = 0.0;
    s = measure(&ms);
    if (s == DG_OK && ms < best) best = ms;
    else b->order = 1 - b->order;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != DG_OK) return s;
  for (const auto& g : b->groups) tune_cache_put(b->arch, g.n, g.nv, g.wm);
  s = upload_items(b);
  if (s != DG_OK) return s;
  drop_graph(b->stream, &b->gexec);
  if (best_ms) *best_ms = best;
  return batch_leave(b);
}

int32_t dg_batch_choice(const dg_batch* b, int32_t* host_out) {
  if (!b) return 0;
  const int nk = static_cast<int>(b->groups.size());
  if (host_out) {
    host_out[0] = 0;   // kinds' launches one after another
    host_out[1] = b->order;
    for (int q = 0; q < nk; ++q) {
      host_out[2 + 4 * q] = b->groups[q].n;
      host_out[3 + 4 * q] = b->groups[q].nv;
      host_out[4 + 4 * q] = b->groups[q].wm;
      host_out[5 + 4 * q] = b->groups[q].grid;
    }
  }
  return nk;
}

dg_status dg_batch_set_choice(dg_batch* b, const int32_t* choice, int32_t nint) {
  if (!b) return DG_ERR_INVALID;
  const int nk = static_cast<int>(b->groups.size());
  if (!choice || nint != 2 + 4 * nk) return bfail(b, DG_ERR_INVALID, "dg_batch_set_choice: need 2 + 4 * kinds ints");
  if (choice[0] == 1)
    return bfail(b, DG_ERR_UNSUPPORTED, "dg_batch_set_choice: concurrent kind launches are switched off");
  if (choice[0] != 0 || (choice[1] != 0 && choice[1] != 1))
    return bfail(b, DG_ERR_INVALID, "dg_batch_set_choice: concurrent and order must be 0 or 1");
  for (int q = 0; q < nk; ++q) {
    const auto& g = b->groups[q];
    if (choice[2 + 4 * q] != g.n || choice[3 + 4 * q] != g.nv)
      return bfail(b, DG_ERR_INVALID, "dg_batch_set_choice: kinds differ from this batch's");
    if (choice[4 + 4 * q] < 0)
      return bfail(b, DG_ERR_INVALID, "dg_batch_set_choice: work-groups per CU must be >= 0 (0: one per tile)");
  }
  b->order = choice[1];
  for (int q = 0; q < nk; ++q) b->groups[q].wm = choice[4 + 4 * q];
  drop_graph(b->stream, &b->gexec);
  return upload_items(b);
}

int32_t dg_batch_grid(const dg_batch* b) {
  if (!b) return 0;
  int total = 0;
  for (const auto& g : b->groups) total += g.grid;
  return total;
}

const char* dg_batch_last_error(const dg_batch* b) {
  if (b) return b->err.c_str();
  std::lock_guard<std::mutex> lk(g_err_mu);
  return g_init_error.c_str();
}

}  // extern "C"
