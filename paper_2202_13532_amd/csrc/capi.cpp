// C ABI of the DG Vlasov-Poisson library: configuration checks, workspace
// layout, host setup uploads, stage orchestration and HIP-graph replay of
// SSP-RK3 steps.  Every entry point is declared and documented in dg.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/dg.h"
#include "dg_host.h"
#include "dg_kernels.h"

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

std::mutex g_err_mu;
std::string g_init_error = "no error";

// Workspace layout derived from a validated configuration.
struct Layout {
  size_t esize = 0, dof = 0;
  int naxes = 0, n = 0, Nx = 0, Nu = 1, Nv = 0, nvchunks = 0, pmax = 0;
  int ntiles_slab = 0, ntiles = 0;
  size_t off_B, off_C, off_part, off_mom, off_dens, off_E, off_cpart, off_mpart, off_coef, off_ring,
      off_last, off_ctr, off_T, off_z1, off_wx, off_wu, off_wv, off_uc, off_vc, off_uc64, off_vc64, total;
};

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
  if (c->reserved != 0) return "reserved must be 0";
  return nullptr;
}

Layout make_layout(const dg_config* c) {
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
  const size_t nx = static_cast<size_t>(L.Nx) * L.n;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += align_up(bytes); return r; };
  L.off_B = take(L.dof * L.esize);
  L.off_C = take(L.dof * L.esize);
  L.off_part = take(nx * L.ntiles_slab * 8);
  L.off_mom = take(static_cast<size_t>(L.ntiles) * 4 * 8);
  L.off_dens = take(nx * 8);
  L.off_E = take(nx * 8);
  L.off_cpart = take(static_cast<size_t>(L.Nx) * L.pmax * 16);
  L.off_mpart = take(static_cast<size_t>(L.Nx) * 8);
  L.off_coef = take(static_cast<size_t>(L.pmax) * 16);
  L.off_ring = take(static_cast<size_t>(dgk::kRing) * 64);
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
  L.total = o;
  return L;
}

}  // namespace

struct dg_ctx {
  dg_config cfg{};
  Layout L;
  dgh::Basis basis;
  double courant = 0.0;
  double dx[3] = {0, 0, 0};
  char* ws = nullptr;
  hipStream_t user = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  double t = 0.0;
  std::string err = "no error";
  // cached step graph
  hipGraphExec_t gexec = nullptr;
  const void* g_f = nullptr;
  double g_dt = 0.0;
  bool g_diag = false;

  template <typename P> P* at(size_t off) const { return reinterpret_cast<P*>(ws + off); }
  bool f64() const { return cfg.storage == DG_F64; }
};

namespace {

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
  a.hu = c->cfg.nv == 2 ? 0.5 * c->dx[1] : 1.0;
  a.Nx = L.Nx;
  a.Nu = L.Nu;
  a.Nv = L.Nv;
  a.nvchunks = L.nvchunks;
  a.zero_inflow = c->cfg.vbc == DG_VBC_ZERO_INFLOW ? 1 : 0;
  a.Jx = static_cast<T>(2.0 / c->dx[0]);
  if (c->cfg.nv == 2) {
    a.Ju = static_cast<T>(2.0 / c->dx[1]);
    a.Jv = static_cast<T>(2.0 / c->dx[2]);
  } else {
    a.Ju = T(0);
    a.Jv = static_cast<T>(2.0 / c->dx[1]);
  }
  a.wc = static_cast<T>(c->cfg.omega_c);
  a.c_un = static_cast<T>(c_un);
  a.c_in = static_cast<T>(c_in);
  a.c_dt = static_cast<T>(c_dt);
}

// One fused stage kernel: out = c_un un + c_in fin + c_dt L(fin) (L with field E).
dg_status stage(dg_ctx* c, const void* fin, const void* fun, void* out, const double* E,
                double* partials, double c_un, double c_in, double c_dt) {
  hipError_t e;
  if (c->f64()) {
    dgk::StageArgs<double> p;
    fill_pack(c, &p, fin, fun, out, E, partials, c_un, c_in, c_dt);
    e = dgk::launch_stage(c->cfg.nv, c->L.n, true, &p, c->L.ntiles, c->stream);
  } else {
    dgk::StageArgs<float> p;
    fill_pack(c, &p, fin, fun, out, E, partials, c_un, c_in, c_dt);
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

dg_status field(dg_ctx* c, double* E, double* coeffs, bool record) {
  const Layout& L = c->L;
  dgk::FieldArgs a{};
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
dg_status enqueue_step(dg_ctx* c, void* f, double dt, bool diag) {
  void* B = c->ws + c->L.off_B;
  void* C = c->ws + c->L.off_C;
  double* E = c->at<double>(c->L.off_E);
  double* part = c->at<double>(c->L.off_part);
  DG_TRY(stage(c, f, nullptr, B, E, part, 0.0, 1.0, dt));
  DG_TRY(field(c, E, nullptr, false));
  DG_TRY(stage(c, B, f, C, E, part, 0.75, 0.25, 0.25 * dt));
  DG_TRY(field(c, E, nullptr, false));
  DG_TRY(stage(c, C, f, f, E, part, 1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0 * dt));
  DG_TRY(field(c, E, nullptr, diag));
  if (diag) DG_TRY(moments(c, f));
  return DG_OK;
}

dg_status build_graph(dg_ctx* c, void* f, double dt, bool diag) {
  if (c->gexec && c->g_f == f && c->g_dt == dt && c->g_diag == diag) return DG_OK;
  if (c->gexec) {
    hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
  DG_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  dg_status s = enqueue_step(c, f, dt, diag);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (s != DG_OK) {
    if (g) hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) {
    c->gexec = nullptr;
    return hip_fail(c, e, "hipGraphInstantiate");
  }
  c->g_f = f;
  c->g_dt = dt;
  c->g_diag = diag;
  return DG_OK;
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

}  // namespace

extern "C" {

size_t dg_workspace_bytes(const dg_config* cfg) {
  if (validate(cfg)) return 0;
  if (cfg->n > dgk::kMaxN) return 0;
  return make_layout(cfg).total;
}

dg_status dg_init(const dg_config* cfg, void* workspace, size_t workspace_bytes, void* hip_stream, dg_ctx** out) {
  auto init_fail = [](dg_status s, const std::string& m) {
    std::lock_guard<std::mutex> lk(g_err_mu);
    g_init_error = m;
    return s;
  };
  if (!out) return init_fail(DG_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (const char* why = validate(cfg)) return init_fail(DG_ERR_INVALID, why);
  if (cfg->n > dgk::kMaxN) return init_fail(DG_ERR_UNSUPPORTED, "n above 9 is not built");
  const Layout L = make_layout(cfg);
  if (!workspace) return init_fail(DG_ERR_INVALID, "workspace is NULL");
  if (workspace_bytes < L.total) return init_fail(DG_ERR_OOM, "workspace smaller than dg_workspace_bytes()");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return init_fail(DG_ERR_INVALID, "workspace must be 256-byte aligned");
  if (L.ntiles <= 0 || static_cast<long long>(L.Nx) * L.ntiles_slab > 0x7fffffffLL)
    return init_fail(DG_ERR_UNSUPPORTED, "grid too large");

  dg_ctx* c = new (std::nothrow) dg_ctx();
  if (!c) return init_fail(DG_ERR_INVALID, "host allocation failed");
  c->cfg = *cfg;
  c->L = L;
  c->ws = static_cast<char*>(workspace);
  c->user = static_cast<hipStream_t>(hip_stream);
  try {
    c->basis = dgh::make_basis(cfg->n);
    c->courant = dgh::courant_number(cfg->n);
  } catch (const std::exception& ex) {
    delete c;
    return init_fail(DG_ERR_INVALID, std::string("basis setup failed: ") + ex.what());
  }
  for (int a = 0; a <= cfg->nv; ++a) c->dx[a] = (cfg->hi[a] - cfg->lo[a]) / cfg->nelem[a];

  auto cleanup = [&](hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (c->stream) hipStreamDestroy(c->stream);
    if (c->ev_in) hipEventDestroy(c->ev_in);
    if (c->ev_out) hipEventDestroy(c->ev_out);
    delete c;
    return init_fail(DG_ERR_DEVICE, m);
  };
  hipError_t e;
  if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess) return cleanup(e, "hipStreamCreate");
  if ((e = hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming)) != hipSuccess) return cleanup(e, "hipEventCreate");
  if ((e = hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming)) != hipSuccess) return cleanup(e, "hipEventCreate");

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

dg_status dg_destroy(dg_ctx* ctx) {
  if (!ctx) return DG_OK;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (ctx->gexec) hipGraphExecDestroy(ctx->gexec);
  hipEventDestroy(ctx->ev_in);
  hipEventDestroy(ctx->ev_out);
  hipStreamDestroy(ctx->stream);
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

namespace {
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
}  // namespace

dg_status dg_rk_step(dg_ctx* ctx, void* f, double dt, int32_t nsteps, dg_diag* host_diag) {
  if (!ctx) return DG_ERR_INVALID;
  if (nsteps == 0 && f && dt > 0.0) return DG_OK;
  DG_TRY(begin_steps(ctx, f, dt, nsteps));
  const Layout& L = ctx->L;
  const bool diag = host_diag != nullptr;
  DG_TRY(build_graph(ctx, f, dt, diag));
  int done = 0;
  bool bad = false;
  while (done < nsteps) {
    const int chunk = std::min(nsteps - done, dgk::kRing);
    if (diag) {
      hipError_t e = dgk::launch_reset_counter(ctx->at<int>(L.off_ctr), ctx->stream);
      if (e != hipSuccess) return hip_fail(ctx, e, "counter reset");
    }
    for (int s = 0; s < chunk; ++s) DG_HIP(ctx, hipGraphLaunch(ctx->gexec, ctx->stream));
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
      st = stage(ctx, ins[k], f, outs[k], E, part, cu[k], ci[k], cd[k]);
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
  for (auto& e : ev) hipEventDestroy(e);
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
