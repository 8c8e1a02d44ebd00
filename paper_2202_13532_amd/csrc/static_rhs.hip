// dg_rhs_static: the right-hand side of dg_rhs without a context or a caller
// workspace, for callers that cannot allocate device memory.  Its scratch
// (node tables, connection tensor, density partials, Fourier partials, E)
// lives in a file-scope device array, one copy per GPU, whose device address
// is looked up once per device and passed to the kernels.  The tables that
// dg_init computes on the host are built here by a device kernel from the
// same formulas (LGL nodes and weights as compile-time constants, the
// connection tensor of eq. spectral_transform), so no host-to-device copy is
// needed either.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <mutex>
#include <string>

#include "../../include/dg.h"
#include "ctx.h"
#include "dg_kernels.h"
#include "dg_ops_constexpr.h"
#include "spherical_bessel.h"

namespace {

constexpr size_t kScratchBytes = size_t(8) << 20;   // DG_RHS_STATIC_SCRATCH_BYTES
static_assert(kScratchBytes == DG_RHS_STATIC_SCRATCH_BYTES, "scratch size mismatch with dg.h");

// Host code must not pass `scratch` itself to a kernel (in host code the name
// stands for a host-side shadow): kernels receive the address returned by
// hipGetSymbolAddress for the current device.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_base[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
dg_status scratch_base(char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return dgi::global_fail(DG_ERR_DEVICE, std::string("dg_rhs_static: hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return dgi::global_fail(DG_ERR_DEVICE, "dg_rhs_static: device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_base[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return dgi::global_fail(DG_ERR_DEVICE, std::string("dg_rhs_static: hipGetSymbolAddress: ") + hipGetErrorString(e));
    g_base[dev] = p;
  }
  *out = static_cast<char*>(g_base[dev]);
  return DG_OK;
}

// Node tables and the connection tensor in the layout make_ctx uploads.
struct TableArgs {
  double *wx, *wu, *wv, *uc64, *vc64, *T, *z1;
  void *uc, *vc;   // storage precision
  int nv, f64, Nx, Nu, Nv, pmax;
  double lo[3], hi[3];
};

template <int N>
__global__ void __launch_bounds__(256) tables_kernel(TableArgs a) {
  constexpr dgc::OpsC<N> K = dgc::make_ops<N>();
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int nxn = a.Nx * N;
  // node coordinates and quadrature weights of axis `ax` (element m, node j)
  auto axis = [&](int ax, int Ne, long long q, double* w, double* c64, void* c) {
    const int m = static_cast<int>(q / N), j = static_cast<int>(q % N);
    const double d = (a.hi[ax] - a.lo[ax]) / Ne;
    const double x = a.lo[ax] + (m + 0.5) * d + K.xi[j] * 0.5 * d;
    w[q] = K.w[j] * 0.5 * d;
    c64[q] = x;
    if (a.f64) static_cast<double*>(c)[q] = x;
    else static_cast<float*>(c)[q] = static_cast<float>(x);
  };
  if (i < nxn) {
    const int m = static_cast<int>(i / N), j = static_cast<int>(i % N);
    const double d = (a.hi[0] - a.lo[0]) / a.Nx;
    a.wx[i] = K.w[j] * 0.5 * d;
    const double x = a.lo[0] + (m + 0.5) * d + K.xi[j] * 0.5 * d;
    double sn, cs;
    sincos(2.0 * dgc::kPi / (a.hi[0] - a.lo[0]) * x, &sn, &cs);
    a.z1[2 * i] = cs;
    a.z1[2 * i + 1] = sn;
  }
  if (a.nv == 2) {
    if (i < a.Nu * N) axis(1, a.Nu, i, a.wu, a.uc64, a.uc);
    if (i < a.Nv * N) axis(2, a.Nv, i, a.wv, a.vc64, a.vc);
  } else {
    if (i < N) {   // no u axis: unit weights, zero coordinates
      a.wu[i] = 1.0;
      a.uc64[i] = 0.0;
      if (a.f64) static_cast<double*>(a.uc)[i] = 0.0;
      else static_cast<float*>(a.uc)[i] = 0.0f;
    }
    if (i < a.Nv * N) axis(1, a.Nv, i, a.wv, a.vc64, a.vc);
  }
  // T_p^{mj} = (dx/L) e^{-i k_p xbar_m} w_j sum_s gamma_s^-1 (-i)^s P_s(xi_j) j_s(k_p / J),
  // stored node-major: [(m n + j) pmax + p - 1]
  if (i < static_cast<long long>(nxn) * a.pmax) {
    const int q = static_cast<int>(i / a.pmax), p = static_cast<int>(i % a.pmax) + 1;
    const int m = q / N, j = q % N;
    const double L = a.hi[0] - a.lo[0], d = L / a.Nx, J = 2.0 / d;
    const double kp = 2.0 * dgc::kPi * p / L;
    double re = 0.0, im = 0.0;
    for (int s = 0; s < N; ++s) {
      const double gam = s < N - 1 ? 2.0 / (2.0 * s + 1.0) : 2.0 / (N - 1.0);
      const double v = dgc::c_leg(s, K.xi[j]) * dgh::sph_bessel_j(s, kp / J) / gam;
      switch (s % 4) {   // (-i)^s
        case 0: re += v; break;
        case 1: im -= v; break;
        case 2: re -= v; break;
        default: im += v; break;
      }
    }
    re *= K.w[j];
    im *= K.w[j];
    double sn, cs;
    sincos(-kp * (a.lo[0] + (m + 0.5) * d), &sn, &cs);
    const double pr = d / L * cs, pi = d / L * sn;
    a.T[2 * i] = pr * re - pi * im;
    a.T[2 * i + 1] = pr * im + pi * re;
  }
}

hipError_t launch_tables(int n, const TableArgs& a, long long threads, hipStream_t s) {
  const unsigned grid = static_cast<unsigned>((threads + 255) / 256);
  switch (n) {
#define DG_TAB_CASE(NN) \
  case NN: hipLaunchKernelGGL(tables_kernel<NN>, dim3(grid), dim3(256), 0, s, a); break;
    DG_TAB_CASE(2) DG_TAB_CASE(3) DG_TAB_CASE(4) DG_TAB_CASE(5) DG_TAB_CASE(6) DG_TAB_CASE(7) DG_TAB_CASE(8)
    DG_TAB_CASE(9) DG_TAB_CASE(10) DG_TAB_CASE(11) DG_TAB_CASE(12)
#undef DG_TAB_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

extern "C" {

dg_status dg_rhs_static(const dg_config* cfg, const void* f, const double* E, void* rhs, void* hip_stream) {
  dg_status st;
  if (const char* why = dgi::config_error(cfg, &st)) return dgi::global_fail(st, std::string("dg_rhs_static: ") + why);
  if (!f || !rhs) return dgi::global_fail(DG_ERR_INVALID, "dg_rhs_static: f and rhs must be non-NULL");
  if (f == rhs) return dgi::global_fail(DG_ERR_INVALID, "dg_rhs_static: f and rhs must not overlap");
  const dgi::Layout L = dgi::scratch_layout(cfg);
  if (L.total > kScratchBytes) {
    char buf[192];
    std::snprintf(buf, sizeof(buf),
                  "dg_rhs_static: this configuration needs %zu bytes of scratch, above the maximum of %zu bytes",
                  L.total, kScratchBytes);
    return dgi::global_fail(DG_ERR_OOM, buf);
  }
  char* base = nullptr;
  if ((st = scratch_base(&base)) != DG_OK) return st;
  // a context on the host stack over the scratch array: no device allocation
  dg_ctx c;
  c.cfg = *cfg;
  c.L = L;
  c.ws = base;
  c.user = c.stream = static_cast<hipStream_t>(hip_stream);
  c.owns_stream = false;
  for (int a = 0; a <= cfg->nv; ++a) c.dx[a] = (cfg->hi[a] - cfg->lo[a]) / cfg->nelem[a];
  TableArgs ta{};
  ta.wx = c.at<double>(L.off_wx);
  ta.wu = c.at<double>(L.off_wu);
  ta.wv = c.at<double>(L.off_wv);
  ta.uc64 = c.at<double>(L.off_uc64);
  ta.vc64 = c.at<double>(L.off_vc64);
  ta.uc = c.ws + L.off_uc;
  ta.vc = c.ws + L.off_vc;
  ta.T = c.at<double>(L.off_T);
  ta.z1 = c.at<double>(L.off_z1);
  ta.nv = cfg->nv;
  ta.f64 = c.f64() ? 1 : 0;
  ta.Nx = L.Nx;
  ta.Nu = L.Nu;
  ta.Nv = L.Nv;
  ta.pmax = L.pmax;
  for (int a = 0; a < 3; ++a) {
    ta.lo[a] = cfg->lo[a];
    ta.hi[a] = cfg->hi[a];
  }
  long long threads = static_cast<long long>(L.Nx) * L.n * L.pmax;
  threads = std::max(threads, static_cast<long long>(std::max(L.Nu, L.Nv)) * L.n);
  hipError_t e = launch_tables(L.n, ta, threads, c.stream);
  if (e != hipSuccess) return dgi::global_fail(DG_ERR_DEVICE, std::string("dg_rhs_static: table kernel launch: ") + hipGetErrorString(e));
  const double* Ef = E;
  if (!Ef) {
    double* Es = c.at<double>(L.off_E);
    if ((st = dgi::density(&c, f)) != DG_OK || (st = dgi::field(&c, Es, nullptr, false)) != DG_OK)
      return dgi::global_fail(st, "dg_rhs_static: " + c.err);
    Ef = Es;
  }
  if ((st = dgi::stage(&c, f, nullptr, rhs, Ef, nullptr, 0.0, 0.0, 1.0)) != DG_OK)
    return dgi::global_fail(st, "dg_rhs_static: " + c.err);
  return DG_OK;
}

}  // extern "C"
