// C ABI of the learned coarse-grid correction: the per-element network
// (BF16 MFMA forward / backward, AdamW), the fine -> coarse L2 projection used
// to build its training data, the feature gather and the corrected coarse
// SSP-RK3 step.  Every entry point is declared and documented in dg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/dg.h"
#include "ctx.h"
#include "dg_host.h"
#include "dg_kernels.h"
#include "nn_kernels.h"

namespace {

constexpr size_t kAlign = 256;
constexpr int kMseBlocks = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
inline int pad16(int x) { return (x + 15) / 16 * 16; }

std::mutex g_nn_mu;
std::string g_nn_init_error = "no error";

struct NNLayout {
  int L = 0, max_rows = 0, wmax = 0, ldmax = 0;
  std::vector<int> sizes, ld;
  std::vector<size_t> offW, offb;     // element offsets into the parameter vector
  size_t nparam = 0;
  size_t off_P, off_Pbf, off_G, off_m, off_v, off_Ytmp, off_dA, off_dZ, off_dZb, off_loss, off_sum, off_sumsq,
      off_Xf, off_Yo, off_corr, off_xm1, off_xm2, off_gpart, off_cpart, total;
  size_t gpart_floats = 0;   // split-K scratch of the GEMMs
  std::vector<size_t> off_A, off_Z;   // A[l]: BF16 input of layer l (l >= 1); Z[l]: pre-activation of layer l
  std::vector<int> kp;                // K of layer l padded to a multiple of 32 (fused inference)
  std::vector<size_t> off_Wt;         // layer l's weights transposed, out x kp BF16 (fused inference)
  bool fusable = false;               // the shape fits the fused inference kernel
};

const char* nn_validate(const int32_t* sizes, int32_t nlayers, int32_t max_rows) {
  if (!sizes) return "sizes is NULL";
  if (nlayers < 1 || nlayers > 16) return "nlayers must be in 1..16";
  for (int l = 0; l <= nlayers; ++l)
    if (sizes[l] < 1 || sizes[l] > 8192) return "layer widths must be in 1..8192";
  if (max_rows < 1 || max_rows > (1 << 24)) return "max_rows must be in 1..2^24";
  return nullptr;
}

NNLayout nn_layout(const int32_t* sizes, int32_t nlayers, int32_t max_rows) {
  NNLayout N;
  N.L = nlayers;
  N.max_rows = max_rows;
  N.sizes.assign(sizes, sizes + nlayers + 1);
  for (int l = 0; l <= nlayers; ++l) N.ld.push_back(pad16(sizes[l]));
  for (int l = 0; l < nlayers; ++l) {
    N.offW.push_back(N.nparam);
    N.nparam += static_cast<size_t>(sizes[l]) * sizes[l + 1];
    N.offb.push_back(N.nparam);
    N.nparam += sizes[l + 1];
  }
  for (int l = 1; l <= nlayers; ++l) {
    N.wmax = std::max(N.wmax, sizes[l]);
    N.ldmax = std::max(N.ldmax, N.ld[l]);
  }
  const size_t R = static_cast<size_t>(max_rows);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += align_up(bytes); return r; };
  N.off_P = take(N.nparam * 4);
  N.off_Pbf = take(N.nparam * 2);
  N.off_G = take(N.nparam * 4);
  N.off_m = take(N.nparam * 4);
  N.off_v = take(N.nparam * 4);
  N.off_A.assign(nlayers + 1, 0);
  N.off_Z.assign(nlayers + 1, 0);
  for (int l = 1; l < nlayers; ++l) N.off_A[l] = take(R * N.ld[l] * 2);
  for (int l = 0; l + 1 < nlayers; ++l) N.off_Z[l] = take(R * sizes[l + 1] * 4);
  N.off_Ytmp = take(R * N.wmax * 4);
  N.off_dA = take(R * N.wmax * 4);
  N.off_dZ = take(R * N.wmax * 4);
  N.off_dZb = take(R * N.ldmax * 2);
  N.off_loss = take(kMseBlocks * 8);
  const int cmax = std::max(N.ld[0], N.ldmax);
  N.off_sum = take(static_cast<size_t>(cmax) * 8);
  N.off_sumsq = take(static_cast<size_t>(cmax) * 8);
  N.off_Xf = take(R * N.ld[0] * 2);
  N.off_Yo = take(R * sizes[nlayers] * 4);
  N.off_corr = take(R * sizes[nlayers] * 4);
  N.off_xm1 = take(R * sizes[nlayers] * 4);
  N.off_xm2 = take(R * sizes[nlayers] * 4);
  size_t wmm = 0;
  for (int l = 0; l < nlayers; ++l) wmm = std::max(wmm, static_cast<size_t>(sizes[l]) * sizes[l + 1]);
  N.gpart_floats = std::max(4 * R * static_cast<size_t>(N.wmax), 32 * wmm);
  N.off_gpart = take(N.gpart_floats * 4);
  N.off_cpart = take(static_cast<size_t>(dgn::kColsumPart) * N.wmax * 4);
  N.fusable = nlayers <= dgn::kMlpMaxLayers && ((sizes[0] + 31) / 32) * 32 <= dgn::kMlpMaxIn;
  for (int l = 0; l < nlayers; ++l) {
    N.kp.push_back((sizes[l] + 31) / 32 * 32);
    if (sizes[l + 1] > dgn::kMlpMaxOut) N.fusable = false;
  }
  for (int l = 0; l < nlayers; ++l) N.off_Wt.push_back(N.fusable ? take(static_cast<size_t>(sizes[l + 1]) * N.kp[l] * 2) : 0);
  N.total = o;
  return N;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_q from the
// Chebyshev guesses); exact for polynomials of degree <= 2q - 1.
void gauss_legendre(int q, std::vector<double>* x, std::vector<double>* w) {
  x->assign(q, 0.0);
  w->assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    double t = -std::cos(M_PI * (i + 0.75) / (q + 0.5));
    for (int it = 0; it < 100; ++it) {
      const double dt = dgh::legendre(q, t) / dgh::legendre_deriv(q, t);
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    const double d = dgh::legendre_deriv(q, t);
    (*x)[i] = t;
    (*w)[i] = 2.0 / ((1.0 - t * t) * d * d);
  }
}

double lagrange(const std::vector<double>& nodes, int i, double x) {
  double v = 1.0;
  for (size_t k = 0; k < nodes.size(); ++k)
    if (static_cast<int>(k) != i) v *= (x - nodes[k]) / (nodes[i] - nodes[k]);
  return v;
}

// One-axis L2 projection from r fine elements (nf LGL nodes each) onto the
// coarse element that contains them (nc LGL nodes): P = Mc^{-1} B with the
// exact mass matrix Mc_ij = int l^c_i l^c_j and coupling B_ik = int l^c_i l^f_k
// over the coarse reference element, both by Gauss-Legendre quadrature on each
// fine sub-element.  Row-major nc x (r nf).
std::vector<double> projection_matrix(int nc, int nf, int r) {
  const dgh::Basis bc = dgh::make_basis(nc), bf = dgh::make_basis(nf);
  std::vector<double> gx, gw;
  gauss_legendre(nc + nf + 4, &gx, &gw);
  const int span = r * nf;
  std::vector<double> M(static_cast<size_t>(nc) * nc, 0.0), B(static_cast<size_t>(nc) * span, 0.0);
  for (int s = 0; s < r; ++s) {
    const double a = -1.0 + 2.0 * s / r, b = -1.0 + 2.0 * (s + 1) / r;
    for (size_t q = 0; q < gx.size(); ++q) {
      const double x = 0.5 * (a + b) + 0.5 * (b - a) * gx[q];
      const double wq = 0.5 * (b - a) * gw[q];
      for (int i = 0; i < nc; ++i) {
        const double li = lagrange(bc.xi, i, x) * wq;
        for (int j = 0; j < nc; ++j) M[i * nc + j] += li * lagrange(bc.xi, j, x);
        for (int k = 0; k < nf; ++k) B[i * span + s * nf + k] += li * lagrange(bf.xi, k, gx[q]);
      }
    }
  }
  // Gaussian elimination with partial pivoting on [M | B].
  for (int col = 0; col < nc; ++col) {
    int piv = col;
    for (int i = col + 1; i < nc; ++i)
      if (std::fabs(M[i * nc + col]) > std::fabs(M[piv * nc + col])) piv = i;
    if (piv != col) {
      for (int j = 0; j < nc; ++j) std::swap(M[col * nc + j], M[piv * nc + j]);
      for (int j = 0; j < span; ++j) std::swap(B[col * span + j], B[piv * span + j]);
    }
    for (int i = 0; i < nc; ++i) {
      if (i == col) continue;
      const double f = M[i * nc + col] / M[col * nc + col];
      for (int j = 0; j < nc; ++j) M[i * nc + j] -= f * M[col * nc + j];
      for (int j = 0; j < span; ++j) B[i * span + j] -= f * B[col * span + j];
    }
  }
  for (int i = 0; i < nc; ++i)
    for (int j = 0; j < span; ++j) B[i * span + j] /= M[i * nc + i];
  return B;
}

}  // namespace

struct dg_nn {
  NNLayout N;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  int cus = 256;   // compute units of the device (split-K sizing)
  int64_t t = 0;   // AdamW step count
  bool have_grads = false;
  bool wt_stale = true;   // the transposed weight copies lag the parameters
  bool fused = true;      // inference through the fused kernel when the shape fits
  std::string err = "no error";
  // cached graph of one corrected coarse step and what it was captured for
  hipGraphExec_t gexec = nullptr;
  uint64_t g_ctx = 0;                 // id of the coarse context it was captured for
  const void* g_f = nullptr;
  const void* g_mean = nullptr;
  const void* g_inv = nullptr;
  double g_dt = 0.0;
  float g_scale = 0.0f;
  bool g_diag = false;
  template <typename P> P* at(size_t off) const { return reinterpret_cast<P*>(ws + off); }
};

namespace {

dg_status nfail(dg_nn* nn, dg_status s, const std::string& m) {
  if (nn) nn->err = m;
  return s;
}

#define NN_HIP(nn, expr)                                                                   \
  do {                                                                                     \
    hipError_t e__ = (expr);                                                               \
    if (e__ != hipSuccess) return nfail(nn, DG_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e__)); \
  } while (0)

#define NN_TRY(expr)              \
  do {                            \
    dg_status s__ = (expr);       \
    if (s__ != DG_OK) return s__; \
  } while (0)

dgn::GemmArgs gemm(const uint16_t* A, size_t sam, size_t sak, const uint16_t* B, size_t sbk, size_t sbn, float* C,
                   size_t scm, int M, int Nn, int K) {
  dgn::GemmArgs g{};
  g.A = A;
  g.B = B;
  g.C = C;
  g.sam = sam;
  g.sak = sak;
  g.sbk = sbk;
  g.sbn = sbn;
  g.scm = scm;
  g.scn = 1;
  g.M = M;
  g.N = Nn;
  g.K = K;
  g.beta = 0.0f;
  return g;
}

hipError_t run_gemm(dg_nn* nn, const dgn::GemmArgs& g, hipStream_t s) {
  return dgn::launch_gemm_tiled(g, nn->at<float>(nn->N.off_gpart), nn->N.gpart_floats, nn->cus, s);
}

// Forward pass on `s`: X (rows x ld[0] BF16) -> Y (rows x sizes[L] FP32).  With
// `keep`, the pre-activations are stored for the backward pass.
dg_status forward_on(dg_nn* nn, const uint16_t* X, int rows, float* Y, bool keep, hipStream_t s) {
  const NNLayout& N = nn->N;
  const uint16_t* A = X;
  for (int l = 0; l < N.L; ++l) {
    const int in = N.sizes[l], out = N.sizes[l + 1];
    const bool last = l == N.L - 1;
    // bias, GELU and the BF16 copy for the next layer in the GEMM's epilogue
    // (the activation buffers' padding columns are zero from initialisation
    // and never written)
    dgn::GemmArgs g = gemm(A, N.ld[l], 1, nn->at<uint16_t>(N.off_Pbf) + N.offW[l], out, 1, nullptr, out, rows, out, in);
    g.epi = 1;
    g.gelu = last ? 0 : 1;
    g.bias = nn->at<float>(N.off_P) + N.offb[l];
    g.Z = (!last && keep) ? nn->at<float>(N.off_Z[l]) : nullptr;
    g.Af = last ? Y : nullptr;
    g.Abf = last ? nullptr : nn->at<uint16_t>(N.off_A[l + 1]);
    g.lda = N.ld[l + 1];
    NN_HIP(nn, run_gemm(nn, g, s));
    if (!last) A = nn->at<uint16_t>(N.off_A[l + 1]);
  }
  return DG_OK;
}

// Transposed BF16 weight copies for the fused kernel, if the parameters
// changed since they were made (enqueued on s).
dg_status refresh_wt(dg_nn* nn, hipStream_t s) {
  const NNLayout& N = nn->N;
  if (!N.fusable || !nn->wt_stale) return DG_OK;
  for (int l = 0; l < N.L; ++l)
    NN_HIP(nn, dgn::launch_transpose_weights(nn->at<uint16_t>(N.off_Pbf) + N.offW[l], N.sizes[l], N.sizes[l + 1], N.kp[l],
                                             nn->at<uint16_t>(N.off_Wt[l]), s));
  nn->wt_stale = false;
  return DG_OK;
}

// Inference Y = NN(X): one fused launch when the shape fits (and fused
// inference is on), else one GEMM launch per layer.  The transposed weights
// must be current (refresh_wt).
dg_status forward_infer(dg_nn* nn, const uint16_t* X, int rows, float* Y, hipStream_t s) {
  const NNLayout& N = nn->N;
  if (!N.fusable || !nn->fused) return forward_on(nn, X, rows, Y, false, s);
  if (nn->wt_stale) return nfail(nn, DG_ERR_INVALID, "internal: transposed weights are stale");
  dgn::MlpArgs a{};
  a.X = X;
  a.ldx = N.ld[0];
  a.rows = rows;
  a.L = N.L;
  for (int l = 0; l < N.L; ++l) {
    a.in[l] = N.sizes[l];
    a.out[l] = N.sizes[l + 1];
    a.kp[l] = N.kp[l];
    a.Wt[l] = nn->at<uint16_t>(N.off_Wt[l]);
    a.bias[l] = nn->at<float>(N.off_P) + N.offb[l];
  }
  a.Y = Y;
  NN_HIP(nn, dgn::launch_mlp_fused(a, s));
  return DG_OK;
}

dg_status check_rows(dg_nn* nn, int rows) {
  if (rows < 1 || rows > nn->N.max_rows) return nfail(nn, DG_ERR_INVALID, "rows must be in 1..max_rows");
  return DG_OK;
}

// The coarse grid of a correction must be 1D2V FP32 with n^3 outputs and
// 7 n^3 + n inputs.
// The coarse grid of a correction must be 1D2V FP32 with n^3 outputs.  Input
// width 7 n^3 + n: whole values (own block, six neighbour blocks, E); 8 n^3 + n:
// fluctuation features (the blocks minus the x average of the state, E, then
// the own block's x average) and an x-mean-free correction.
const char* coarse_mismatch(const dg_ctx* c, const dg_nn* nn, bool* fluct = nullptr) {
  if (c->cfg.nv != 2) return "the learned correction needs a 1D2V grid";
  if (c->cfg.storage != DG_F32) return "the learned correction needs FP32 storage";
  if (c->cfg.vbc != DG_VBC_PERIODIC) return "the learned correction assumes periodic velocity boundaries";
  if (c->cfg.layout != DG_LAYOUT_DENSE) return "the learned correction needs DG_LAYOUT_DENSE states";
  if (c->bg) return "the learned correction needs whole-f states (no background set)";
  if (!nn) return nullptr;
  const int n = c->L.n, nb = n * n * n;
  if (nn->N.sizes[0] != 7 * nb + n && nn->N.sizes[0] != 8 * nb + n) return "network input width must be 7 n^3 + n or 8 n^3 + n";
  if (fluct) *fluct = nn->N.sizes[0] == 8 * nb + n;
  if (nn->N.sizes[nn->N.L] != nb) return "network output width must be n^3";
  const size_t ne = static_cast<size_t>(c->L.Nx) * c->L.Nu * c->L.Nv;
  if (ne > static_cast<size_t>(nn->N.max_rows)) return "coarse element count exceeds max_rows";
  return nullptr;
}

// values per x node of a coarse state (the inner size of [Nx*n, Nu*n*Nv*n])
size_t inner_of(const dg_ctx* c) { return static_cast<size_t>(c->L.Nu) * c->L.n * c->L.Nv * c->L.n; }

dgn::GatherArgs gather_args(const dg_ctx* c, const void* f, const double* E, const float* mean, const float* inv_std,
                            uint16_t* X, int ld, const float* xmean) {
  dgn::GatherArgs g{};
  g.xmean = xmean;
  g.f = static_cast<const float*>(f);
  g.E = E;
  g.mean = mean;
  g.inv_std = inv_std;
  g.X = X;
  g.Nx = c->L.Nx;
  g.Nu = c->L.Nu;
  g.Nv = c->L.Nv;
  g.n = c->L.n;
  g.nfeat = (xmean ? 8 : 7) * c->L.n * c->L.n * c->L.n + c->L.n;
  g.ld = ld;
  return g;
}

}  // namespace

extern "C" {

size_t dg_nn_workspace_bytes(const int32_t* sizes, int32_t nlayers, int32_t max_rows) {
  if (nn_validate(sizes, nlayers, max_rows)) return 0;
  return nn_layout(sizes, nlayers, max_rows).total;
}

dg_status dg_nn_init(const int32_t* sizes, int32_t nlayers, int32_t max_rows, void* workspace, size_t workspace_bytes,
                     void* hip_stream, dg_nn** out) {
  auto init_fail = [](dg_status s, const std::string& m) {
    std::lock_guard<std::mutex> lk(g_nn_mu);
    g_nn_init_error = m;
    return s;
  };
  if (!out) return init_fail(DG_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (const char* why = nn_validate(sizes, nlayers, max_rows)) return init_fail(DG_ERR_INVALID, why);
  NNLayout N = nn_layout(sizes, nlayers, max_rows);
  if (!workspace) return init_fail(DG_ERR_INVALID, "workspace is NULL");
  if (workspace_bytes < N.total) return init_fail(DG_ERR_OOM, "workspace smaller than dg_nn_workspace_bytes()");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return init_fail(DG_ERR_INVALID, "workspace must be 256-byte aligned");
  dg_nn* nn = new (std::nothrow) dg_nn();
  if (!nn) return init_fail(DG_ERR_INVALID, "host allocation failed");
  nn->N = std::move(N);
  nn->ws = static_cast<char*>(workspace);
  nn->stream = static_cast<hipStream_t>(hip_stream);
  {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) nn->cus = prop.multiProcessorCount;
  }
  hipError_t e = hipEventCreateWithFlags(&nn->ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    delete nn;
    return init_fail(DG_ERR_DEVICE, std::string("hipEventCreate: ") + hipGetErrorString(e));
  }
  // parameters and optimiser state start at zero (the caller sets parameters)
  const NNLayout& L = nn->N;
  e = hipMemsetAsync(nn->ws + L.off_P, 0, L.off_Ytmp - L.off_P, nn->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(nn->stream);
  if (e != hipSuccess) {
    (void)hipEventDestroy(nn->ev);
    delete nn;
    return init_fail(DG_ERR_DEVICE, std::string("workspace clear: ") + hipGetErrorString(e));
  }
  *out = nn;
  return DG_OK;
}

dg_status dg_nn_destroy(dg_nn* nn) {
  if (!nn) return DG_OK;
  hipError_t e = hipStreamSynchronize(nn->stream);
  if (nn->gexec) (void)hipGraphExecDestroy(nn->gexec);
  (void)hipEventDestroy(nn->ev);
  delete nn;
  return e == hipSuccess ? DG_OK : DG_ERR_DEVICE;
}

int64_t dg_nn_param_count(const dg_nn* nn) { return nn ? static_cast<int64_t>(nn->N.nparam) : 0; }

int32_t dg_nn_input_ld(const dg_nn* nn) { return nn ? nn->N.ld[0] : 0; }

dg_status dg_nn_set_params(dg_nn* nn, const float* host_params) {
  if (!nn) return DG_ERR_INVALID;
  if (!host_params) return nfail(nn, DG_ERR_INVALID, "host_params is NULL");
  const NNLayout& L = nn->N;
  for (size_t i = 0; i < L.nparam; ++i)
    if (!std::isfinite(host_params[i])) return nfail(nn, DG_ERR_NONFINITE, "parameters must be finite");
  // BF16 copies rounded to nearest even on the host, as the device does
  std::vector<uint16_t> bf(L.nparam);
  for (size_t i = 0; i < L.nparam; ++i) {
    uint32_t u;
    std::memcpy(&u, &host_params[i], 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    bf[i] = static_cast<uint16_t>(u >> 16);
  }
  NN_HIP(nn, hipMemcpyAsync(nn->ws + L.off_P, host_params, L.nparam * 4, hipMemcpyHostToDevice, nn->stream));
  NN_HIP(nn, hipMemcpyAsync(nn->ws + L.off_Pbf, bf.data(), L.nparam * 2, hipMemcpyHostToDevice, nn->stream));
  // optimiser state restarts with new parameters
  NN_HIP(nn, hipMemsetAsync(nn->ws + L.off_m, 0, L.off_v - L.off_m + L.nparam * 4, nn->stream));
  NN_HIP(nn, hipStreamSynchronize(nn->stream));
  nn->t = 0;
  nn->have_grads = false;
  nn->wt_stale = true;
  return DG_OK;
}

dg_status dg_nn_get_params(dg_nn* nn, float* host_params) {
  if (!nn) return DG_ERR_INVALID;
  if (!host_params) return nfail(nn, DG_ERR_INVALID, "host_params is NULL");
  NN_HIP(nn, hipMemcpyAsync(host_params, nn->ws + nn->N.off_P, nn->N.nparam * 4, hipMemcpyDeviceToHost, nn->stream));
  NN_HIP(nn, hipStreamSynchronize(nn->stream));
  return DG_OK;
}

dg_status dg_nn_forward(dg_nn* nn, const uint16_t* X, int32_t rows, float* Y) {
  if (!nn) return DG_ERR_INVALID;
  if (!X || !Y) return nfail(nn, DG_ERR_INVALID, "X and Y must be non-NULL");
  NN_TRY(check_rows(nn, rows));
  NN_TRY(refresh_wt(nn, nn->stream));
  return forward_infer(nn, X, rows, Y, nn->stream);
}

dg_status dg_nn_set_fused(dg_nn* nn, int32_t on) {
  if (!nn) return DG_ERR_INVALID;
  if (on != 0 && on != 1) return nfail(nn, DG_ERR_INVALID, "dg_nn_set_fused: on must be 0 or 1");
  if (on != 0 && !nn->N.fusable) return nfail(nn, DG_ERR_UNSUPPORTED, "this network's shape has no fused form");
  if ((on != 0) != nn->fused) {
    nn->fused = on != 0;
    // a cached corrected step holds the other form
    if (nn->gexec) {
      (void)hipDeviceSynchronize();
      (void)hipGraphExecDestroy(nn->gexec);
      nn->gexec = nullptr;
    }
  }
  return DG_OK;
}

dg_status dg_nn_loss_grad(dg_nn* nn, const uint16_t* X, const float* T, int32_t rows, double* loss, float* host_grads) {
  if (!nn) return DG_ERR_INVALID;
  if (!X || !T) return nfail(nn, DG_ERR_INVALID, "X and T must be non-NULL");
  NN_TRY(check_rows(nn, rows));
  const NNLayout& N = nn->N;
  hipStream_t s = nn->stream;
  float* Yo = nn->at<float>(N.off_Yo);
  NN_TRY(forward_on(nn, X, rows, Yo, true, s));
  const int nout = N.sizes[N.L];
  float* dZ = nn->at<float>(N.off_dZ);
  uint16_t* dZb = nn->at<uint16_t>(N.off_dZb);
  double* part = nn->at<double>(N.off_loss);
  const float inv = static_cast<float>(1.0 / (static_cast<double>(rows) * nout));
  NN_HIP(nn, dgn::launch_mse(Yo, T, rows, nout, N.ld[N.L], inv, dZ, dZb, part, kMseBlocks, s));
  float* G = nn->at<float>(N.off_G);
  const uint16_t* Wbf = nn->at<uint16_t>(N.off_Pbf);
  for (int l = N.L - 1; l >= 0; --l) {
    const int in = N.sizes[l], out = N.sizes[l + 1];
    const uint16_t* A = l == 0 ? X : nn->at<uint16_t>(N.off_A[l]);
    NN_HIP(nn, dgn::launch_colsum(dZ, rows, out, G + N.offb[l], nn->at<float>(N.off_cpart), s));
    // dW = A^T dZ  (in x out, K = rows)
    NN_HIP(nn, run_gemm(nn, gemm(A, 1, N.ld[l], dZb, N.ld[l + 1], 1, G + N.offW[l], out, in, out, rows), s));
    if (l > 0) {
      // dA = dZ W^T  (rows x in, K = out), then through the GELU of layer l-1
      float* dA = nn->at<float>(N.off_dA);
      NN_HIP(nn, run_gemm(nn, gemm(dZb, N.ld[l + 1], 1, Wbf + N.offW[l], 1, out, dA, in, rows, in, out), s));
      NN_HIP(nn, dgn::launch_gelu_back(dA, nn->at<float>(N.off_Z[l - 1]), dZ, dZb, rows, in, N.ld[l], s));
    }
  }
  nn->have_grads = true;
  if (loss) {
    double h[kMseBlocks];
    NN_HIP(nn, hipMemcpyAsync(h, part, sizeof(h), hipMemcpyDeviceToHost, s));
    NN_HIP(nn, hipStreamSynchronize(s));
    double acc = 0.0;
    for (int i = 0; i < kMseBlocks; ++i) acc += h[i];
    *loss = acc / (static_cast<double>(rows) * nout);
  }
  if (host_grads) {
    NN_HIP(nn, hipMemcpyAsync(host_grads, G, N.nparam * 4, hipMemcpyDeviceToHost, s));
    NN_HIP(nn, hipStreamSynchronize(s));
  }
  return DG_OK;
}

dg_status dg_nn_adamw(dg_nn* nn, float lr, float weight_decay) {
  if (!nn) return DG_ERR_INVALID;
  if (!nn->have_grads) return nfail(nn, DG_ERR_INVALID, "dg_nn_adamw: no gradients (call dg_nn_loss_grad first)");
  if (!(lr >= 0.0f) || !std::isfinite(lr) || !(weight_decay >= 0.0f)) return nfail(nn, DG_ERR_INVALID, "bad lr or weight_decay");
  const NNLayout& N = nn->N;
  nn->t += 1;
  const double b1 = 0.9, b2 = 0.999;
  for (int l = 0; l < N.L; ++l) {
    for (int part = 0; part < 2; ++part) {
      const size_t off = part == 0 ? N.offW[l] : N.offb[l];
      const size_t cnt = part == 0 ? static_cast<size_t>(N.sizes[l]) * N.sizes[l + 1] : N.sizes[l + 1];
      dgn::AdamArgs a{};
      a.p = nn->at<float>(N.off_P) + off;
      a.grad = nn->at<float>(N.off_G) + off;
      a.m = nn->at<float>(N.off_m) + off;
      a.v = nn->at<float>(N.off_v) + off;
      a.bf = nn->at<uint16_t>(N.off_Pbf) + off;
      a.count = cnt;
      a.lr = lr;
      a.b1 = static_cast<float>(b1);
      a.b2 = static_cast<float>(b2);
      a.eps = 1e-8f;
      a.wd = part == 0 ? weight_decay : 0.0f;
      a.c1 = static_cast<float>(1.0 - std::pow(b1, static_cast<double>(nn->t)));
      a.c2 = static_cast<float>(1.0 - std::pow(b2, static_cast<double>(nn->t)));
      NN_HIP(nn, dgn::launch_adamw(a, nn->stream));
    }
  }
  nn->wt_stale = true;
  return DG_OK;
}

dg_status dg_nn_column_stats(dg_nn* nn, const float* X, int64_t rows, int32_t cols, double* host_sum, double* host_sumsq) {
  if (!nn) return DG_ERR_INVALID;
  if (!X || !host_sum || !host_sumsq) return nfail(nn, DG_ERR_INVALID, "NULL argument");
  const int cmax = std::max(nn->N.ld[0], nn->N.ldmax);
  if (rows < 1 || cols < 1 || cols > cmax) return nfail(nn, DG_ERR_INVALID, "rows >= 1 and 1 <= cols <= max(input ld, widest layer)");
  double* s = nn->at<double>(nn->N.off_sum);
  double* q = nn->at<double>(nn->N.off_sumsq);
  NN_HIP(nn, dgn::launch_colstats(X, static_cast<size_t>(rows), cols, cols, s, q, nn->stream));
  NN_HIP(nn, hipMemcpyAsync(host_sum, s, cols * 8, hipMemcpyDeviceToHost, nn->stream));
  NN_HIP(nn, hipMemcpyAsync(host_sumsq, q, cols * 8, hipMemcpyDeviceToHost, nn->stream));
  NN_HIP(nn, hipStreamSynchronize(nn->stream));
  return DG_OK;
}

const char* dg_nn_last_error(const dg_nn* nn) {
  if (nn) return nn->err.c_str();
  std::lock_guard<std::mutex> lk(g_nn_mu);
  return g_nn_init_error.c_str();
}

dg_status dg_projection_matrix(int32_t nc, int32_t nf, int32_t r, double* out) {
  if (nc < 2 || nc > 9 || nf < 2 || nf > 9 || r < 1 || nc * r * nf > dgn::kMaxProj || !out) return DG_ERR_INVALID;
  auto P = projection_matrix(nc, nf, r);
  std::memcpy(out, P.data(), P.size() * sizeof(double));
  return DG_OK;
}

dg_status dg_project(dg_ctx* fine, dg_ctx* coarse, const void* f_fine, void* f_coarse) {
  if (!fine || !coarse) return DG_ERR_INVALID;
  if (!f_fine || !f_coarse) return dgi::fail(coarse, DG_ERR_INVALID, "dg_project: NULL state");
  const dg_config& F = fine->cfg;
  const dg_config& C = coarse->cfg;
  const bool fin32 = F.storage == DG_F32, cout32 = C.storage == DG_F32;
  if (F.nv != C.nv) return dgi::fail(coarse, DG_ERR_INVALID, "dg_project: grids differ in dimension");
  if (F.layout != DG_LAYOUT_DENSE || C.layout != DG_LAYOUT_DENSE)
    return dgi::fail(coarse, DG_ERR_INVALID, "dg_project: states must use DG_LAYOUT_DENSE");
  if (fine->bg || coarse->bg) return dgi::fail(coarse, DG_ERR_INVALID, "dg_project: states must be whole f (no background)");
  const int naxes = 1 + F.nv;
  int r[3] = {1, 1, 1};
  for (int a = 0; a < naxes; ++a) {
    if (F.lo[a] != C.lo[a] || F.hi[a] != C.hi[a]) return dgi::fail(coarse, DG_ERR_INVALID, "dg_project: domains differ");
    if (F.nelem[a] % C.nelem[a]) return dgi::fail(coarse, DG_ERR_INVALID, "dg_project: fine element counts must be multiples of the coarse ones");
    r[a] = F.nelem[a] / C.nelem[a];
    if (C.n * r[a] * F.n > dgn::kMaxProj) return dgi::fail(coarse, DG_ERR_UNSUPPORTED, "dg_project: refinement ratio too large");
  }
  // Plan: axes whose fine and coarse spaces coincide (r = 1, same n) are the
  // identity and skipped; the others run in order of increasing size ratio
  // nc / (r nf), so the intermediates shrink as early as possible.  Scratch:
  // the fine context's two stage buffers hold the FP64 intermediates.
  const size_t cap = fine->L.dof * fine->L.esize;
  double* buf[2] = {fine->at<double>(fine->L.off_B), fine->at<double>(fine->L.off_C)};
  std::vector<int> order;
  for (int a = 0; a < naxes; ++a)
    if (!(r[a] == 1 && C.n == F.n)) order.push_back(a);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return C.n * r[y] < C.n * r[x]; });
  std::vector<dgn::ProjArgs> plan;
  {
    std::vector<size_t> dims(naxes);   // current node count per axis
    for (int a = 0; a < naxes; ++a) dims[a] = static_cast<size_t>(F.nelem[a]) * F.n;
    for (size_t k = 0; k < order.size(); ++k) {
      const int a = order[k];
      dgn::ProjArgs p{};
      auto P = projection_matrix(C.n, F.n, r[a]);
      std::memcpy(p.P, P.data(), P.size() * sizeof(double));
      size_t outer = 1, inner = 1;
      for (int b = 0; b < a; ++b) outer *= dims[b];
      for (int b = a + 1; b < naxes; ++b) inner *= dims[b];
      const size_t out_count = outer * static_cast<size_t>(C.nelem[a]) * C.n * inner;
      if (out_count * 8 > cap)
        return dgi::fail(coarse, DG_ERR_UNSUPPORTED, "dg_project: intermediate does not fit the fine stage buffers");
      if (outer > 0x7fffffff || inner > 0x7fffffff) return dgi::fail(coarse, DG_ERR_UNSUPPORTED, "dg_project: grid too large");
      p.in_f32 = (k == 0 && fin32) ? 1 : 0;
      // an FP64 coarse state takes the last axis directly
      p.out = (k + 1 == order.size() && !cout32) ? static_cast<double*>(f_coarse) : buf[k % 2];
      p.outer = static_cast<int>(outer);
      p.inner = static_cast<int>(inner);
      p.Nc = C.nelem[a];
      p.nc = C.n;
      p.nf = F.n;
      p.r = r[a];
      plan.push_back(p);
      dims[a] = static_cast<size_t>(C.nelem[a]) * C.n;
    }
  }
  NN_TRY(dgi::enter(fine));
  {  // the fine stream also orders after the coarse caller's stream
    hipError_t e = hipEventRecord(coarse->ev_in, coarse->user);
    if (e == hipSuccess) e = hipStreamWaitEvent(fine->stream, coarse->ev_in, 0);
    if (e != hipSuccess) return dgi::hip_fail(coarse, e, "stream ordering");
  }
  hipStream_t s = fine->stream;
  const void* in = f_fine;
  for (auto& p : plan) {
    p.in = in;
    hipError_t e = dgn::launch_project_axis(p, s);
    if (e != hipSuccess) return dgi::hip_fail(coarse, e, "projection launch");
    in = p.out;
  }
  hipError_t e = hipSuccess;
  const size_t dof = coarse->L.dof;
  if (plan.empty()) {   // identical spaces: a copy, converting the precision if needed
    if (fin32 == cout32) e = hipMemcpyAsync(f_coarse, f_fine, dof * (cout32 ? 4 : 8), hipMemcpyDeviceToDevice, s);
    else if (cout32) e = dgn::launch_f64_to_f32(static_cast<const double*>(f_fine), static_cast<float*>(f_coarse), dof, s);
    else e = dgn::launch_f32_to_f64(static_cast<const float*>(f_fine), static_cast<double*>(f_coarse), dof, s);
  } else if (cout32) {
    e = dgn::launch_f64_to_f32(static_cast<const double*>(in), static_cast<float*>(f_coarse), dof, s);
  }
  if (e != hipSuccess) return dgi::hip_fail(coarse, e, "conversion launch");
  NN_TRY(dgi::leave(fine));
  // the coarse caller's stream orders after the fine stream
  hipEvent_t ev = fine->ev_out;
  if ((e = hipStreamWaitEvent(coarse->user, ev, 0)) != hipSuccess) return dgi::hip_fail(coarse, e, "hipStreamWaitEvent");
  return DG_OK;
}

dg_status dg_nn_features(dg_ctx* coarse, const dg_nn* nn, const void* f, const double* E, const float* mean,
                         const float* inv_std, uint16_t* X) {
  if (!coarse) return DG_ERR_INVALID;
  if (!nn || !f || !E || !mean || !inv_std || !X) return dgi::fail(coarse, DG_ERR_INVALID, "dg_nn_features: NULL argument");
  bool fluct = false;
  if (const char* why = coarse_mismatch(coarse, nn, &fluct)) return dgi::fail(coarse, DG_ERR_INVALID, why);
  NN_TRY(dgi::enter(coarse));
  float* xm = nullptr;
  hipError_t e = hipSuccess;
  if (fluct) {   // x average of f into the context's stage scratch
    xm = coarse->at<float>(coarse->L.off_B);
    e = dgn::launch_xmean(static_cast<const float*>(f), coarse->at<double>(coarse->L.off_wx), xm, coarse->L.Nx * coarse->L.n,
                          inner_of(coarse), coarse->stream);
  }
  if (e == hipSuccess) e = dgn::launch_gather(gather_args(coarse, f, E, mean, inv_std, X, nn->N.ld[0], xm), coarse->stream);
  if (e != hipSuccess) return dgi::hip_fail(coarse, e, "gather launch");
  return dgi::leave(coarse);
}

dg_status dg_nn_features_raw(dg_ctx* coarse, const void* f, const double* E, int32_t fluct, float* out) {
  if (!coarse) return DG_ERR_INVALID;
  if (!f || !E || !out) return dgi::fail(coarse, DG_ERR_INVALID, "dg_nn_features_raw: NULL argument");
  if (const char* why = coarse_mismatch(coarse, nullptr)) return dgi::fail(coarse, DG_ERR_INVALID, why);
  NN_TRY(dgi::enter(coarse));
  float* xm = nullptr;
  hipError_t e = hipSuccess;
  if (fluct) {
    xm = coarse->at<float>(coarse->L.off_B);
    e = dgn::launch_xmean(static_cast<const float*>(f), coarse->at<double>(coarse->L.off_wx), xm, coarse->L.Nx * coarse->L.n,
                          inner_of(coarse), coarse->stream);
  }
  if (e == hipSuccess) e = dgn::launch_gather_raw(gather_args(coarse, f, E, nullptr, nullptr, nullptr, 0, xm), out, coarse->stream);
  if (e != hipSuccess) return dgi::hip_fail(coarse, e, "gather launch");
  return dgi::leave(coarse);
}

dg_status dg_nn_to_elements(dg_ctx* coarse, const void* x, const void* sub, float scale, int32_t fluct, float* out) {
  if (!coarse) return DG_ERR_INVALID;
  if (!x || !out) return dgi::fail(coarse, DG_ERR_INVALID, "dg_nn_to_elements: NULL argument");
  if (coarse->cfg.nv != 2) return dgi::fail(coarse, DG_ERR_INVALID, "the learned correction needs a 1D2V grid");
  if (coarse->cfg.layout != DG_LAYOUT_DENSE)
    return dgi::fail(coarse, DG_ERR_INVALID, "the learned correction needs DG_LAYOUT_DENSE states");
  if (coarse->bg) return dgi::fail(coarse, DG_ERR_INVALID, "the learned correction needs whole-f states (no background set)");
  const bool f64 = coarse->cfg.storage == DG_F64;
  if (!std::isfinite(scale)) return dgi::fail(coarse, DG_ERR_INVALID, "dg_nn_to_elements: scale must be finite");
  NN_TRY(dgi::enter(coarse));
  const dgi::Layout& L = coarse->L;
  const size_t inner = inner_of(coarse);
  float* xm = nullptr;
  hipError_t e = hipSuccess;
  if (f64) {   // FP64 inputs (training targets from FP64 right-hand sides)
    double* xm64 = nullptr;
    if (fluct) {
      xm64 = coarse->at<double>(L.off_B);
      e = dgn::launch_xmean_diff64(static_cast<const double*>(x), static_cast<const double*>(sub),
                                   coarse->at<double>(L.off_wx), xm64, L.Nx * L.n, inner, coarse->stream);
    }
    if (e == hipSuccess)
      e = dgn::launch_to_elements64(static_cast<const double*>(x), static_cast<const double*>(sub), xm64, scale, out, L.n, L.Nx,
                                    L.Nu, L.Nv, coarse->stream);
  } else {
    if (fluct) {   // x average of (x - sub), by linearity mean(x) - mean(sub), in the stage scratch
      xm = coarse->at<float>(L.off_B);
      const double* wx = coarse->at<double>(L.off_wx);
      e = dgn::launch_xmean(static_cast<const float*>(x), wx, xm, L.Nx * L.n, inner, coarse->stream);
      if (e == hipSuccess && sub) {
        float* xs = xm + inner;
        e = dgn::launch_xmean(static_cast<const float*>(sub), wx, xs, L.Nx * L.n, inner, coarse->stream);
        if (e == hipSuccess) e = dgn::launch_axpy(xm, xs, nullptr, -1.0f, 1, inner, coarse->stream);
      }
    }
    if (e == hipSuccess)
      e = dgn::launch_to_elements(static_cast<const float*>(x), static_cast<const float*>(sub), xm, scale, out, L.n, L.Nx, L.Nu,
                                  L.Nv, coarse->stream);
  }
  if (e != hipSuccess) return dgi::hip_fail(coarse, e, "to_elements launch");
  return dgi::leave(coarse);
}

}  // extern "C"

namespace {

// One corrected SSP-RK3 stage: out = c_un un + c_in fin + c_dt (L(fin) + s NN(fin)),
// then the field of out for the next stage.
dg_status corrected_stage(dg_ctx* c, dg_nn* nn, const float* mean, const float* inv_std, float scale, const void* fin,
                          const void* fun, void* out, double c_un, double c_in, double c_dt, bool record) {
  const dgi::Layout& L = c->L;
  hipStream_t s = c->stream;
  double* E = c->at<double>(L.off_E);
  const int rows = L.Nx * L.Nu * L.Nv;
  const int nx = L.Nx * L.n;
  const size_t inner = inner_of(c);
  bool fluct = false;
  coarse_mismatch(c, nn, &fluct);
  uint16_t* Xf = nn->at<uint16_t>(nn->N.off_Xf);
  float* Yo = nn->at<float>(nn->N.off_Yo);
  float* corr = nn->at<float>(nn->N.off_corr);
  float* xm_f = fluct ? nn->at<float>(nn->N.off_xm1) : nullptr;
  float* xm_c = fluct ? nn->at<float>(nn->N.off_xm2) : nullptr;
  hipError_t e = hipSuccess;
  if (fluct) e = dgn::launch_xmean(static_cast<const float*>(fin), c->at<double>(L.off_wx), xm_f, nx, inner, s);
  if (e == hipSuccess) e = dgn::launch_gather(gather_args(c, fin, E, mean, inv_std, Xf, nn->N.ld[0], xm_f), s);
  if (e != hipSuccess) return dgi::hip_fail(c, e, "gather launch");
  {
    dg_status st = forward_infer(nn, Xf, rows, Yo, s);
    if (st != DG_OK) return dgi::fail(c, st, nn->err);
  }
  dgn::ScatterArgs sc{};
  sc.Y = Yo;
  sc.out = corr;
  for (int j = 0; j < L.n; ++j) sc.w[j] = static_cast<float>(c->basis.w[j]);
  sc.scale = scale;
  sc.Nx = L.Nx;
  sc.Nu = L.Nu;
  sc.Nv = L.Nv;
  sc.n = L.n;
  sc.ldy = L.n * L.n * L.n;
  // whole-value correction: mass-neutral per element; fluctuation correction:
  // its x average is removed below (which also keeps the total mass)
  sc.mass_neutral = fluct ? 0 : 1;
  if ((e = dgn::launch_scatter(sc, s)) != hipSuccess) return dgi::hip_fail(c, e, "scatter launch");
  if (fluct && (e = dgn::launch_xmean(corr, c->at<double>(L.off_wx), xm_c, nx, inner, s)) != hipSuccess)
    return dgi::hip_fail(c, e, "xmean launch");
  // the stage adds c_dt (corr - xm_c) to its update and forms the density
  // partials of the result itself
  NN_TRY(dgi::stage(c, fin, fun, out, E, c->at<double>(L.off_part), c_un, c_in, c_dt, false, corr, xm_c));
  return dgi::field(c, E, nullptr, record);
}

// One corrected SSP-RK3 step (three corrected stages; moments when diag).
dg_status corrected_step(dg_ctx* c, dg_nn* nn, const float* mean, const float* inv_std, float scale, void* f,
                         double dt, bool diag) {
  void* B = c->ws + c->L.off_B;
  void* C = c->ws + c->L.off_C;
  NN_TRY(corrected_stage(c, nn, mean, inv_std, scale, f, nullptr, B, 0.0, 1.0, dt, false));
  NN_TRY(corrected_stage(c, nn, mean, inv_std, scale, B, f, C, 0.75, 0.25, 0.25 * dt, false));
  NN_TRY(corrected_stage(c, nn, mean, inv_std, scale, C, f, f, 1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0 * dt, diag));
  if (diag) NN_TRY(dgi::moments(c, f));
  return DG_OK;
}

// The corrected step is ~45 short launches; it is captured once per
// (context, state, dt, statistics, scale, diag) and replayed.  Parameter
// updates need no new capture: the network's buffers keep their addresses.
dg_status build_corrected_graph(dg_ctx* c, dg_nn* nn, const float* mean, const float* inv_std, float scale, void* f,
                                double dt, bool diag) {
  if (nn->gexec && nn->g_ctx == c->id && nn->g_f == f && nn->g_mean == mean && nn->g_inv == inv_std && nn->g_dt == dt &&
      nn->g_scale == scale && nn->g_diag == diag)
    return DG_OK;
  if (nn->gexec) {
    // the old graph may still replay, on this or another context's stream
    (void)hipDeviceSynchronize();
    (void)hipGraphExecDestroy(nn->gexec);
    nn->gexec = nullptr;
  }
  hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return dgi::hip_fail(c, e, "hipStreamBeginCapture");
  dg_status s = corrected_step(c, nn, mean, inv_std, scale, f, dt, diag);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(c->stream, &g);
  if (s != DG_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return dgi::hip_fail(c, e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&nn->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    nn->gexec = nullptr;
    return dgi::hip_fail(c, e, "hipGraphInstantiate");
  }
  nn->g_ctx = c->id;
  nn->g_f = f;
  nn->g_mean = mean;
  nn->g_inv = inv_std;
  nn->g_dt = dt;
  nn->g_scale = scale;
  nn->g_diag = diag;
  return DG_OK;
}

}  // namespace

extern "C" {

dg_status dg_nn_rk_step(dg_ctx* coarse, dg_nn* nn, const float* mean, const float* inv_std, float out_scale, void* f,
                        double dt, int32_t nsteps, dg_diag* host_diag) {
  if (!coarse) return DG_ERR_INVALID;
  if (!nn || !mean || !inv_std) return dgi::fail(coarse, DG_ERR_INVALID, "dg_nn_rk_step: NULL argument");
  if (const char* why = coarse_mismatch(coarse, nn)) return dgi::fail(coarse, DG_ERR_INVALID, why);
  if (!std::isfinite(out_scale)) return dgi::fail(coarse, DG_ERR_INVALID, "out_scale must be finite");
  if (nsteps == 0 && f && dt > 0.0) return DG_OK;
  // transposed weights for the fused network, then order after the network's
  // stream (parameter updates, that refresh) as well
  if (dg_status st = refresh_wt(nn, nn->stream); st != DG_OK) return dgi::fail(coarse, st, nn->err);
  hipError_t e = hipEventRecord(nn->ev, nn->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(coarse->stream, nn->ev, 0);
  if (e != hipSuccess) return dgi::hip_fail(coarse, e, "network stream ordering");
  NN_TRY(dgi::begin_steps(coarse, f, dt, nsteps));
  const dgi::Layout& L = coarse->L;
  const bool diag = host_diag != nullptr;
  NN_TRY(build_corrected_graph(coarse, nn, mean, inv_std, out_scale, f, dt, diag));
  bool bad = false;
  int done = 0;
  while (done < nsteps) {
    const int chunk = std::min(nsteps - done, dgk::kRing);
    if (diag && (e = dgk::launch_reset_counter(coarse->at<int>(L.off_ctr), coarse->stream)) != hipSuccess)
      return dgi::hip_fail(coarse, e, "counter reset");
    for (int k = 0; k < chunk; ++k)
      if ((e = hipGraphLaunch(nn->gexec, coarse->stream)) != hipSuccess) return dgi::hip_fail(coarse, e, "hipGraphLaunch");
    if (diag) {
      std::vector<double> ring(static_cast<size_t>(chunk) * 8);
      e = hipMemcpyAsync(ring.data(), coarse->at<double>(L.off_ring), ring.size() * 8, hipMemcpyDeviceToHost, coarse->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(coarse->stream);
      if (e != hipSuccess) return dgi::hip_fail(coarse, e, "diagnostics readback");
      for (int k = 0; k < chunk; ++k) {
        dgi::copy_record(&ring[static_cast<size_t>(k) * 8], coarse->t + (done + k + 1) * dt, &host_diag[done + k]);
        host_diag[done + k].step = done + k;
        if (!host_diag[done + k].finite) bad = true;
      }
    }
    done += chunk;
  }
  coarse->t += nsteps * dt;
  NN_TRY(dgi::leave(coarse));
  // the network's stream orders after the step (its buffers were used)
  if ((e = hipStreamWaitEvent(nn->stream, coarse->ev_out, 0)) != hipSuccess) return dgi::hip_fail(coarse, e, "hipStreamWaitEvent");
  if (bad) return dgi::fail(coarse, DG_ERR_NONFINITE, "a step produced non-finite diagnostics");
  return DG_OK;
}

}  // extern "C"
