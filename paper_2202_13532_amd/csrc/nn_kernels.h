// Launch interface of the learned-correction kernels (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace dgn {

constexpr int kMaxProj = 324;   // nc * r * nf entries of a projection matrix

struct ProjArgs {
  const void* in;     // [outer, Nc*r*nf, inner], FP32 if in_f32 else FP64
  double* out;        // [outer, Nc*nc, inner]
  double P[kMaxProj]; // nc x (r*nf), row-major
  int outer, inner, Nc, nc, nf, r, in_f32;
};

struct GatherArgs {
  const float* f;       // coarse state [Nx, n, Nu, n, Nv, n]
  const double* E;      // Nx*n field
  const float* mean;    // nfeat
  const float* inv_std; // nfeat
  uint16_t* X;          // rows x ld (BF16)
  const float* xmean;   // x average of f per (u, v) node, or nullptr (whole values)
  int Nx, Nu, Nv, n, nfeat, ld;
};

struct ScatterArgs {
  const float* Y;       // rows x ldy network output (element-major)
  float* out;           // state layout
  float w[16];          // n reference LGL weights
  float scale;
  int Nx, Nu, Nv, n, ldy, mass_neutral;
};

struct GemmArgs {
  const uint16_t* A;    // A(m,k) = A[m*sam + k*sak]
  const uint16_t* B;    // B(k,n) = B[k*sbk + n*sbn]
  float* C;             // C(m,n) = C[m*scm + n*scn]
  size_t sam, sak, sbk, sbn, scm, scn;
  int M, N, K;
  float beta;
  // Fused layer epilogue instead of storing C (when epi != 0):
  //   z = acc + bias[n];  Z[m*N + n] = z;  v = gelu ? GELU(z) : z;
  //   Af[m*N + n] = v;  Abf[m*lda + n] = BF16(v)   (each output optional)
  int epi, gelu, lda;
  const float* bias;
  float* Z;
  float* Af;
  uint16_t* Abf;
};

struct AdamArgs {
  float* p;
  const float* grad;
  float* m;
  float* v;
  uint16_t* bf;         // BF16 copy (or nullptr)
  size_t count;
  float lr, b1, b2, eps, wd, c1, c2;   // c1 = 1 - b1^t, c2 = 1 - b2^t
};

// Whole-network inference in one launch: every layer's GEMM, bias and GELU
// for RM rows per work-group, activations kept in LDS.  Shapes: at most
// kMlpMaxLayers layers, input width <= kMlpMaxIn, every layer output <= kMlpMaxOut.
constexpr int kMlpMaxLayers = 8, kMlpMaxIn = 1024, kMlpMaxOut = 128;
struct MlpArgs {
  const uint16_t* X;                  // rows x ldx BF16 inputs (columns >= in[0] are zero)
  int ldx, rows, L;
  int in[kMlpMaxLayers], out[kMlpMaxLayers];
  int kp[kMlpMaxLayers];              // K padded to a multiple of 32
  const uint16_t* Wt[kMlpMaxLayers];  // out x kp BF16: W transposed, zero for k >= in
  const float* bias[kMlpMaxLayers];
  float* Y;                           // rows x out[L-1] FP32 (no GELU on the last layer)
};
hipError_t launch_mlp_fused(const MlpArgs& a, hipStream_t s);
// Wt[n * kp + k] = W[k * out + n] for k < in, 0 for in <= k < kp (BF16)
hipError_t launch_transpose_weights(const uint16_t* W, int in, int out, int kp, uint16_t* Wt, hipStream_t s);

hipError_t launch_project_axis(const ProjArgs& a, hipStream_t s);
hipError_t launch_f32_to_f64(const float* in, double* out, size_t n, hipStream_t s);
hipError_t launch_f64_to_f32(const double* in, float* out, size_t n, hipStream_t s);
hipError_t launch_gather(const GatherArgs& a, hipStream_t s);
hipError_t launch_gather_raw(const GatherArgs& a, float* out, hipStream_t s);
hipError_t launch_scatter(const ScatterArgs& a, hipStream_t s);
hipError_t launch_gemm(const GemmArgs& g, hipStream_t s);
// LDS-tiled MFMA GEMM with split-K (falls back to launch_gemm when an operand
// has no unit stride or is not 16-byte aligned).  `part`: device scratch of
// part_floats floats for the split-K slices; `cus`: compute units.
hipError_t launch_gemm_tiled(const GemmArgs& g, float* part, size_t part_floats, int cus, hipStream_t s);
hipError_t launch_gelu_back(const float* dA, const float* Z, float* dZ, uint16_t* dZb, int rows, int cols, int ld, hipStream_t s);
hipError_t launch_mse(const float* Y, const float* T, int rows, int cols, int ld, float inv_count, float* dY, uint16_t* dYb,
                      double* partial, int nblocks, hipStream_t s);
// column sums (bias gradients); part: 32 x cols floats of scratch
constexpr int kColsumPart = 32;
hipError_t launch_colsum(const float* in, int rows, int cols, float* out, float* part, hipStream_t s);
hipError_t launch_adamw(const AdamArgs& a, hipStream_t s);
hipError_t launch_colstats(const float* X, size_t rows, int ld, int cols, double* sum, double* sumsq, hipStream_t s);
// out = scale * (in - sub - xm) element-major (sub, xm optional; xm per (u, v) node)
hipError_t launch_to_elements(const float* in, const float* sub, const float* xm, float scale, float* out, int n, int Nx,
                              int Nu, int Nv, hipStream_t s);
// y += a * (x - xm) (xm optional, per inner index: the state is [outer, inner])
hipError_t launch_axpy(float* y, const float* x, const float* xm, float a, size_t outer, size_t inner, hipStream_t s);
// FP64 inputs: x average of (x - sub) (sub optional) and the element-major
// FP32 copy of scale * (in - sub - xm)
hipError_t launch_xmean_diff64(const double* x, const double* sub, const double* wx, double* out, int outer, size_t inner,
                               hipStream_t s);
hipError_t launch_to_elements64(const double* in, const double* sub, const double* xm, float scale, float* out, int n, int Nx,
                                int Nu, int Nv, hipStream_t s);
// x average of a state [Nx*n, inner] with the x quadrature weights wx (Nx*n,
// FP64): out[q] = sum_o wx[o] in[o, q] / sum_o wx[o], FP64 sums
hipError_t launch_xmean(const float* in, const double* wx, float* out, int outer, size_t inner, hipStream_t s);

}  // namespace dgn
