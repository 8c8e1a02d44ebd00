// Learned coarse-grid correction: data movement between DG grids and a
// per-element MLP trained and evaluated with BF16 MFMA (FP32 accumulate).
//
//   project_axis_kernel  L2 projection of a fine DG function onto a coarse
//                        grid along one axis (matrix per coarse element).
//   gather_kernel        per coarse element: own n^3 block, the six face
//                        neighbours' blocks and E at the n x nodes, normalised
//                        and converted to BF16 (one row per element).
//   scatter_kernel       network output (element-major) -> state layout, with
//                        the element's weighted mean removed (mass neutral).
//   gemm_bf16_kernel     C = A B with v_mfma_f32_16x16x16_bf16: one wave per
//                        16x16 tile of C; A and B addressed by strides so the
//                        same kernel serves X W, dY W^T and X^T dY.
//   bias_act_kernel, gelu_back_kernel, mse_kernel, colsum_kernel,
//   adamw_kernel, colstats_kernel: elementwise / reduction helpers.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "nn_kernels.h"

namespace dgn {

constexpr int kWave = 64;

__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);   // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);                                                         // round to nearest even
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __builtin_bit_cast(float, static_cast<uint32_t>(h) << 16); }

// Exact GELU x Phi(x) and its derivative Phi(x) + x phi(x).
__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// ---------------------------------------------------------------------------
// Projection along one axis.  The state is viewed as [outer, Nf*nf, inner];
// the result is [outer, Nc*nc, inner] with out[o, c*nc + i, q] =
// sum_m P[i, m] in[o, c*r*nf + m, q], m < r*nf.  One thread per output value.
// ---------------------------------------------------------------------------
__global__ void project_axis_kernel(ProjArgs a) {
  const size_t total = static_cast<size_t>(a.outer) * a.Nc * a.nc * a.inner;
  const size_t tid = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tid >= total) return;
  const size_t q = tid % a.inner;
  const size_t rest = tid / a.inner;
  const int row = static_cast<int>(rest % (static_cast<size_t>(a.Nc) * a.nc));
  const size_t o = rest / (static_cast<size_t>(a.Nc) * a.nc);
  const int c = row / a.nc, i = row % a.nc;
  const int span = a.r * a.nf;
  const size_t in_rows = static_cast<size_t>(a.Nc) * span;
  const size_t base = (o * in_rows + static_cast<size_t>(c) * span) * a.inner + q;
  double s = 0.0;
  if (a.in_f32) {
    const float* src = static_cast<const float*>(a.in) + base;
    for (int m = 0; m < span; ++m)
      s = __builtin_fma(a.P[i * span + m], static_cast<double>(src[static_cast<size_t>(m) * a.inner]), s);
  } else {
    const double* src = static_cast<const double*>(a.in) + base;
    for (int m = 0; m < span; ++m) s = __builtin_fma(a.P[i * span + m], src[static_cast<size_t>(m) * a.inner], s);
  }
  a.out[tid] = s;
}

__global__ void f32_to_f64_kernel(const float* in, double* out, size_t n) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = static_cast<double>(in[i]);
}
__global__ void f64_to_f32_kernel(const double* in, float* out, size_t n) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = static_cast<float>(in[i]);
}

// ---------------------------------------------------------------------------
// Feature gather on a 1D2V coarse grid [Nx, n, Nu, n, Nv, n] (FP32 state).
// Row e = (ix*Nu + iu)*Nv + iv; columns: own block (n^3, order jx, ju, jv),
// then the x-1, x+1, u-1, u+1, v-1, v+1 neighbour blocks (periodic), then E at
// the element's n x nodes, then zero padding up to ld.  Column c is
// normalised as (value - mean[c]) * inv_std[c] before conversion to BF16.
// One thread per (row, column).
// ---------------------------------------------------------------------------
__global__ void gather_kernel(GatherArgs a) {
  const int n = a.n, nb = n * n * n;
  const size_t total = static_cast<size_t>(a.Nx) * a.Nu * a.Nv * a.ld;
  const size_t tid = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tid >= total) return;
  const int col = static_cast<int>(tid % a.ld);
  const size_t e = tid / a.ld;
  const int iv = static_cast<int>(e % a.Nv);
  const int iu = static_cast<int>((e / a.Nv) % a.Nu);
  const int ix = static_cast<int>(e / (static_cast<size_t>(a.Nv) * a.Nu));
  float val = 0.0f;
  if (col < 7 * nb) {
    const int blk = col / nb, loc = col % nb;
    int ex = ix, eu = iu, ev = iv;
    switch (blk) {
      case 1: ex = ix == 0 ? a.Nx - 1 : ix - 1; break;
      case 2: ex = ix == a.Nx - 1 ? 0 : ix + 1; break;
      case 3: eu = iu == 0 ? a.Nu - 1 : iu - 1; break;
      case 4: eu = iu == a.Nu - 1 ? 0 : iu + 1; break;
      case 5: ev = iv == 0 ? a.Nv - 1 : iv - 1; break;
      case 6: ev = iv == a.Nv - 1 ? 0 : iv + 1; break;
      default: break;
    }
    const int jx = loc / (n * n), ju = (loc / n) % n, jv = loc % n;
    const size_t idx = ((((static_cast<size_t>(ex) * n + jx) * a.Nu + eu) * n + ju) * a.Nv + ev) * n + jv;
    val = a.f[idx];
  } else if (col < 7 * nb + n) {
    val = static_cast<float>(a.E[ix * n + (col - 7 * nb)]);
  }
  const bool real = col < a.nfeat;
  const float z = real ? (val - a.mean[col]) * a.inv_std[col] : 0.0f;
  a.X[tid] = f2bf(z);
}

// Network output Y[e][loc] (loc = (jx*n + ju)*n + jv), scaled by `scale`,
// minus its element mean under the product LGL weights w_jx w_ju w_jv, written
// to the state layout (FP32).  One thread per element.
__global__ void scatter_kernel(ScatterArgs a) {
  const int n = a.n;
  const size_t ne = static_cast<size_t>(a.Nx) * a.Nu * a.Nv;
  const size_t e = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int iv = static_cast<int>(e % a.Nv);
  const int iu = static_cast<int>((e / a.Nv) % a.Nu);
  const int ix = static_cast<int>(e / (static_cast<size_t>(a.Nv) * a.Nu));
  const float* y = a.Y + e * a.ldy;
  double num = 0.0, den = 0.0;   // FP64: the removed mean must not carry a rounding bias
  for (int jx = 0; jx < n; ++jx)
    for (int ju = 0; ju < n; ++ju)
      for (int jv = 0; jv < n; ++jv) {
        const double w = static_cast<double>(a.w[jx]) * a.w[ju] * a.w[jv];
        num += w * y[(jx * n + ju) * n + jv];
        den += w;
      }
  const float mean = a.mass_neutral ? static_cast<float>(num / den) : 0.0f;
  for (int jx = 0; jx < n; ++jx)
    for (int ju = 0; ju < n; ++ju)
      for (int jv = 0; jv < n; ++jv) {
        const size_t idx = ((((static_cast<size_t>(ix) * n + jx) * a.Nu + iu) * n + ju) * a.Nv + iv) * n + jv;
        a.out[idx] = a.scale * (y[(jx * n + ju) * n + jv] - mean);
      }
}

// ---------------------------------------------------------------------------
// BF16 MFMA GEMM.  C(m, n) = sum_k A(m, k) B(k, n) with
//   A(m, k) = A[m*sam + k*sak], B(k, n) = B[k*sbk + n*sbn]   (BF16),
// FP32 accumulation, C stored FP32 at C[m*scm + n*scn] (beta: C = acc + beta C).
// v_mfma_f32_16x16x16_bf16 lane layout (wave of 64, lane = l):
//   A operand: row l % 16, k = 4 (l / 16) + t,  t = 0..3
//   B operand: col l % 16, k = 4 (l / 16) + t
//   D:         col l % 16, row 4 (l / 16) + t
// Out-of-range rows, columns and k are read as zero and not stored.
// ---------------------------------------------------------------------------
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kWave) gemm_bf16_kernel(GemmArgs g) {
  const int lane = threadIdx.x;
  const int m0 = blockIdx.x * 16, n0 = blockIdx.y * 16;
  const int r = lane % 16, kb = 4 * (lane / 16);
  const int am = m0 + r, bn = n0 + r;
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    bf16x4 av, bv;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = k0 + kb + t;
      const bool ka = am < g.M && k < g.K;
      const bool kbv = bn < g.N && k < g.K;
      av[t] = ka ? static_cast<short>(g.A[static_cast<size_t>(am) * g.sam + static_cast<size_t>(k) * g.sak]) : short(0);
      bv[t] = kbv ? static_cast<short>(g.B[static_cast<size_t>(k) * g.sbk + static_cast<size_t>(bn) * g.sbn]) : short(0);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
  }
  const int cn = n0 + lane % 16;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int cm = m0 + kb + t;
    if (cm < g.M && cn < g.N) {
      float* c = g.C + static_cast<size_t>(cm) * g.scm + static_cast<size_t>(cn) * g.scn;
      *c = g.beta != 0.0f ? acc[t] + g.beta * *c : acc[t];
    }
  }
}

// Z = Y + bias (per column), stored FP32; A = act(Z) stored BF16 (ld columns,
// padding columns set to zero) and optionally FP32.
__global__ void bias_act_kernel(BiasActArgs a) {
  const size_t total = static_cast<size_t>(a.rows) * a.ld;
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int col = static_cast<int>(i % a.ld);
  const size_t row = i / a.ld;
  if (col >= a.cols) {
    if (a.Abf) a.Abf[i] = 0;
    return;
  }
  const size_t zi = row * a.cols + col;
  const float z = a.Y[zi] + (a.bias ? a.bias[col] : 0.0f);
  if (a.Z) a.Z[zi] = z;
  const float v = a.gelu ? gelu(z) : z;
  if (a.Af) a.Af[zi] = v;
  if (a.Abf) a.Abf[i] = f2bf(v);
}

// dZ = dA * gelu'(Z) (FP32), and its BF16 copy with ld columns.
__global__ void gelu_back_kernel(const float* dA, const float* Z, float* dZ, uint16_t* dZb, int rows, int cols, int ld) {
  const size_t total = static_cast<size_t>(rows) * ld;
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int col = static_cast<int>(i % ld);
  const size_t row = i / ld;
  if (col >= cols) {
    dZb[i] = 0;
    return;
  }
  const size_t zi = row * cols + col;
  const float d = dA[zi] * gelu_grad(Z[zi]);
  dZ[zi] = d;
  dZb[i] = f2bf(d);
}

// MSE: per-block partial sums of (y - t)^2 and dY = 2 (y - t) / count (FP32
// and BF16 copy with ld columns).
__global__ void mse_kernel(const float* Y, const float* T, int rows, int cols, int ld, float inv_count,
                           float* dY, uint16_t* dYb, double* partial) {
  __shared__ double red[256];
  const size_t total = static_cast<size_t>(rows) * cols;
  double s = 0.0;
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const float d = Y[i] - T[i];
    s += static_cast<double>(d) * d;
    const float g = 2.0f * d * inv_count;
    dY[i] = g;
    const size_t row = i / cols, col = i % cols;
    dYb[row * ld + col] = f2bf(g);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Column sums (bias gradients): out[c] = sum_rows in[row*cols + c]; one block
// per column, fixed-order tree.
__global__ void colsum_kernel(const float* in, int rows, int cols, float* out) {
  __shared__ float red[256];
  const int c = blockIdx.x;
  float s = 0.0f;
  for (int r = threadIdx.x; r < rows; r += blockDim.x) s += in[static_cast<size_t>(r) * cols + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}

// AdamW on FP32 master parameters; refreshes the BF16 copy (W stored
// [in, out] with the padded BF16 copy [in_pad, out] when `bf` is set).
__global__ void adamw_kernel(AdamArgs a) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.count) return;
  const float g = a.grad[i];
  const float m = a.b1 * a.m[i] + (1.0f - a.b1) * g;
  const float v = a.b2 * a.v[i] + (1.0f - a.b2) * g * g;
  a.m[i] = m;
  a.v[i] = v;
  const float mh = m / a.c1, vh = v / a.c2;
  const float p = a.p[i] - a.lr * (mh / (sqrtf(vh) + a.eps) + a.wd * a.p[i]);
  a.p[i] = p;
  if (a.bf) a.bf[i] = f2bf(p);
}

// Per-column mean and sum of squares over `rows` rows of an FP32 matrix with
// ld columns (FP64 accumulation), one block per column.
__global__ void colstats_kernel(const float* X, size_t rows, int ld, double* sum, double* sumsq) {
  __shared__ double r1[256], r2[256];
  const int c = blockIdx.x;
  double s = 0.0, q = 0.0;
  for (size_t r = threadIdx.x; r < rows; r += blockDim.x) {
    const double v = X[r * ld + c];
    s += v;
    q += v * v;
  }
  r1[threadIdx.x] = s;
  r2[threadIdx.x] = q;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      r1[threadIdx.x] += r1[threadIdx.x + w];
      r2[threadIdx.x] += r2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sum[c] = r1[0];
    sumsq[c] = r2[0];
  }
}

// Raw feature values (no normalisation, FP32) for statistics.
__global__ void gather_raw_kernel(GatherArgs a, float* out) {
  const int n = a.n, nb = n * n * n;
  const size_t total = static_cast<size_t>(a.Nx) * a.Nu * a.Nv * a.nfeat;
  const size_t tid = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tid >= total) return;
  const int col = static_cast<int>(tid % a.nfeat);
  const size_t e = tid / a.nfeat;
  const int iv = static_cast<int>(e % a.Nv);
  const int iu = static_cast<int>((e / a.Nv) % a.Nu);
  const int ix = static_cast<int>(e / (static_cast<size_t>(a.Nv) * a.Nu));
  float val;
  if (col < 7 * nb) {
    const int blk = col / nb, loc = col % nb;
    int ex = ix, eu = iu, ev = iv;
    switch (blk) {
      case 1: ex = ix == 0 ? a.Nx - 1 : ix - 1; break;
      case 2: ex = ix == a.Nx - 1 ? 0 : ix + 1; break;
      case 3: eu = iu == 0 ? a.Nu - 1 : iu - 1; break;
      case 4: eu = iu == a.Nu - 1 ? 0 : iu + 1; break;
      case 5: ev = iv == 0 ? a.Nv - 1 : iv - 1; break;
      case 6: ev = iv == a.Nv - 1 ? 0 : iv + 1; break;
      default: break;
    }
    const int jx = loc / (n * n), ju = (loc / n) % n, jv = loc % n;
    val = a.f[((((static_cast<size_t>(ex) * n + jx) * a.Nu + eu) * n + ju) * a.Nv + ev) * n + jv];
  } else {
    val = static_cast<float>(a.E[ix * n + (col - 7 * nb)]);
  }
  out[tid] = val;
}

// Element-major copy of scale * (in - sub) (sub optional) for a state-layout
// array (training targets).
__global__ void to_elements_kernel(const float* in, const float* sub, float scale, float* out, int n, int Nx, int Nu, int Nv) {
  const int nb = n * n * n;
  const size_t total = static_cast<size_t>(Nx) * Nu * Nv * nb;
  const size_t tid = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tid >= total) return;
  const int loc = static_cast<int>(tid % nb);
  const size_t e = tid / nb;
  const int iv = static_cast<int>(e % Nv);
  const int iu = static_cast<int>((e / Nv) % Nu);
  const int ix = static_cast<int>(e / (static_cast<size_t>(Nv) * Nu));
  const int jx = loc / (n * n), ju = (loc / n) % n, jv = loc % n;
  const size_t src = ((((static_cast<size_t>(ix) * n + jx) * Nu + iu) * n + ju) * Nv + iv) * n + jv;
  out[tid] = scale * (sub ? in[src] - sub[src] : in[src]);
}

__global__ void axpy_kernel(float* y, const float* x, float a, size_t n) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = __builtin_fmaf(a, x[i], y[i]);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(size_t n, int b) { return static_cast<unsigned>((n + b - 1) / b); }

hipError_t launch_project_axis(const ProjArgs& a, hipStream_t s) {
  const size_t total = static_cast<size_t>(a.outer) * a.Nc * a.nc * a.inner;
  hipLaunchKernelGGL(project_axis_kernel, dim3(nblk(total, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_f32_to_f64(const float* in, double* out, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(f32_to_f64_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}
hipError_t launch_f64_to_f32(const double* in, float* out, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}
hipError_t launch_gather(const GatherArgs& a, hipStream_t s) {
  const size_t total = static_cast<size_t>(a.Nx) * a.Nu * a.Nv * a.ld;
  hipLaunchKernelGGL(gather_kernel, dim3(nblk(total, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_gather_raw(const GatherArgs& a, float* out, hipStream_t s) {
  const size_t total = static_cast<size_t>(a.Nx) * a.Nu * a.Nv * a.nfeat;
  hipLaunchKernelGGL(gather_raw_kernel, dim3(nblk(total, 256)), dim3(256), 0, s, a, out);
  return hipGetLastError();
}
hipError_t launch_scatter(const ScatterArgs& a, hipStream_t s) {
  const size_t ne = static_cast<size_t>(a.Nx) * a.Nu * a.Nv;
  hipLaunchKernelGGL(scatter_kernel, dim3(nblk(ne, 128)), dim3(128), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_gemm(const GemmArgs& g, hipStream_t s) {
  hipLaunchKernelGGL(gemm_bf16_kernel, dim3((g.M + 15) / 16, (g.N + 15) / 16), dim3(kWave), 0, s, g);
  return hipGetLastError();
}
hipError_t launch_bias_act(const BiasActArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(bias_act_kernel, dim3(nblk(static_cast<size_t>(a.rows) * a.ld, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_gelu_back(const float* dA, const float* Z, float* dZ, uint16_t* dZb, int rows, int cols, int ld, hipStream_t s) {
  hipLaunchKernelGGL(gelu_back_kernel, dim3(nblk(static_cast<size_t>(rows) * ld, 256)), dim3(256), 0, s, dA, Z, dZ, dZb, rows, cols, ld);
  return hipGetLastError();
}
hipError_t launch_mse(const float* Y, const float* T, int rows, int cols, int ld, float inv_count, float* dY, uint16_t* dYb,
                      double* partial, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(mse_kernel, dim3(nblocks), dim3(256), 0, s, Y, T, rows, cols, ld, inv_count, dY, dYb, partial);
  return hipGetLastError();
}
hipError_t launch_colsum(const float* in, int rows, int cols, float* out, hipStream_t s) {
  hipLaunchKernelGGL(colsum_kernel, dim3(cols), dim3(256), 0, s, in, rows, cols, out);
  return hipGetLastError();
}
hipError_t launch_adamw(const AdamArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(adamw_kernel, dim3(nblk(a.count, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_colstats(const float* X, size_t rows, int ld, int cols, double* sum, double* sumsq, hipStream_t s) {
  hipLaunchKernelGGL(colstats_kernel, dim3(cols), dim3(256), 0, s, X, rows, ld, sum, sumsq);
  return hipGetLastError();
}
hipError_t launch_to_elements(const float* in, const float* sub, float scale, float* out, int n, int Nx, int Nu, int Nv, hipStream_t s) {
  const size_t total = static_cast<size_t>(Nx) * Nu * Nv * n * n * n;
  hipLaunchKernelGGL(to_elements_kernel, dim3(nblk(total, 256)), dim3(256), 0, s, in, sub, scale, out, n, Nx, Nu, Nv);
  return hipGetLastError();
}
hipError_t launch_axpy(float* y, const float* x, float a, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(axpy_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, y, x, a, n);
  return hipGetLastError();
}

}  // namespace dgn
