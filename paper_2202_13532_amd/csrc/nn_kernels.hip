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

#include <algorithm>
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
    const size_t q = ((static_cast<size_t>(eu) * n + ju) * a.Nv + ev) * n + jv;
    const size_t idx = (static_cast<size_t>(ex) * n + jx) * (static_cast<size_t>(a.Nu) * n * a.Nv * n) + q;
    val = a.xmean ? a.f[idx] - a.xmean[q] : a.f[idx];
  } else if (col < 7 * nb + n) {
    val = static_cast<float>(a.E[ix * n + (col - 7 * nb)]);
  } else if (a.xmean && col < 8 * nb + n) {
    const int loc = col - 7 * nb - n;
    const int ju = (loc / n) % n, jv = loc % n;
    val = a.xmean[((static_cast<size_t>(iu) * n + ju) * a.Nv + iv) * n + jv];
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

// ---------------------------------------------------------------------------
// LDS-tiled BF16 MFMA GEMM for the network's shapes (rows = 4096 per coarse
// state, or several states per training step; inner and outer sizes
// 64..464).  A 256-thread work-group computes a 64 x 64 tile of C, each wave
// a 32 x 32 quarter as 2 x 2 tiles of v_mfma_f32_16x16x32_bf16 (FP32
// accumulate).  Every global load of the work-group's k range (at most
// kMaxKT tiles of 32) is issued before the first MFMA into registers, so
// the load latency is paid once instead of once per k tile; the tiles then
// pass through a double-buffered LDS stage (one barrier per tile), stored
// with k contiguous so that each lane reads its 8 k values of a row or
// column with one 16-byte LDS read.  Global loads are 16 bytes (8 BF16)
// along the operand's contiguous direction: A with k (AK) or m contiguous,
// B with n (BN) or k contiguous.  Split-K: work-group z covers k in
// [z ks, (z+1) ks); with more than one slice, partial tiles go to `part`
// (slice-major, M x N each) and gemm_reduce_kernel adds the slices in order
// (deterministic).
// MFMA lane layout (16x16x32): A row l mod 16, k = 8 floor(l/16) + t,
// t = 0..7; B column l mod 16, same k; D column l mod 16, rows 4 floor(l/16)
// + t, t = 0..3.
// ---------------------------------------------------------------------------
constexpr int kTM = 64, kTN = 64, kTK = 32, kTLd = kTK + 8;   // LDS row: 40 BF16 (80 bytes)
constexpr int kMaxKT = 16;                                   // k tiles held in registers (k range <= 512)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// 8 consecutive BF16 base[start .. start + 8), zero at and beyond `bound`
// (base + start is 16-byte aligned when the 8 values are all in range)
__device__ __forceinline__ uint4 load8v(const uint16_t* base, int start, int bound) {
  if (start + 8 <= bound) return *reinterpret_cast<const uint4*>(base + start);
  uint16_t v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = start + i < bound ? base[start + i] : uint16_t(0);
  return uint4{v[0] | (uint32_t(v[1]) << 16), v[2] | (uint32_t(v[3]) << 16), v[4] | (uint32_t(v[5]) << 16),
               v[6] | (uint32_t(v[7]) << 16)};
}

// 8 values of one uint4 to LDS entries tile[(c + i) * kTLd + kk] (a transpose)
__device__ __forceinline__ void scatter8(uint16_t* tile, int c, int kk, uint4 v) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    tile[(c + 2 * i) * kTLd + kk] = static_cast<uint16_t>(w[i] & 0xffffu);
    tile[(c + 2 * i + 1) * kTLd + kk] = static_cast<uint16_t>(w[i] >> 16);
  }
}

template <bool AK, bool BN>
__global__ void __launch_bounds__(256) gemm_bf16_tiled_kernel(GemmArgs g, float* part, int ks) {
  __shared__ uint16_t As[2][kTM * kTLd];
  __shared__ uint16_t Bs[2][kTN * kTLd];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * kTM, n0 = blockIdx.y * kTN;
  const int kb = blockIdx.z * ks, ke = min(g.K, kb + ks);
  const int nt = (ke - kb + kTK - 1) / kTK;   // <= kMaxKT (launch_gemm_tiled bounds ks)
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  // load roles: (row r, k chunk 8 q) for operands stored with k contiguous,
  // (k row kk, chunk of 8 along m or n) for the others
  const int r4 = tid >> 2, q4 = (tid & 3) * 8, kk8 = tid >> 3, c8 = (tid & 7) * 8;
  uint4 ra[kMaxKT], rb[kMaxKT];
#pragma unroll
  for (int t = 0; t < kMaxKT; ++t) {
    if (t < nt) {
      const int k0 = kb + t * kTK;
      if (AK) {
        const int m = m0 + r4;
        ra[t] = m < g.M ? load8v(g.A + static_cast<size_t>(m) * g.sam, k0 + q4, ke) : uint4{0, 0, 0, 0};
      } else {
        const int k = k0 + kk8;
        ra[t] = k < ke ? load8v(g.A + static_cast<size_t>(k) * g.sak, m0 + c8, g.M) : uint4{0, 0, 0, 0};
      }
      if (BN) {
        const int k = k0 + kk8;
        rb[t] = k < ke ? load8v(g.B + static_cast<size_t>(k) * g.sbk, n0 + c8, g.N) : uint4{0, 0, 0, 0};
      } else {
        const int n = n0 + r4;
        rb[t] = n < g.N ? load8v(g.B + static_cast<size_t>(n) * g.sbn, k0 + q4, ke) : uint4{0, 0, 0, 0};
      }
    }
  }
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int t = 0; t < kMaxKT; ++t) {
    if (t < nt) {   // uniform over the work-group
      // buffer t & 1 was last read in tile t - 2, before every thread passed
      // the barrier of tile t - 1
      uint16_t* as = As[t & 1];
      uint16_t* bs = Bs[t & 1];
      if (AK) *reinterpret_cast<uint4*>(&as[r4 * kTLd + q4]) = ra[t];
      else scatter8(as, c8, kk8, ra[t]);
      if (BN) scatter8(bs, c8, kk8, rb[t]);
      else *reinterpret_cast<uint4*>(&bs[r4 * kTLd + q4]) = rb[t];
      __syncthreads();
      const int kq = 8 * (lane >> 4);
      bf16x8 af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        af[i] = *reinterpret_cast<const bf16x8*>(&as[(wm + 16 * i + (lane & 15)) * kTLd + kq]);
        bf[i] = *reinterpret_cast<const bf16x8*>(&bs[(wn + 16 * i + (lane & 15)) * kTLd + kq]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  }
  // D layout: column lane % 16, rows 4 (lane / 16) + t
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn + 16 * j + (lane & 15);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + t;
        if (m < g.M && n < g.N) {
          if (part) part[(static_cast<size_t>(blockIdx.z) * g.M + m) * g.N + n] = acc[i][j][t];
          else g.C[static_cast<size_t>(m) * g.scm + static_cast<size_t>(n) * g.scn] = acc[i][j][t];
        }
      }
    }
}

// C(m, n) = sum over the slices in order.
__global__ void gemm_reduce_kernel(const float* part, int slices, GemmArgs g) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t mn = static_cast<size_t>(g.M) * g.N;
  if (i >= mn) return;
  float s = 0.0f;
#pragma unroll 8
  for (int z = 0; z < slices; ++z) s += part[z * mn + i];
  const size_t m = i / g.N, n = i % g.N;
  g.C[m * g.scm + n * g.scn] = s;
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
    const size_t q = ((static_cast<size_t>(eu) * n + ju) * a.Nv + ev) * n + jv;
    const size_t idx = (static_cast<size_t>(ex) * n + jx) * (static_cast<size_t>(a.Nu) * n * a.Nv * n) + q;
    val = a.xmean ? a.f[idx] - a.xmean[q] : a.f[idx];
  } else if (col < 7 * nb + n) {
    val = static_cast<float>(a.E[ix * n + (col - 7 * nb)]);
  } else if (a.xmean) {
    const int loc = col - 7 * nb - n;
    const int ju = (loc / n) % n, jv = loc % n;
    val = a.xmean[((static_cast<size_t>(iu) * n + ju) * a.Nv + iv) * n + jv];
  }
  out[tid] = val;
}

// Element-major copy of scale * (in - sub - xm) (sub, xm optional) for a
// state-layout array (training targets; xm per (u, v) node).
__global__ void to_elements_kernel(const float* in, const float* sub, const float* xm, float scale, float* out, int n, int Nx,
                                   int Nu, int Nv) {
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
  const size_t q = ((static_cast<size_t>(iu) * n + ju) * Nv + iv) * n + jv;
  const size_t src = (static_cast<size_t>(ix) * n + jx) * (static_cast<size_t>(Nu) * n * Nv * n) + q;
  float v = sub ? in[src] - sub[src] : in[src];
  if (xm) v -= xm[q];
  out[tid] = scale * v;
}

// FP64 versions for targets built from FP64 right-hand sides: the x average
// of (x - sub) in FP64, and the element-major FP32 copy of scale * (x - sub - xm).
__global__ void xmean_diff64_kernel(const double* x, const double* sub, const double* wx, double* out, int outer, size_t inner) {
  const size_t q = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= inner) return;
  double s = 0.0, w = 0.0;
  for (int o = 0; o < outer; ++o) {
    const size_t i = static_cast<size_t>(o) * inner + q;
    s += wx[o] * (sub ? x[i] - sub[i] : x[i]);
    w += wx[o];
  }
  out[q] = s / w;
}

__global__ void to_elements64_kernel(const double* in, const double* sub, const double* xm, float scale, float* out, int n,
                                     int Nx, int Nu, int Nv) {
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
  const size_t q = ((static_cast<size_t>(iu) * n + ju) * Nv + iv) * n + jv;
  const size_t src = (static_cast<size_t>(ix) * n + jx) * (static_cast<size_t>(Nu) * n * Nv * n) + q;
  double v = sub ? in[src] - sub[src] : in[src];
  if (xm) v -= xm[q];
  out[tid] = static_cast<float>(static_cast<double>(scale) * v);
}

__global__ void axpy_kernel(float* y, const float* x, const float* xm, float a, size_t outer, size_t inner) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= outer * inner) return;
  const float v = xm ? x[i] - xm[i % inner] : x[i];
  y[i] = __builtin_fmaf(a, v, y[i]);
}

// LGL-weighted average over the outer (x node) index, one thread per inner
// index, FP64 sum in a fixed order.
__global__ void xmean_kernel(const float* in, const double* wx, float* out, int outer, size_t inner) {
  const size_t q = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= inner) return;
  double s = 0.0, w = 0.0;
  for (int o = 0; o < outer; ++o) {
    const double wo = wx[o];
    s += wo * in[static_cast<size_t>(o) * inner + q];
    w += wo;
  }
  out[q] = static_cast<float>(s / w);
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

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

hipError_t launch_gemm_tiled(const GemmArgs& g, float* part, size_t part_floats, int cus, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.K <= 0) return hipErrorInvalidValue;
  const bool ak = g.sak == 1, bn = g.sbn == 1;
  const bool am = !ak && g.sam == 1, bk = !bn && g.sbk == 1;
  // the 16-byte loads need 16-byte aligned rows of the contiguous direction
  const size_t sa = ak ? g.sam : g.sak, sb = bn ? g.sbk : g.sbn;
  if (!(ak || am) || !(bn || bk) || !aligned16(g.A) || !aligned16(g.B) || (sa % 8) || (sb % 8)) return launch_gemm(g, s);
  const int tiles = ((g.M + kTM - 1) / kTM) * ((g.N + kTN - 1) / kTN);
  // split K (the weight gradients: K = rows) until there are about two
  // work-groups per CU, keeping slices of >= 256 so the reduction stays short
  int slices = 1;
  while (tiles * slices < 2 * cus && g.K / (2 * slices) >= 256) slices *= 2;
  // each slice's k range must fit the kernel's register stage
  int smin = 1;
  while (static_cast<long long>(smin) * kMaxKT * kTK < g.K) smin *= 2;
  slices = std::max(slices, smin);
  while (slices > smin && static_cast<size_t>(slices) * g.M * g.N > part_floats) slices /= 2;
  if (slices > 1 && static_cast<size_t>(slices) * g.M * g.N > part_floats) return launch_gemm(g, s);
  const int ks = ((g.K + slices - 1) / slices + kTK - 1) / kTK * kTK;
  slices = (g.K + ks - 1) / ks;
  if (ks > kMaxKT * kTK) return hipErrorInvalidValue;
  float* p = slices > 1 ? part : nullptr;
  const dim3 grid((g.M + kTM - 1) / kTM, (g.N + kTN - 1) / kTN, slices);
  if (ak && bn) hipLaunchKernelGGL((gemm_bf16_tiled_kernel<true, true>), grid, dim3(256), 0, s, g, p, ks);
  else if (ak) hipLaunchKernelGGL((gemm_bf16_tiled_kernel<true, false>), grid, dim3(256), 0, s, g, p, ks);
  else if (bn) hipLaunchKernelGGL((gemm_bf16_tiled_kernel<false, true>), grid, dim3(256), 0, s, g, p, ks);
  else hipLaunchKernelGGL((gemm_bf16_tiled_kernel<false, false>), grid, dim3(256), 0, s, g, p, ks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || slices == 1) return e;
  const size_t mn = static_cast<size_t>(g.M) * g.N;
  hipLaunchKernelGGL(gemm_reduce_kernel, dim3(nblk(mn, 256)), dim3(256), 0, s, part, slices, g);
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
hipError_t launch_to_elements(const float* in, const float* sub, const float* xm, float scale, float* out, int n, int Nx,
                              int Nu, int Nv, hipStream_t s) {
  const size_t total = static_cast<size_t>(Nx) * Nu * Nv * n * n * n;
  hipLaunchKernelGGL(to_elements_kernel, dim3(nblk(total, 256)), dim3(256), 0, s, in, sub, xm, scale, out, n, Nx, Nu, Nv);
  return hipGetLastError();
}
hipError_t launch_axpy(float* y, const float* x, const float* xm, float a, size_t outer, size_t inner, hipStream_t s) {
  hipLaunchKernelGGL(axpy_kernel, dim3(nblk(outer * inner, 256)), dim3(256), 0, s, y, x, xm, a, outer, inner);
  return hipGetLastError();
}
hipError_t launch_xmean_diff64(const double* x, const double* sub, const double* wx, double* out, int outer, size_t inner,
                               hipStream_t s) {
  hipLaunchKernelGGL(xmean_diff64_kernel, dim3(nblk(inner, 256)), dim3(256), 0, s, x, sub, wx, out, outer, inner);
  return hipGetLastError();
}
hipError_t launch_to_elements64(const double* in, const double* sub, const double* xm, float scale, float* out, int n, int Nx,
                                int Nu, int Nv, hipStream_t s) {
  const size_t total = static_cast<size_t>(Nx) * Nu * Nv * n * n * n;
  hipLaunchKernelGGL(to_elements64_kernel, dim3(nblk(total, 256)), dim3(256), 0, s, in, sub, xm, scale, out, n, Nx, Nu, Nv);
  return hipGetLastError();
}
hipError_t launch_xmean(const float* in, const double* wx, float* out, int outer, size_t inner, hipStream_t s) {
  hipLaunchKernelGGL(xmean_kernel, dim3(nblk(inner, 256)), dim3(256), 0, s, in, wx, out, outer, inner);
  return hipGetLastError();
}

}  // namespace dgn
