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
//   gemm_bf16_tiled_kernel  C = A B with v_mfma_f32_16x16x32_bf16, a 64x64
//                        tile of C per work-group, split K with an ordered
//                        reduction (gemm_reduce_kernel); the same kernel
//                        serves X W, dY W^T and X^T dY, and the forward
//                        layers take bias + GELU + BF16 conversion in its
//                        epilogue.
//   gemm_bf16_kernel     fallback for operands without a unit stride: one
//                        wave per 16x16 tile with v_mfma_f32_16x16x16_bf16.
//   gelu_back_kernel, mse_kernel, colsum_kernel,
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

// Final value of C(m, n): a plain store, or the fused layer epilogue.
__device__ __forceinline__ void gemm_store(const GemmArgs& g, int m, int n, float acc) {
  if (!g.epi) {
    g.C[static_cast<size_t>(m) * g.scm + static_cast<size_t>(n) * g.scn] = acc;
    return;
  }
  const float z = acc + (g.bias ? g.bias[n] : 0.0f);
  const size_t zi = static_cast<size_t>(m) * g.N + n;
  if (g.Z) g.Z[zi] = z;
  const float v = g.gelu ? gelu(z) : z;
  if (g.Af) g.Af[zi] = v;
  if (g.Abf) g.Abf[static_cast<size_t>(m) * g.lda + n] = f2bf(v);
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
// One work-group per row; 32-bit index arithmetic (launch_gather checks that
// rows x ld and the state size fit).  With one thread per (row, column) and
// the node count a run-time value, ten integer divisions per feature made
// the kernel 12.5 us for 4096 rows of 464 columns.
// ---------------------------------------------------------------------------
// Feature `col` of the row of element (ix, iu, iv), normalised (0 for
// padding columns); N = a.n, a compile-time constant so that the node
// indices come from multiply-shift sequences instead of divisions.
template <int N>
__device__ __forceinline__ float gather_value(const GatherArgs& a, int ix, int iu, int iv, int col) {
  constexpr int nb = N * N * N;
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
    const int jx = loc / (N * N), ju = (loc / N) % N, jv = loc % N;
    const unsigned q = ((static_cast<unsigned>(eu) * N + ju) * a.Nv + ev) * N + jv;
    const unsigned idx = (static_cast<unsigned>(ex) * N + jx) * (static_cast<unsigned>(a.Nu) * N * a.Nv * N) + q;
    val = a.xmean ? a.f[idx] - a.xmean[q] : a.f[idx];
  } else if (col < 7 * nb + N) {
    val = static_cast<float>(a.E[ix * N + (col - 7 * nb)]);
  } else if (a.xmean && col < 8 * nb + N) {
    const int loc = col - 7 * nb - N;
    const int ju = (loc / N) % N, jv = loc % N;
    val = a.xmean[((static_cast<unsigned>(iu) * N + ju) * a.Nv + iv) * N + jv];
  }
  return col < a.nfeat ? (val - a.mean[col]) * a.inv_std[col] : 0.0f;
}

// One work-group per row (element): the element's indices once, in scalar
// registers; the threads stride over the row's ld columns.
template <int N>
__global__ void __launch_bounds__(256) gather_kernel(GatherArgs a) {
  const unsigned e = blockIdx.x;
  const int iv = static_cast<int>(e % static_cast<unsigned>(a.Nv));
  const unsigned e2 = e / static_cast<unsigned>(a.Nv);
  const int iu = static_cast<int>(e2 % static_cast<unsigned>(a.Nu));
  const int ix = static_cast<int>(e2 / static_cast<unsigned>(a.Nu));
  uint16_t* row = a.X + static_cast<size_t>(e) * a.ld;
  for (int col = threadIdx.x; col < a.ld; col += 256) row[col] = f2bf(gather_value<N>(a, ix, iu, iv, col));
}

// Network output Y[e][loc] (loc = (jx*n + ju)*n + jv), scaled by `scale`,
// minus its element mean under the product LGL weights w_jx w_ju w_jv, written
// to the state layout (FP32).  One 64-lane wave per element: the lanes stride
// over the n^3 nodes, the weighted sum is formed in FP64 and combined by a
// fixed butterfly (reproducible), and the outputs are written by node.
__global__ void __launch_bounds__(kWave) scatter_kernel(ScatterArgs a) {
  const int n = a.n, nn = n * n, nb = nn * n;
  const unsigned e = blockIdx.x;   // element, v fastest
  const int lane = threadIdx.x;
  const int iv = static_cast<int>(e % static_cast<unsigned>(a.Nv));
  const unsigned e2 = e / static_cast<unsigned>(a.Nv);
  const int iu = static_cast<int>(e2 % static_cast<unsigned>(a.Nu));
  const int ix = static_cast<int>(e2 / static_cast<unsigned>(a.Nu));
  const float* y = a.Y + static_cast<size_t>(e) * a.ldy;
  float mean = 0.0f;
  if (a.mass_neutral) {
    double num = 0.0;   // FP64: the removed mean must not carry a rounding bias
    for (int i = lane; i < nb; i += kWave) {
      const int jx = i / nn, ju = (i / n) % n, jv = i % n;
      num += static_cast<double>(a.w[jx]) * a.w[ju] * a.w[jv] * y[i];
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) num += __shfl_xor(num, off);
    double sw = 0.0;
    for (int j = 0; j < n; ++j) sw += a.w[j];
    mean = static_cast<float>(num / (sw * sw * sw));
  }
  for (int i = lane; i < nb; i += kWave) {
    const int jx = i / nn, ju = (i / n) % n, jv = i % n;
    const size_t idx = ((((static_cast<size_t>(ix) * n + jx) * a.Nu + iu) * n + ju) * a.Nv + iv) * n + jv;
    a.out[idx] = a.scale * (y[i] - mean);
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
      if (g.epi) {
        gemm_store(g, cm, cn, acc[t]);
      } else {
        float* c = g.C + static_cast<size_t>(cm) * g.scm + static_cast<size_t>(cn) * g.scn;
        *c = g.beta != 0.0f ? acc[t] + g.beta * *c : acc[t];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// LDS-tiled BF16 MFMA GEMM for the network's shapes (rows = 4096 per coarse
// state, or several states per training step; inner and outer sizes
// 64..464).  A 256-thread work-group computes a 64 x 64 tile of C, each wave
// a 32 x 32 quarter as 2 x 2 tiles of v_mfma_f32_16x16x32_bf16 (FP32
// accumulate); when 64-row tiles would leave CUs idle, 32-row tiles (each
// wave 16 x 32) double the work-groups.  Every global load of the work-group's k range (at most
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

template <bool AK, bool BN, int TM>
__global__ void __launch_bounds__(256) gemm_bf16_tiled_kernel(GemmArgs g, float* part, int ks) {
  constexpr int MI = TM / 32;   // 16-row MFMA tiles per wave along m
  __shared__ uint16_t As[2][TM * kTLd];
  __shared__ uint16_t Bs[2][kTN * kTLd];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * TM, n0 = blockIdx.y * kTN;
  const int kb = blockIdx.z * ks, ke = min(g.K, kb + ks);
  const int nt = (ke - kb + kTK - 1) / kTK;   // <= kMaxKT (launch_gemm_tiled bounds ks)
  const int wm = (wave >> 1) * (TM / 2), wn = (wave & 1) * 32;
  // load roles: (row r, k chunk 8 q) for operands stored with k contiguous,
  // (k row kk, chunk of 8 along m or n) for the others; with TM = 32 half of
  // the threads have no A role
  const int r4 = tid >> 2, q4 = (tid & 3) * 8, kk8 = tid >> 3, c8 = (tid & 7) * 8;
  const bool arole = AK ? r4 < TM : c8 < TM;
  uint4 ra[kMaxKT], rb[kMaxKT];
#pragma unroll
  for (int t = 0; t < kMaxKT; ++t) {
    if (t < nt) {
      const int k0 = kb + t * kTK;
      if (!arole) {
        ra[t] = uint4{0, 0, 0, 0};
      } else if (AK) {
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
  f32x4 acc[MI][2];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int t = 0; t < kMaxKT; ++t) {
    if (t < nt) {   // uniform over the work-group
      // buffer t & 1 was last read in tile t - 2, before every thread passed
      // the barrier of tile t - 1
      uint16_t* as = As[t & 1];
      uint16_t* bs = Bs[t & 1];
      if (arole) {
        if (AK) *reinterpret_cast<uint4*>(&as[r4 * kTLd + q4]) = ra[t];
        else scatter8(as, c8, kk8, ra[t]);
      }
      if (BN) scatter8(bs, c8, kk8, rb[t]);
      else *reinterpret_cast<uint4*>(&bs[r4 * kTLd + q4]) = rb[t];
      __syncthreads();
      const int kq = 8 * (lane >> 4);
      bf16x8 af[MI], bf[2];
#pragma unroll
      for (int i = 0; i < MI; ++i) af[i] = *reinterpret_cast<const bf16x8*>(&as[(wm + 16 * i + (lane & 15)) * kTLd + kq]);
#pragma unroll
      for (int i = 0; i < 2; ++i) bf[i] = *reinterpret_cast<const bf16x8*>(&bs[(wn + 16 * i + (lane & 15)) * kTLd + kq]);
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  }
  // D layout: column lane % 16, rows 4 (lane / 16) + t
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn + 16 * j + (lane & 15);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + t;
        if (m < g.M && n < g.N) {
          if (part) part[(static_cast<size_t>(blockIdx.z) * g.M + m) * g.N + n] = acc[i][j][t];
          else gemm_store(g, m, n, acc[i][j][t]);
        }
      }
    }
}

// ---------------------------------------------------------------------------
// Fused inference: a work-group of kMlpWaves waves takes kMlpRows rows
// through every layer.  The input rows are staged in LDS (k contiguous, zero
// beyond ldx); each layer's 16-column output tiles are dealt round-robin to
// the waves (one each at width 128: the per-wave chain of dependent
// instructions is what bounds this latency-bound kernel),
// each tile's B operand read straight from the transposed weights (8 k
// values of one column = one 16-byte load).  The weights do not depend on
// the activations, so their loads are not left on the critical path: layer
// 0's (its k range up to kMlpKT0 tiles) go out before the input staging,
// and each hidden layer's (at most kMlpMaxOut / 32 k tiles) while the layer
// before it computes.  The epilogue adds the bias, applies GELU (hidden
// layers) and writes the BF16 activations to the other LDS buffer, or the
// FP32 outputs (last layer).  One row tile of 16: the weights are read once
// per work-group, from L2, and 16-row work-groups spread a few thousand rows
// over all CUs.
// ---------------------------------------------------------------------------
constexpr int kMlpRows = 16, kMlpWaves = 8, kMlpThreads = 64 * kMlpWaves;
constexpr int kMlpTilesPerWave = (kMlpMaxOut / 16 + kMlpWaves - 1) / kMlpWaves;
constexpr int kMlpKT0 = 16;                  // layer-0 k tiles held in registers (inputs <= 512 in one pass)
constexpr int kMlpXB = 4;                    // input-staging loads in flight per thread
constexpr int kMlpKTH = kMlpMaxOut / 32;     // k tiles of a hidden layer
constexpr int kMlpHLd = kMlpMaxOut + 8;      // hidden LDS row (BF16), padded against bank conflicts
constexpr int kMlpXLd = kMlpMaxIn + 8;

// B operand of k tile kt for the wave's tile j of a layer (zero where the
// column or k tile is out of range)
__device__ __forceinline__ bf16x8 mlp_b(const uint16_t* Wt, int kp, int out, int ntiles, int wave, int j, int kt, int nkt,
                                       int lane) {
  const int col = (wave + kMlpWaves * j) * 16 + (lane & 15);
  if (wave + kMlpWaves * j >= ntiles || col >= out || kt >= nkt) return bf16x8{};
  return *reinterpret_cast<const bf16x8*>(Wt + static_cast<size_t>(col) * kp + 32 * kt + 8 * (lane >> 4));
}

__global__ void __launch_bounds__(kMlpThreads) mlp_fused_kernel(MlpArgs a) {
  __shared__ uint16_t Xs[kMlpRows * kMlpXLd];
  __shared__ uint16_t Hs[2][kMlpRows * kMlpHLd];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * kMlpRows;
  // layer-0 weights (first kMlpKT0 k tiles) first: the longest loads
  bf16x8 b0[kMlpTilesPerWave][kMlpKT0];
  {
    const int nkt = a.kp[0] / 32, nt = (a.out[0] + 15) / 16;
#pragma unroll
    for (int j = 0; j < kMlpTilesPerWave; ++j)
#pragma unroll
      for (int q = 0; q < kMlpKT0; ++q) b0[j][q] = mlp_b(a.Wt[0], a.kp[0], a.out[0], nt, wave, j, q, nkt, lane);
  }
  // input rows, 8 BF16 per thread and load, kMlpXB loads in flight, zero
  // past the row's end
  const int kp0 = a.kp[0], xtot = kMlpRows * kp0;
  for (int e0 = tid * 8; e0 < xtot; e0 += kMlpThreads * 8 * kMlpXB) {
    uint4 v[kMlpXB];
#pragma unroll
    for (int i = 0; i < kMlpXB; ++i) {
      const int e = e0 + kMlpThreads * 8 * i, r = e / kp0, k = e % kp0, m = m0 + r;
      v[i] = (e < xtot && m < a.rows) ? load8v(a.X + static_cast<size_t>(m) * a.ldx, k, a.ldx) : uint4{0, 0, 0, 0};
    }
#pragma unroll
    for (int i = 0; i < kMlpXB; ++i) {
      const int e = e0 + kMlpThreads * 8 * i, r = e / kp0, k = e % kp0;
      if (e < xtot) *reinterpret_cast<uint4*>(&Xs[r * kMlpXLd + k]) = v[i];
    }
  }
  __syncthreads();
  bf16x8 bh[kMlpTilesPerWave][kMlpKTH];   // the current hidden layer's weights
  for (int l = 0; l < a.L; ++l) {
    const uint16_t* As = l == 0 ? Xs : Hs[(l - 1) & 1];
    const int lda = l == 0 ? kMlpXLd : kMlpHLd;
    const int out = a.out[l], kp = a.kp[l], nkt = kp / 32;
    const bool last = l == a.L - 1;
    const int ntiles = (out + 15) / 16;
    // next layer's weights, in flight while this layer computes
    bf16x8 bnext[kMlpTilesPerWave][kMlpKTH];
    if (!last) {
      const int kpn = a.kp[l + 1], ntn = (a.out[l + 1] + 15) / 16;
#pragma unroll
      for (int j = 0; j < kMlpTilesPerWave; ++j)
#pragma unroll
        for (int q = 0; q < kMlpKTH; ++q) bnext[j][q] = mlp_b(a.Wt[l + 1], kpn, a.out[l + 1], ntn, wave, j, q, kpn / 32, lane);
    }
    const uint16_t* arow = As + (lane & 15) * lda + 8 * (lane >> 4);
    f32x4 acc[kMlpTilesPerWave];
#pragma unroll
    for (int j = 0; j < kMlpTilesPerWave; ++j) acc[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    if (l == 0) {
#pragma unroll
      for (int q = 0; q < kMlpKT0; ++q) {
        if (q < nkt) {   // uniform
          const bf16x8 af = *reinterpret_cast<const bf16x8*>(arow + 32 * q);
#pragma unroll
          for (int j = 0; j < kMlpTilesPerWave; ++j)
            if (wave + kMlpWaves * j < ntiles) acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, b0[j][q], acc[j], 0, 0, 0);
        }
      }
      // inputs wider than kMlpKT0 k tiles: the rest, loaded as it is used
      for (int q = kMlpKT0; q < nkt; ++q) {
        const bf16x8 af = *reinterpret_cast<const bf16x8*>(arow + 32 * q);
#pragma unroll
        for (int j = 0; j < kMlpTilesPerWave; ++j)
          if (wave + kMlpWaves * j < ntiles)
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, mlp_b(a.Wt[0], kp, out, ntiles, wave, j, q, nkt, lane),
                                                             acc[j], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int q = 0; q < kMlpKTH; ++q) {
        if (q < nkt) {   // uniform
          const bf16x8 af = *reinterpret_cast<const bf16x8*>(arow + 32 * q);
#pragma unroll
          for (int j = 0; j < kMlpTilesPerWave; ++j)
            if (wave + kMlpWaves * j < ntiles) acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bh[j][q], acc[j], 0, 0, 0);
        }
      }
    }
    // epilogue: D column lane % 16, rows 4 (lane / 16) + t
    uint16_t* Hn = Hs[l & 1];
    const int kpn = last ? 0 : a.kp[l + 1];
#pragma unroll
    for (int j = 0; j < kMlpTilesPerWave; ++j) {
      const int col = (wave + kMlpWaves * j) * 16 + (lane & 15);
      if (wave + kMlpWaves * j >= ntiles) continue;
      const float b = col < out ? a.bias[l][col] : 0.0f;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = 4 * (lane >> 4) + t, m = m0 + r;
        const float z = acc[j][t] + b;
        if (last) {
          if (m < a.rows && col < out) a.Y[static_cast<size_t>(m) * out + col] = z;
        } else if (col < kpn) {
          // zero in the padding columns: the next layer reads k up to kp
          Hn[r * kMlpHLd + col] = col < out ? f2bf(gelu(z)) : uint16_t(0);
        }
      }
    }
    // padding columns of the next layer's input beyond the last output tile
    if (!last) {
      if (ntiles * 16 < kpn) {   // uniform: only when out is not a multiple of 16 below kpn
        for (int e = tid; e < kMlpRows * kpn; e += kMlpThreads) {
          const int r = e / kpn, k = e % kpn;
          if (k >= ntiles * 16) Hn[r * kMlpHLd + k] = 0;
        }
      }
#pragma unroll
      for (int j = 0; j < kMlpTilesPerWave; ++j)
#pragma unroll
        for (int q = 0; q < kMlpKTH; ++q) bh[j][q] = bnext[j][q];
    }
    __syncthreads();
  }
}

// Wt[n * kp + k] = W[k * out + n] (zero for k >= in).
__global__ void transpose_weights_kernel(const uint16_t* W, int in, int out, int kp, uint16_t* Wt) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= static_cast<size_t>(out) * kp) return;
  const int n = static_cast<int>(i / kp), k = static_cast<int>(i % kp);
  Wt[i] = k < in ? W[static_cast<size_t>(k) * out + n] : uint16_t(0);
}

// C(m, n) = sum over the slices in order.
__global__ void gemm_reduce_kernel(const float* part, int slices, GemmArgs g) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t mn = static_cast<size_t>(g.M) * g.N;
  if (i >= mn) return;
  float s = 0.0f;
#pragma unroll 8
  for (int z = 0; z < slices; ++z) s += part[z * mn + i];
  gemm_store(g, static_cast<int>(i / g.N), static_cast<int>(i % g.N), s);
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

// Column sums of a rows x cols FP32 matrix in two fixed-order passes:
// colsum_part_kernel: work-group (column block of 64, row slice z) -> each
// thread sums every 4th row of the slice for one column (coalesced 256-byte
// rows), the four row groups are added in order -> part[z][col];
// colsum_final_kernel: out[col] = sum over the slices in order.
__global__ void __launch_bounds__(256) colsum_part_kernel(const float* in, int rows, int cols, int per, float* part) {
  __shared__ float red[256];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), g = threadIdx.x >> 6;
  const int r0 = blockIdx.y * per, r1 = min(rows, r0 + per);
  float acc = 0.0f;
  // unrolled so that the loads are in flight together (the sum order is fixed)
  if (c < cols) {
#pragma unroll 16
    for (int r = r0 + g; r < r1; r += 4) acc += in[static_cast<size_t>(r) * cols + c];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if (g == 0 && c < cols)
    part[static_cast<size_t>(blockIdx.y) * cols + c] =
        ((red[threadIdx.x] + red[threadIdx.x + 64]) + red[threadIdx.x + 128]) + red[threadIdx.x + 192];
}
__global__ void colsum_final_kernel(const float* part, int slices, int cols, float* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  // all loads issued before the first add (clamped rows, then masked), the
  // additions in slice order
  float v[kColsumPart];
#pragma unroll
  for (int z = 0; z < kColsumPart; ++z) v[z] = part[static_cast<size_t>(min(z, slices - 1)) * cols + c];
  float acc = 0.0f;
#pragma unroll
  for (int z = 0; z < kColsumPart; ++z) acc += z < slices ? v[z] : 0.0f;
  out[c] = acc;
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
#pragma unroll 8
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
  const size_t rows = static_cast<size_t>(a.Nx) * a.Nu * a.Nv;
  const size_t state = rows * a.n * a.n * a.n;
  if (rows * a.ld > 0x7fffffff || state > 0x7fffffff) return hipErrorInvalidValue;   // 32-bit indices
  const dim3 g(static_cast<unsigned>(rows));
  switch (a.n) {
#define DGN_GATHER_CASE(NN) \
  case NN: hipLaunchKernelGGL(gather_kernel<NN>, g, dim3(256), 0, s, a); break;
    DGN_GATHER_CASE(2) DGN_GATHER_CASE(3) DGN_GATHER_CASE(4) DGN_GATHER_CASE(5) DGN_GATHER_CASE(6)
    DGN_GATHER_CASE(7) DGN_GATHER_CASE(8) DGN_GATHER_CASE(9) DGN_GATHER_CASE(10) DGN_GATHER_CASE(11)
    DGN_GATHER_CASE(12)
#undef DGN_GATHER_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_gather_raw(const GatherArgs& a, float* out, hipStream_t s) {
  const size_t total = static_cast<size_t>(a.Nx) * a.Nu * a.Nv * a.nfeat;
  hipLaunchKernelGGL(gather_raw_kernel, dim3(nblk(total, 256)), dim3(256), 0, s, a, out);
  return hipGetLastError();
}
hipError_t launch_scatter(const ScatterArgs& a, hipStream_t s) {
  const size_t ne = static_cast<size_t>(a.Nx) * a.Nu * a.Nv;
  if (ne > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(scatter_kernel, dim3(static_cast<unsigned>(ne)), dim3(kWave), 0, s, a);
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
  // split K (the weight gradients: K = rows) until there are about two
  // work-groups per CU, keeping slices of >= 256 so the reduction stays short;
  // each slice's k range must also fit the kernel's register stage
  int smin = 1;
  while (static_cast<long long>(smin) * kMaxKT * kTK < g.K) smin *= 2;
  auto split = [&](int tiles) {
    int sl = 1;
    while (tiles * sl < 2 * cus && g.K / (2 * sl) >= 256) sl *= 2;
    return std::max(sl, smin);
  };
  // 64-row tiles while tiles x slices fill the CUs, else 32-row tiles (twice
  // the work-groups)
  int tm = kTM;
  int tiles = ((g.M + tm - 1) / tm) * ((g.N + kTN - 1) / kTN);
  int slices = split(tiles);
  if (tiles * slices < cus) {
    tm = kTM / 2;
    tiles = ((g.M + tm - 1) / tm) * ((g.N + kTN - 1) / kTN);
    slices = split(tiles);
  }
  while (slices > smin && static_cast<size_t>(slices) * g.M * g.N > part_floats) slices /= 2;
  if (slices > 1 && static_cast<size_t>(slices) * g.M * g.N > part_floats) return launch_gemm(g, s);
  const int ks = ((g.K + slices - 1) / slices + kTK - 1) / kTK * kTK;
  slices = (g.K + ks - 1) / ks;
  if (ks > kMaxKT * kTK) return hipErrorInvalidValue;
  float* p = slices > 1 ? part : nullptr;
  const dim3 grid((g.M + tm - 1) / tm, (g.N + kTN - 1) / kTN, slices);
  if (tm == kTM) {
    if (ak && bn) hipLaunchKernelGGL((gemm_bf16_tiled_kernel<true, true, kTM>), grid, dim3(256), 0, s, g, p, ks);
    else if (ak) hipLaunchKernelGGL((gemm_bf16_tiled_kernel<true, false, kTM>), grid, dim3(256), 0, s, g, p, ks);
    else if (bn) hipLaunchKernelGGL((gemm_bf16_tiled_kernel<false, true, kTM>), grid, dim3(256), 0, s, g, p, ks);
    else hipLaunchKernelGGL((gemm_bf16_tiled_kernel<false, false, kTM>), grid, dim3(256), 0, s, g, p, ks);
  } else {
    if (ak && bn) hipLaunchKernelGGL((gemm_bf16_tiled_kernel<true, true, kTM / 2>), grid, dim3(256), 0, s, g, p, ks);
    else if (ak) hipLaunchKernelGGL((gemm_bf16_tiled_kernel<true, false, kTM / 2>), grid, dim3(256), 0, s, g, p, ks);
    else if (bn) hipLaunchKernelGGL((gemm_bf16_tiled_kernel<false, true, kTM / 2>), grid, dim3(256), 0, s, g, p, ks);
    else hipLaunchKernelGGL((gemm_bf16_tiled_kernel<false, false, kTM / 2>), grid, dim3(256), 0, s, g, p, ks);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || slices == 1) return e;
  const size_t mn = static_cast<size_t>(g.M) * g.N;
  hipLaunchKernelGGL(gemm_reduce_kernel, dim3(nblk(mn, 256)), dim3(256), 0, s, part, slices, g);
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
hipError_t launch_colsum(const float* in, int rows, int cols, float* out, float* part, hipStream_t s) {
  const int per = (rows + kColsumPart - 1) / kColsumPart;   // at most kColsumPart slices
  const int slices = (rows + per - 1) / per;
  hipLaunchKernelGGL(colsum_part_kernel, dim3((cols + 63) / 64, slices), dim3(256), 0, s, in, rows, cols, per, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(colsum_final_kernel, dim3((cols + 255) / 256), dim3(256), 0, s, part, slices, cols, out);
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

hipError_t launch_mlp_fused(const MlpArgs& a, hipStream_t s) {
  if (a.L < 1 || a.L > kMlpMaxLayers || a.rows < 1 || a.kp[0] > kMlpMaxIn) return hipErrorInvalidValue;
  if (!a.X || a.ldx < a.in[0]) return hipErrorInvalidValue;
  for (int l = 0; l < a.L; ++l) {
    if (a.out[l] < 1 || a.out[l] > kMlpMaxOut || a.kp[l] % 32 || a.kp[l] < a.in[l]) return hipErrorInvalidValue;
    if (l > 0 && (a.in[l] != a.out[l - 1] || a.kp[l] > kMlpMaxOut)) return hipErrorInvalidValue;
  }
  const int blocks = (a.rows + kMlpRows - 1) / kMlpRows;
  hipLaunchKernelGGL(mlp_fused_kernel, dim3(blocks), dim3(kMlpThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_transpose_weights(const uint16_t* W, int in, int out, int kp, uint16_t* Wt, hipStream_t s) {
  const size_t total = static_cast<size_t>(out) * kp;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(transpose_weights_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, s, W, in, out,
                     kp, Wt);
  return hipGetLastError();
}

}  // namespace dgn
