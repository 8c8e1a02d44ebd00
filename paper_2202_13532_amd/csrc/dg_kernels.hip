// HIP kernels for gfx950: fused DG stage (flux, per-axis contraction, upwind
// lift, SSP-RK3 axpy, FP64 density partials), density/moment reductions and
// the FP64 spectral field solve.
//
// Work decomposition of the stage kernel (one 64-lane wave per work-group):
//   a tile is one x element x one u element x TV = 64/n consecutive v
//   elements.  Lane l holds v node (iv0*n + l) of the tile and keeps the whole
//   n x n (x-node, u-node) slab of that v node in registers, so
//     * global loads/stores are coalesced rows of 64 contiguous values
//       (the v index is innermost in the state layout),
//     * the x and u contractions run in registers with the operator entries
//       as scalar operands,
//     * the v contraction exchanges the row through LDS: each lane then owns
//       one v pencil (n contiguous nodes plus the two face neighbours).
//   The face value of each axis is taken only from the upwind side (App. A);
//   each axis speed is independent of that axis's own coordinate (eq. vlasov),
//   so the flux contraction is the speed times the contraction of f.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "field_bodies.h"
#include "stage_tiles.h"

namespace dgk {



// -------------------------------------------------------------------------
// Density partials only (same tiles and partial layout as the stage kernels).
// -------------------------------------------------------------------------
template <typename T, int N, int NV>
__global__ void __launch_bounds__(kWave) density_kernel(StageArgs<T> a) {
  constexpr int TV = kWave / N;
  const int lane = threadIdx.x;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int vc = bid % a.nvchunks;
  const int t1 = bid / a.nvchunks;
  const int iu = NV == 2 ? t1 % a.Nu : 0;
  const int ix = NV == 2 ? t1 / a.Nu : t1;
  const int iv0 = vc * TV;
  const int tva = min(TV, a.Nv - iv0);
  const bool act = lane < tva * N;
  const int jl = act ? lane : 0;
  const size_t LP = static_cast<size_t>(a.lpitch);   // row pitch
  const size_t NUn = static_cast<size_t>(NV == 2 ? a.Nu : 1) * N;
  const T* __restrict__ fin = a.fin + static_cast<size_t>(vc) * a.cpitch + jl;
  const double wvl = act ? a.wv[iv0 * N + jl] : 0.0;
  const int ntiles = (NV == 2 ? a.Nu : 1) * a.nvchunks;
#pragma unroll
  for (int jx = 0; jx < N; ++jx) {
    double s = 0.0;
    if (NV == 2) {
#pragma unroll
      for (int ju = 0; ju < N; ++ju) {
        const size_t r = ((static_cast<size_t>(ix) * N + jx) * NUn + static_cast<size_t>(iu) * N + ju) * LP;
        s = __builtin_fma(a.wu[iu * N + ju], static_cast<double>(fin[r]), s);
      }
    } else {
      s = static_cast<double>(fin[(static_cast<size_t>(ix) * N + jx) * LP]);
    }
    s = wave_sum(act ? s * wvl : 0.0);
    if (lane == 0) a.partials[static_cast<size_t>(ix * N + jx) * ntiles + iu * a.nvchunks + vc] = s;
  }
}

// Layout conversion between a dense state (rows of nvn values) and one
// with rows of lp values holding chunks of cp values, the first tvn used.
template <typename T>
__global__ void pack_rows_kernel(const T* __restrict__ dense, T* __restrict__ out, size_t total, unsigned lp,
                                 unsigned cp, unsigned tvn, unsigned nvn) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const size_t row = i / lp;
    const unsigned m = static_cast<unsigned>(i - row * lp);
    const unsigned c = m / cp, k = m - c * cp, node = c * tvn + k;
    out[i] = (k < tvn && node < nvn) ? dense[row * nvn + node] : T(0);
  }
}
template <typename T>
__global__ void unpack_rows_kernel(const T* __restrict__ in, T* __restrict__ dense, size_t total, unsigned lp,
                                   unsigned cp, unsigned tvn, unsigned nvn) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const size_t row = i / nvn;
    const unsigned node = static_cast<unsigned>(i - row * nvn);
    const unsigned c = node / tvn;
    dense[i] = in[row * lp + c * cp + (node - c * tvn)];
  }
}

// Per-tile moments: [mass, kinetic energy, l2sq, nonfinite count], product
// LGL quadrature over all axes (weights wx * wu * wv).
template <typename T, int N, int NV>
__global__ void __launch_bounds__(kWave) moments_kernel(StageArgs<T> a, double* mom) {
  constexpr int TV = kWave / N;
  constexpr int NU = NV == 2 ? N : 1;
  const int lane = threadIdx.x;
  const int bid = blockIdx.x;
  const int vc = bid % a.nvchunks;
  const int t1 = bid / a.nvchunks;
  const int iu = NV == 2 ? t1 % a.Nu : 0;
  const int ix = NV == 2 ? t1 / a.Nu : t1;
  const int iv0 = vc * TV;
  const int tva = min(TV, a.Nv - iv0);
  const bool act = lane < tva * N;
  const int jl = act ? lane : 0;
  const size_t LP = static_cast<size_t>(a.lpitch);   // row pitch
  const size_t NUn = static_cast<size_t>(NV == 2 ? a.Nu : 1) * N;
  const T* __restrict__ fin = a.fin + static_cast<size_t>(vc) * a.cpitch + jl;
  const double wvl = act ? a.wv[iv0 * N + jl] : 0.0;
  const double v = a.vc64[iv0 * N + jl];
  double m = 0.0, k = 0.0, l2 = 0.0, bad = 0.0;
  for (int jx = 0; jx < N; ++jx) {
    const double wxv = a.wx[ix * N + jx];
    for (int ju = 0; ju < NU; ++ju) {
      const size_t r = NV == 2
          ? ((static_cast<size_t>(ix) * N + jx) * NUn + static_cast<size_t>(iu) * N + ju) * LP
          : (static_cast<size_t>(ix) * N + jx) * LP;
      double fv = act ? static_cast<double>(fin[r]) : 0.0;
      if (a.bg64 && act) fv += a.bg64[static_cast<size_t>(NV == 2 ? iu * N + ju : 0) * (a.Nv * N) + iv0 * N + jl];
      const double wuv = NV == 2 ? a.wu[iu * N + ju] : 1.0;
      const double u = NV == 2 ? a.uc64[iu * N + ju] : 0.0;
      const double W = wxv * wuv * wvl;
      if (!isfinite(fv)) bad += 1.0;
      m = __builtin_fma(W, fv, m);
      k = __builtin_fma(W * 0.5 * (u * u + v * v), fv, k);
      l2 = __builtin_fma(W * fv, fv, l2);
    }
  }
  m = wave_sum(m);
  k = wave_sum(k);
  l2 = wave_sum(l2);
  bad = wave_sum(bad);
  if (lane == 0) {
    mom[bid * 4 + 0] = m;
    mom[bid * 4 + 1] = k;
    mom[bid * 4 + 2] = l2;
    mom[bid * 4 + 3] = bad;
  }
}

__global__ void __launch_bounds__(kFieldA) fieldA_kernel(FieldArgs a) { fieldA_body<16, true>(a, blockIdx.x); }
__global__ void __launch_bounds__(kFieldB) fieldB_kernel(FieldArgs a) { fieldB_body(a); }

constexpr int kFieldThreads = 256;

__global__ void moments_reduce_kernel(const double* mom, int ntiles, double* ring, const int* counter) {
  __shared__ double red[3][kFieldThreads];
  const int tid = threadIdx.x;
  double s[3] = {0.0, 0.0, 0.0};
  double bad = 0.0;
  for (int t = tid; t < ntiles; t += kFieldThreads) {
    s[0] += mom[4 * t + 0];
    s[1] += mom[4 * t + 1];
    s[2] += mom[4 * t + 2];
    bad += mom[4 * t + 3];
  }
  for (int q = 0; q < 3; ++q) red[q][tid] = s[q];
  __syncthreads();
  for (int w = kFieldThreads / 2; w > 0; w >>= 1) {
    if (tid < w)
      for (int q = 0; q < 3; ++q) red[q][tid] += red[q][tid + w];
    __syncthreads();
  }
  // bad counts are summed separately to keep the tree above fixed
  __shared__ double rb[kFieldThreads];
  rb[tid] = bad;
  __syncthreads();
  for (int w = kFieldThreads / 2; w > 0; w >>= 1) {
    if (tid < w) rb[tid] += rb[tid + w];
    __syncthreads();
  }
  if (tid == 0) {
    const int k = *counter - 1;
    double* r = ring + 8 * ((k < 0 ? 0 : k) % kRing);
    r[3] = red[1][0];
    r[4] = red[2][0];
    const bool fin = isfinite(red[0][0]) && isfinite(red[1][0]) && isfinite(red[2][0]) && rb[0] == 0.0;
    if (!fin) r[6] = 0.0;
  }
}

__global__ void reset_counter_kernel(int* c) { *c = 0; }

// -------------------------------------------------------------------------
// Copy references for the bandwidth measurements (bench.py --pattern-copy):
//   linear_copy_kernel: 16-byte loads and stores, grid-stride, about four per thread;
//   pattern_copy_kernel: the 1D2V stage kernel's access pattern without its
//     halos or arithmetic: one wave per tile (same tiles, XCD remap and
//     buffer resources), the tile's n x n rows of one v chunk loaded, then
//     stored (unused slots of padded rows written as zeros); optionally
//     held to the stage-1 kernel's residency per CU;
//   empty_kernel: no work; a chain of them on one stream gives the time of
//     one dependent launch (dispatch, the kernel-boundary cache operations,
//     completion), the floor under every kernel of the step.
// -------------------------------------------------------------------------
__global__ void __launch_bounds__(kWave) empty_kernel() {}

constexpr int kLdsPerCu = 160 * 1024;   // LDS of one gfx950 CU
constexpr int kLdsGranule = 512;        // LDS allocation granularity (bytes)

__global__ void __launch_bounds__(256) linear_copy_kernel(const float4* __restrict__ in, float4* __restrict__ out,
                                                          size_t n16) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n16;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    out[i] = in[i];
}

template <typename T, int N>
__global__ void __launch_bounds__(kWave) pattern_copy_kernel(StageArgs<T> a) {
  using B = Buf<T>;
  constexpr unsigned S = sizeof(T);
  constexpr int TV = kWave / N;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const unsigned lane = threadIdx.x;
  const int vc = bid % a.nvchunks, t1 = bid / a.nvchunks, iu = t1 % a.Nu, ix = t1 / a.Nu;
  const int tva = min(TV, a.Nv - vc * TV);
  const unsigned NUn = static_cast<unsigned>(a.Nu) * N, LP = a.lpitch, CP = a.cpitch, m0 = vc * CP;
  const size_t xstride = static_cast<size_t>(N) * NUn * LP;
  const unsigned xbytes = static_cast<unsigned>(xstride * S), rowb = LP * S;
  const unsigned vo = lane < static_cast<unsigned>(tva * N) ? lane * S : kOffOOB;
  const unsigned vs = (lane < CP && m0 + lane < LP) ? lane * S : kOffOOB;
  const auto rf = xelem_rsrc(a.fin, xstride, ix, xbytes);
  const auto ro = xelem_rsrc(a.out, xstride, ix, xbytes);
  T f[N][N];
#pragma unroll
  for (int jx = 0; jx < N; ++jx)
#pragma unroll
    for (int ju = 0; ju < N; ++ju) f[jx][ju] = B::ld(rf, vo + ((jx * NUn + iu * N) * LP + m0) * S, ju * rowb);
#pragma unroll
  for (int jx = 0; jx < N; ++jx)
#pragma unroll
    for (int ju = 0; ju < N; ++ju) {
      const unsigned o = vs + ((jx * NUn + iu * N) * LP + m0) * S;
      if (a.nt_store) B::st_nt(f[jx][ju], ro, o, ju * rowb);
      else B::st(f[jx][ju], ro, o, ju * rowb);
    }
}

// -------------------------------------------------------------------------
// Spectral tools on the x grid (Sec. 5.3).
//   fourier_kernel: c_p = sum_q T_p^q g_q for p = 1..pmax (eq. spectral_transform)
//     on arbitrary nodal values g; block b serves modes 64b..64b+63, four
//     groups of 64 threads each add a contiguous quarter of the nodes, the
//     quarters are then added in order.
//   xfilter_kernel: out[r, c] = sum_q M[r, q] in[q, c] for a state seen as an
//     (Nx n) x C matrix (x outermost); block (bx, by) computes a 64-column x
//     64-row tile through 16-deep LDS slabs of M and of the state.
// -------------------------------------------------------------------------
__global__ void __launch_bounds__(256) fourier_kernel(const double* __restrict__ T, const double* __restrict__ g,
                                                      int nodes, int pmax, double* __restrict__ out) {
  __shared__ double red[2][256];
  const int tid = threadIdx.x, p = blockIdx.x * 64 + tid % 64, grp = tid / 64;
  double cr = 0.0, ci = 0.0;
  if (p < pmax) {
    const int q0 = grp * nodes / 4, q1 = (grp + 1) * nodes / 4;
    for (int q = q0; q < q1; ++q) {
      const double v = g[q];
      const double* t = T + 2 * (static_cast<size_t>(q) * pmax + p);
      cr = __builtin_fma(t[0], v, cr);
      ci = __builtin_fma(t[1], v, ci);
    }
  }
  red[0][tid] = cr;
  red[1][tid] = ci;
  __syncthreads();
  if (tid < 64 && p < pmax) {
    out[2 * p] = (red[0][tid] + red[0][64 + tid]) + (red[0][128 + tid] + red[0][192 + tid]);
    out[2 * p + 1] = (red[1][tid] + red[1][64 + tid]) + (red[1][128 + tid] + red[1][192 + tid]);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) xfilter_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                      const T* __restrict__ M, int R, size_t C) {
  __shared__ T Ms[64][17];
  __shared__ T Fs[16][64];
  const int tid = threadIdx.x, lane = tid % 64, grp = tid / 64;
  const size_t col = static_cast<size_t>(blockIdx.x) * 64 + lane;
  const int r0 = blockIdx.y * 64;
  T acc[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = T(0);
  for (int k0 = 0; k0 < R; k0 += 16) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int kk = grp * 4 + i, q = k0 + kk;
      Fs[kk][lane] = (q < R && col < C) ? in[static_cast<size_t>(q) * C + col] : T(0);
      const int e = tid + 256 * i, mr = e / 16, mk = e % 16;   // 64 x 16 slab of M
      Ms[mr][mk] = (r0 + mr < R && k0 + mk < R) ? M[static_cast<size_t>(r0 + mr) * R + k0 + mk] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const T fv = Fs[kk][lane];
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = fmadd(Ms[grp * 16 + r][kk], fv, acc[r]);
    }
    __syncthreads();
  }
  if (col < C) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = r0 + grp * 16 + r;
      if (row < R) out[static_cast<size_t>(row) * C + col] = acc[r];
    }
  }
}

// -------------------------------------------------------------------------
// Host launchers.
// -------------------------------------------------------------------------
template <typename T, int N, bool BG>
static void stage_bg(int nv, bool un, const StageArgs<T>& a, int ntiles, hipStream_t s) {
  if (nv == 2) {
    // u^n loads take the non-temporal hint together with the stores
    if (un && a.nt_store) hipLaunchKernelGGL((stage2v_kernel<T, N, true, BG, false, true>), dim3(ntiles), dim3(kWave), 0, s, a);
    else if (un) hipLaunchKernelGGL((stage2v_kernel<T, N, true, BG>), dim3(ntiles), dim3(kWave), 0, s, a);
    else hipLaunchKernelGGL((stage2v_kernel<T, N, false, BG>), dim3(ntiles), dim3(kWave), 0, s, a);
  } else {
    if (un) hipLaunchKernelGGL((stage1v_kernel<T, N, true, BG>), dim3(ntiles), dim3(kWave), 0, s, a);
    else hipLaunchKernelGGL((stage1v_kernel<T, N, false, BG>), dim3(ntiles), dim3(kWave), 0, s, a);
  }
}

template <typename T, int N>
static hipError_t stage_t(int nv, const void* args, int ntiles, hipStream_t s) {
  const StageArgs<T>& a = *static_cast<const StageArgs<T>*>(args);
  const bool un = a.c_un != T(0);
  if (a.corr) {
    // the learned correction's stage: FP32 1D2V, no background
    if constexpr (sizeof(T) == 4) {
      if (nv != 2 || a.bg_u) return hipErrorInvalidValue;
      if (un && a.nt_store) hipLaunchKernelGGL((stage2v_kernel<T, N, true, false, true, true>), dim3(ntiles), dim3(kWave), 0, s, a);
      else if (un) hipLaunchKernelGGL((stage2v_kernel<T, N, true, false, true>), dim3(ntiles), dim3(kWave), 0, s, a);
      else hipLaunchKernelGGL((stage2v_kernel<T, N, false, false, true>), dim3(ntiles), dim3(kWave), 0, s, a);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  if (a.bg_u) stage_bg<T, N, true>(nv, un, a, ntiles, s);
  else stage_bg<T, N, false>(nv, un, a, ntiles, s);
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t density_t(int nv, const void* args, int ntiles, hipStream_t s) {
  const StageArgs<T>& a = *static_cast<const StageArgs<T>*>(args);
  if (nv == 2)
    hipLaunchKernelGGL((density_kernel<T, N, 2>), dim3(ntiles), dim3(kWave), 0, s, a);
  else
    hipLaunchKernelGGL((density_kernel<T, N, 1>), dim3(ntiles), dim3(kWave), 0, s, a);
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t moments_t(int nv, const void* args, double* mom, int ntiles, hipStream_t s) {
  const StageArgs<T>& a = *static_cast<const StageArgs<T>*>(args);
  if (nv == 2)
    hipLaunchKernelGGL((moments_kernel<T, N, 2>), dim3(ntiles), dim3(kWave), 0, s, a, mom);
  else
    hipLaunchKernelGGL((moments_kernel<T, N, 1>), dim3(ntiles), dim3(kWave), 0, s, a, mom);
  return hipGetLastError();
}

#define DG_DISPATCH_N(FN, T, ...)                 \
  switch (n) {                                    \
    case 2: return FN<T, 2>(__VA_ARGS__);         \
    case 3: return FN<T, 3>(__VA_ARGS__);         \
    case 4: return FN<T, 4>(__VA_ARGS__);         \
    case 5: return FN<T, 5>(__VA_ARGS__);         \
    case 6: return FN<T, 6>(__VA_ARGS__);         \
    case 7: return FN<T, 7>(__VA_ARGS__);         \
    case 8: return FN<T, 8>(__VA_ARGS__);         \
    case 9: return FN<T, 9>(__VA_ARGS__);         \
    case 10: return FN<T, 10>(__VA_ARGS__);       \
    case 11: return FN<T, 11>(__VA_ARGS__);       \
    case 12: return FN<T, 12>(__VA_ARGS__);       \
    default: return hipErrorInvalidValue;         \
  }

hipError_t launch_stage(int nv, int n, bool f64, const void* args, int ntiles, hipStream_t s) {
  if (f64) { DG_DISPATCH_N(stage_t, double, nv, args, ntiles, s) }
  DG_DISPATCH_N(stage_t, float, nv, args, ntiles, s)
}

hipError_t launch_density(int nv, int n, bool f64, const void* args, int ntiles, hipStream_t s) {
  if (f64) { DG_DISPATCH_N(density_t, double, nv, args, ntiles, s) }
  DG_DISPATCH_N(density_t, float, nv, args, ntiles, s)
}

hipError_t launch_moments(int nv, int n, bool f64, const void* args, double* mom, int ntiles, hipStream_t s) {
  if (f64) { DG_DISPATCH_N(moments_t, double, nv, args, mom, ntiles, s) }
  DG_DISPATCH_N(moments_t, float, nv, args, mom, ntiles, s)
}

hipError_t launch_field(const FieldArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(fieldA_kernel, dim3(a.Nx), dim3(kFieldA), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fieldB_kernel, dim3(1), dim3(kFieldB), 2 * a.pmax * sizeof(double), s, a);
  return hipGetLastError();
}

hipError_t launch_moments_reduce(const double* mom, int ntiles, double* ring, const int* counter, hipStream_t s) {
  hipLaunchKernelGGL(moments_reduce_kernel, dim3(1), dim3(kFieldThreads), 0, s, mom, ntiles, ring, counter);
  return hipGetLastError();
}


hipError_t launch_empty(hipStream_t s) {
  hipLaunchKernelGGL(empty_kernel, dim3(1), dim3(kWave), 0, s);
  return hipGetLastError();
}

hipError_t launch_linear_copy(const void* in, void* out, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  // about four 16-byte copies per thread: many short waves keep more requests
  // in flight than a grid sized to the resident-wave count (on a 446 MB
  // buffer 5.7 TB/s against 5.25 TB/s with 8192 work-groups)
  const unsigned grid = static_cast<unsigned>(std::min<size_t>(std::max<size_t>(n16 / 1024, 1), size_t(1) << 16));
  hipLaunchKernelGGL(linear_copy_kernel, dim3(grid), dim3(256), 0, s, static_cast<const float4*>(in),
                     static_cast<float4*>(out), n16);
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t pattern_copy_t(int nv, const void* args, int ntiles, bool stage_residency, hipStream_t s) {
  if (nv != 2) return hipErrorInvalidValue;
  size_t lds = 0;
  if (stage_residency) {
    // unused LDS per work-group, sized so that no more of them fit on a CU
    // than work-groups of the stage-1 kernel of this shape (the copy alone
    // would keep more waves resident)
    int per_cu = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, stage2v_kernel<T, N, false, false, false>, kWave, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 3) return hipErrorInvalidValue;   // would need more than 64 KiB per work-group
    lds = static_cast<size_t>(kLdsPerCu / per_cu) / kLdsGranule * kLdsGranule;
  }
  hipLaunchKernelGGL((pattern_copy_kernel<T, N>), dim3(ntiles), dim3(kWave), lds, s, *static_cast<const StageArgs<T>*>(args));
  return hipGetLastError();
}

hipError_t launch_pattern_copy(int nv, int n, bool f64, const void* args, int ntiles, bool stage_residency,
                               hipStream_t s) {
  if (f64) { DG_DISPATCH_N(pattern_copy_t, double, nv, args, ntiles, stage_residency, s) }
  DG_DISPATCH_N(pattern_copy_t, float, nv, args, ntiles, stage_residency, s)
}

hipError_t launch_fourier(const double* T, const double* g, int nodes, int pmax, double* out, hipStream_t s) {
  hipLaunchKernelGGL(fourier_kernel, dim3((pmax + 63) / 64), dim3(256), 0, s, T, g, nodes, pmax, out);
  return hipGetLastError();
}

hipError_t launch_xfilter(bool f64, const void* in, void* out, const void* M, int R, size_t C, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>((C + 63) / 64), static_cast<unsigned>((R + 63) / 64));
  if (f64)
    hipLaunchKernelGGL(xfilter_kernel<double>, grid, dim3(256), 0, s, static_cast<const double*>(in),
                       static_cast<double*>(out), static_cast<const double*>(M), R, C);
  else
    hipLaunchKernelGGL(xfilter_kernel<float>, grid, dim3(256), 0, s, static_cast<const float*>(in),
                       static_cast<float*>(out), static_cast<const float*>(M), R, C);
  return hipGetLastError();
}

hipError_t launch_reset_counter(int* counter, hipStream_t s) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, counter);
  return hipGetLastError();
}

hipError_t launch_repack(bool pack, bool f64, const void* in, void* out, size_t rows, unsigned lp, unsigned cp,
                         unsigned tvn, unsigned nvn, hipStream_t s) {
  const size_t total = rows * (pack ? lp : nvn);
  if (total == 0) return hipSuccess;
  const unsigned grid = static_cast<unsigned>(std::min<size_t>((total + 255) / 256, 65536));
  if (pack) {
    if (f64) hipLaunchKernelGGL(pack_rows_kernel<double>, dim3(grid), dim3(256), 0, s, static_cast<const double*>(in), static_cast<double*>(out), total, lp, cp, tvn, nvn);
    else hipLaunchKernelGGL(pack_rows_kernel<float>, dim3(grid), dim3(256), 0, s, static_cast<const float*>(in), static_cast<float*>(out), total, lp, cp, tvn, nvn);
  } else {
    if (f64) hipLaunchKernelGGL(unpack_rows_kernel<double>, dim3(grid), dim3(256), 0, s, static_cast<const double*>(in), static_cast<double*>(out), total, lp, cp, tvn, nvn);
    else hipLaunchKernelGGL(unpack_rows_kernel<float>, dim3(grid), dim3(256), 0, s, static_cast<const float*>(in), static_cast<float*>(out), total, lp, cp, tvn, nvn);
  }
  return hipGetLastError();
}

}  // namespace dgk
