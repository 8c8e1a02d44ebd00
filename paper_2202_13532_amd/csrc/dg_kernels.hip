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

#include "dg_kernels.h"

namespace dgk {

// Work-groups are dispatched round-robin over the 8 XCDs.  Re-map so that each
// XCD walks a contiguous range of logical tiles: neighbouring tiles (which
// share halo rows) then run at the same time on the same L2.
__device__ __forceinline__ int xcd_remap(int b, int g) {
  const int q = g >> 3, r = g & 7, c = b & 7;
  return c * q + min(c, r) + (b >> 3);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// t_i = sum_k Ups_ik g_k + Xl_i fL - Xr_i fR  for one pencil; res_i = s t_i (+ res_i).
template <typename T, int N, bool ACC, typename G>
__device__ __forceinline__ void contract(const Ops<T>& op, G g, T fL, T fR, T s, T* res) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T t = op.xl[i] * fL - op.xr[i] * fR;
#pragma unroll
    for (int k = 0; k < N; ++k) t = fmadd(op.ups[i * kMaxN + k], g(k), t);
    res[i] = ACC ? fmadd(s, t, res[i]) : s * t;
  }
}

// -------------------------------------------------------------------------
// 1D2V stage kernel.  state [Nx, N, Nu, N, Nv, N].
// -------------------------------------------------------------------------
template <typename T, int N>
__global__ void __launch_bounds__(kWave) stage2v_kernel(StageArgs<T> a, Ops<T> op) {
  constexpr int TV = kWave / N;
  constexpr int ROW = kWave + 2;   // >= TV*N + 2; lane+1 stays inside a row
  __shared__ T lds[N * ROW];
  __shared__ T hbuf[N * N];

  const int lane = threadIdx.x;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int vc = bid % a.nvchunks;
  const int t1 = bid / a.nvchunks;
  const int iu = t1 % a.Nu;
  const int ix = t1 / a.Nu;
  const int iv0 = vc * TV;
  const int tva = min(TV, a.Nv - iv0);
  const int nact = tva * N;
  const bool act = lane < nact;
  const int jl = act ? lane : 0;
  const size_t NVn = static_cast<size_t>(a.Nv) * N;
  const size_t NUn = static_cast<size_t>(a.Nu) * N;
  // first element of the row (ix, jx, iu, ju, :)
  auto row = [&](int ixe, int jx, int iue, int ju) -> size_t {
    return ((static_cast<size_t>(ixe) * N + jx) * NUn + static_cast<size_t>(iue) * N + ju) * NVn;
  };
  const T* __restrict__ fin = a.fin + static_cast<size_t>(iv0) * N + jl;

  T f[N][N];
#pragma unroll
  for (int jx = 0; jx < N; ++jx)
#pragma unroll
    for (int ju = 0; ju < N; ++ju) f[jx][ju] = fin[row(ix, jx, iu, ju)];

  // x faces: the x speed u is uniform per u node, so the upwind side is too.
  const int ixl = ix == 0 ? a.Nx - 1 : ix - 1;
  const int ixr = ix == a.Nx - 1 ? 0 : ix + 1;
  T xh[N];
#pragma unroll
  for (int ju = 0; ju < N; ++ju) {
    const T uu = a.ucoord[iu * N + ju];
    xh[ju] = uu > T(0) ? fin[row(ixl, N - 1, iu, ju)] : (uu < T(0) ? fin[row(ixr, 0, iu, ju)] : T(0));
  }

  // u faces: the u speed -E(x) - v B varies per lane (v) and per x node.
  const T vv = a.vcoord[iv0 * N + jl];
  const int iul = iu == 0 ? a.Nu - 1 : iu - 1;
  const int iur = iu == a.Nu - 1 ? 0 : iu + 1;
  const bool zl = a.zero_inflow && iu == 0;
  const bool zr = a.zero_inflow && iu == a.Nu - 1;
  T uh[N], su[N];
#pragma unroll
  for (int jx = 0; jx < N; ++jx) {
    const T au = -static_cast<T>(a.E[ix * N + jx]) - vv * a.wc;
    su[jx] = a.Ju * au;
    const T* p = au > T(0) ? fin + row(ix, jx, iul, N - 1) : fin + row(ix, jx, iur, 0);
    const T val = *p;
    const bool zero = (au == T(0)) || (au > T(0) ? zl : zr);
    uh[jx] = zero ? T(0) : val;
  }

  // v faces: the v speed u B is uniform per u node; one halo value per
  // (x node, u node) row, from the upwind neighbouring v element.
  {
    const T* base = a.fin;
    for (int h = lane; h < N * N; h += kWave) {
      const int jx = h / N, ju = h % N;
      const T av = a.ucoord[iu * N + ju] * a.wc;
      size_t jv;
      bool outside;
      if (av > T(0)) {
        outside = iv0 == 0;
        jv = outside ? NVn - 1 : static_cast<size_t>(iv0) * N - 1;
      } else {
        const int e = iv0 + tva;
        outside = e == a.Nv;
        jv = outside ? 0 : static_cast<size_t>(e) * N;
      }
      const T val = base[row(ix, jx, iu, ju) + jv];
      hbuf[h] = (av == T(0) || (outside && a.zero_inflow)) ? T(0) : val;
    }
  }

  T acc[N][N];
  // x axis: contract over the x node index (column ju of the slab).
#pragma unroll
  for (int ju = 0; ju < N; ++ju) {
    const T uu = a.ucoord[iu * N + ju];
    const T fL = uu > T(0) ? xh[ju] : f[0][ju];
    const T fR = uu > T(0) ? f[N - 1][ju] : xh[ju];
    T r[N];
    contract<T, N, false>(op, [&](int k) { return f[k][ju]; }, fL, fR, a.Jx * uu, r);
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i][ju] = r[i];
  }
  // u axis: contract over the u node index (row jx of the slab).
#pragma unroll
  for (int jx = 0; jx < N; ++jx) {
    const bool pos = su[jx] > T(0);
    const T fL = pos ? uh[jx] : f[jx][0];
    const T fR = pos ? f[jx][N - 1] : uh[jx];
    contract<T, N, true>(op, [&](int k) { return f[jx][k]; }, fL, fR, su[jx], acc[jx]);
  }
  // v axis through LDS, one x node at a time.  Pencil owner: row pr (= u
  // node), element pv of the chunk.
  const bool pact = lane < N * tva;
  const int pr = pact ? lane / tva : 0;
  const int pv = pact ? lane % tva : 0;
  const T sv = a.Jv * a.ucoord[iu * N + pr] * a.wc;
  const int hside = (lane < N && a.ucoord[iu * N + lane] * a.wc > T(0)) ? 0 : nact + 1;
#pragma unroll
  for (int jx = 0; jx < N; ++jx) {
    __syncthreads();
    if (act) {
#pragma unroll
      for (int ju = 0; ju < N; ++ju) lds[ju * ROW + 1 + lane] = f[jx][ju];
    }
    if (lane < N) lds[lane * ROW + hside] = hbuf[jx * N + lane];
    __syncthreads();
    T g[N + 2];
#pragma unroll
    for (int k = 0; k < N + 2; ++k) g[k] = lds[pr * ROW + pv * N + k];
    const T fL = sv > T(0) ? g[0] : g[1];
    const T fR = sv > T(0) ? g[N] : g[N + 1];
    T r[N];
    contract<T, N, false>(op, [&](int k) { return g[k + 1]; }, fL, fR, sv, r);
    __syncthreads();
    if (pact) {
#pragma unroll
      for (int i = 0; i < N; ++i) lds[pr * ROW + pv * N + 1 + i] = r[i];
    }
    __syncthreads();
#pragma unroll
    for (int ju = 0; ju < N; ++ju) acc[jx][ju] += lds[ju * ROW + 1 + lane];
  }

  // epilogue: stage combination, store, FP64 density partials.
  const T* __restrict__ fun = a.fun + static_cast<size_t>(iv0) * N + jl;
  T* __restrict__ out = a.out + static_cast<size_t>(iv0) * N + jl;
  const bool use_un = a.c_un != T(0);
#pragma unroll
  for (int jx = 0; jx < N; ++jx)
#pragma unroll
    for (int ju = 0; ju < N; ++ju) {
      T v = fmadd(a.c_dt, acc[jx][ju], a.c_in * f[jx][ju]);
      if (use_un) v = fmadd(a.c_un, fun[row(ix, jx, iu, ju)], v);
      f[jx][ju] = v;
      if (act) out[row(ix, jx, iu, ju)] = v;
    }
  if (a.partials) {
    const double wvl = act ? a.wv[iv0 * N + jl] : 0.0;
    const int ntiles = a.Nu * a.nvchunks;
#pragma unroll
    for (int jx = 0; jx < N; ++jx) {
      double s = 0.0;
#pragma unroll
      for (int ju = 0; ju < N; ++ju) s = __builtin_fma(a.wu[iu * N + ju], static_cast<double>(f[jx][ju]), s);
      // lanes past the ragged end of the chunk hold garbage: select, never multiply by 0
      s = wave_sum(act ? s * wvl : 0.0);
      if (lane == 0) a.partials[static_cast<size_t>(ix * N + jx) * ntiles + iu * a.nvchunks + vc] = s;
    }
  }
}

// -------------------------------------------------------------------------
// 1D1V stage kernel.  state [Nx, N, Nv, N]; x speed v, v speed -E(x).
// -------------------------------------------------------------------------
template <typename T, int N>
__global__ void __launch_bounds__(kWave) stage1v_kernel(StageArgs<T> a, Ops<T> op) {
  constexpr int TV = kWave / N;
  constexpr int ROW = kWave + 2;   // >= TV*N + 2; lane+1 stays inside a row
  __shared__ T lds[N * ROW];

  const int lane = threadIdx.x;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int vc = bid % a.nvchunks;
  const int ix = bid / a.nvchunks;
  const int iv0 = vc * TV;
  const int tva = min(TV, a.Nv - iv0);
  const int nact = tva * N;
  const bool act = lane < nact;
  const int jl = act ? lane : 0;
  const size_t NVn = static_cast<size_t>(a.Nv) * N;
  auto row = [&](int ixe, int jx) -> size_t { return (static_cast<size_t>(ixe) * N + jx) * NVn; };
  const T* __restrict__ fin = a.fin + static_cast<size_t>(iv0) * N + jl;

  T f[N];
#pragma unroll
  for (int jx = 0; jx < N; ++jx) f[jx] = fin[row(ix, jx)];
  const T vv = a.vcoord[iv0 * N + jl];
  const int ixl = ix == 0 ? a.Nx - 1 : ix - 1;
  const int ixr = ix == a.Nx - 1 ? 0 : ix + 1;
  const T xh = vv > T(0) ? fin[row(ixl, N - 1)] : (vv < T(0) ? fin[row(ixr, 0)] : T(0));

  T acc[N];
  {
    const T fL = vv > T(0) ? xh : f[0];
    const T fR = vv > T(0) ? f[N - 1] : xh;
    contract<T, N, false>(op, [&](int k) { return f[k]; }, fL, fR, a.Jx * vv, acc);
  }
  // v faces, one per x node row, from the side selected by the sign of -E.
  T hval = T(0);
  int hside = 0;
  if (lane < N) {
    const T av = -static_cast<T>(a.E[ix * N + lane]);
    size_t jv;
    bool outside;
    if (av > T(0)) {
      outside = iv0 == 0;
      jv = outside ? NVn - 1 : static_cast<size_t>(iv0) * N - 1;
      hside = 0;
    } else {
      const int e = iv0 + tva;
      outside = e == a.Nv;
      jv = outside ? 0 : static_cast<size_t>(e) * N;
      hside = nact + 1;
    }
    const T val = a.fin[row(ix, lane) + jv];
    hval = (av == T(0) || (outside && a.zero_inflow)) ? T(0) : val;
  }
  if (act) {
#pragma unroll
    for (int jx = 0; jx < N; ++jx) lds[jx * ROW + 1 + lane] = f[jx];
  }
  if (lane < N) lds[lane * ROW + hside] = hval;
  __syncthreads();
  const bool pact = lane < N * tva;
  const int pr = pact ? lane / tva : 0;
  const int pv = pact ? lane % tva : 0;
  const T sv = -a.Jv * static_cast<T>(a.E[ix * N + pr]);
  T g[N + 2];
#pragma unroll
  for (int k = 0; k < N + 2; ++k) g[k] = lds[pr * ROW + pv * N + k];
  {
    const T fL = sv > T(0) ? g[0] : g[1];
    const T fR = sv > T(0) ? g[N] : g[N + 1];
    T r[N];
    contract<T, N, false>(op, [&](int k) { return g[k + 1]; }, fL, fR, sv, r);
    __syncthreads();
    if (pact) {
#pragma unroll
      for (int i = 0; i < N; ++i) lds[pr * ROW + pv * N + 1 + i] = r[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int jx = 0; jx < N; ++jx) acc[jx] += lds[jx * ROW + 1 + lane];

  const T* __restrict__ fun = a.fun + static_cast<size_t>(iv0) * N + jl;
  T* __restrict__ out = a.out + static_cast<size_t>(iv0) * N + jl;
  const bool use_un = a.c_un != T(0);
#pragma unroll
  for (int jx = 0; jx < N; ++jx) {
    T v = fmadd(a.c_dt, acc[jx], a.c_in * f[jx]);
    if (use_un) v = fmadd(a.c_un, fun[row(ix, jx)], v);
    f[jx] = v;
    if (act) out[row(ix, jx)] = v;
  }
  if (a.partials) {
    const double wvl = act ? a.wv[iv0 * N + jl] : 0.0;
#pragma unroll
    for (int jx = 0; jx < N; ++jx) {
      const double s = wave_sum(act ? wvl * static_cast<double>(f[jx]) : 0.0);
      if (lane == 0) a.partials[static_cast<size_t>(ix * N + jx) * a.nvchunks + vc] = s;
    }
  }
}

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
  const size_t NVn = static_cast<size_t>(a.Nv) * N;
  const size_t NUn = static_cast<size_t>(NV == 2 ? a.Nu : 1) * N;
  const T* __restrict__ fin = a.fin + static_cast<size_t>(iv0) * N + jl;
  const double wvl = act ? a.wv[iv0 * N + jl] : 0.0;
  const int ntiles = (NV == 2 ? a.Nu : 1) * a.nvchunks;
#pragma unroll
  for (int jx = 0; jx < N; ++jx) {
    double s = 0.0;
    if (NV == 2) {
#pragma unroll
      for (int ju = 0; ju < N; ++ju) {
        const size_t r = ((static_cast<size_t>(ix) * N + jx) * NUn + static_cast<size_t>(iu) * N + ju) * NVn;
        s = __builtin_fma(a.wu[iu * N + ju], static_cast<double>(fin[r]), s);
      }
    } else {
      s = static_cast<double>(fin[(static_cast<size_t>(ix) * N + jx) * NVn]);
    }
    s = wave_sum(act ? s * wvl : 0.0);
    if (lane == 0) a.partials[static_cast<size_t>(ix * N + jx) * ntiles + iu * a.nvchunks + vc] = s;
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
  const size_t NVn = static_cast<size_t>(a.Nv) * N;
  const size_t NUn = static_cast<size_t>(NV == 2 ? a.Nu : 1) * N;
  const T* __restrict__ fin = a.fin + static_cast<size_t>(iv0) * N + jl;
  const double wvl = act ? a.wv[iv0 * N + jl] : 0.0;
  const double v = a.vc64[iv0 * N + jl];
  double m = 0.0, k = 0.0, l2 = 0.0, bad = 0.0;
  for (int jx = 0; jx < N; ++jx) {
    const double wxv = a.wx[ix * N + jx];
    for (int ju = 0; ju < NU; ++ju) {
      const size_t r = NV == 2
          ? ((static_cast<size_t>(ix) * N + jx) * NUn + static_cast<size_t>(iu) * N + ju) * NVn
          : (static_cast<size_t>(ix) * N + jx) * NVn;
      const double fv = act ? static_cast<double>(fin[r]) : 0.0;
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

// -------------------------------------------------------------------------
// Field solve (FP64).  Stage A: one block per x element reduces the density
// partials in a fixed order, forms that element's Fourier partial sums
// sum_j T_p^{mj} (n_mj - 1) and its mass.  Stage B: one block sums the
// partials over elements in order, synthesises E at every x node
// (eq. electric_sol) and records mass, field energy and max|E|.
// -------------------------------------------------------------------------
constexpr int kFieldThreads = 256;

__global__ void __launch_bounds__(kFieldThreads) fieldA_kernel(FieldArgs a) {
  __shared__ double red[kFieldThreads];
  __shared__ double dens[kMaxN];
  const int ix = blockIdx.x, tid = threadIdx.x, n = a.n;
  for (int jx = 0; jx < n; ++jx) {
    const double* p = a.partials + static_cast<size_t>(ix * n + jx) * a.ntiles;
    double s = 0.0;
    for (int t = tid; t < a.ntiles; t += kFieldThreads) s += p[t];
    red[tid] = s;
    __syncthreads();
    for (int w = kFieldThreads / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) dens[jx] = red[0];
    __syncthreads();
  }
  if (tid < n) a.dens[ix * n + tid] = dens[tid];
  if (tid == 0) {
    double m = 0.0;
    for (int j = 0; j < n; ++j) m += a.wx[ix * n + j] * dens[j];
    a.mpart[ix] = m;
  }
  const int nodes = a.Nx * n;
  for (int p = tid; p < a.pmax; p += kFieldThreads) {
    double cr = 0.0, ci = 0.0;
    for (int j = 0; j < n; ++j) {
      const double* t = a.T + 2 * (static_cast<size_t>(p) * nodes + ix * n + j);
      const double s = dens[j] - 1.0;
      cr += t[0] * s;
      ci += t[1] * s;
    }
    a.cpart[2 * (static_cast<size_t>(ix) * a.pmax + p) + 0] = cr;
    a.cpart[2 * (static_cast<size_t>(ix) * a.pmax + p) + 1] = ci;
  }
}

__global__ void __launch_bounds__(kFieldThreads) fieldB_kernel(FieldArgs a) {
  extern __shared__ double sh[];          // 2 * pmax coefficients
  __shared__ double red[kFieldThreads];
  __shared__ double redm[kFieldThreads];
  const int tid = threadIdx.x, n = a.n, nodes = a.Nx * a.n;
  for (int p = tid; p < a.pmax; p += kFieldThreads) {
    double cr = 0.0, ci = 0.0;
    for (int ix = 0; ix < a.Nx; ++ix) {
      cr += a.cpart[2 * (static_cast<size_t>(ix) * a.pmax + p) + 0];
      ci += a.cpart[2 * (static_cast<size_t>(ix) * a.pmax + p) + 1];
    }
    sh[2 * p] = cr;
    sh[2 * p + 1] = ci;
    if (a.coeffs) {
      a.coeffs[2 * p] = cr;
      a.coeffs[2 * p + 1] = ci;
    }
  }
  __syncthreads();
  double fe = 0.0, mx = 0.0;
  for (int node = tid; node < nodes; node += kFieldThreads) {
    double e = 0.0;
    for (int p = 0; p < a.pmax; ++p) {
      const double* g = a.G + 2 * (static_cast<size_t>(p) * nodes + node);
      e += 2.0 * (sh[2 * p] * g[0] - sh[2 * p + 1] * g[1]);
    }
    a.E[node] = e;
    fe += a.wx[node] * e * e;
    mx = fmax(mx, fabs(e));
  }
  red[tid] = fe;
  redm[tid] = mx;
  __syncthreads();
  for (int w = kFieldThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
      red[tid] += red[tid + w];
      redm[tid] = fmax(redm[tid], redm[tid + w]);
    }
    __syncthreads();
  }
  if (tid == 0) {
    double m = 0.0;
    for (int ix = 0; ix < a.Nx; ++ix) m += a.mpart[ix];
    const double fen = 0.5 * red[0];
    const bool fin = isfinite(m) && isfinite(fen) && isfinite(redm[0]);
    const int k = (a.record && a.ring) ? *a.counter : -1;
    double rec[8] = {0.0, m, fen, 0.0, 0.0, redm[0], fin ? 1.0 : 0.0, static_cast<double>(k)};
    for (int q = 0; q < 8; ++q) a.last[q] = rec[q];
    if (k >= 0) {
      double* r = a.ring + 8 * (k % kRing);
      for (int q = 0; q < 8; ++q) r[q] = rec[q];
      *a.counter = k + 1;
    }
  }
  (void)n;
}

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
// Host launchers.
// -------------------------------------------------------------------------
template <typename T, int N>
static hipError_t stage_t(int nv, const void* args, int ntiles, hipStream_t s) {
  const StageArgs<T>& a = static_cast<const StagePack<T>*>(args)->a;
  const Ops<T>& op = static_cast<const StagePack<T>*>(args)->op;
  if (nv == 2)
    hipLaunchKernelGGL((stage2v_kernel<T, N>), dim3(ntiles), dim3(kWave), 0, s, a, op);
  else
    hipLaunchKernelGGL((stage1v_kernel<T, N>), dim3(ntiles), dim3(kWave), 0, s, a, op);
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t density_t(int nv, const void* args, int ntiles, hipStream_t s) {
  const StageArgs<T>& a = static_cast<const StagePack<T>*>(args)->a;
  if (nv == 2)
    hipLaunchKernelGGL((density_kernel<T, N, 2>), dim3(ntiles), dim3(kWave), 0, s, a);
  else
    hipLaunchKernelGGL((density_kernel<T, N, 1>), dim3(ntiles), dim3(kWave), 0, s, a);
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t moments_t(int nv, const void* args, double* mom, int ntiles, hipStream_t s) {
  const StageArgs<T>& a = static_cast<const StagePack<T>*>(args)->a;
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
  hipLaunchKernelGGL(fieldA_kernel, dim3(a.Nx), dim3(kFieldThreads), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fieldB_kernel, dim3(1), dim3(kFieldThreads), 2 * a.pmax * sizeof(double), s, a);
  return hipGetLastError();
}

hipError_t launch_moments_reduce(const double* mom, int ntiles, double* ring, const int* counter, hipStream_t s) {
  hipLaunchKernelGGL(moments_reduce_kernel, dim3(1), dim3(kFieldThreads), 0, s, mom, ntiles, ring, counter);
  return hipGetLastError();
}

hipError_t launch_reset_counter(int* counter, hipStream_t s) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, counter);
  return hipGetLastError();
}

}  // namespace dgk
