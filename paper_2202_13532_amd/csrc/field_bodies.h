// FP64 field-solve bodies shared by the single-run and the batched field
// kernels (dg_kernels.hip, batched_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "dg_kernels.h"
#include "stage_tiles.h"

namespace dgk {

// -------------------------------------------------------------------------
// Field solve (FP64), two launches per stage (a kernel boundary orders the
// hand-over; a device-scope fence would write back and invalidate L2).
//   fieldA: block ix (256 threads) reduces the density partials of its x
//           element in a fixed order (each wave whole rows) and forms its
//           Fourier sums
//           sum_j T_p^{mj} (n_mj - 1)  (eq. spectral_transform) and its mass.
//   fieldB: one block sums those in element order, synthesises E at every x
//           node, E_mj = sum_{p=1..pmax} 2 Re((i / k_p) c_p e^{i k_p x_mj})
//           (eq. electric_sol), as a polynomial in z = e^{i k_1 x_mj}
//           evaluated by Horner's scheme, and writes the diagnostics record.
// Each kernel issues every read that does not depend on its reduction in the
// first memory round trip.
// No float atomics: results are bitwise reproducible.
// -------------------------------------------------------------------------
constexpr int kFieldB = 1024;

constexpr int kFieldA = 256;

// fieldA variants: LOADS partials per lane, row and pass (one pass covers
// LOADS * 64 values of each of the wave's rows, all loads of a pass in
// flight together; the per-lane sums add the values in index order whatever
// LOADS is, so both forms give the same bits); TPRE: fetch
// the connection-tensor entries of the thread's first mode in the same
// round trip as the partials.  The single-run solve (one block per x
// element, never more than a few hundred blocks) takes the lowest-latency
// form <16, true>; the batched solve (thousands of blocks) the
// register-lean <8, false>, which keeps more blocks resident per CU.

template <int LOADS, bool TPRE>
__device__ __forceinline__ void fieldA_body(const FieldArgs& a, int ix) {
  // every fused multiply-add is written out (fmadd): the rounding then does
  // not depend on the kernel this code is inlined into
  #pragma clang fp contract(off)
  __shared__ double dens[kMaxN];
  __shared__ double wxs[kMaxN];
  const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave, n = a.n;
  // Reads that do not depend on the density go out with the partials, in
  // one memory round trip: the connection-tensor entries of this thread's
  // first mode and the quadrature weights of the element (for its mass).
  double tr[TPRE ? kMaxN : 1], ti[TPRE ? kMaxN : 1];
  if (TPRE && tid < a.pmax) {
#pragma unroll
    for (int j = 0; j < kMaxN; ++j)
      if (j < n) {
        const double* t = a.T + 2 * (static_cast<size_t>(ix * n + j) * a.pmax + tid);
        tr[j] = t[0];
        ti[j] = t[1];
      }
  }
  const double wxj = tid < n ? a.wx[ix * n + tid] : 0.0;
  // The element's partials are n rows of ntiles values, contiguous: wave w
  // sums rows w, w + 4, w + 8 (lane-strided, every load of a pass in flight
  // together), then its lanes in a fixed exchange pattern.
  constexpr int kWaves = kFieldA / kWave;
  constexpr int RW = (kMaxN + kWaves - 1) / kWaves;
  const double* base = a.partials + static_cast<size_t>(ix * n) * a.ntiles;
  const int nt = a.ntiles;
  double s[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) s[r] = 0.0;
  for (int q0 = 0; q0 < nt; q0 += kWave * LOADS) {
    double v[RW][LOADS];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int j = wid + r * kWaves;
#pragma unroll
      for (int q = 0; q < LOADS; ++q) {
        const int idx = q0 + q * kWave + lane;
        v[r][q] = (j < n && idx < nt) ? base[static_cast<size_t>(j) * nt + idx] : 0.0;
      }
    }
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int q = 0; q < LOADS; ++q) s[r] += v[r][q];
  }
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    const int j = wid + r * kWaves;
    if (j < n) {
      const double d = wave_sum(s[r]);
      if (lane == 0) {
        dens[j] = d;
        a.dens[ix * n + j] = d;
      }
    }
  }
  if (tid < n) wxs[tid] = wxj;
  __syncthreads();
  for (int p = tid; p < a.pmax; p += kFieldA) {
    double cr = 0.0, ci = 0.0;
    if (TPRE && p == tid) {
#pragma unroll
      for (int j = 0; j < kMaxN; ++j)
        if (j < n) {
          const double sj = dens[j] - 1.0;
          cr = __builtin_fma(tr[TPRE ? j : 0], sj, cr);
          ci = __builtin_fma(ti[TPRE ? j : 0], sj, ci);
        }
    } else {
      for (int j = 0; j < n; ++j) {
        const double* t = a.T + 2 * (static_cast<size_t>(ix * n + j) * a.pmax + p);
        const double sj = dens[j] - 1.0;
        cr = __builtin_fma(t[0], sj, cr);
        ci = __builtin_fma(t[1], sj, ci);
      }
    }
    a.cpart[2 * (static_cast<size_t>(ix) * a.pmax + p) + 0] = cr;
    a.cpart[2 * (static_cast<size_t>(ix) * a.pmax + p) + 1] = ci;
  }
  if (tid == 0) {
    double m = 0.0;
    for (int j = 0; j < n; ++j) m = __builtin_fma(wxs[j], dens[j], m);
    a.mpart[ix] = m;
  }
}

__device__ __forceinline__ void fieldB_body(const FieldArgs& a) {
  // every fused multiply-add is written out (fmadd): the rounding then does
  // not depend on the kernel this code is inlined into
  #pragma clang fp contract(off)
  extern __shared__ double csh[];          // 2 * pmax scaled coefficients
  __shared__ double red[2][kFieldB];
  __shared__ double wred[2][kFieldB / kWave];
  __shared__ double mass_sh;
  const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
  const int nodes = a.Nx * a.n;
  // Reads that do not depend on the coefficients go out first, in the same
  // round trip as the element partials: this thread's first x node (z_1 and
  // its weight), the first 64 mass partials and the record counter.
  double z1r0 = 0.0, z1i0 = 0.0, wx0 = 0.0;
  if (tid < nodes) {
    z1r0 = a.z1[2 * tid];
    z1i0 = a.z1[2 * tid + 1];
    wx0 = a.wx[tid];
  }
  const double mp0 = (wid == 0 && lane < a.Nx) ? a.mpart[lane] : 0.0;
  const int k = (tid == 0 && a.record && a.ring) ? *a.counter : -1;
  // c_p = sum over elements of the element partials, 64 modes at a time:
  // G = 16 groups of threads, each adding a contiguous G-th of the elements
  // for one mode (its loads in flight together), the groups' sums then added
  // in order.
  constexpr int PB = kWave, G = kFieldB / PB;
  for (int base = 0; base < a.pmax; base += PB) {
    const int p = base + tid % PB;
    const int g = tid / PB;
    double cr = 0.0, ci = 0.0;
    if (p < a.pmax) {
      const int e0 = g * a.Nx / G, e1 = (g + 1) * a.Nx / G;
#pragma unroll 8
      for (int e = e0; e < e1; ++e) {
        cr += a.cpart[2 * (static_cast<size_t>(e) * a.pmax + p) + 0];
        ci += a.cpart[2 * (static_cast<size_t>(e) * a.pmax + p) + 1];
      }
    }
    red[0][tid] = cr;
    red[1][tid] = ci;
    __syncthreads();
    if (tid < PB && base + tid < a.pmax) {
      double r = 0.0, i = 0.0;
      for (int q = 0; q < G; ++q) {
        r += red[0][q * PB + tid];
        i += red[1][q * PB + tid];
      }
      if (a.coeffs) {
        a.coeffs[2 * (base + tid)] = r;
        a.coeffs[2 * (base + tid) + 1] = i;
      }
      // 2 Re((i / k_p) c_p z) = -(2 / k_p) Im(c_p z): fold -2 / k_p in once
      const double sc = -2.0 / ((base + tid + 1) * a.k1);
      csh[2 * (base + tid)] = sc * r;
      csh[2 * (base + tid) + 1] = sc * i;
    }
    __syncthreads();
  }
  // mass: wave 0 adds the element partials (lane-strided, then a fixed
  // exchange pattern)
  if (wid == 0) {
    double mp = mp0;
    for (int e = lane + kWave; e < a.Nx; e += kWave) mp += a.mpart[e];
    mp = wave_sum(mp);
    if (lane == 0) mass_sh = mp;
  }
  // E at every x node: E = Im(sum_p a_p z^p) with z = e^{i k_1 x} and a_p
  // the scaled coefficients, by Horner's scheme, S = z (a_1 + z (a_2 + ...
  // + z a_pmax)): four fused multiply-adds per mode
  double fe = 0.0, mx = 0.0;
  for (int node = tid; node < nodes; node += kFieldB) {
    const bool first = node == tid;
    const double z1r = first ? z1r0 : a.z1[2 * node];
    const double z1i = first ? z1i0 : a.z1[2 * node + 1];
    const double w = first ? wx0 : a.wx[node];
    double ar = 0.0, ai = 0.0;
    for (int p = a.pmax - 1; p >= 0; --p) {
      const double nr = __builtin_fma(z1r, ar, __builtin_fma(-z1i, ai, csh[2 * p]));
      const double ni = __builtin_fma(z1r, ai, __builtin_fma(z1i, ar, csh[2 * p + 1]));
      ar = nr;
      ai = ni;
    }
    const double e = __builtin_fma(z1r, ai, z1i * ar);
    a.E[node] = e;
    fe = __builtin_fma(w * e, e, fe);
    mx = fmax(mx, fabs(e));
  }
  // field energy and max |E|: per wave, then the waves in order
  fe = wave_sum(fe);
  mx = wave_max(mx);
  if (lane == 0) {
    wred[0][wid] = fe;
    wred[1][wid] = mx;
  }
  __syncthreads();
  if (tid == 0) {
    double fsum = 0.0, fmx = 0.0;
    for (int w = 0; w < kFieldB / kWave; ++w) {
      fsum += wred[0][w];
      fmx = fmax(fmx, wred[1][w]);
    }
    const double m = mass_sh + a.mass0;
    const double fen = 0.5 * fsum;
    const bool fin = isfinite(m) && isfinite(fen) && isfinite(fmx);
    double rec[8] = {0.0, m, fen, 0.0, 0.0, fmx, fin ? 1.0 : 0.0, static_cast<double>(k)};
    for (int q = 0; q < 8; ++q) a.last[q] = rec[q];
    if (k >= 0) {
      double* r = a.ring + 8 * (k % kRing);
      for (int q = 0; q < 8; ++q) r[q] = rec[q];
      *a.counter = k + 1;
    }
  }
}

}  // namespace dgk
