// Stage code shared by the single-run and the batched kernels: wave
// reductions, buffer access, the 1D2V and 1D1V stage tiles and the
// single-run stage kernel templates.  Included by dg_kernels.hip and
// batched_kernels.hip (each instantiates what it launches).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dg_kernels.h"
#include "dg_ops_constexpr.h"

namespace dgk {


// Work-groups are dispatched round-robin over the 8 XCDs.  Re-map so that each
// XCD walks a contiguous range of logical tiles: neighbouring tiles (which
// share halo rows) then run at the same time on the same L2.
__device__ __forceinline__ int xcd_remap(int b, int g) {
  const int q = g >> 3, r = g & 7, c = b & 7;
  return c * q + min(c, r) + (b >> 3);
}

// Sum over the 64 lanes of a wave, result valid in every lane.  Within each
// 16-lane row the butterfly uses DPP (quad_perm xor 1, xor 2, row_ror 4, 8),
// so no LDS round trip is needed; the four row sums are combined through
// readlane.  Fixed order: bitwise reproducible.
__device__ __forceinline__ double dpp_f64(double v, int ctrl_sel) {
  typedef int i32x2 __attribute__((ext_vector_type(2)));
  i32x2 x = __builtin_bit_cast(i32x2, v);
  i32x2 y;
  switch (ctrl_sel) {
    case 0:
      y.x = __builtin_amdgcn_mov_dpp(x.x, 0xB1, 0xF, 0xF, true);
      y.y = __builtin_amdgcn_mov_dpp(x.y, 0xB1, 0xF, 0xF, true);
      break;
    case 1:
      y.x = __builtin_amdgcn_mov_dpp(x.x, 0x4E, 0xF, 0xF, true);
      y.y = __builtin_amdgcn_mov_dpp(x.y, 0x4E, 0xF, 0xF, true);
      break;
    case 2:
      y.x = __builtin_amdgcn_mov_dpp(x.x, 0x124, 0xF, 0xF, true);
      y.y = __builtin_amdgcn_mov_dpp(x.y, 0x124, 0xF, 0xF, true);
      break;
    default:
      y.x = __builtin_amdgcn_mov_dpp(x.x, 0x128, 0xF, 0xF, true);
      y.y = __builtin_amdgcn_mov_dpp(x.y, 0x128, 0xF, 0xF, true);
      break;
  }
  return __builtin_bit_cast(double, y);
}

__device__ __forceinline__ double lane_f64(double v, int l) {
  typedef int i32x2 __attribute__((ext_vector_type(2)));
  i32x2 x = __builtin_bit_cast(i32x2, v);
  i32x2 y;
  y.x = __builtin_amdgcn_readlane(x.x, l);
  y.y = __builtin_amdgcn_readlane(x.y, l);
  return __builtin_bit_cast(double, y);
}

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64(v, 0);   // lane ^ 1
  v += dpp_f64(v, 1);   // lane ^ 2
  v += dpp_f64(v, 2);   // rotate by 4 within the row
  v += dpp_f64(v, 3);   // rotate by 8 within the row: every lane holds its row sum
  return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

// Maximum over the 64 lanes (same exchange pattern), valid in every lane.
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_f64(v, 0));
  v = fmax(v, dpp_f64(v, 1));
  v = fmax(v, dpp_f64(v, 2));
  v = fmax(v, dpp_f64(v, 3));
  return fmax(fmax(lane_f64(v, 0), lane_f64(v, 16)), fmax(lane_f64(v, 32), lane_f64(v, 48)));
}

// The stage kernels run one wave per work-group.  LDS instructions of one
// wave execute in program order, so exchanging data through LDS between the
// lanes of that wave only needs the compiler not to reorder the accesses; a
// work-group barrier would also wait for every outstanding global load.
__device__ __forceinline__ void wave_lds_order() { __asm__ volatile("" ::: "memory"); }

__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// t_i = sum_k Ups_ik g_k + Xl_i fL - Xr_i fR for one pencil (operator entries
// are compile-time literals); res_i = s t_i, or res_i += s t_i when ACC.
//
// Even/odd form: on the symmetric LGL nodes Upsilon is centro-antisymmetric
// (Ups[n-1-i][n-1-k] = -Ups[i][k]) and the face columns mirror each other
// (Xr[i] = Xl[n-1-i]).  With e_k = g_k + g_{n-1-k}, o_k = g_k - g_{n-1-k},
// S = fL + fR, D = fL - fR and m = n/2, every output pair (i, n-1-i) is
//   P = sum_{k<m} A_ik e_k + Ups_ic g_c + (Xl_i - Xr_i)/2 S,
//   Q = sum_{k<m} B_ik o_k + (Xl_i + Xr_i)/2 D,
//   t_i = P + Q,  t_{n-1-i} = Q - P,
// A = (Ups_ik + Ups_i,n-1-k)/2, B = (Ups_ik - Ups_i,n-1-k)/2, c the middle
// node (odd n); the middle output is sum_k B_ck o_k + Xl_c D.
template <typename T, int N, bool ACC, typename G>
__device__ __forceinline__ void contract(G g, T fL, T fR, T s, T* res) {
  // every fused multiply-add is written out (fmadd): the rounding then does
  // not depend on the kernel this code is inlined into
  #pragma clang fp contract(off)
  static_assert(dgc::reflection_symmetric<N>(), "LGL operators must be reflection symmetric");
  constexpr dgc::OpsC<N> K = dgc::make_ops<N>();
  constexpr int M = N / 2;
  const T S = fL + fR, D = fL - fR;
  T e[M], o[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    e[k] = g(k) + g(N - 1 - k);
    o[k] = g(k) - g(N - 1 - k);
  }
#pragma unroll
  for (int i = 0; i < M; ++i) {
    T P = static_cast<T>(0.5 * (K.xl[i] - K.xr[i])) * S;
#pragma unroll
    for (int k = 0; k < M; ++k) P = fmadd(static_cast<T>(0.5 * (K.ups[i][k] + K.ups[i][N - 1 - k])), e[k], P);
    if (N % 2) P = fmadd(static_cast<T>(K.ups[i][M]), g(M), P);
    T Q = static_cast<T>(0.5 * (K.xl[i] + K.xr[i])) * D;
#pragma unroll
    for (int k = 0; k < M; ++k) Q = fmadd(static_cast<T>(0.5 * (K.ups[i][k] - K.ups[i][N - 1 - k])), o[k], Q);
    const T ti = P + Q, tm = Q - P;
    res[i] = ACC ? fmadd(s, ti, res[i]) : s * ti;
    res[N - 1 - i] = ACC ? fmadd(s, tm, res[N - 1 - i]) : s * tm;
  }
  if (N % 2) {
    T Q = static_cast<T>(K.xl[M]) * D;
#pragma unroll
    for (int k = 0; k < M; ++k) Q = fmadd(static_cast<T>(K.ups[M][k]), o[k], Q);
    res[M] = ACC ? fmadd(s, Q, res[M]) : s * Q;
  }
}

// Raw buffer access.  A resource covers one x element of a state array; the
// per-row offset goes in the scalar offset and the lane offset in the vector
// offset.  st_nt stores with the non-temporal hint: a stage's output is read
// only by the next kernel, and when the three state buffers exceed the
// last-level (Infinity) cache, stores that allocate there leave dirty lines
// whose write-back then competes with the next kernel's reads.  Lanes past the ragged end of a v chunk get an out-of-range vector
// offset: the hardware range check returns 0 for their loads and drops their
// stores, so no lane mask or branch is needed around memory operations.
constexpr unsigned kRsrcWord3 = 0x00020000u;   // gfx9 raw-buffer format word
constexpr unsigned kOffOOB = 0x80000000u;
constexpr int kCpolNT = 2;                     // cache-policy operand: non-temporal

template <typename T> struct Buf;
template <> struct Buf<float> {
  __device__ static float ld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
  }
  __device__ static float ld_nt(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, kCpolNT));
  }
  __device__ static void st(float v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), r, vo, so, 0);
  }
  __device__ static void st_nt(float v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), r, vo, so, kCpolNT);
  }
};
template <> struct Buf<double> {
  __device__ static double ld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
  }
  __device__ static double ld_nt(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, kCpolNT));
  }
  __device__ static void st(double v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, vo, so, 0);
  }
  __device__ static void st_nt(double v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, vo, so, kCpolNT);
  }
};

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t xelem_rsrc(const T* base, size_t xstride, int ix, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base + ix * xstride), 0, static_cast<int>(bytes), kRsrcWord3);
}

// LDS row stride for the v exchange: the smallest R >= TV*n + 2 for which the
// pencil start addresses pr*R + pv*n (lane = pv*n + pr) fall in distinct banks
// modulo 64, so the n+2 pencil reads of a wave are free of bank conflicts.
template <int N>
constexpr int lds_row() {
  constexpr int TV = kWave / N;
  for (int R = TV * N + 2; R < TV * N + 2 + 128; ++R) {
    bool seen[64] = {};
    bool ok = true;
    for (int pv = 0; pv < TV && ok; ++pv)
      for (int pr = 0; pr < N && ok; ++pr) {
        const int b = (pr * R + pv * N) % 64;
        if (seen[b]) ok = false;
        seen[b] = true;
      }
    if (ok) return R;
  }
  return TV * N + 2;
}
template <int N>
constexpr int lds_words_2v() { return 3 * (N + 1) * lds_row<N>(); }
// FP32 tiles with n >= 7 reduce their density partials through LDS once per
// tile (N x 64 doubles); the others (FP64: LDS would cost occupancy; small n:
// many resident tiles per CU) reduce each row with DPP.
template <typename T, int N>
constexpr bool dens_lds() { return sizeof(T) == 4 && N >= 7; }
template <typename T, int N>
constexpr int dens_words() { return dens_lds<T, N>() ? N * kWave : 1; }
template <int N>
constexpr int lds_words_1v() { return (N + 1) * lds_row<N>(); }

// -------------------------------------------------------------------------
// 1D2V stage kernel.  state [Nx, N, Nu, N, rows of lpitch values]: a row
// holds the Nv*N v values (one x node, one u node) as nvchunks chunks of TV
// elements, chunk c starting at position c*cpitch (cpitch = TV*N dense, 64
// padded).  UN: stage reads u^n.
// -------------------------------------------------------------------------
// lds: lds_words_2v<N>() words (input rows + 2 result buffers; row N of each
// is the scratch row of idle lanes); hbuf: N*N words; dsum: dens_words<T, N>()
// doubles.
// BG: the state holds g = f - f0 for an x-uniform background f0(u, v)
// (dg_set_background); the RHS then adds L(f0) = -E(x) G_u(u, v) + G_b(u, v),
// two FP64-built tables in the state's row layout.
// CORR (FP32, dense rows): L + (corr - corr_xm) in place of L, the
// correction read one row ahead like u^n (the learned correction's stage).
template <typename T, int N, bool UN, bool BG = false, bool CORR = false, bool UNNT = false>
__device__ __forceinline__ void stage2v_tile(const StageArgs<T> a, int bid, T* lds, T* hbuf, double* dsum) {
  // every fused multiply-add is written out (fmadd): the rounding then does
  // not depend on the kernel this code is inlined into
  #pragma clang fp contract(off)
  using B = Buf<T>;
  constexpr unsigned S = sizeof(T);
  constexpr int TV = kWave / N;
  constexpr int ROW = lds_row<N>();
  constexpr dgc::OpsC<N> K = dgc::make_ops<N>();

  const unsigned lane = threadIdx.x;
  const int vc = bid % a.nvchunks;
  const int t1 = bid / a.nvchunks;
  const int iu = t1 % a.Nu;
  const int ix = t1 / a.Nu;
  const int iv0 = vc * TV;
  const int tva = min(TV, a.Nv - iv0);
  const unsigned nact = tva * N;
  const bool act = lane < nact;
  const unsigned vo = act ? lane * S : kOffOOB;
  const unsigned NUn = static_cast<unsigned>(a.Nu) * N;
  const unsigned LP = static_cast<unsigned>(a.lpitch);          // values per row (v line) in memory
  const unsigned CP = static_cast<unsigned>(a.cpitch);          // values per v chunk in memory
  const size_t xstride = static_cast<size_t>(N) * NUn * LP;     // values per x element
  const unsigned xbytes = static_cast<unsigned>(xstride * S);
  const unsigned c0 = iv0 * N;                                  // first v node of the chunk
  const unsigned m0 = vc * CP;                                  // its position in a row
  const unsigned gap = CP - TV * N;                             // unused slots after a full chunk
  // position of the row's last v node (end of the last, possibly ragged, chunk)
  const unsigned mlast = (a.nvchunks - 1) * CP + (a.Nv - (a.nvchunks - 1) * TV) * N - 1;
  // byte offset of (row (jx, iu', ju), chunk start) inside one x element
  auto soff = [&](int jx, int iue, int ju) -> unsigned { return ((jx * NUn + iue * N + ju) * LP + m0) * S; };
  // Rows (jx, iu, 0..N-1) are rowb bytes apart: their common part goes in the
  // lane offset (one VALU add per x node; idle lanes stay out of range) and
  // ju * rowb in the scalar offset, so only N distinct scalar offsets are live
  // instead of one per row of the slab.
  const unsigned rowb = LP * S;
  auto vrow = [&](int jx, int iue) -> unsigned { return vo + ((jx * NUn + iue * N) * LP + m0) * S; };
  // Store offset: the active lanes, plus the unused slots that end a padded
  // chunk, which receive zeros, so that every memory line of a row is written
  // whole (left unwritten, the partly written lines made the padded layout
  // slower than the dense one).  For dense rows this is exactly the active
  // lanes.
  const unsigned vs = (lane < CP && m0 + lane < LP) ? lane * S : kOffOOB;
  const auto rf = xelem_rsrc(a.fin, xstride, ix, xbytes);
  const auto ru = xelem_rsrc(a.fun, xstride, ix, xbytes);
  const auto ro = xelem_rsrc(a.out, xstride, ix, xbytes);

  // v halo through an idle lane: when the chunk leaves lane nact idle and the
  // v speeds u_ju B of all rows share a sign (zeros aside), that lane fetches
  // each row's upwind neighbour node (just before or after the chunk, or the
  // periodic wrap) in the same load instruction as the row, nearly for free;
  // otherwise the N*N halo values are gathered separately below.
  bool vpos = false, vneg = false;
#pragma unroll
  for (int ju = 0; ju < N; ++ju) {
    const T av = a.ucoord[iu * N + ju] * a.wc;
    vpos = vpos || av > T(0);
    vneg = vneg || av < T(0);
  }
  const bool lane_halo = nact < static_cast<unsigned>(kWave) && !(vpos && vneg);
  unsigned vo_ld = vo;
  if (lane_halo && lane == nact) {
    int off;   // row positions relative to the chunk start
    bool outside;
    if (vpos) {
      outside = iv0 == 0;
      off = outside ? static_cast<int>(mlast) : -static_cast<int>(gap) - 1;
    } else {
      outside = iv0 + tva == a.Nv;
      off = outside ? -static_cast<int>(m0) : static_cast<int>(CP);
    }
    vo_ld = (outside && a.zero_inflow) ? kOffOOB : static_cast<unsigned>(off * static_cast<int>(S));
  }

  T f[N][N];
#pragma unroll
  for (int jx = 0; jx < N; ++jx) {
    const unsigned vj = vo_ld + ((jx * NUn + iu * N) * LP + m0) * S;
#pragma unroll
    for (int ju = 0; ju < N; ++ju) f[jx][ju] = B::ld(rf, vj, ju * rowb);
  }

  // x faces: the x speed u is uniform per u node, so the upwind side (left
  // neighbour's last node or right neighbour's first node) is too.
  const int ixl = ix == 0 ? a.Nx - 1 : ix - 1;
  const int ixr = ix == a.Nx - 1 ? 0 : ix + 1;
  T xh[N];
  {
    const auto rxl = xelem_rsrc(a.fin, xstride, ixl, xbytes);
    const auto rxr = xelem_rsrc(a.fin, xstride, ixr, xbytes);
#pragma unroll
    for (int ju = 0; ju < N; ++ju) {
      const T uu = a.ucoord[iu * N + ju];
      T h;
      if (uu > T(0)) h = B::ld(rxl, vrow(N - 1, iu), ju * rowb);
      else h = B::ld(rxr, vrow(0, iu), ju * rowb);
      xh[ju] = uu == T(0) ? T(0) : h;
    }
  }

  // u faces: the u speed -E(x) - v B varies per lane (v) and per x node; the
  // two candidate rows share one scalar base and differ in the vector offset.
  const T vv = a.vcoord[c0 + (act ? lane : 0u)];
  const int iul = iu == 0 ? a.Nu - 1 : iu - 1;
  const int iur = iu == a.Nu - 1 ? 0 : iu + 1;
  const bool zl = a.zero_inflow && iu == 0;
  const bool zr = a.zero_inflow && iu == a.Nu - 1;
  auto uspeed = [&](int jx) -> T { return fmadd(-vv, a.wc, -static_cast<T>(a.E[ix * N + jx])); };
  auto uface = [&](int jx) -> T {
    const T au = uspeed(jx);
    const unsigned oL = soff(jx, iul, N - 1), oR = soff(jx, iur, 0);
    const unsigned ob = min(oL, oR);
    const unsigned vu = act ? lane * S + ((au > T(0) ? oL : oR) - ob) : kOffOOB;
    const T val = B::ld(rf, vu, ob);
    const bool zero = (au == T(0)) || (au > T(0) ? zl : zr);
    return zero ? T(0) : val;
  };

  // v faces: the v speed u B is uniform per u node; one halo value per
  // (x node, u node) row, from the upwind neighbouring v element.
  for (unsigned h = lane_halo ? N * N : lane; h < N * N; h += kWave) {
    const int jx = h / N, ju = h % N;
    const T av = a.ucoord[iu * N + ju] * a.wc;
    unsigned jv;   // row position of the upwind neighbour node
    bool outside;
    if (av > T(0)) {
      outside = iv0 == 0;
      jv = outside ? mlast : m0 - gap - 1;
    } else {
      outside = iv0 + tva == a.Nv;
      jv = outside ? 0u : m0 + CP;
    }
    const T val = B::ld(rf, ((jx * NUn + iu * N + ju) * LP + jv) * S, 0u);
    hbuf[h] = (av == T(0) || (outside && a.zero_inflow)) ? T(0) : val;
  }

  // v-axis pencil owner: lane = pv*N + pr (row pr = u node, element pv of the
  // chunk); idle lanes work on the scratch row N.
  const bool pact = lane < N * tva;
  const int pr = pact ? lane % N : N;
  const int pv = pact ? lane / N : 0;
  const T sv = pact ? a.Jv * a.ucoord[iu * N + pr] * a.wc : T(0);
  const int hside = (lane < N && a.ucoord[iu * N + lane] * a.wc > T(0)) ? 0 : nact + 1;
  // upwind side of the pencil's faces.  It follows the halo slot that is
  // written: with the idle-lane halo only the tile's upwind slot holds data,
  // so a row with zero speed reads that side too (its flux is 0 * t, and t
  // must be finite: the other slot holds whatever LDS held before).
  const bool vleft = pact && (lane_halo ? vpos : a.ucoord[iu * N + pr] * a.wc > T(0));
  // column of this lane's value in an LDS row: the halo lane's goes to the
  // upwind end (slot 0 or nact + 1)
  const unsigned pcol = (lane_halo && lane == nact && vpos) ? 0u : 1u + lane;
  const double wvl = act ? a.wv[c0 + lane] * a.hu : 0.0;    // v weight times du/2
  const int ntiles = a.Nu * a.nvchunks;

  // background rows G_u, G_b of this (u element, v chunk): the same for every x node
  T bgu[BG ? N : 1], bgb[BG ? N : 1];
  if constexpr (BG) {
    const unsigned tb = static_cast<unsigned>(a.Nu) * N * LP * S;
    const auto rgu = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(a.bg_u), 0, static_cast<int>(tb), kRsrcWord3);
    const auto rgb = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(a.bg_b), 0, static_cast<int>(tb), kRsrcWord3);
    const unsigned vb = vo + (iu * N * LP + m0) * S;
#pragma unroll
    for (int ju = 0; ju < N; ++ju) {
      bgu[ju] = B::ld(rgu, vb, ju * rowb);
      bgb[ju] = B::ld(rgb, vb, ju * rowb);
    }
  }
  // rows of u^n and of the u face are fetched one row ahead of their use.
  // u^n rows are read by this tile only; UNNT (the launchers set it where
  // the stage outputs take the non-temporal hint, i.e. buffers larger than
  // the last-level cache) loads them with that hint too.  The slab rows keep
  // the default policy, since neighbouring tiles read their faces and v
  // edge values.  The hint is an immediate of the load instruction, so the
  // two policies are two kernel instances, not a branch.
  auto ld_un = [&](unsigned vo, unsigned so) -> T {
    if constexpr (UNNT) return B::ld_nt(ru, vo, so);
    else return B::ld(ru, vo, so);
  };
  T unr[N];
  if (UN) {
#pragma unroll
    for (int ju = 0; ju < N; ++ju) unr[ju] = ld_un(vrow(0, iu), ju * rowb);
  }
  // correction rows (one ahead) and its x average (the same for every x node)
  T crr[CORR ? N : 1], cxm[CORR ? N : 1];
  const auto rc = CORR ? xelem_rsrc(reinterpret_cast<const T*>(a.corr), xstride, ix, xbytes) : rf;
  if constexpr (CORR) {
#pragma unroll
    for (int ju = 0; ju < N; ++ju) {
      crr[ju] = B::ld(rc, vrow(0, iu), ju * rowb);
      cxm[ju] = (a.corr_xm && act) ? static_cast<T>(a.corr_xm[(iu * N + ju) * static_cast<unsigned>(LP) + m0 + lane])
                                   : T(0);
    }
  }
  // u-face values: without u^n (stage 1) the registers allow fetching all N
  // of them with the slab; with u^n they are fetched one row ahead
  constexpr int NUH = UN ? 1 : N;
  T uhs[NUH];
#pragma unroll
  for (int q = 0; q < NUH; ++q) uhs[q] = uface(q);

  // LDS: lin holds the current x node's row of f (input of the v pencils),
  // lout[2] the v-axis results of the last two rows (double buffered).
  T* const lin = lds;
  T* const lout0 = lds + (N + 1) * ROW;
  T* const lout1 = lds + 2 * (N + 1) * ROW;
  auto put_row = [&](int jx) {
#pragma unroll
    for (int ju = 0; ju < N; ++ju) lin[ju * ROW + pcol] = f[jx][ju];
    if (!lane_halo && lane < N) lin[lane * ROW + hside] = hbuf[jx * N + lane];
  };
  // stage combination, store and FP64 density partial of a finished row
  auto finish_row = [&](int jx, const T* acc, const T* lo) {
    T vout[N];
    const T mE = BG ? -static_cast<T>(a.E[ix * N + jx]) : T(0);
#pragma unroll
    for (int ju = 0; ju < N; ++ju) {
      T rhs = acc[ju] + lo[ju * ROW + 1 + lane];
      if constexpr (BG) rhs += fmadd(mE, bgu[ju], bgb[ju]);
      if constexpr (CORR) rhs += crr[ju] - cxm[ju];
      // with u^n: f + c_un (u^n - f) = c_un u^n + (1 - c_un) f; a nearly
      // steady state then stays bit-identical instead of picking up the same
      // rounding every step (a mass drift in FP32)
      const T base = UN ? fmadd(a.c_un, unr[ju] - f[jx][ju], f[jx][ju]) : a.c_in * f[jx][ju];
      vout[ju] = fmadd(a.c_dt, rhs, base);
    }
    // next u^n row issued before this row's stores (loads and stores share one
    // in-order completion counter)
    if (UN && jx + 1 < N) {
      const unsigned vj = vrow(jx + 1, iu);
#pragma unroll
      for (int ju = 0; ju < N; ++ju) unr[ju] = ld_un(vj, ju * rowb);
    }
    if constexpr (CORR) {
      if (jx + 1 < N) {
        const unsigned vj = vrow(jx + 1, iu);
#pragma unroll
        for (int ju = 0; ju < N; ++ju) crr[ju] = B::ld(rc, vj, ju * rowb);
      }
    }
    // density partial: (du/2) sum_ju w_ju v, reference weights as literals
    double sum = 0.0;
    const unsigned vj = vs + ((jx * NUn + iu * N) * LP + m0) * S;
    if (a.nt_store) {   // uniform branch
#pragma unroll
      for (int ju = 0; ju < N; ++ju) B::st_nt(act ? vout[ju] : T(0), ro, vj, ju * rowb);
    } else {
#pragma unroll
      for (int ju = 0; ju < N; ++ju) B::st(act ? vout[ju] : T(0), ro, vj, ju * rowb);
    }
#pragma unroll
    for (int ju = 0; ju < N; ++ju) sum = __builtin_fma(K.w[ju], static_cast<double>(vout[ju]), sum);
    if (a.partials) {
      // idle lanes: select, never multiply by a zero weight
      sum = act ? sum * wvl : 0.0;
      if constexpr (dens_lds<T, N>()) {
        dsum[jx * kWave + lane] = sum;   // reduced once per tile, after the last row
      } else {
        sum = wave_sum(sum);
        if (lane == 0) a.partials[static_cast<size_t>(ix * N + jx) * ntiles + iu * a.nvchunks + vc] = sum;
      }
    }
  };

  // Software-pipelined loop over the x nodes (rows of the slab).  Row jx:
  // its f row goes to LDS, the register-only x and u parts run while the LDS
  // write and the pencil reads are in flight, the v result goes to lout, and
  // the row is finished during the next iteration, after that row's register
  // work has covered the LDS latency.  LDS accesses of one wave execute in
  // order, so only compiler ordering is needed.
  put_row(0);
  T accp[N];     // x+u parts of the previous row, finished one iteration late
#pragma unroll
  for (int jx = 0; jx < N; ++jx) {
    T acc[N];
    // x axis: acc_ju = Jx u_ju (sum_k Ups[jx][k] f[k][ju] + Xl[jx] fL - Xr[jx] fR)
#pragma unroll
    for (int ju = 0; ju < N; ++ju) {
      const T uu = a.ucoord[iu * N + ju];
      const T fL = uu > T(0) ? xh[ju] : f[0][ju];
      const T fR = uu > T(0) ? f[N - 1][ju] : xh[ju];
      T t = fmadd(static_cast<T>(K.xl[jx]), fL, -(static_cast<T>(K.xr[jx]) * fR));
#pragma unroll
      for (int k = 0; k < N; ++k) t = fmadd(static_cast<T>(K.ups[jx][k]), f[k][ju], t);
      acc[ju] = (a.Jx * uu) * t;
    }
    wave_lds_order();
    T g[N + 2];
#pragma unroll
    for (int k = 0; k < N + 2; ++k) g[k] = lin[pr * ROW + pv * N + k];
    // u axis along the row (covers the pencil read latency)
    {
      const T su = a.Ju * uspeed(jx);
      const bool pos = su > T(0);
      const T uh = uhs[UN ? 0 : jx];
      const T fL = pos ? uh : f[jx][0];
      const T fR = pos ? f[jx][N - 1] : uh;
      contract<T, N, true>([&](int k) { return f[jx][k]; }, fL, fR, su, acc);
    }
    if (UN && jx + 1 < N) uhs[0] = uface(jx + 1);
    // v axis on the pencil
    {
      const T fL = vleft ? g[0] : g[1];
      const T fR = vleft ? g[N] : g[N + 1];
      T r[N];
      contract<T, N, false>([&](int k) { return g[k + 1]; }, fL, fR, sv, r);
      T* lo = (jx & 1) ? lout1 : lout0;
      wave_lds_order();
#pragma unroll
      for (int i = 0; i < N; ++i) lo[pr * ROW + pv * N + 1 + i] = r[i];
    }
    if (jx + 1 < N) put_row(jx + 1);
    wave_lds_order();
    if (jx > 0) finish_row(jx - 1, accp, (jx & 1) ? lout0 : lout1);
#pragma unroll
    for (int i = 0; i < N; ++i) accp[i] = acc[i];
  }
  wave_lds_order();
  finish_row(N - 1, accp, ((N - 1) & 1) ? lout1 : lout0);
  if constexpr (dens_lds<T, N>()) {
    if (a.partials) {
      // lane 4r + q (r < N) adds the row-r partials of lanes 16q .. 16q+15 in
      // lane order; the four quarters are then added in a fixed order
      // ((q0 + q1) + (q2 + q3)) by two quad exchanges, and lane 4r writes.
      wave_lds_order();
      const int r = lane >> 2, q = lane & 3;
      double t = 0.0;
      if (r < N) {
#pragma unroll
        for (int i = 0; i < 16; ++i) t += dsum[r * kWave + 16 * q + i];
      }
      t += dpp_f64(t, 0);   // lane ^ 1
      t += dpp_f64(t, 1);   // lane ^ 2
      if (r < N && q == 0) a.partials[static_cast<size_t>(ix * N + r) * ntiles + iu * a.nvchunks + vc] = t;
    }
  }
}

// -------------------------------------------------------------------------
// 1D1V stage kernel.  state [Nx, N, Nv, N]; x speed v, v speed -E(x).
// -------------------------------------------------------------------------
template <typename T, int N, bool UN, bool BG = false>
__device__ __forceinline__ void stage1v_tile(const StageArgs<T> a, int bid, T* lds) {
  // every fused multiply-add is written out (fmadd): the rounding then does
  // not depend on the kernel this code is inlined into
  #pragma clang fp contract(off)
  using B = Buf<T>;
  constexpr unsigned S = sizeof(T);
  constexpr int TV = kWave / N;
  constexpr int ROW = lds_row<N>();

  const unsigned lane = threadIdx.x;
  const int vc = bid % a.nvchunks;
  const int ix = bid / a.nvchunks;
  const int iv0 = vc * TV;
  const int tva = min(TV, a.Nv - iv0);
  const unsigned nact = tva * N;
  const bool act = lane < nact;
  const unsigned vo = act ? lane * S : kOffOOB;
  const unsigned NVn = static_cast<unsigned>(a.Nv) * N;
  const size_t xstride = static_cast<size_t>(N) * NVn;
  const unsigned xbytes = static_cast<unsigned>(xstride * S);
  const unsigned c0 = iv0 * N;
  auto soff = [&](int jx) -> unsigned { return (jx * NVn + c0) * S; };
  const auto rf = xelem_rsrc(a.fin, xstride, ix, xbytes);

  T f[N];
#pragma unroll
  for (int jx = 0; jx < N; ++jx) f[jx] = B::ld(rf, vo, soff(jx));
  const T vv = a.vcoord[c0 + (act ? lane : 0u)];
  const int ixl = ix == 0 ? a.Nx - 1 : ix - 1;
  const int ixr = ix == a.Nx - 1 ? 0 : ix + 1;
  // x faces: the x speed v varies per lane; both candidate rows are coalesced.
  const T hl = B::ld(xelem_rsrc(a.fin, xstride, ixl, xbytes), vo, soff(N - 1));
  const T hr = B::ld(xelem_rsrc(a.fin, xstride, ixr, xbytes), vo, soff(0));
  const T xh = vv > T(0) ? hl : (vv < T(0) ? hr : T(0));

  T acc[N];
  {
    const T fL = vv > T(0) ? xh : f[0];
    const T fR = vv > T(0) ? f[N - 1] : xh;
    // unscaled (s = 1 is exact): the x speed multiplies in the final fused
    // multiply-add with the v part
    contract<T, N, false>([&](int k) { return f[k]; }, fL, fR, T(1), acc);
  }
  // v faces, one per x node row, from the side selected by the sign of -E.
  T hval = T(0);
  int hside = 0;
  if (lane < N) {
    const T av = -static_cast<T>(a.E[ix * N + lane]);
    unsigned jv;
    bool outside;
    if (av > T(0)) {
      outside = iv0 == 0;
      jv = outside ? NVn - 1 : c0 - 1;
      hside = 0;
    } else {
      const int e = iv0 + tva;
      outside = e == a.Nv;
      jv = outside ? 0u : static_cast<unsigned>(e) * N;
      hside = nact + 1;
    }
    const T val = B::ld(rf, (lane * NVn + jv) * S, 0u);
    hval = (av == T(0) || (outside && a.zero_inflow)) ? T(0) : val;
  }
#pragma unroll
  for (int jx = 0; jx < N; ++jx) lds[jx * ROW + 1 + lane] = f[jx];
  if (lane < N) lds[lane * ROW + hside] = hval;
  wave_lds_order();
  const bool pact = lane < N * tva;
  const int pr = pact ? lane % N : N;
  const int pv = pact ? lane / N : 0;
  const T sv = pact ? -a.Jv * static_cast<T>(a.E[ix * N + pr]) : T(0);
  {
    T g[N + 2];
#pragma unroll
    for (int k = 0; k < N + 2; ++k) g[k] = lds[pr * ROW + pv * N + k];
    const T fL = sv > T(0) ? g[0] : g[1];
    const T fR = sv > T(0) ? g[N] : g[N + 1];
    T r[N];
    contract<T, N, false>([&](int k) { return g[k + 1]; }, fL, fR, sv, r);
    wave_lds_order();
#pragma unroll
    for (int i = 0; i < N; ++i) lds[pr * ROW + pv * N + 1 + i] = r[i];
  }
  wave_lds_order();
  const auto ru = xelem_rsrc(a.fun, xstride, ix, xbytes);
  const auto ro = xelem_rsrc(a.out, xstride, ix, xbytes);
  const double wvl = act ? a.wv[c0 + lane] : 0.0;
  const T sx = a.Jx * vv;
  // background (1D1V): L(f0) = -E(x) G_v(v)
  const T bgv = BG ? a.bg_u[act ? c0 + lane : 0u] : T(0);
#pragma unroll
  for (int jx = 0; jx < N; ++jx) {
    T rhs = fmadd(sx, acc[jx], lds[jx * ROW + 1 + lane]);
    if constexpr (BG) rhs = fmadd(-static_cast<T>(a.E[ix * N + jx]), bgv, rhs);
    const T base = UN ? fmadd(a.c_un, B::ld(ru, vo, soff(jx)) - f[jx], f[jx]) : a.c_in * f[jx];
    const T v = fmadd(a.c_dt, rhs, base);
    if (a.nt_store) B::st_nt(v, ro, vo, soff(jx));
    else B::st(v, ro, vo, soff(jx));
    if (a.partials) {
      const double s = wave_sum(act ? wvl * static_cast<double>(v) : 0.0);
      if (lane == 0) a.partials[static_cast<size_t>(ix * N + jx) * a.nvchunks + vc] = s;
    }
  }
}

// -------------------------------------------------------------------------
// Single-run stage kernels: one tile per work-group.
// -------------------------------------------------------------------------
// FP64 slabs of n = 9 do not fit 256 VGPRs; at one wave per SIMD the
// compiler may also use the accumulation registers instead of spilling to
// scratch memory.  FP64 n = 12 (476 registers at one wave per SIMD) is built
// for two waves per SIMD with scratch spills: the one-wave build of this
// same source returned wrong values for one v pencil (x node 6, u node 4,
// first element of each chunk) whenever the v term was active, while the
// two-wave build matches the oracle to 1.7e-15.
template <typename T, int N>
constexpr int stage_min_waves() { return sizeof(T) == 8 && N >= 9 && N <= 11 ? 1 : 2; }

template <typename T, int N, bool UN, bool BG, bool CORR = false, bool UNNT = false>
__global__ void __launch_bounds__(kWave, (stage_min_waves<T, N>())) stage2v_kernel(StageArgs<T> a) {
  __shared__ T lds[lds_words_2v<N>()];
  __shared__ T hbuf[N * N];
  __shared__ double dsum[dens_words<T, N>()];
  // reversed order: the tiles the previous stage wrote last are read first
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  stage2v_tile<T, N, UN, BG, CORR, UNNT>(a, a.reverse ? static_cast<int>(gridDim.x) - 1 - b : b, lds, hbuf, dsum);
}

template <typename T, int N, bool UN, bool BG>
__global__ void __launch_bounds__(kWave) stage1v_kernel(StageArgs<T> a) {
  __shared__ T lds[lds_words_1v<N>()];
  stage1v_tile<T, N, UN, BG>(a, xcd_remap(blockIdx.x, gridDim.x), lds);
}

}  // namespace dgk
