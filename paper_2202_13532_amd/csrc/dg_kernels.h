// Launch interface of the HIP kernels (host side, C++ linkage).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace dgk {

constexpr int kWave = 64;
constexpr int kMaxN = 12;
constexpr int kRing = 1024;   // diagnostics records per device ring

// v-elements covered by one wave for n nodes: the wave's lanes hold the
// contiguous v-nodes of whole elements.
inline int tv_of(int n) { return kWave / n; }

template <typename T>
struct StageArgs {
  const T* fin;           // argument of L (u^(k-1))
  const T* fun;           // u^n, read only when c_un != 0
  T* out;                 // c_un u^n + c_in fin + c_dt L(fin)
  const double* E;        // Nx*n field at the x nodes
  const T* ucoord;        // Nu*n u-node coordinates (nv = 2)
  const T* vcoord;        // Nv*n v-node coordinates
  const double* wu;       // Nu*n u quadrature weights (dx/2 w_j), nv = 2
  const double* wv;       // Nv*n v quadrature weights
  const double* wx;       // Nx*n x quadrature weights (moments only)
  const double* uc64;     // Nu*n u-node coordinates in FP64 (moments only)
  const double* vc64;     // Nv*n v-node coordinates in FP64 (moments only)
  double* partials;       // density partials or nullptr
  const T* bg_u;          // background tables (state-row layout, storage precision) or nullptr:
  const T* bg_b;          //   1D2V G_u, G_b of L(f0) = -E G_u + G_b; 1D1V bg_u = G_v (Nv*n)
  const double* bg64;     // background f0 (FP64, dense [Nu*n][Nv*n] or [Nv*n]) for the moments, or nullptr
  const float* corr;      // FP32 1D2V dense states: a correction added to L (state layout), or nullptr
  const float* corr_xm;   //   and its x average per (u node, v node), subtracted, or nullptr
  double hu;              // du/2 (u-axis Jacobian inverse), nv = 2
  int Nx, Nu, Nv, nvchunks;
  int cpitch, lpitch;     // values per v chunk / per (x node, u node) row of the arrays
  int nt_store;           // 1: non-temporal stores (the run's three state buffers exceed the last-level cache)
  int reverse;            // 1: 1D2V tiles visited in reverse order (single-run stage launches)
  int zero_inflow;        // 1: zero outside the velocity box
  int n1v;                // batched launches: n of a 1D1V run, 0 for a 1D2V run
  T Jx, Ju, Jv, wc;       // Jacobians 2/dx per axis, omega_c
  T c_un, c_in, c_dt;     // stage coefficients
};

struct FieldArgs {
  const double* partials;  // [(Nx*n) * ntiles]
  int ntiles;              // partials per x node
  int Nx, n, pmax;
  double k1;               // 2 pi / L
  const double* T;         // connection tensor, complex (re,im), [(Nx*n) x pmax]
  const double* z1;        // e^{i k_1 x_mj}, complex, [Nx*n]
  const double* wx;        // Nx*n x quadrature weights
  double* dens;            // Nx*n density
  double* cpart;           // Nx * pmax complex partial Fourier sums
  double* mpart;           // Nx mass partials
  double* E;               // Nx*n field out
  double* coeffs;          // pmax complex coefficients out
  double* ring;            // diagnostics ring (dg_diag records as 8 doubles) or nullptr
  double* last;            // always receives the newest record (8 doubles)
  int* counter;            // ring write counter
  int record;              // 1: append a record
  double mass0;            // mass of the background f0 (added to the recorded mass)
};

// Launchers return hipSuccess or the launch error.  `args` points to a
// StageArgs<float> or StageArgs<double> matching f64.
hipError_t launch_stage(int nv, int n, bool f64, const void* args, int ntiles, hipStream_t s);
hipError_t launch_density(int nv, int n, bool f64, const void* args, int ntiles, hipStream_t s);
hipError_t launch_moments(int nv, int n, bool f64, const void* args, double* mom, int ntiles, hipStream_t s);
hipError_t launch_field(const FieldArgs& a, hipStream_t s);
hipError_t launch_moments_reduce(const double* mom, int ntiles, double* ring, const int* counter, hipStream_t s);
hipError_t launch_reset_counter(int* counter, hipStream_t s);
// copy references: a 16-byte grid-stride copy of `bytes` (multiple of 16),
// and the 1D2V stage kernel's tile access pattern without halos or arithmetic
hipError_t launch_linear_copy(const void* in, void* out, size_t bytes, hipStream_t s);
hipError_t launch_empty(hipStream_t s);
hipError_t launch_pattern_copy(int nv, int n, bool f64, const void* args, int ntiles, bool stage_residency,
                               hipStream_t s);
// c_p (2*pmax doubles) = T (node-major [nodes][pmax] complex) applied to g (nodes)
hipError_t launch_fourier(const double* T, const double* g, int nodes, int pmax, double* out, hipStream_t s);
// out = M in along the x rows: M R x R, states R x C, storage precision
hipError_t launch_xfilter(bool f64, const void* in, void* out, const void* M, int R, size_t C, hipStream_t s);
// dense rows of nvn values <-> rows of lp values in chunks of cp (tvn used);
// pack writes rows*lp values (zeros in unused slots), unpack rows*nvn
hipError_t launch_repack(bool pack, bool f64, const void* in, void* out, size_t rows, unsigned lp, unsigned cp,
                         unsigned tvn, unsigned nvn, hipStream_t s);

// Batched persistent stage of one kind: `runs` (device) holds one
// StageArgs<float> per run of the batch, `items` (device) the kind's (run,
// tile) work list, `xcd_begin` (device, 9 entries, relative to `items`) its
// split over the 8 XCDs.  nv = 2: the 1D2V runs of n nodes; nv = 1: the 1D1V
// runs of any n (StageArgs::n1v; n ignored).  un_nt: the 1D2V u^n loads take
// the non-temporal hint (the runs' buffers exceed the last-level cache).
hipError_t launch_stage_batched(bool un, bool un_nt, int n, int nv, const StageArgs<float>* runs, const int2* items,
                                const int* xcd_begin, int grid, hipStream_t s);
// Batched field solve: `fa` (device) one FieldArgs per run, `xitems` (device)
// the (run, x element) list.
hipError_t launch_field_batched(const FieldArgs* fa, const int2* xitems, int nxitems, int nruns, int max_pmax, hipStream_t s);
// Resident work-groups per CU of the batched stage kernel of a kind.
int batched_occupancy(bool un, int n, int nv);

}  // namespace dgk
