// Batched persistent stage kernels and the batched field solve (many
// independent runs stepped together, FP32 storage), with their launchers.
#include <hip/hip_runtime.h>

#include "field_bodies.h"
#include "stage_tiles.h"

namespace dgk {

// -------------------------------------------------------------------------
// Batched stage kernels: many independent runs (1D1V and 1D2V, n in 2..12,
// FP32 storage).  The 1D2V runs are grouped by kind (n); each kind gets one
// launch per RK stage, specialised like the single-run kernels (a single
// launch for every kind would carry the largest kind's register allocation
// and run every kind at its occupancy).  The host builds each kind's (run,
// tile) work list, ordered by decreasing tile cost (or run-interleaved) and
// split into 8 contiguous ranges, one per XCD; work-group b serves range
// b % 8 with a stride of the number of work-groups on that XCD, so the waves
// of one XCD walk neighbouring tiles together.  The grid is the kind's
// launch shape: persistent (a few work-groups per CU, each looping over its
// range) or one work-group per tile.
// The 1D1V runs of a batch, whatever their n, share one launch per stage (a
// launch per n and stage costs a fixed ~10 us, often for ~1 % of the DOF;
// inside a 1D2V kind's launch their latency-bound tiles ran slower still, at
// that kind's occupancy); each item branches on its run's n1v, a
// wave-uniform value.
// -------------------------------------------------------------------------
template <bool UN>
__device__ __forceinline__ void stage1v_any_n(const StageArgs<float>& a, int tile, float* lds) {
  switch (a.n1v) {
    case 2: stage1v_tile<float, 2, UN>(a, tile, lds); break;
    case 3: stage1v_tile<float, 3, UN>(a, tile, lds); break;
    case 4: stage1v_tile<float, 4, UN>(a, tile, lds); break;
    case 5: stage1v_tile<float, 5, UN>(a, tile, lds); break;
    case 6: stage1v_tile<float, 6, UN>(a, tile, lds); break;
    case 7: stage1v_tile<float, 7, UN>(a, tile, lds); break;
    case 8: stage1v_tile<float, 8, UN>(a, tile, lds); break;
    case 9: stage1v_tile<float, 9, UN>(a, tile, lds); break;
    case 10: stage1v_tile<float, 10, UN>(a, tile, lds); break;
    case 11: stage1v_tile<float, 11, UN>(a, tile, lds); break;
    case 12: stage1v_tile<float, 12, UN>(a, tile, lds); break;
    default: break;
  }
}

constexpr int max_lds_words_1v() {
  int m = 0;
  const int w[] = {lds_words_1v<2>(), lds_words_1v<3>(), lds_words_1v<4>(), lds_words_1v<5>(),
                   lds_words_1v<6>(), lds_words_1v<7>(), lds_words_1v<8>(), lds_words_1v<9>(),
                   lds_words_1v<10>(), lds_words_1v<11>(), lds_words_1v<12>()};
  for (int x : w) m = x > m ? x : m;
  return m;
}

// Work-list walk shared by both batched kernels: work-group b serves XCD
// range b % 8; the item (run, tile) is the same for every lane, so it and the
// run's arguments stay in scalar registers.
template <typename F>
__device__ __forceinline__ void batched_walk(const StageArgs<float>* __restrict__ runs, const int2* __restrict__ items,
                                             const int* __restrict__ xcd_begin, F&& tile_fn) {
  const int b = blockIdx.x, c = b & 7, slot = b >> 3, g = gridDim.x;
  const int slots = (g >> 3) + (c < (g & 7) ? 1 : 0);
  const int end = xcd_begin[c + 1];
  for (int i = xcd_begin[c] + slot; i < end; i += slots) {
    const int2 it = items[i];
    const int run = __builtin_amdgcn_readfirstlane(it.x);
    const int tile = __builtin_amdgcn_readfirstlane(it.y);
    tile_fn(runs[run], tile);
    wave_lds_order();
  }
}

template <bool UN, int N, bool UNNT = false>
__global__ void __launch_bounds__(kWave, 2) stage_batched_kernel(const StageArgs<float>* __restrict__ runs,
                                                                  const int2* __restrict__ items,
                                                                  const int* __restrict__ xcd_begin) {
  __shared__ float lds[lds_words_2v<N>()];
  __shared__ float hbuf[N * N];
  __shared__ double dsum[dens_words<float, N>()];
  batched_walk(runs, items, xcd_begin, [&](const StageArgs<float>& a, int tile) {
    stage2v_tile<float, N, UN, false, false, UNNT>(a, tile, lds, hbuf, dsum);
  });
}

template <bool UN>
__global__ void __launch_bounds__(kWave) stage_batched_1v_kernel(const StageArgs<float>* __restrict__ runs,
                                                                  const int2* __restrict__ items,
                                                                  const int* __restrict__ xcd_begin) {
  __shared__ float lds[max_lds_words_1v()];
  batched_walk(runs, items, xcd_begin, [&](const StageArgs<float>& a, int tile) { stage1v_any_n<UN>(a, tile, lds); });
}

// Batched field solve: block q of fieldA serves (run, x element) item q;
// block r of fieldB serves run r.
__global__ void __launch_bounds__(kFieldA) fieldA_batched_kernel(const FieldArgs* __restrict__ fa, const int2* __restrict__ items) {
  const int2 it = items[blockIdx.x];
  fieldA_body<8, false>(fa[it.x], it.y);
}
__global__ void __launch_bounds__(kFieldB) fieldB_batched_kernel(const FieldArgs* __restrict__ fa) {
  fieldB_body(fa[blockIdx.x]);
}


template <int N>
static hipError_t stage_batched_t(bool un, bool un_nt, const StageArgs<float>* runs, const int2* items,
                                  const int* xcd_begin, int grid, hipStream_t s) {
  if (un && un_nt)
    hipLaunchKernelGGL((stage_batched_kernel<true, N, true>), dim3(grid), dim3(kWave), 0, s, runs, items, xcd_begin);
  else if (un) hipLaunchKernelGGL((stage_batched_kernel<true, N>), dim3(grid), dim3(kWave), 0, s, runs, items, xcd_begin);
  else hipLaunchKernelGGL((stage_batched_kernel<false, N>), dim3(grid), dim3(kWave), 0, s, runs, items, xcd_begin);
  return hipGetLastError();
}

template <typename K>
static int occ_of_kernel(K kernel) {
  int nb = 0;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kWave, 0) == hipSuccess ? nb : 0;
}

hipError_t launch_stage_batched(bool un, bool un_nt, int n, int nv, const StageArgs<float>* runs, const int2* items,
                                const int* xcd_begin, int grid, hipStream_t s) {
  if (grid < 1) return hipErrorInvalidValue;
  if (nv == 1) {
    if (un) hipLaunchKernelGGL(stage_batched_1v_kernel<true>, dim3(grid), dim3(kWave), 0, s, runs, items, xcd_begin);
    else hipLaunchKernelGGL(stage_batched_1v_kernel<false>, dim3(grid), dim3(kWave), 0, s, runs, items, xcd_begin);
    return hipGetLastError();
  }
  switch (n) {
#define DG_BATCH_CASE(NN) \
  case NN: return stage_batched_t<NN>(un, un_nt, runs, items, xcd_begin, grid, s);
    DG_BATCH_CASE(2) DG_BATCH_CASE(3) DG_BATCH_CASE(4) DG_BATCH_CASE(5)
    DG_BATCH_CASE(6) DG_BATCH_CASE(7) DG_BATCH_CASE(8) DG_BATCH_CASE(9)
    DG_BATCH_CASE(10) DG_BATCH_CASE(11) DG_BATCH_CASE(12)
#undef DG_BATCH_CASE
    default: return hipErrorInvalidValue;
  }
}

int batched_occupancy(bool un, int n, int nv) {
  if (nv == 1) return un ? occ_of_kernel(stage_batched_1v_kernel<true>) : occ_of_kernel(stage_batched_1v_kernel<false>);
  switch (n) {
#define DG_BATCH_CASE(NN) \
  case NN: return un ? occ_of_kernel(stage_batched_kernel<true, NN>) : occ_of_kernel(stage_batched_kernel<false, NN>);
    DG_BATCH_CASE(2) DG_BATCH_CASE(3) DG_BATCH_CASE(4) DG_BATCH_CASE(5)
    DG_BATCH_CASE(6) DG_BATCH_CASE(7) DG_BATCH_CASE(8) DG_BATCH_CASE(9)
    DG_BATCH_CASE(10) DG_BATCH_CASE(11) DG_BATCH_CASE(12)
#undef DG_BATCH_CASE
    default: return 0;
  }
}

hipError_t launch_field_batched(const FieldArgs* fa, const int2* xitems, int nxitems, int nruns, int max_pmax, hipStream_t s) {
  hipLaunchKernelGGL(fieldA_batched_kernel, dim3(nxitems), dim3(kFieldA), 0, s, fa, xitems);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fieldB_batched_kernel, dim3(nruns), dim3(kFieldB), 2 * max_pmax * sizeof(double), s, fa);
  return hipGetLastError();
}


}  // namespace dgk
