// Internal: the context structure and the stage / field helpers shared by
// the single-run entry points and the learned-correction entry points.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/dg.h"
#include "dg_host.h"

namespace dgi {

// Workspace layout derived from a validated configuration.
struct Layout {
  size_t esize = 0, dof = 0;
  int naxes = 0, n = 0, Nx = 0, Nu = 1, Nv = 0, nvchunks = 0, pmax = 0;
  int ntiles_slab = 0, ntiles = 0;
  int cpitch = 0, lpitch = 0;   // values per v chunk and per row of a state array (dg_layout)
  size_t selems = 0;            // values in a state array
  size_t off_B, off_C, off_part, off_mom, off_dens, off_E, off_cpart, off_mpart, off_coef, off_ring,
      off_last, off_ctr, off_T, off_z1, off_wx, off_wu, off_wv, off_uc, off_vc, off_uc64, off_vc64,
      off_bgu, off_bgb, off_bg64, off_M, total;
};

}  // namespace dgi

struct dg_ctx {
  dg_config cfg{};
  uint64_t id = 0;   // unique per context in the process (keys of cached graphs held elsewhere)
  dgi::Layout L;
  dgh::Basis basis;
  double courant = 0.0;
  double dx[3] = {0, 0, 0};
  char* ws = nullptr;
  hipStream_t user = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  bool owns_stream = true;
  double t = 0.0;
  std::string err = "no error";
  // cached step graph
  hipGraphExec_t gexec = nullptr;
  const void* g_f = nullptr;
  double g_dt = 0.0;
  bool g_diag = false;
  // background f0 (dg_set_background): states hold g = f - f0
  bool bg = false;
  double mass0 = 0.0;

  template <typename P> P* at(size_t off) const { return reinterpret_cast<P*>(ws + off); }
  bool f64() const { return cfg.storage == DG_F64; }
};

namespace dgi {

dg_status fail(dg_ctx* c, dg_status s, const std::string& msg);
dg_status hip_fail(dg_ctx* c, hipError_t e, const char* what);
// out = c_un un + c_in fin + c_dt L(fin) with field E; density partials of out
// into `partials` when non-NULL.
dg_status stage(dg_ctx* c, const void* fin, const void* fun, void* out, const double* E, double* partials,
                double c_un, double c_in, double c_dt, bool reverse = false, const float* corr = nullptr,
                const float* corr_xm = nullptr);
// Density partials of f (FP64) into the workspace.
dg_status density(dg_ctx* c, const void* f);
// Velocity moments of f into the diagnostics ring (after a recording field solve).
dg_status moments(dg_ctx* c, const void* f);
// Field solve from the workspace density partials.
dg_status field(dg_ctx* c, double* E, double* coeffs, bool record);
dg_status enter(dg_ctx* c);
dg_status leave(dg_ctx* c);
// Field of f, CFL check of dt (synchronises).
dg_status begin_steps(dg_ctx* ctx, void* f, double dt, int32_t nsteps);
void copy_record(const double* r, double t, dg_diag* out);
// Workspace layout without stage buffers (the stage's scratch only).
Layout scratch_layout(const dg_config* cfg);
// Reason cfg is rejected (and the status in *st), or NULL.
const char* config_error(const dg_config* cfg, dg_status* st);
// Record msg as the context-free error (dg_last_error(NULL)) and return s.
dg_status global_fail(dg_status s, const std::string& msg);

// Destroy an executable graph once the stream that replays it is idle (a
// caller may have launched it and returned without waiting); *g = NULL.
inline void drop_graph(hipStream_t stream, hipGraphExec_t* g) {
  if (!*g) return;
  (void)hipStreamSynchronize(stream);
  (void)hipGraphExecDestroy(*g);
  *g = nullptr;
}

}  // namespace dgi
