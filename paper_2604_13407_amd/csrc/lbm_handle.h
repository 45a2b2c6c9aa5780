// The lattice handle behind the opaque lbm_lattice of the C-ABI, and the host
// helpers shared by the forward (lbm_api.cpp) and adjoint (lbm_adjoint_api.cpp)
// entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/pplbm.h"
#include "lbm_params.h"

// State of the last lbm_adjoint_forward, consumed by lbm_adjoint_backward.
struct AdjointRecord {
  bool ready = false;
  lbm_adjoint_cfg cfg{};
  char* ws = nullptr;      // caller's adjoint workspace
  size_t ws_bytes = 0;
  double inv_den = 0.0;    // velocity-error loss: 1 / sum u_target^2
};

struct lbm_lattice {
  lbm_config cfg;
  lbm_buffers buf;
  hipStream_t stream;
  pplbm::StepParams prm;
  // user-facing parameters kept to rebuild prm
  double s[9];
  int scheme;
  double eps, k1, k2;
  int q2_policy;
  double rho_s;
  int cur = 0;  // 0: f_a holds the current state, 1: f_b
  int64_t steps = 0;
  // float storage: lbm_step re-references after every step whose count is a
  // multiple of this (0: never)
  int64_t reref_every = 0;
  bool initialized = false;
  int seg_len = 64;
  // workspace carve-up
  double* partials = nullptr;
  size_t max_parts = 0;
  double* log = nullptr;
  double* red_tmp = nullptr;
  double* fin_tmp = nullptr;  // the reduction finish's first-stage sums
  void* psi = nullptr;
  // masked lattices on the masked strip march: the per-node link words (in
  // the workspace), whether they have been written since the handle was
  // created (a handle on the library's static workspace, which other handles
  // share, writes them again at every call that steps), and whether the
  // masked strip march is enabled (1, default) or the tile kernel is used (0)
  uint16_t* links = nullptr;
  // ... and, with moving walls, the tiles that hold nodes beside the walls
  // (flags, list, count) and those tiles' reduction partials
  unsigned* tile_flags = nullptr;
  int* tile_list = nullptr;
  int* tile_count = nullptr;
  double* moving_partials = nullptr;
  bool links_ok = false;
  bool static_ws = false;
  int masked_strips = 1;
  AdjointRecord adj;
  std::string err;
};

namespace pplbm_host {

size_t align256(size_t v);
size_t elem_size(const lbm_config* c);
size_t state_bytes_of(const lbm_config* c);
int fail(lbm_lattice* h, int code, const std::string& msg);
int hip_fail(lbm_lattice* h, hipError_t e, const char* what);
bool config_ok(const lbm_config* c, std::string& why);
// Calls without a handle (lbm_create, lbm_create_static and the size queries)
// keep their last message here; lbm_last_error(NULL) returns it.
extern std::string g_create_error;
// Records `msg` as the message of a call without a handle and returns `code`.
int fail_query(int code, const std::string& msg);
// One step from f_in to f_out with the handle's kernels and launch shape;
// reduce = 1 writes reduction partials (n_parts_of(h) of them); `traj` (NULL,
// or [4][ny][nx] doubles: the step's rho - rho_ref, j_x, j_y, psi) only where
// replay_writes_traj(h).
hipError_t step_between(lbm_lattice* h, const void* f_in, void* f_out, int reduce, double* traj = nullptr);
// Whether the step kernel can write the adjoint trajectory itself.
bool replay_writes_traj(const lbm_lattice* h);
// Called by every entry point that steps: a handle on the shared static
// workspace writes its link words again before its first step.
void begin_stepping(lbm_lattice* h);
int n_parts_of(const lbm_lattice* h);
void* state_ptr(lbm_lattice* h, int which);
void fill_record(const double* v, int64_t step, lbm_reduction* r);
int fault_status(lbm_lattice* h, const lbm_reduction& r);

}  // namespace pplbm_host
