// Launch interface between the C-ABI host code and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pplbm.h"
#include "lbm_params.h"

namespace pplbm {

struct StepLaunch {
  const void* f_in;
  void* f_out;
  const uint8_t* mask;
  const double* wall_u;
  void* psi;          // two-pass pseudopotential field (double)
  double* partials;   // per-block / per-wave reduction partials
  int kernel;         // 0 fused, 1 two-pass
  int seg_len;        // fused: rows per wavefront
  int reduce;         // 1: write reduction partials this step
  int fast;           // fused: use the specialised strip kernel (no mask, no moving walls, 32-bit offsets)
  double* traj;       // adjoint replay: also write rho - rho_ref, j_x, j_y, psi per node ([4][ny][nx]);
                      // aligned strip kernel only, without reductions; NULL otherwise
  int interleave;     // aligned strip kernel: the XCDs take successive runs of rows in turn (0: each XCD
                      // takes one contiguous band of runs)
  int aligned;        // fused, no mask or moving walls: the strip march over 64-column strips (the last
                      // one partial where the width is not a multiple of 64)
  int masked;         // fused, solid mask or moving walls: the masked strip march
  const uint16_t* links;  // masked strip march: the per-node link words ([ny][nx], launch_links)
  // masked strip march with moving walls: the tiles holding nodes beside the
  // walls (launch_links) and their reduction partials
  const int* tile_list;
  const int* tile_count;
  double* moving_partials;
  int lockstep;       // aligned strip kernel (unmasked): the 4 waves of a block march in lockstep
};

int two_pass_blocks(int nx, int ny);
// Blocks (one reduction record each) of the fused tile kernel, which takes the
// lattices the strip kernels do not.
int tile_blocks(int nx, int ny);
// Strip and segment counts of the fused strip kernels (one reduction record
// per strip and segment): aligned, 64-column strips (the last one partial
// where the width is not a multiple of 64); otherwise 62-column strips.
void fused_shape(int nx, int ny, int seg_len, bool aligned, int* n_strips, int* n_segs);

template <class S>
hipError_t launch_init(const StepParams& p, const double* rho0, const double* ux0, const double* uy0,
                       const uint8_t* mask, void* fa, void* fb, hipStream_t s);
template <class S>
hipError_t launch_step(const StepParams& p, const StepLaunch& L, hipStream_t s);
template <class S>
hipError_t launch_fields(const StepParams& p, const void* f, const uint8_t* mask, const double* wall_u, void* psi,
                         double* rho, double* ux, double* uy, double* fx, double* fy, double* psi_o,
                         double* partials, int reduce, hipStream_t s);
// Link words of a masked lattice for the masked strip march (bit 0 solid
// node, bits 1-8 pull source solid or beyond a wall, bit 9 moving-wall term).
// With moving walls, also the list of the tile kernel's 32 x 8 tiles that hold
// a fluid node beside a moving wall (in increasing tile index) and its count;
// tile_flags, tile_list: one entry per tile.
hipError_t launch_links(const StepParams& p, const uint8_t* mask, int moving, uint16_t* links, unsigned* tile_flags,
                        int* tile_list, int* tile_count, hipStream_t s);
// Float storage: the reference density of every node becomes its current
// density (both population arrays hold the current state).
hipError_t launch_reref(const StepParams& p, void* fa, void* fb, const uint8_t* mask, hipStream_t s);
// Fixed-order sum of n_parts partials (and of *extra_count more at extra, when
// extra is non-NULL) into out[RED_COUNT], through tmp (kFinalizeBlocks *
// RED_COUNT doubles).
constexpr int kFinalizeBlocks = 128;
hipError_t launch_finalize(const double* partials, int n_parts, double* out, double* tmp, hipStream_t s,
                           const double* extra = nullptr, const int* extra_count = nullptr);

// Size of the library-owned workspace of lbm_create_static handles, and its
// address on the current device (resolved once per device).
constexpr size_t kStaticWorkspaceBytes = LBM_STATIC_WORKSPACE_BYTES;
hipError_t static_workspace(void** ptr);

}  // namespace pplbm
