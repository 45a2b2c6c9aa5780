// Host side of liblbm.so: the C-ABI declared in include/pplbm.h.
//
// The handle keeps the caller's device pointers, a parameter block and the
// index of the population array holding the current state.  All device work
// is enqueued on the caller's stream; no device memory is allocated here.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pplbm.h"
#include "lbm_handle.h"
#include "lbm_internal.h"
#include "lbm_node.h"

using pplbm::RED_COUNT;
using pplbm::StepParams;

namespace pplbm_host {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t elem_size(const lbm_config* c) { return c->precision == LBM_FP64 ? sizeof(double) : sizeof(float); }

// 9 population planes, plus the reference plane for float storage.
size_t state_bytes_of(const lbm_config* c) {
  const size_t planes = c->precision == LBM_FP64 ? 9 : 10;
  return planes * (size_t)c->nx * (size_t)c->ny * elem_size(c);
}

int fail(lbm_lattice* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}

int hip_fail(lbm_lattice* h, hipError_t e, const char* what) {
  return fail(h, LBM_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// The specialised strip kernel handles lattices without a mask or moving walls
// whose population arrays fit 32-bit byte offsets.
bool fast_path(const lbm_lattice* h) {
  // 32-bit byte offsets into the population array
  double bytes = (double)state_bytes_of(&h->cfg);
  return h->cfg.kernel == LBM_KERNEL_FUSED && !h->buf.mask && !h->buf.wall_u && bytes < 4294967040.0;
}

// Whether the two population arrays exceed the 256 MB last-level cache, so
// that every step streams them from HBM.
bool streams_from_hbm(const lbm_config* c) { return 2.0 * (double)state_bytes_of(c) > 256.0 * 1048576.0; }

// Widths that are not a multiple of 64 end in a partial strip.  The strip
// march takes them for float storage (1.6-2.8x the tile kernel: 1000 x 1000
// droplet 22.4k -> 41.9k MLUPS, 2000 x 4096 20.3k -> 56.2k, 1000 x 1000 annulus
// with moving walls 16.6k -> 26.6k) and for lattices that stream from HBM
// (double storage, 2000 x 4096: the 62-column kernel 30.8k, the march 34.7k).
// Double storage on lattices that sit in the last-level cache keeps the
// 62-column kernel (1000 x 1000 droplet: 29.5k against 27.3k) or the tile
// kernel (the annulus: 24.5k against 21.8k).
bool strip_width_ok(const lbm_lattice* h) {
  return h->cfg.nx % 64 == 0 || h->cfg.precision == LBM_FP32_DEV || streams_from_hbm(&h->cfg);
}

// Lattices with a solid mask or moving walls (whose population arrays fit
// 32-bit byte offsets) take the masked strip march unless the tile kernel was
// asked for (lbm_set_masked_strips).
bool masked_march(const lbm_lattice* h) {
  double bytes = (double)state_bytes_of(&h->cfg);
  return h->cfg.kernel == LBM_KERNEL_FUSED && (h->buf.mask || h->buf.wall_u) && bytes < 4294967040.0 &&
         h->masked_strips && strip_width_ok(h);
}

// Whether the fused step marches 64-column strips.
bool aligned_march(const lbm_lattice* h) { return masked_march(h) || (fast_path(h) && strip_width_ok(h)); }

void begin_stepping(lbm_lattice* h) {
  if (h->static_ws) h->links_ok = false;
}

bool replay_writes_traj(const lbm_lattice* h) {
  // the aligned strip kernel, with 32-bit byte offsets into the trajectory
  return fast_path(h) && strip_width_ok(h) &&
         32.0 * (double)h->cfg.nx * (double)h->cfg.ny < 4294967040.0;
}

hipError_t step_between(lbm_lattice* h, const void* f_in, void* f_out, int reduce, double* traj) {
  pplbm::StepLaunch L;
  L.f_in = f_in;
  L.f_out = f_out;
  L.mask = h->buf.mask;
  L.wall_u = h->buf.wall_u;
  L.psi = h->psi;
  L.partials = h->partials;
  L.kernel = h->cfg.kernel;
  L.seg_len = h->seg_len;
  L.reduce = reduce;
  L.fast = fast_path(h) ? 1 : 0;
  L.traj = traj;
  L.interleave = (h->cfg.precision == LBM_FP32_DEV && streams_from_hbm(&h->cfg)) ? 1 : 0;
  L.masked = masked_march(h) ? 1 : 0;
  L.aligned = (!L.masked && aligned_march(h)) ? 1 : 0;
  // lattices that stream from HBM: the waves of a block march in lockstep
  L.lockstep = streams_from_hbm(&h->cfg) ? 1 : 0;
  L.links = h->links;
  L.tile_list = h->tile_list;
  L.tile_count = h->tile_count;
  L.moving_partials = h->moving_partials;
  if (L.masked && !h->links_ok) {
    hipError_t e = pplbm::launch_links(h->prm, h->buf.mask, h->buf.wall_u ? 1 : 0, h->links, h->tile_flags,
                                       h->tile_list, h->tile_count, h->stream);
    if (e != hipSuccess) return e;
    h->links_ok = true;
  }
  return (h->cfg.precision == LBM_FP64) ? pplbm::launch_step<double>(h->prm, L, h->stream)
                                        : pplbm::launch_step<float>(h->prm, L, h->stream);
}

int n_parts_of(const lbm_lattice* h) {
  const int nx = h->cfg.nx, ny = h->cfg.ny;
  if (h->cfg.kernel == LBM_KERNEL_TWO_PASS) return pplbm::two_pass_blocks(nx, ny);
  // the fused kernels, as launch_step picks them
  const bool fast = fast_path(h);
  if (aligned_march(h) || (fast && h->cfg.precision == LBM_FP64)) {
    int n_strips, n_segs;
    pplbm::fused_shape(nx, ny, h->seg_len, aligned_march(h), &n_strips, &n_segs);
    return n_strips * n_segs;
  }
  return pplbm::tile_blocks(nx, ny);
}

void* state_ptr(lbm_lattice* h, int which) { return which == 0 ? h->buf.f_a : h->buf.f_b; }

std::string g_create_error;

int fail_query(int code, const std::string& msg) {
  g_create_error = msg;
  return code;
}

bool config_ok(const lbm_config* c, std::string& why) {
  if (!c) {
    why = "config is NULL";
    return false;
  }
  if (c->nx < 1 || c->ny < 1) {
    why = "nx and ny must be >= 1";
    return false;
  }
  if (9.0 * (double)c->nx * (double)c->ny >= 2147483647.0) {
    why = "9*nx*ny must be < 2^31";
    return false;
  }
  if (c->precision != LBM_FP64 && c->precision != LBM_FP32_DEV) {
    why = "unknown precision";
    return false;
  }
  if (c->kernel != LBM_KERNEL_FUSED && c->kernel != LBM_KERNEL_TWO_PASS) {
    why = "unknown kernel";
    return false;
  }
  if (!std::isfinite(c->rho_ref)) {
    why = "rho_ref must be finite";
    return false;
  }
  if (c->log_capacity < 1 || c->log_capacity > (1 << 24)) {
    why = "log_capacity must be in [1, 2^24]";
    return false;
  }
  return true;
}

constexpr int kMinSegLen = 1;

// Float storage re-references every node to its current density every this
// many steps by default.  Without it the references of a moving interface go
// stale and the rounding of the (then large) stored deviations accumulates:
// on the 2048 x 16384 falling droplet, FP32 against FP64 after 100,000 steps
// (max-norm, density relative / velocity of the peak): never 3.6e-3 / 3.4e-3;
// every 1,000 steps 2.2e-5 / 4.3e-5; every 100 steps 4.1e-5 / 4.1e-5.  One
// re-reference costs about two steps' worth of memory traffic.
constexpr int64_t kDefaultRerefEvery = 1000;

// Rows each wavefront marches: the longest of 24, 16, 14, 12, 8, 6 rows that
// still gives the launch enough wavefronts to fill the chip (2,560 for float
// storage, which fits 3 per SIMD, 1,024 for double).  A run recomputes the
// pseudopotential of the two rows beside it, so longer runs read and compute
// less; but a run keeps only a few rows of loads in flight, so the chip needs
// many runs at once.  Lattices whose two population arrays exceed the 256 MB
// last-level cache stream from HBM, and there short runs are faster: the
// waves resident at one time then read fewer, fuller DRAM rows.  Those take
// at most 14 rows (float) or 8 (double).  Measured on gfx950 (MLUPS):
// 2048 x 16384, float: 8 rows 63.2k, 12 64.3k, 16 63.9k, 24 61.8k, 32 62.0k;
// double: 4 rows 34.3k, 8 35.6k, 16 34.9k, 24 34.0k.  512 x 2048 (cache
// resident), float: 8 rows 48.5k, 16 rows 42.2k; double: 16 rows 35.2k, 8
// rows 33.4k.  With the waves of a block in lockstep (lattices that stream
// from HBM), 2048 x 16384, ms per step, float: 12 rows 0.504, 14 0.502, 16
// 0.503, 20 0.504; double: 8 rows 0.914, 10 0.918, 16 0.935.  Lattices too
// small to fill the chip with 6-row runs take
// shorter ones, down to one row per wavefront (which pulls 3 rows for the 1
// it stores): the 256 x 256 masked oblique channel, float storage, 11.4 us
// per step at 4 rows, 9.9 at 3, 8.5 at 2, 6.9 at 1.
int default_seg_len(const lbm_lattice* h) {
  const int nx = h->cfg.nx, ny = std::max(h->cfg.ny, 1);
  int n_strips, n_segs;
  const bool aligned = aligned_march(h);
  const bool fp64 = h->cfg.precision == LBM_FP64;
  const long target = fp64 ? 1024 : 2560;
  const int cap = streams_from_hbm(&h->cfg) ? (fp64 ? 8 : 14) : 24;
  for (int rows : {24, 16, 14, 12, 8, 6, 4, 3, 2}) {
    if (rows > cap) continue;
    pplbm::fused_shape(nx, ny, rows, aligned, &n_strips, &n_segs);
    if ((long)n_strips * n_segs >= target) return std::min(rows, ny);
  }
  return std::min(kMinSegLen, ny);
}

size_t max_parts_for(const lbm_config* c) {
  int n_strips, n_segs;
  pplbm::fused_shape(c->nx, c->ny, kMinSegLen, false, &n_strips, &n_segs);  // the larger count
  size_t fused = (size_t)n_strips * n_segs;
  size_t two = (size_t)pplbm::two_pass_blocks(c->nx, c->ny);
  size_t tiles = (size_t)pplbm::tile_blocks(c->nx, c->ny);
  return std::max(fused, std::max(two, tiles));
}

struct Layout {
  size_t partials, log, red_tmp, fin_tmp, psi, links, tiles, moving_partials, total;
};

Layout layout_for(const lbm_config* c) {
  Layout L;
  size_t off = 0;
  L.partials = off;
  off = align256(off + max_parts_for(c) * RED_COUNT * sizeof(double));
  L.log = off;
  off = align256(off + (size_t)c->log_capacity * RED_COUNT * sizeof(double));
  L.red_tmp = off;
  off = align256(off + RED_COUNT * sizeof(double));
  L.fin_tmp = off;
  off = align256(off + (size_t)pplbm::kFinalizeBlocks * RED_COUNT * sizeof(double));
  L.psi = off;
  off = align256(off + (size_t)c->nx * c->ny * sizeof(double));
  L.links = off;
  off = align256(off + (size_t)c->nx * c->ny * sizeof(uint16_t));
  // tile flags, tile list, count (masked lattices with moving walls)
  const size_t n_tiles = (size_t)pplbm::tile_blocks(c->nx, c->ny);
  L.tiles = off;
  off = align256(off + (2 * n_tiles + 1) * sizeof(int));
  L.moving_partials = off;
  off = align256(off + n_tiles * RED_COUNT * sizeof(double));
  L.total = off;
  return L;
}

void rebuild_params(lbm_lattice* h) {
  h->adj.ready = false;
  StepParams& p = h->prm;
  for (int k = 0; k < 9; ++k) {
    p.s[k] = h->s[k];
    p.h[k] = 1.0 - 0.5 * h->s[k];
  }
  double k1 = std::isnan(h->k1) ? -h->eps / 16.0 : h->k1;
  double k2 = std::isnan(h->k2) ? -h->eps / 16.0 : h->k2;
  p.q1 = 3.0 * (k1 + 2.0 * k2);
  int q2 = h->q2_policy;
  if (q2 == LBM_Q2_DEFAULT) q2 = (h->scheme == LBM_SCHEME_IMPROVED) ? LBM_Q2_NEG_HALF_Q1 : LBM_Q2_NEG_Q1;
  p.q2 = (q2 == LBM_Q2_NEG_Q1) ? -1.0 : -0.5;
  p.q7 = k1;
  if (h->scheme == LBM_SCHEME_IMPROVED) {
    p.qa = (30.0 * h->eps - 15.0) / 16.0;
    p.qb = 3.0 * h->eps / 8.0;
  } else {
    p.qa = 0.0;
    p.qb = 0.0;
  }
  double q = pplbm::psi_squared(p, h->rho_s);
  p.psi_solid = std::sqrt(q > 0.0 ? q : 0.0);
  p.gmag = std::sqrt(p.fx * p.fx + p.fy * p.fy);
  p.ghx = p.gmag > 0 ? p.fx / p.gmag : 0.0;
  p.ghy = p.gmag > 0 ? p.fy / p.gmag : 0.0;
}

bool all_finite(std::initializer_list<double> v) {
  for (double d : v)
    if (!std::isfinite(d)) return false;
  return true;
}



void fill_record(const double* v, int64_t step, lbm_reduction* r) {
  r->mass = v[pplbm::RED_MASS];
  r->mom_x = v[pplbm::RED_MOMX];
  r->mom_y = v[pplbm::RED_MOMY];
  r->wall_x = v[pplbm::RED_WALLX];
  r->wall_y = v[pplbm::RED_WALLY];
  r->uc_num = v[pplbm::RED_UC_NUM];
  r->uc_den = v[pplbm::RED_UC_DEN];
  r->buoy = v[pplbm::RED_BUOY];
  r->pphi = v[pplbm::RED_PPHI];
  r->faults = v[pplbm::RED_FAULTS];
  r->step = step;
}

int fault_status(lbm_lattice* h, const lbm_reduction& r) {
  if (r.faults > 0.0) {
    char msg[160];
    std::snprintf(msg, sizeof msg, "step %lld: %.0f node(s) with rho <= 0, negative psi^2 or non-finite values",
                  (long long)r.step, r.faults);
    return fail(h, std::isfinite(r.mass) ? LBM_ERR_EOS_DOMAIN : LBM_ERR_NONFINITE, msg);
  }
  return LBM_OK;
}

}  // namespace pplbm_host

using namespace pplbm_host;

extern "C" {

int lbm_abi_version(void) { return LBM_ABI_VERSION; }

int lbm_state_bytes(const lbm_config* cfg, size_t* bytes) {
  g_create_error.clear();
  std::string why;
  if (!bytes) return fail_query(LBM_ERR_INVALID_ARG, "bytes is NULL");
  if (!config_ok(cfg, why)) return fail_query(LBM_ERR_INVALID_ARG, why);
  *bytes = state_bytes_of(cfg);
  return LBM_OK;
}

int lbm_workspace_bytes(const lbm_config* cfg, size_t* bytes) {
  g_create_error.clear();
  std::string why;
  if (!bytes) return fail_query(LBM_ERR_INVALID_ARG, "bytes is NULL");
  if (!config_ok(cfg, why)) return fail_query(LBM_ERR_INVALID_ARG, why);
  *bytes = layout_for(cfg).total;
  return LBM_OK;
}

int lbm_create_static(const lbm_config* cfg, const lbm_buffers* buf, void* hip_stream, lbm_lattice** out) {
  g_create_error.clear();
  if (!out) {
    g_create_error = "out is NULL";
    return LBM_ERR_INVALID_ARG;
  }
  *out = nullptr;
  std::string why;
  if (!config_ok(cfg, why)) {
    g_create_error = why;
    return LBM_ERR_INVALID_ARG;
  }
  if (!buf || buf->workspace) {
    g_create_error = "buf must be non-NULL with workspace NULL (the library's static workspace is used)";
    return LBM_ERR_INVALID_ARG;
  }
  const size_t need = layout_for(cfg).total;
  if (need > pplbm::kStaticWorkspaceBytes) {
    g_create_error = "the lattice needs a " + std::to_string(need) + "-byte workspace; the static workspace holds " +
                     std::to_string(pplbm::kStaticWorkspaceBytes) + " bytes (use lbm_create with a caller buffer)";
    return LBM_ERR_INVALID_ARG;
  }
  void* ws = nullptr;
  hipError_t e = pplbm::static_workspace(&ws);
  if (e != hipSuccess) {
    g_create_error = std::string("static workspace: ") + hipGetErrorString(e);
    return LBM_ERR_HIP;
  }
  lbm_buffers b = *buf;
  b.workspace = ws;
  const int rc = lbm_create(cfg, &b, hip_stream, out);
  if (rc == LBM_OK) (*out)->static_ws = true;
  return rc;
}

int lbm_create(const lbm_config* cfg, const lbm_buffers* buf, void* hip_stream, lbm_lattice** out) {
  g_create_error.clear();
  if (!out) {
    g_create_error = "out is NULL";
    return LBM_ERR_INVALID_ARG;
  }
  *out = nullptr;
  std::string why;
  if (!config_ok(cfg, why)) {
    g_create_error = why;
    return LBM_ERR_INVALID_ARG;
  }
  if (!buf || !buf->f_a || !buf->f_b || !buf->workspace || buf->f_a == buf->f_b) {
    g_create_error = "f_a, f_b and workspace must be distinct non-NULL device pointers";
    return LBM_ERR_INVALID_ARG;
  }
  if (((uintptr_t)buf->workspace & 255u) != 0) {
    g_create_error = "workspace must be 256-byte aligned";
    return LBM_ERR_INVALID_ARG;
  }
  lbm_lattice* h = new (std::nothrow) lbm_lattice();
  if (!h) {
    g_create_error = "out of host memory";
    return LBM_ERR_INVALID_ARG;
  }
  h->cfg = *cfg;
  h->buf = *buf;
  h->stream = (hipStream_t)hip_stream;
  std::memset(&h->prm, 0, sizeof(h->prm));
  h->prm.nx = cfg->nx;
  h->prm.ny = cfg->ny;
  h->prm.periodic_x = cfg->periodic_x ? 1 : 0;
  h->prm.periodic_y = cfg->periodic_y ? 1 : 0;
  h->prm.rho_ref = (cfg->precision == LBM_FP32_DEV) ? cfg->rho_ref : 0.0;
  // defaults: Carnahan-Starling a = 1, b = 4, R = 1, T = 0.7 T_c
  h->prm.eos_kind = LBM_EOS_CS;
  h->prm.a = 1.0;
  h->prm.b = 4.0;
  h->prm.RT = 0.7 * 0.3773 / 4.0;
  h->prm.k_eos = 1.0;
  h->prm.G = -1.0;
  h->prm.force_mode = LBM_FORCE_CONST;
  h->prm.rho_g = 0.0;
  h->prm.rho_l = 1.0;
  for (int k = 0; k < 9; ++k) h->s[k] = 1.0;
  h->scheme = LBM_SCHEME_IMPROVED;
  h->eps = 0.0;
  h->k1 = NAN;
  h->k2 = NAN;
  h->q2_policy = LBM_Q2_DEFAULT;
  h->rho_s = 0.0;
  h->seg_len = default_seg_len(h);
  h->reref_every = cfg->precision == LBM_FP32_DEV ? kDefaultRerefEvery : 0;
  Layout L = layout_for(cfg);
  char* ws = (char*)buf->workspace;
  h->partials = (double*)(ws + L.partials);
  h->max_parts = max_parts_for(cfg);
  h->log = (double*)(ws + L.log);
  h->red_tmp = (double*)(ws + L.red_tmp);
  h->fin_tmp = (double*)(ws + L.fin_tmp);
  h->psi = (void*)(ws + L.psi);
  h->links = (uint16_t*)(ws + L.links);
  {
    const size_t n_tiles = (size_t)pplbm::tile_blocks(cfg->nx, cfg->ny);
    h->tile_flags = (unsigned*)(ws + L.tiles);
    h->tile_list = (int*)(ws + L.tiles) + n_tiles;
    h->tile_count = (int*)(ws + L.tiles) + 2 * n_tiles;
  }
  h->moving_partials = (double*)(ws + L.moving_partials);
  rebuild_params(h);
  *out = h;
  return LBM_OK;
}

int lbm_destroy(lbm_lattice* h) {
  delete h;
  return LBM_OK;
}

const char* lbm_last_error(const lbm_lattice* h) { return h ? h->err.c_str() : g_create_error.c_str(); }

int lbm_set_eos(lbm_lattice* h, int32_t kind, double a, double b, double R, double T, double k_eos) {
  if (!h) return LBM_ERR_INVALID_ARG;
  if (kind != LBM_EOS_VDW && kind != LBM_EOS_CS) return fail(h, LBM_ERR_INVALID_ARG, "unknown EOS kind");
  if (!all_finite({a, b, R, T, k_eos}) || b <= 0 || R <= 0 || T <= 0 || k_eos <= 0 || a < 0)
    return fail(h, LBM_ERR_INVALID_ARG, "EOS constants must be finite, b, R, T, k_eos > 0, a >= 0");
  h->prm.eos_kind = kind;
  h->prm.a = a;
  h->prm.b = b;
  h->prm.RT = R * T;
  h->prm.k_eos = k_eos;
  rebuild_params(h);
  return LBM_OK;
}

int lbm_set_G(lbm_lattice* h, double G) {
  if (!h) return LBM_ERR_INVALID_ARG;
  if (!std::isfinite(G) || G == 0.0) return fail(h, LBM_ERR_INVALID_ARG, "G must be finite and non-zero");
  h->prm.G = G;
  rebuild_params(h);
  return LBM_OK;
}

int lbm_set_relaxation(lbm_lattice* h, const double* s) {
  if (!h) return LBM_ERR_INVALID_ARG;
  if (!s) return fail(h, LBM_ERR_INVALID_ARG, "rates pointer is NULL");
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(s[k]) || s[k] < 0.0 || s[k] > 2.0)
      return fail(h, LBM_ERR_INVALID_ARG, "every rate must be in [0, 2]");
  for (int k = 0; k < 9; ++k) h->s[k] = s[k];
  rebuild_params(h);
  return LBM_OK;
}

int lbm_set_scheme(lbm_lattice* h, int32_t scheme, double eps, double k1, double k2, int32_t q2_policy) {
  if (!h) return LBM_ERR_INVALID_ARG;
  if (scheme != LBM_SCHEME_ORIGINAL && scheme != LBM_SCHEME_IMPROVED)
    return fail(h, LBM_ERR_INVALID_ARG, "unknown scheme");
  if (q2_policy < LBM_Q2_DEFAULT || q2_policy > LBM_Q2_NEG_HALF_Q1)
    return fail(h, LBM_ERR_INVALID_ARG, "unknown q2 policy");
  if (!std::isfinite(eps) || (!std::isnan(k1) && !std::isfinite(k1)) || (!std::isnan(k2) && !std::isfinite(k2)))
    return fail(h, LBM_ERR_INVALID_ARG, "eps, k1, k2 must be finite (k1, k2 may be NaN)");
  h->scheme = scheme;
  h->eps = eps;
  h->k1 = k1;
  h->k2 = k2;
  h->q2_policy = q2_policy;
  rebuild_params(h);
  return LBM_OK;
}

int lbm_set_body_force(lbm_lattice* h, int32_t mode, double fx, double fy) {
  if (!h) return LBM_ERR_INVALID_ARG;
  if (mode != LBM_FORCE_CONST && mode != LBM_FORCE_BUOYANT) return fail(h, LBM_ERR_INVALID_ARG, "unknown force mode");
  if (!all_finite({fx, fy})) return fail(h, LBM_ERR_INVALID_ARG, "force must be finite");
  h->prm.force_mode = mode;
  h->prm.fx = fx;
  h->prm.fy = fy;
  rebuild_params(h);
  return LBM_OK;
}

int lbm_set_phase_densities(lbm_lattice* h, double rho_g, double rho_l) {
  if (!h) return LBM_ERR_INVALID_ARG;
  if (!all_finite({rho_g, rho_l}) || !(rho_g > 0.0) || !(rho_l > rho_g))
    return fail(h, LBM_ERR_INVALID_ARG, "need 0 < rho_g < rho_l");
  h->prm.rho_g = rho_g;
  h->prm.rho_l = rho_l;
  rebuild_params(h);
  return LBM_OK;
}

int lbm_set_walls(lbm_lattice* h, double rho_s) {
  if (!h) return LBM_ERR_INVALID_ARG;
  if (!std::isfinite(rho_s) || rho_s < 0.0) return fail(h, LBM_ERR_INVALID_ARG, "rho_s must be finite and >= 0");
  h->rho_s = rho_s;
  rebuild_params(h);
  return LBM_OK;
}

int lbm_init_equilibrium(lbm_lattice* h, const double* rho0, const double* ux0, const double* uy0) {
  if (!h) return LBM_ERR_INVALID_ARG;
  if (!rho0) return fail(h, LBM_ERR_INVALID_ARG, "rho0 is NULL");
  hipError_t e = (h->cfg.precision == LBM_FP64)
                     ? pplbm::launch_init<double>(h->prm, rho0, ux0, uy0, h->buf.mask, h->buf.f_a, h->buf.f_b,
                                                  h->stream)
                     : pplbm::launch_init<float>(h->prm, rho0, ux0, uy0, h->buf.mask, h->buf.f_a, h->buf.f_b,
                                                 h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "init launch");
  h->cur = 0;
  h->steps = 0;
  h->initialized = true;
  return LBM_OK;
}

int lbm_step(lbm_lattice* h, int64_t n, int32_t reduce_every, lbm_reduction* out, int64_t n_out) {
  if (!h) return LBM_ERR_INVALID_ARG;
  if (!h->initialized) return fail(h, LBM_ERR_STATE, "lbm_step before lbm_init_equilibrium / lbm_set_state");
  if (n < 0 || reduce_every < 0 || n_out < 0) return fail(h, LBM_ERR_INVALID_ARG, "negative count");
  int64_t records = 0;
  if (reduce_every > 0) records = (h->steps + n) / reduce_every - h->steps / reduce_every;
  if (records > h->cfg.log_capacity)
    return fail(h, LBM_ERR_INVALID_ARG, "more reduction records than log_capacity in one call");
  std::vector<int64_t> rec_steps;
  rec_steps.reserve((size_t)records);
  begin_stepping(h);
  const int parts = n_parts_of(h);
  for (int64_t t = 0; t < n; ++t) {
    int64_t idx = h->steps + 1;
    int reduce = (reduce_every > 0 && idx % reduce_every == 0) ? 1 : 0;
    hipError_t e = step_between(h, state_ptr(h, h->cur), state_ptr(h, 1 - h->cur), reduce);
    if (e != hipSuccess) return hip_fail(h, e, "step launch");
    if (reduce) {
      const bool mv = masked_march(h) && h->buf.wall_u;
      e = pplbm::launch_finalize(h->partials, parts, h->log + rec_steps.size() * RED_COUNT, h->fin_tmp, h->stream,
                                 mv ? h->moving_partials : nullptr, mv ? h->tile_count : nullptr);
      if (e != hipSuccess) return hip_fail(h, e, "reduction launch");
      rec_steps.push_back(idx);
    }
    h->cur = 1 - h->cur;
    h->steps = idx;
    if (h->cfg.precision == LBM_FP32_DEV && h->reref_every > 0 && idx % h->reref_every == 0) {
      e = pplbm::launch_reref(h->prm, state_ptr(h, h->cur), state_ptr(h, 1 - h->cur), h->buf.mask, h->stream);
      if (e != hipSuccess) return hip_fail(h, e, "rereference launch");
    }
  }
  if (out && !rec_steps.empty() && n_out > 0) {
    size_t ncopy = (size_t)std::min<int64_t>(n_out, (int64_t)rec_steps.size());
    std::vector<double> host(ncopy * RED_COUNT);
    hipError_t e = hipMemcpyAsync(host.data(), h->log, host.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "reduction copy");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "stream synchronize");
    int status = LBM_OK;
    for (size_t r = 0; r < ncopy; ++r) {
      fill_record(&host[r * RED_COUNT], rec_steps[r], &out[r]);
      if (status == LBM_OK) status = fault_status(h, out[r]);
    }
    return status;
  }
  return LBM_OK;
}

int lbm_set_rows_per_wave(lbm_lattice* h, int32_t rows) {
  if (!h) return LBM_ERR_INVALID_ARG;
  if (rows == 0) {
    h->seg_len = default_seg_len(h);
    return LBM_OK;
  }
  if (rows < kMinSegLen || rows > 4096) return fail(h, LBM_ERR_INVALID_ARG, "rows per wave must be in [1, 4096]");
  h->seg_len = rows;
  return LBM_OK;
}

int lbm_set_masked_strips(lbm_lattice* h, int32_t on) {
  if (!h) return LBM_ERR_INVALID_ARG;
  if (on != 0 && on != 1) return fail(h, LBM_ERR_INVALID_ARG, "masked strips: 0 or 1");
  h->masked_strips = on;
  h->seg_len = default_seg_len(h);
  return LBM_OK;
}

int lbm_set_rereference_every(lbm_lattice* h, int64_t k) {
  if (!h) return LBM_ERR_INVALID_ARG;
  if (k < 0) return fail(h, LBM_ERR_INVALID_ARG, "rereference interval must be >= 0");
  h->reref_every = k;
  return LBM_OK;
}

int lbm_step_count(const lbm_lattice* h, int64_t* steps) {
  if (!h || !steps) return LBM_ERR_INVALID_ARG;
  *steps = h->steps;
  return LBM_OK;
}

int lbm_read_fields(lbm_lattice* h, double* rho, double* ux, double* uy, double* fx, double* fy, double* psi) {
  if (!h) return LBM_ERR_INVALID_ARG;
  if (!h->initialized) return fail(h, LBM_ERR_STATE, "read before init");
  const void* f = state_ptr(h, h->cur);
  hipError_t e = (h->cfg.precision == LBM_FP64)
                     ? pplbm::launch_fields<double>(h->prm, f, h->buf.mask, h->buf.wall_u, h->psi, rho, ux, uy, fx,
                                                    fy, psi, h->partials, 0, h->stream)
                     : pplbm::launch_fields<float>(h->prm, f, h->buf.mask, h->buf.wall_u, h->psi, rho, ux, uy, fx, fy,
                                                   psi, h->partials, 0, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "fields launch");
  return LBM_OK;
}

int lbm_reduce(lbm_lattice* h, lbm_reduction* out) {
  if (!h || !out) return LBM_ERR_INVALID_ARG;
  if (!h->initialized) return fail(h, LBM_ERR_STATE, "reduce before init");
  const void* f = state_ptr(h, h->cur);
  hipError_t e = (h->cfg.precision == LBM_FP64)
                     ? pplbm::launch_fields<double>(h->prm, f, h->buf.mask, h->buf.wall_u, h->psi, nullptr, nullptr,
                                                    nullptr, nullptr, nullptr, nullptr, h->partials, 1, h->stream)
                     : pplbm::launch_fields<float>(h->prm, f, h->buf.mask, h->buf.wall_u, h->psi, nullptr, nullptr,
                                                   nullptr, nullptr, nullptr, nullptr, h->partials, 1, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "fields launch");
  e = pplbm::launch_finalize(h->partials, pplbm::two_pass_blocks(h->cfg.nx, h->cfg.ny), h->red_tmp, h->fin_tmp,
                             h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "reduction launch");
  double host[RED_COUNT];
  e = hipMemcpyAsync(host, h->red_tmp, sizeof host, hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "reduction copy");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "stream synchronize");
  fill_record(host, h->steps + 1, out);
  return fault_status(h, *out);
}

int lbm_rereference(lbm_lattice* h) {
  if (!h) return LBM_ERR_INVALID_ARG;
  if (!h->initialized) return fail(h, LBM_ERR_STATE, "rereference before init");
  if (h->cfg.precision != LBM_FP32_DEV) return LBM_OK;
  h->adj.ready = false;
  hipError_t e = pplbm::launch_reref(h->prm, state_ptr(h, h->cur), state_ptr(h, 1 - h->cur), h->buf.mask, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "rereference launch");
  return LBM_OK;
}

int lbm_state_ptr(const lbm_lattice* h, void** f) {
  if (!h || !f) return LBM_ERR_INVALID_ARG;
  *f = h->cur == 0 ? h->buf.f_a : h->buf.f_b;
  return LBM_OK;
}

int lbm_get_state(lbm_lattice* h, void* dst) {
  if (!h || !dst) return LBM_ERR_INVALID_ARG;
  if (!h->initialized) return fail(h, LBM_ERR_STATE, "get_state before init");
  size_t bytes = state_bytes_of(&h->cfg);
  hipError_t e = hipMemcpyAsync(dst, state_ptr(h, h->cur), bytes, hipMemcpyDeviceToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "state copy");
  return LBM_OK;
}

int lbm_set_state(lbm_lattice* h, const void* src, int64_t step) {
  if (!h || !src || step < 0) return LBM_ERR_INVALID_ARG;
  size_t bytes = state_bytes_of(&h->cfg);
  hipError_t e = hipMemcpyAsync(h->buf.f_a, src, bytes, hipMemcpyDeviceToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "state copy");
  e = hipMemcpyAsync(h->buf.f_b, src, bytes, hipMemcpyDeviceToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "state copy");
  h->cur = 0;
  h->steps = step;
  h->initialized = true;
  return LBM_OK;
}

}  // extern "C"
