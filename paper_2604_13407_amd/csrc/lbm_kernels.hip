// HIP kernels of one pseudopotential MRT step for gfx950 (CDNA4, wave64).
//
// Step implementations, all on the node arithmetic of lbm_node.h:
//  * the aligned strip march: a wavefront owns 64 aligned columns (the last
//    strip of a width that is not a multiple of 64 fewer) and marches up a
//    run of rows; each row
//    is pulled once, its density and pseudopotential are computed in
//    registers, the x-neighbours' psi comes through DPP lane shifts and the
//    y-neighbours' from the rows kept in registers, and the middle row is
//    collided and stored as whole aligned lines.  Masked lattices (solid
//    nodes, moving walls) take the same march with bounce-back chosen per link
//    from a 16-bit link word per node; the nodes beside moving walls are
//    stepped first by the tile kernel, on the tiles that hold them only;
//  * the 62-column strip march (double storage, widths that are not a
//    multiple of 64, on lattices that sit in the last-level cache);
//  * the tile kernel (every other lattice): one node per thread, psi of a
//    32 x 8 tile and its one-node ring in LDS;
//  * the two-pass kernels: a psi pass writes the pseudopotential field, then
//    a collide pass pulls again, reads psi of the 8 neighbours and collides.
//    Simple, one node per thread; the reference for the fused kernels.
// Reductions (every reduce_every steps) are FP64 per-wave or per-block partial
// sums finished by a fixed-order kernel, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lbm_internal.h"
#include "lbm_node.h"

namespace pplbm {

constexpr int WAVE = 64;
constexpr int STRIP = WAVE - 2;  // interior columns per wavefront

template <class T>
__device__ inline T shfl_up1(T v) {
  return __shfl_up(v, 1, WAVE);
}
template <class T>
__device__ inline T shfl_down1(T v) {
  return __shfl_down(v, 1, WAVE);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// ------------------------------------------------------------------ init
template <class S>
__global__ void init_kernel(StepParams p, const double* __restrict__ rho0, const double* __restrict__ ux0,
                            const double* __restrict__ uy0, const uint8_t* __restrict__ mask, S* __restrict__ fa,
                            S* __restrict__ fb) {
  int x = blockIdx.x * blockDim.x + threadIdx.x;
  int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= p.nx || y >= p.ny) return;
  size_t k = (size_t)y * p.nx + x;
  double r = rho0[k];
  double u = ux0 ? ux0[k] : 0.0;
  double v = uy0 ? uy0[k] : 0.0;
  double usq = u * u + v * v;
  // float storage: every node's reference offset is c = rhat - rho_ref with
  // rhat its initial density (as a 16-bit float); population i is stored
  // relative to the offset of the node that pulls it (x + e_i, or x across a
  // wall)
  double cd[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) cd[i] = 0.0;
  if constexpr (sizeof(S) == 4) {
    const RefT cf = (RefT)(r - p.rho_ref);
    const size_t rk = ref_at(p.nx, y, x);
    ref_base(fa)[rk] = cf;
    ref_base(fb)[rk] = cf;
    // the run's unused second half is zero, so the whole state is defined
    ref_base(fa)[rk + p.nx] = (RefT)0;
    ref_base(fb)[rk + p.nx] = (RefT)0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      int xd, yd;
      bool inside;
      const bool sol = solid_at(p, mask, x + ex(i), y + ey(i), xd, yd, inside);
      cd[i] = (double)(sol ? cf : (RefT)(rho0[(size_t)yd * p.nx + xd] - p.rho_ref));
    }
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    double eu = ex(i) * u + ey(i) * v;
    // f_eq - w (rho_ref + c) = w [(rho - rho_ref - c) + rho (3 e.u + 9/2 (e.u)^2 - 3/2 u^2)]
    double dv = wgt(i) * ((r - p.rho_ref - cd[i]) + r * (3.0 * eu + 4.5 * eu * eu - 1.5 * usq));
    fa[pop_at<S>(p.nx, y, i, x)] = (S)dv;
    fb[pop_at<S>(p.nx, y, i, x)] = (S)dv;
  }
}

// Re-reference (float storage), three passes over the current array `fa`:
// the new offset of every fluid node (the density of its current
// post-collision populations) goes to the reference offsets of `fb`; then
// every stored population moves from its puller's old offset to the new one,
// in both arrays; then the new offsets are copied into `fa`.  The state is
// unchanged up to one rounding per population.
__global__ void reref_new_kernel(StepParams p, const float* __restrict__ fa, float* __restrict__ fb,
                                 const uint8_t* mask) {
  int x = blockIdx.x * blockDim.x + threadIdx.x;
  int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= p.nx || y >= p.ny) return;
  const size_t k = (size_t)y * p.nx + x;
  const size_t rk = ref_at(p.nx, y, x);
  if (mask && mask[k]) {
    ref_base(fb)[rk] = ref_base(fa)[rk];
    return;
  }
  double cd[9];
  dest_refs<float>(p, fa, mask, x, y, cd);
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) s += (double)fa[pop_at<float>(p.nx, y, i, x)] + wgt(i) * cd[i];
  ref_base(fb)[rk] = (RefT)s;
}

__global__ void reref_shift_kernel(StepParams p, float* __restrict__ fa, float* __restrict__ fb, const uint8_t* mask) {
  int x = blockIdx.x * blockDim.x + threadIdx.x;
  int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= p.nx || y >= p.ny) return;
  const size_t k = (size_t)y * p.nx + x;
  if (mask && mask[k]) return;
  double co[9], cn[9];
  dest_refs<float>(p, fa, mask, x, y, co);
  dest_refs<float>(p, fb, mask, x, y, cn);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const size_t e = pop_at<float>(p.nx, y, i, x);
    const float v = (float)((double)fa[e] + wgt(i) * (co[i] - cn[i]));
    fa[e] = v;
    fb[e] = v;
  }
}

__global__ void reref_copy_kernel(StepParams p, float* __restrict__ fa, const float* __restrict__ fb) {
  int x = blockIdx.x * blockDim.x + threadIdx.x;
  int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= p.nx || y >= p.ny) return;
  const size_t rk = ref_at(p.nx, y, x);
  ref_base(fa)[rk] = ref_base(fb)[rk];
}

// ------------------------------------------------------------------ two-pass: psi
template <class S>
__global__ void psi_kernel(StepParams p, const S* __restrict__ f, const uint8_t* __restrict__ mask,
                           const double* __restrict__ wall_u, double* __restrict__ psi_out) {
  int x = blockIdx.x * blockDim.x + threadIdx.x;
  int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= p.nx || y >= p.ny) return;
  size_t k = (size_t)y * p.nx + x;
  if (mask && mask[k]) {
    psi_out[k] = p.psi_solid;
    return;
  }
  double d[9], c;
  pull_node<S>(p, f, mask, wall_u, x, y, d, nullptr, c);
  double drho, jx, jy;
  node_sums<S>(d, c, drho, jx, jy);
  bool bad;
  psi_out[k] = psi_of(p, p.rho_ref + drho, bad);
}

__device__ inline double psi_at(const StepParams& p, const double* __restrict__ psi, const uint8_t* __restrict__ mask,
                                int x, int y) {
  int xw, yw;
  bool inside;
  bool sol = solid_at(p, mask, x, y, xw, yw, inside);
  if (!inside) return p.psi_solid;
  (void)sol;  // a masked solid node already holds psi_solid in the field
  return psi[(size_t)yw * p.nx + xw];
}

// Per-block deterministic reduction of acc[RED_COUNT] -> partials[block].
__device__ inline void block_reduce_store(double* acc, double* __restrict__ partials, int block_id) {
  __shared__ double lds[RED_COUNT][16];
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int lane = tid % WAVE;
  const int wid = tid / WAVE;
  const int nw = (blockDim.x * blockDim.y) / WAVE;
#pragma unroll
  for (int q = 0; q < RED_COUNT; ++q) {
    double v = wave_sum(acc[q]);
    if (lane == 0) lds[q][wid] = v;
  }
  __syncthreads();
  if (tid < RED_COUNT) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += lds[tid][w];
    partials[(size_t)block_id * RED_COUNT + tid] = s;
  }
}

// ------------------------------------------------------------------ two-pass: collide
template <class S, bool REDUCE>
__global__ void collide_kernel(StepParams p, const S* __restrict__ f, S* __restrict__ fo,
                               const uint8_t* __restrict__ mask, const double* __restrict__ wall_u,
                               const double* __restrict__ psi, double* __restrict__ partials) {
  int x = blockIdx.x * blockDim.x + threadIdx.x;
  int y = blockIdx.y * blockDim.y + threadIdx.y;
  double acc[RED_COUNT];
#pragma unroll
  for (int q = 0; q < RED_COUNT; ++q) acc[q] = 0.0;
  bool active = (x < p.nx && y < p.ny);
  size_t k = active ? (size_t)y * p.nx + x : 0;
  if (active && !(mask && mask[k])) {
    double d[9];
    double wall[2] = {0.0, 0.0};
    double c;
    float cd[9];
    pull_node<S>(p, f, mask, wall_u, x, y, d, REDUCE ? wall : nullptr, c, cd);
    double drho, jx, jy;
    node_sums<S>(d, c, drho, jx, jy);
    double Sx, Sy;
    stencil_sums(psi_at(p, psi, mask, x + 1, y), psi_at(p, psi, mask, x, y + 1), psi_at(p, psi, mask, x - 1, y),
                 psi_at(p, psi, mask, x, y - 1), psi_at(p, psi, mask, x + 1, y + 1), psi_at(p, psi, mask, x - 1, y + 1),
                 psi_at(p, psi, mask, x - 1, y - 1), psi_at(p, psi, mask, x + 1, y - 1), Sx, Sy);
    NodeMacro mac = collide_node<S>(p, d, c, drho, jx, jy, psi[k], Sx, Sy);
#pragma unroll
    for (int i = 0; i < 9; ++i)
      fo[pop_at<S>(p.nx, y, i, x)] = store_value<S>(d[i], wgt(i), sizeof(S) == 4 ? (double)cd[i] : 0.0);
    if (REDUCE) {
      bool bad;
      double rho = p.rho_ref + drho;
      psi_of(p, rho, bad);
      acc[RED_WALLX] += wall[0];
      acc[RED_WALLY] += wall[1];
      accumulate_node(p, acc, rho, jx, jy, mac, bad);
    }
  }
  if (REDUCE) block_reduce_store(acc, partials, blockIdx.y * gridDim.x + blockIdx.x);
}

// ------------------------------------------------------------------ read-out
template <class S>
__global__ void fields_kernel(StepParams p, const S* __restrict__ f, const uint8_t* __restrict__ mask,
                              const double* __restrict__ wall_u, const double* __restrict__ psi, double* rho_o,
                              double* ux_o, double* uy_o, double* fx_o, double* fy_o, double* psi_o,
                              double* __restrict__ partials, int reduce) {
  int x = blockIdx.x * blockDim.x + threadIdx.x;
  int y = blockIdx.y * blockDim.y + threadIdx.y;
  double acc[RED_COUNT];
#pragma unroll
  for (int q = 0; q < RED_COUNT; ++q) acc[q] = 0.0;
  bool active = (x < p.nx && y < p.ny);
  if (active) {
    size_t k = (size_t)y * p.nx + x;
    double r = 0.0, u = 0.0, v = 0.0, fxi = 0.0, fyi = 0.0;
    double ps = psi[k];
    if (!(mask && mask[k])) {
      double d[9];
      double wall[2] = {0.0, 0.0};
      double c;
      pull_node<S>(p, f, mask, wall_u, x, y, d, reduce ? wall : nullptr, c);
      double drho, jx, jy;
      node_sums<S>(d, c, drho, jx, jy);
      r = p.rho_ref + drho;
      double Sx, Sy;
      stencil_sums(psi_at(p, psi, mask, x + 1, y), psi_at(p, psi, mask, x, y + 1), psi_at(p, psi, mask, x - 1, y),
                   psi_at(p, psi, mask, x, y - 1), psi_at(p, psi, mask, x + 1, y + 1),
                   psi_at(p, psi, mask, x - 1, y + 1), psi_at(p, psi, mask, x - 1, y - 1),
                   psi_at(p, psi, mask, x + 1, y - 1), Sx, Sy);
      NodeMacro mac = collide_node<S>(p, d, c, drho, jx, jy, ps, Sx, Sy);
      u = mac.ux;
      v = mac.uy;
      fxi = -p.G * ps * Sx;
      fyi = -p.G * ps * Sy;
      if (reduce) {
        bool bad;
        psi_of(p, r, bad);
        acc[RED_WALLX] += wall[0];
        acc[RED_WALLY] += wall[1];
        accumulate_node(p, acc, r, jx, jy, mac, bad);
      }
    }
    if (rho_o) rho_o[k] = r;
    if (ux_o) ux_o[k] = u;
    if (uy_o) uy_o[k] = v;
    if (fx_o) fx_o[k] = fxi;
    if (fy_o) fy_o[k] = fyi;
    if (psi_o) psi_o[k] = ps;
  }
  if (reduce) block_reduce_store(acc, partials, blockIdx.y * gridDim.x + blockIdx.x);
}

// The kernel's parameters, read again from the kernel-argument segment (the
// StepParams argument is a kernel's first, at offset 0).  The strip march
// calls it once per row and the tile kernel before its collision; the empty
// asm hides that the address does not change, so the ~30 constants of the
// step are scalar loads near their use instead of registers held across the
// kernel; holding them exceeds the scalar register file, and the compiler's
// spills cost a vector instruction per use.
typedef const __attribute__((address_space(4))) StepParams* KernargParams;
__device__ inline const StepParams& kernarg_params() {
  KernargParams kp = (KernargParams)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(kp));
  return *(const StepParams*)kp;
}

// ------------------------------------------------------------------ link words
//
// Per-node 16-bit link word of a masked lattice, read by the masked strip
// march in place of the mask: bit 0 the node is solid; bit i (1..8) the pull
// source x - e_i is solid or lies beyond a wall (the population then comes
// from the node's own opposite one); bit 9 moving walls are given and some
// pull source is a solid node inside the box (the node takes the moving-wall
// term).  Written from the mask and the periodicity.  Bit 10 is never stored:
// the march sets it in registers on the lanes of a partial last strip past
// the lattice's last column (they store nothing), with bit 0 where that
// lane's column does not exist.
constexpr unsigned LINK_SOLID = 1u, LINK_MOVING = 1u << 9, LINK_NOTOWN = 1u << 10;

__global__ __launch_bounds__(256) void links_kernel(StepParams p, const uint8_t* __restrict__ mask, int moving,
                                                   uint16_t* __restrict__ links, unsigned* __restrict__ tile_flags) {
  // one 32 x 8 block per tile of the tile kernel; the tile's flag records
  // whether it holds a fluid node beside a moving wall
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  bool mv = false;
  if (x < p.nx && y < p.ny) {
    const size_t k = (size_t)y * p.nx + x;
    unsigned w = (mask && mask[k]) ? LINK_SOLID : 0u;
    for (int i = 1; i < 9; ++i) {
      int xs, ys;
      bool inside;
      if (solid_at(p, mask, x - ex(i), y - ey(i), xs, ys, inside)) {
        w |= 1u << i;
        if (moving && inside) w |= LINK_MOVING;
      }
    }
    links[k] = (uint16_t)w;
    mv = (w & (LINK_MOVING | LINK_SOLID)) == LINK_MOVING;
  }
  const int any = __syncthreads_or(mv);
  if (threadIdx.x == 0 && threadIdx.y == 0) tile_flags[blockIdx.y * gridDim.x + blockIdx.x] = any ? 1u : 0u;
}

// The flagged tiles, in increasing tile index (one block; a fixed order, so
// the reduction over the tiles' partial sums is reproducible), and their count.
__global__ __launch_bounds__(1024) void compact_tiles_kernel(int n_tiles, const unsigned* __restrict__ flags,
                                                             int* __restrict__ list, int* __restrict__ count) {
  __shared__ int scan[1024];
  const int t = threadIdx.x;
  int base = 0;
  for (int b0 = 0; b0 < n_tiles; b0 += 1024) {
    const int f = (b0 + t < n_tiles && flags[b0 + t]) ? 1 : 0;
    scan[t] = f;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int v = t >= off ? scan[t - off] : 0;
      __syncthreads();
      scan[t] += v;
      __syncthreads();
    }
    if (f) list[base + scan[t] - 1] = b0 + t;
    base += scan[1023];
    __syncthreads();
  }
  if (t == 0) *count = base;
}

// pull_node for the tile step of nodes beside moving walls (ONLY_MOVING):
// the same arithmetic, in the same order, but the solid links come from the
// node's link word and every load (the node's own populations, the pulled
// ones, the reference offsets of the pullers, the wall velocities at the 8
// pull sources) is issued before any is used, so a node costs one memory
// round trip instead of one per moving-wall link.
template <class S>
__device__ inline void pull_links(const StepParams& p, const S* __restrict__ f, const uint16_t* __restrict__ links,
                                  const double* __restrict__ wall_u, int x, int y, double d[9], double* wall,
                                  double& c, float* cdst) {
  const int nx = p.nx;
  const size_t plane = (size_t)nx * p.ny;
  int xs[9], ys[9];
  bool ins[9];
  xs[0] = x;
  ys[0] = y;
  ins[0] = true;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    // the wrapped pull source x - e_i, as solid_at gives it
    int xx = x - ex(i), yy = y - ey(i);
    bool in = true;
    if (xx < 0) {
      in = in && p.periodic_x;
      xx += nx;
    } else if (xx >= nx) {
      in = in && p.periodic_x;
      xx -= nx;
    }
    if (yy < 0) {
      in = in && p.periodic_y;
      yy += p.ny;
    } else if (yy >= p.ny) {
      in = in && p.periodic_y;
      yy -= p.ny;
    }
    xs[i] = xx;
    ys[i] = yy;
    ins[i] = in;
  }
  const unsigned lw = links[(size_t)y * nx + x];
  double own[9], pulled[9], cref[9], uw[9], vw[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) own[q] = (double)f[pop_at<S>(nx, y, q, x)];
#pragma unroll
  for (int i = 1; i < 9; ++i) pulled[i] = (double)f[pop_at<S>(nx, ys[i], i, xs[i])];
  const double c_self = ref_offset<S>(f, nx, y, x);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    // offset of the node that pulls population i from x: x + e_i, the pull
    // source of direction opp(i)
    const int j = opp(i);
    cref[i] = i == 0 ? c_self : ref_offset<S>(f, nx, ys[j], xs[j]);
  }
  if (wall_u) {
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const size_t ks = (size_t)ys[i] * nx + xs[i];
      uw[i] = wall_u[ks];
      vw[i] = wall_u[plane + ks];
    }
  }
  c = c_self;
  bool sol[9];
  sol[0] = false;
#pragma unroll
  for (int i = 1; i < 9; ++i) sol[i] = (lw >> i) & 1u;
  double cd[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    cd[i] = 0.0;
    if constexpr (sizeof(S) == 4) {
      cd[i] = sol[opp(i)] ? c_self : cref[i];
      if (cdst) cdst[i] = (float)cd[i];
    }
  }
  double rho_w = 0.0;
  if (wall_u) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) s += own[q] + wgt(q) * cd[q];
    rho_w = p.rho_ref + s;
  }
  d[0] = own[0];
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    double v = sol[i] ? own[opp(i)] : pulled[i];
    if (sol[i]) {
      double mw = 0.0;
      if (wall_u && ins[i]) {
        const double eu = ex(i) * uw[i] + ey(i) * vw[i];
        mw = 6.0 * wgt(i) * rho_w * eu;
        v += mw;
      }
      if (wall) {
        double fi = v + wgt(i) * (p.rho_ref + c_self);
        double both = 2.0 * fi - mw;
        wall[0] -= ex(i) * both;
        wall[1] -= ey(i) * both;
      }
    }
    d[i] = v;
  }
}

// tile_psi_at from the link words (the pull of pull_links).
template <class S>
__device__ inline double tile_psi_links(const StepParams& p, const S* __restrict__ f,
                                        const uint16_t* __restrict__ links, const double* __restrict__ wall_u,
                                        int x, int y) {
  if (x < -1 || x > p.nx || y < -1 || y > p.ny) return p.psi_solid;
  int xw = x, yw = y;
  bool inside = true;
  if (xw < 0 || xw >= p.nx) {
    inside = inside && p.periodic_x;
    xw = xw < 0 ? xw + p.nx : xw - p.nx;
  }
  if (yw < 0 || yw >= p.ny) {
    inside = inside && p.periodic_y;
    yw = yw < 0 ? yw + p.ny : yw - p.ny;
  }
  if (!inside) return p.psi_solid;
  double d[9], c;
  pull_links<S>(p, f, links, wall_u, xw, yw, d, nullptr, c, nullptr);
  if (links[(size_t)yw * p.nx + xw] & LINK_SOLID) return p.psi_solid;
  double drho, jx, jy;
  node_sums<S>(d, c, drho, jx, jy);
  bool bad;
  return psi_of(p, p.rho_ref + drho, bad);
}

// ------------------------------------------------------------------ fused tile kernel
//
// The fused step for every lattice the strip kernels do not take (double
// storage of masked lattices whose width is not a multiple of 64 and that sit
// in the last-level cache; 64-bit offsets; and masked lattices when asked
// for): a block of 32 x 8 threads owns a 32 x 8 tile, one node per
// thread.  Each thread pulls its node (keeping the pulled populations in
// registers), computes psi and writes it to an LDS tile with a one-node ring;
// 84 threads also compute psi of the ring's nodes.  After one barrier every
// node collides with its neighbours' psi from LDS and is stored.  Many small
// blocks keep enough loads in flight on lattices with solid nodes, where the
// per-node pull is a chain of dependent loads.
constexpr int TILE_X = 32, TILE_Y = 8;
constexpr int TILE_HX = TILE_X + 2, TILE_HY = TILE_Y + 2;
constexpr int TILE_RING = TILE_HX * TILE_HY - TILE_X * TILE_Y;  // 84

// Position h (0..83) of the ring around a tile, in tile-with-ring coordinates.
__device__ inline void tile_ring_pos(int h, int& hx, int& hy) {
  if (h < TILE_HX) {
    hx = h;
    hy = 0;
  } else if (h < 2 * TILE_HX) {
    hx = h - TILE_HX;
    hy = TILE_HY - 1;
  } else {
    const int r = h - 2 * TILE_HX;
    hy = 1 + (r >> 1);
    hx = (r & 1) ? TILE_HX - 1 : 0;
  }
}

// psi of lattice position (x, y), at most one node outside the box: psi_solid
// across a non-periodic edge or on a solid node, else the psi of the pulled
// (wrapped) node.  Positions farther out (the ring of a tile that overhangs the
// box) are no node's neighbour; they get psi_solid without a memory access.
template <class S>
__device__ inline double tile_psi_at(const StepParams& p, const S* __restrict__ f, const uint8_t* __restrict__ mask,
                                     const double* __restrict__ wall_u, int x, int y) {
  if (x < -1 || x > p.nx || y < -1 || y > p.ny) return p.psi_solid;
  int xw, yw;
  bool inside;
  if (solid_at(p, mask, x, y, xw, yw, inside)) return p.psi_solid;
  double d[9], c;
  pull_node<S>(p, f, mask, wall_u, xw, yw, d, nullptr, c);
  double drho, jx, jy;
  node_sums<S>(d, c, drho, jx, jy);
  bool bad;
  return psi_of(p, p.rho_ref + drho, bad);
}

int tile_blocks(int nx, int ny) { return ((nx + TILE_X - 1) / TILE_X) * ((ny + TILE_Y - 1) / TILE_Y); }

// The tile step of the 32 x 8 tile at (x0, y0); `part` receives the tile's
// reduction partial (REDUCE).  ONLY_MOVING: the step of the nodes beside
// moving walls of a masked lattice on the masked strip march, run before the
// march on the tiles that hold such nodes (fluid nodes whose link word has
// LINK_MOVING): the whole tile step, but only those nodes are stored and
// reduced, and their psi goes to `psi_moving`, where the march reads it for
// their neighbours (the march skips them).
template <class S, bool REDUCE, bool ONLY_MOVING>
__device__ inline void tile_step(const StepParams& p, const S* __restrict__ f, S* __restrict__ fo,
                                 const uint8_t* __restrict__ mask, const double* __restrict__ wall_u,
                                 const uint16_t* __restrict__ links, double* __restrict__ psi_moving, int x0, int y0,
                                 double* __restrict__ part) {
  __shared__ double lpsi[TILE_HY][TILE_HX];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int x = x0 + tx, y = y0 + ty;
  const bool active = x < p.nx && y < p.ny;
  const size_t k = active ? (size_t)y * p.nx + x : 0;
  bool moving = false, fluid;
  if (ONLY_MOVING) {
    const unsigned w = active ? links[k] : LINK_SOLID;
    moving = (w & (LINK_MOVING | LINK_SOLID)) == LINK_MOVING;
    fluid = active && !(w & LINK_SOLID);
  } else {
    fluid = active && !(mask && mask[k]);
  }
  double d[9], c = 0.0, drho = 0.0, jx = 0.0, jy = 0.0;
  float cd[9];
  double wall[2] = {0.0, 0.0};
  bool bad = false;
  double ps = p.psi_solid;
  if (fluid) {
    if (ONLY_MOVING)
      pull_links<S>(p, f, links, wall_u, x, y, d, REDUCE ? wall : nullptr, c, sizeof(S) == 4 ? cd : nullptr);
    else
      pull_node<S>(p, f, mask, wall_u, x, y, d, REDUCE ? wall : nullptr, c, sizeof(S) == 4 ? cd : nullptr);
    node_sums<S>(d, c, drho, jx, jy);
    ps = psi_of(p, p.rho_ref + drho, bad);
  } else if (!active) {
    // a tile position past the box's last column or row: the wrapped node, or
    // beyond a wall
    ps = ONLY_MOVING ? tile_psi_links<S>(p, f, links, wall_u, x, y) : tile_psi_at<S>(p, f, mask, wall_u, x, y);
  }
  lpsi[ty + 1][tx + 1] = ps;
  const int tid = ty * TILE_X + tx;
  if (tid < TILE_RING) {
    int hx, hy;
    tile_ring_pos(tid, hx, hy);
    lpsi[hy][hx] = ONLY_MOVING ? tile_psi_links<S>(p, f, links, wall_u, x0 - 1 + hx, y0 - 1 + hy)
                               : tile_psi_at<S>(p, f, mask, wall_u, x0 - 1 + hx, y0 - 1 + hy);
  }
  __syncthreads();

  const StepParams& pc = kernarg_params();
  double acc[RED_COUNT];
#pragma unroll
  for (int q = 0; q < RED_COUNT; ++q) acc[q] = 0.0;
  if (fluid && (!ONLY_MOVING || moving)) {
    if (ONLY_MOVING) psi_moving[k] = ps;
    double Sx, Sy;
    stencil_sums(lpsi[ty + 1][tx + 2], lpsi[ty + 2][tx + 1], lpsi[ty + 1][tx], lpsi[ty][tx + 1], lpsi[ty + 2][tx + 2],
                 lpsi[ty + 2][tx], lpsi[ty][tx], lpsi[ty][tx + 2], Sx, Sy);
    NodeMacro mac = collide_node<S>(pc, d, c, drho, jx, jy, ps, Sx, Sy);
#pragma unroll
    for (int i = 0; i < 9; ++i)
      fo[pop_at<S>(pc.nx, y, i, x)] = store_value<S>(d[i], wgt(i), sizeof(S) == 4 ? (double)cd[i] : 0.0);
    if (REDUCE) {
      acc[RED_WALLX] += wall[0];
      acc[RED_WALLY] += wall[1];
      accumulate_node(pc, acc, pc.rho_ref + drho, jx, jy, mac, bad);
    }
  }
  if (REDUCE) block_reduce_store(acc, part, 0);
}

template <class S, bool REDUCE>
__global__ __launch_bounds__(256) void tile_kernel(StepParams p, const S* __restrict__ f, S* __restrict__ fo,
                                                   const uint8_t* __restrict__ mask,
                                                   const double* __restrict__ wall_u, double* __restrict__ partials) {
  tile_step<S, REDUCE, false>(p, f, fo, mask, wall_u, nullptr, nullptr, blockIdx.x * TILE_X, blockIdx.y * TILE_Y,
                              partials + (size_t)(blockIdx.y * gridDim.x + blockIdx.x) * RED_COUNT);
}

// The tile step of the nodes beside moving walls, over the listed tiles (each
// block takes tiles i, i + gridDim.x, ... of the list; tile i's partial is
// partial i).
template <class S, bool REDUCE>
__global__ __launch_bounds__(256) void moving_tiles_kernel(StepParams p, const S* __restrict__ f, S* __restrict__ fo,
                                                           const uint8_t* __restrict__ mask,
                                                           const double* __restrict__ wall_u,
                                                           const uint16_t* __restrict__ links,
                                                           double* __restrict__ psi_moving,
                                                           const int* __restrict__ list, const int* __restrict__ count,
                                                           int tiles_x, double* __restrict__ partials) {
  const int n = *count;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const int id = list[i];
    const int ty0 = id / tiles_x, tx0 = id - ty0 * tiles_x;
    tile_step<S, REDUCE, true>(p, f, fo, mask, wall_u, links, psi_moving, tx0 * TILE_X, ty0 * TILE_Y,
                               partials + (size_t)i * RED_COUNT);
    __syncthreads();  // the tile's psi in LDS is read before the next tile writes it
  }
}

// ------------------------------------------------------------------ fast strip kernel
//
// The strip kernel specialised for lattices whose only walls are the planes
// across non-periodic axes (no mask, no moving walls) and whose population
// arrays fit 32-bit byte offsets.  Same arithmetic as the tile kernel; what
// differs is the data movement:
//  * loads and stores are buffer instructions whose offset is the plane and
//    row (uniform) plus a lane-constant column; halfway bounce-back is a
//    per-direction select of that offset, not a branch, and columns or rows
//    that are not nodes read out of range (the buffer returns 0, stores are
//    dropped), so the march has no divergent branches;
//  * rows are software-pipelined: the loads of row y+2 are in flight while
//    row y+1 gets its psi and row y collides;
//  * psi of the neighbouring columns comes through DPP wavefront shifts;
//  * blocks are numbered so that each XCD walks a contiguous range of row
//    segments with the neighbouring strips of a segment side by side, so the
//    columns two strips share stay in that XCD's L2.

template <class S>
struct BufIO;
template <>
struct BufIO<float> {
  // byte offset = per-lane `byte_off` + wavefront-uniform `soff`
  static __device__ inline float load(__amdgpu_buffer_rsrc_t r, unsigned byte_off, unsigned soff = 0) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, (int)soff, 0));
  }
  static __device__ inline void store(float v, __amdgpu_buffer_rsrc_t r, unsigned byte_off, unsigned soff = 0) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)byte_off, (int)soff, 0);
  }
};
template <>
struct BufIO<double> {
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  static __device__ inline double load(__amdgpu_buffer_rsrc_t r, unsigned byte_off, unsigned soff = 0) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)byte_off, (int)soff, 0));
  }
  static __device__ inline void store(double v, __amdgpu_buffer_rsrc_t r, unsigned byte_off, unsigned soff = 0) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, (int)byte_off, (int)soff, 0);
  }
};

// A 16-bit float reference offset, widened.
__device__ inline float load_ref16(__amdgpu_buffer_rsrc_t r, unsigned byte_off, unsigned soff) {
  return (float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, (int)byte_off, (int)soff, 0));
}

// A buffer resource over `bytes` bytes at `base`; 0 bytes makes every access
// out of range (loads return 0, stores are dropped).
__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)bytes, 0x00020000);
}

// Lane l receives lane l-1's value (lane 0 keeps its own): DPP wave_shr:1.
__device__ inline double wave_shr1(double v) {
  unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  int lo = (int)(unsigned)b, hi = (int)(unsigned)(b >> 32);
  lo = __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
// Lane l receives lane l+1's value (lane 63 keeps its own): DPP wave_shl:1.
__device__ inline double wave_shl1(double v) {
  unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  int lo = (int)(unsigned)b, hi = (int)(unsigned)(b >> 32);
  lo = __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Lane l receives lane l-1's value and lane 0 receives `fill`: DPP wave_shr:1
// whose destination starts as `fill` (a lane without a source lane keeps it).
// One instruction per half and no lane select: a select around a DPP move
// can be turned into a branch that masks the source lane off.
__device__ inline double wave_shr1_fill(double v, double fill) {
  unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  unsigned long long f = __builtin_bit_cast(unsigned long long, fill);
  int lo = __builtin_amdgcn_update_dpp((int)(unsigned)f, (int)(unsigned)b, 0x138, 0xf, 0xf, false);
  int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(f >> 32), (int)(unsigned)(b >> 32), 0x138, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
// Lane l receives lane l+1's value and lane 63 receives `fill`: DPP wave_shl:1.
__device__ inline double wave_shl1_fill(double v, double fill) {
  unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  unsigned long long f = __builtin_bit_cast(unsigned long long, fill);
  int lo = __builtin_amdgcn_update_dpp((int)(unsigned)f, (int)(unsigned)b, 0x130, 0xf, 0xf, false);
  int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(f >> 32), (int)(unsigned)(b >> 32), 0x130, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Row geometry, uniform across the wavefront.
struct RowGeo {
  bool real;         // the row is a lattice row (in the box, or wrapped periodically)
  unsigned own, bot, top;  // element offsets of rows y, y-1, y+1 (times nx)
  bool wall_b, wall_t;     // y-1 / y+1 lie beyond a non-periodic edge
};

__device__ inline RowGeo row_geo(const StepParams& p, int y) {
  RowGeo g;
  int yw = y;
  g.real = true;
  if (y < 0 || y >= p.ny) {
    if (p.periodic_y)
      yw = y < 0 ? y + p.ny : y - p.ny;
    else
      g.real = false, yw = 0;
  }
  int yb = yw - 1, yt = yw + 1;
  g.wall_b = g.wall_t = false;
  if (yb < 0) {
    if (p.periodic_y) yb += p.ny;
    else g.wall_b = true, yb = 0;
  }
  if (yt >= p.ny) {
    if (p.periodic_y) yt -= p.ny;
    else g.wall_t = true, yt = 0;
  }
  g.own = (unsigned)yw * (unsigned)p.nx;
  g.bot = (unsigned)yb * (unsigned)p.nx;
  g.top = (unsigned)yt * (unsigned)p.nx;
  return g;
}

// Lane geometry, constant along the march.
struct ColGeo {
  bool real;
  unsigned own, left, right;  // wrapped columns x, x-1, x+1
  bool wall_l, wall_r;
};

// Byte offsets of the 9 pulled populations of node (row g, column c);
// `oob` (>= the buffer size) for a node that does not exist.
template <class S>
__device__ inline void pull_offsets(const RowGeo& g, const ColGeo& c, unsigned nx, unsigned oob, unsigned off[9]) {
  constexpr unsigned P = state_planes<S>();
  const unsigned own = P * g.own + c.own;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int exi = ex(i), eyi = ey(i);
    const unsigned row = eyi == 1 ? g.bot : (eyi == -1 ? g.top : g.own);
    const unsigned col = exi == 1 ? c.left : (exi == -1 ? c.right : c.own);
    const bool wall = (eyi == 1 && g.wall_b) || (eyi == -1 && g.wall_t) || (exi == 1 && c.wall_l) ||
                      (exi == -1 && c.wall_r);
    const unsigned e = wall ? (unsigned)opp(i) * nx + own : P * row + (unsigned)i * nx + col;
    off[i] = (g.real && c.real) ? e * (unsigned)sizeof(S) : oob;
  }
}

template <class S>
__device__ inline void load_row(__amdgpu_buffer_rsrc_t in, const unsigned off[9], S v[9]) {
#pragma unroll
  for (int i = 0; i < 9; ++i) v[i] = BufIO<S>::load(in, off[i]);
}

// Per-row quantities carried between pipeline stages.
struct RowScal {
  double drho, jx, jy, psi;
  bool bad;
  RowGeo g;
};

// Density deviation, momentum and psi of a pulled row (psi_solid where the
// node does not exist).
template <class S>
__device__ inline void row_state(const StepParams& p, const S raw[9], bool exists, RowScal& t) {
  double d[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) d[i] = (double)raw[i];
  node_sums<S>(d, 0.0, t.drho, t.jx, t.jy);
  bool bad;
  double ps = psi_of(p, p.rho_ref + t.drho, bad);
  t.psi = exists ? ps : p.psi_solid;
  t.bad = exists && bad;
}

// March state of one wavefront.
struct March {
  __amdgpu_buffer_rsrc_t in, out;
  unsigned N, nx, bytes;
  ColGeo c;
  bool owner;
  int y1;
  // lane-constant byte offset of the pulled column for each direction
  unsigned colB[9];
};

// Byte offsets of row y's pulled populations for an interior strip of a
// y-periodic lattice: plane + source row (uniform) + source column (lane).
template <class S>
__device__ inline void pull_offsets_interior(const March& m, const RowGeo& g, unsigned off[9]) {
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int eyi = ey(i);
    const unsigned row = eyi == 1 ? g.bot : (eyi == -1 ? g.top : g.own);
    off[i] = (state_planes<S>() * row + (unsigned)i * m.nx) * (unsigned)sizeof(S) + m.colB[i];
  }
}

// Issues the 9 pulled loads of row y.  A row that will not be used (`live`
// false: beyond the end of the run) is still issued, with every offset out
// of the buffer's range, so its loads return 0 without touching memory.  The
// loads are then unconditional, and the wait before each row's first use can
// count exactly the loads and stores issued after it (a conditional issue
// makes the wait drain the whole queue, including the rows in flight).
template <class S, bool INTERIOR>
__device__ inline void issue_row(const StepParams& p, const March& m, int y, bool live, S raw[9], RowGeo& g) {
  g = row_geo(p, y);
  unsigned off[9];
  if (INTERIOR)
    pull_offsets_interior<S>(m, g, off);
  else
    pull_offsets<S>(g, m.c, m.nx, m.bytes, off);
#pragma unroll
  for (int i = 0; i < 9; ++i) off[i] = live ? off[i] : m.bytes;
  load_row<S>(m.in, off, raw);
}

// One row of the march: issue the loads of row y+2 into `nxt`, finish row y+1
// (`cur1` into `t1`), then collide and store row y (`cur0`, `t0`) with psi of
// row y-1 from `tm`.
template <class S, bool REDUCE, bool INTERIOR>
__device__ inline void march_row(const StepParams& p, const March& m, int y, const S cur0[9], const S cur1[9],
                                 S nxt[9], const RowScal& tm, const RowScal& t0, RowScal& t1, RowScal& t2,
                                 double* acc) {
  issue_row<S, INTERIOR>(p, m, y + 2, y + 2 <= m.y1, nxt, t2.g);
  row_state<S>(p, cur1, t1.g.real && m.c.real, t1);
  const double pW = wave_shr1(t0.psi), pE = wave_shl1(t0.psi);
  const double pSW = wave_shr1(tm.psi), pSE = wave_shl1(tm.psi);
  const double pNW = wave_shr1(t1.psi), pNE = wave_shl1(t1.psi);
  double d[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) d[i] = (double)cur0[i];
  double Sx, Sy;
  stencil_sums(pE, t1.psi, pW, tm.psi, pNE, pNW, pSW, pSE, Sx, Sy);
  NodeMacro mac = collide_node<S>(p, d, 0.0, t0.drho, t0.jx, t0.jy, t0.psi, Sx, Sy);
  const bool store = m.owner && t0.g.real;
#pragma unroll
  for (int i = 0; i < 9; ++i)
    BufIO<S>::store((S)d[i], m.out,
                    store ? (state_planes<S>() * t0.g.own + (unsigned)i * m.nx + m.c.own) * (unsigned)sizeof(S)
                          : m.bytes);
  if (REDUCE && store) {
    if (!INTERIOR) {
      // bounce-back links: the wall received -(f_i + fbar_opp) e_i = -2 f_i e_i
      double wx = 0.0, wy = 0.0;
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        const int exi = ex(i), eyi = ey(i);
        const bool wall = (eyi == 1 && t0.g.wall_b) || (eyi == -1 && t0.g.wall_t) || (exi == 1 && m.c.wall_l) ||
                          (exi == -1 && m.c.wall_r);
        if (wall) {
          double both = 2.0 * ((double)cur0[i] + wgt(i) * p.rho_ref);
          wx -= exi * both;
          wy -= eyi * both;
        }
      }
      acc[RED_WALLX] += wx;
      acc[RED_WALLY] += wy;
    }
    accumulate_node(p, acc, p.rho_ref + t0.drho, t0.jx, t0.jy, mac, t0.bad);
  }
}

// Depth-2 pipeline: rows y+1 and y+2 are in flight when row y collides; the
// loads of row y+3 go into the slot of row y-1.
template <class S, bool REDUCE, bool INTERIOR>
__device__ inline void march_row4(const StepParams& p, const March& m, int y, const S cur0[9], const S cur1[9],
                                  S nxt[9], const RowScal& tm, const RowScal& t0, RowScal& t1, RowScal& t3,
                                  double* acc) {
  issue_row<S, INTERIOR>(p, m, y + 3, y + 3 <= m.y1, nxt, t3.g);
  row_state<S>(p, cur1, t1.g.real && m.c.real, t1);
  const double pW = wave_shr1(t0.psi), pE = wave_shl1(t0.psi);
  const double pSW = wave_shr1(tm.psi), pSE = wave_shl1(tm.psi);
  const double pNW = wave_shr1(t1.psi), pNE = wave_shl1(t1.psi);
  double d[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) d[i] = (double)cur0[i];
  double Sx, Sy;
  stencil_sums(pE, t1.psi, pW, tm.psi, pNE, pNW, pSW, pSE, Sx, Sy);
  NodeMacro mac = collide_node<S>(p, d, 0.0, t0.drho, t0.jx, t0.jy, t0.psi, Sx, Sy);
  const bool store = m.owner && t0.g.real;
#pragma unroll
  for (int i = 0; i < 9; ++i)
    BufIO<S>::store((S)d[i], m.out,
                    store ? (state_planes<S>() * t0.g.own + (unsigned)i * m.nx + m.c.own) * (unsigned)sizeof(S)
                          : m.bytes);
  if (REDUCE && store) {
    if (!INTERIOR) {
      double wx = 0.0, wy = 0.0;
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        const int exi = ex(i), eyi = ey(i);
        const bool wall = (eyi == 1 && t0.g.wall_b) || (eyi == -1 && t0.g.wall_t) || (exi == 1 && m.c.wall_l) ||
                          (exi == -1 && m.c.wall_r);
        if (wall) {
          double both = 2.0 * ((double)cur0[i] + wgt(i) * p.rho_ref);
          wx -= exi * both;
          wy -= eyi * both;
        }
      }
      acc[RED_WALLX] += wx;
      acc[RED_WALLY] += wy;
    }
    accumulate_node(p, acc, p.rho_ref + t0.drho, t0.jx, t0.jy, mac, t0.bad);
  }
}
// The march over rows y0..y1-1.  Pulled rows live in a ring of slots unrolled
// in the loop body, so no register is copied from one slot to the next:
// float storage uses three slots (row y+2 in flight while row y collides),
// double storage four (rows y+2 and y+3 in flight; each row is twice the
// bytes, so the deeper pipeline is what keeps enough loads outstanding).
template <class S, bool REDUCE, bool INTERIOR>
__device__ inline void march(const StepParams& p, const March& m, int y0, double* acc) {
  if (sizeof(S) == 4) {
    S ra[9], rb[9], rc[9];
    RowScal ta, tb, tc;
    // row r lives in slot (r - y0 + 1) mod 3: y0-1 -> c, y0 -> a, y0+1 -> b
    issue_row<S, INTERIOR>(p, m, y0 - 1, true, rc, tc.g);
    issue_row<S, INTERIOR>(p, m, y0, true, ra, ta.g);
    issue_row<S, INTERIOR>(p, m, y0 + 1, true, rb, tb.g);
    row_state<S>(p, rc, tc.g.real && m.c.real, tc);
    row_state<S>(p, ra, ta.g.real && m.c.real, ta);
    for (int y = y0; y < m.y1; y += 3) {
      march_row<S, REDUCE, INTERIOR>(p, m, y, ra, rb, rc, tc, ta, tb, tc, acc);
      if (y + 1 >= m.y1) break;
      march_row<S, REDUCE, INTERIOR>(p, m, y + 1, rb, rc, ra, ta, tb, tc, ta, acc);
      if (y + 2 >= m.y1) break;
      march_row<S, REDUCE, INTERIOR>(p, m, y + 2, rc, ra, rb, tb, tc, ta, tb, acc);
    }
  } else {
    S r0[9], r1[9], r2[9], r3[9];
    RowScal t0, t1, t2, t3;
    // row r lives in slot (r - y0 + 1) mod 4: y0-1 -> 0, y0 -> 1, y0+1 -> 2, y0+2 -> 3
    issue_row<S, INTERIOR>(p, m, y0 - 1, true, r0, t0.g);
    issue_row<S, INTERIOR>(p, m, y0, true, r1, t1.g);
    issue_row<S, INTERIOR>(p, m, y0 + 1, true, r2, t2.g);
    issue_row<S, INTERIOR>(p, m, y0 + 2, y0 + 2 <= m.y1, r3, t3.g);
    row_state<S>(p, r0, t0.g.real && m.c.real, t0);
    row_state<S>(p, r1, t1.g.real && m.c.real, t1);
    for (int y = y0; y < m.y1; y += 4) {
      march_row4<S, REDUCE, INTERIOR>(p, m, y, r1, r2, r0, t0, t1, t2, t0, acc);
      if (y + 1 >= m.y1) break;
      march_row4<S, REDUCE, INTERIOR>(p, m, y + 1, r2, r3, r1, t1, t2, t3, t1, acc);
      if (y + 2 >= m.y1) break;
      march_row4<S, REDUCE, INTERIOR>(p, m, y + 2, r3, r0, r2, t2, t3, t0, t2, acc);
      if (y + 3 >= m.y1) break;
      march_row4<S, REDUCE, INTERIOR>(p, m, y + 3, r0, r1, r3, t3, t0, t1, t3, acc);
    }
  }
}

template <class S, bool REDUCE>
__global__ __launch_bounds__(256) void fast_kernel(StepParams p, const S* __restrict__ f, S* __restrict__ fo,
                                                   int n_strips, int seg_len, int n_segs, int groups, int per_xcd,
                                                   double* __restrict__ partials) {
  const int b = blockIdx.x;
  const int L = (b & 7) * per_xcd + (b >> 3);
  const int seg = L / groups;
  const int group = L - seg * groups;
  const int wv = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int strip = group * 4 + wv;
  if (seg >= n_segs || strip >= n_strips) return;  // uniform per wavefront

  const int nx = p.nx;
  March m;
  m.N = (unsigned)nx * (unsigned)p.ny;
  m.nx = (unsigned)nx;
  m.bytes = (unsigned)state_planes<S>() * m.N * (unsigned)sizeof(S);
  m.in = __builtin_amdgcn_make_buffer_rsrc((void*)f, (short)0, (int)m.bytes, 0x00020000);
  m.out = __builtin_amdgcn_make_buffer_rsrc((void*)fo, (short)0, (int)m.bytes, 0x00020000);

  // lane geometry
  const int x = strip * STRIP - 1 + lane;
  ColGeo& c = m.c;
  int xw = x;
  c.real = true;
  if (x < 0 || x >= nx) {
    if (p.periodic_x && (x == -1 || x == nx))
      xw = x < 0 ? nx - 1 : 0;
    else
      c.real = false, xw = 0;
  }
  int xl = xw - 1, xr = xw + 1;
  c.wall_l = c.wall_r = false;
  if (xl < 0) {
    if (p.periodic_x) xl += nx;
    else c.wall_l = true, xl = 0;
  }
  if (xr >= nx) {
    if (p.periodic_x) xr -= nx;
    else c.wall_r = true, xr = 0;
  }
  c.own = (unsigned)xw;
  c.left = (unsigned)xl;
  c.right = (unsigned)xr;
  m.owner = lane >= 1 && lane <= STRIP && x < nx;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int exi = ex(i);
    m.colB[i] = (exi == 1 ? c.left : (exi == -1 ? c.right : c.own)) * (unsigned)sizeof(S);
  }

  const int y0 = seg * seg_len;
  m.y1 = min(y0 + seg_len, p.ny);

  double acc[RED_COUNT];
#pragma unroll
  for (int q = 0; q < RED_COUNT; ++q) acc[q] = 0.0;

  // Interior strips (lanes x0-1 .. x0+62 with x0-2 >= 0 and x0+63 <= nx-1: no
  // column wall, no wrap, every lane a node) of y-periodic lattices take the
  // select-free path; strips at the x edges and y-walled lattices the general one.
  const int x0 = strip * STRIP;
  const bool interior = p.periodic_y && x0 >= 2 && x0 + STRIP + 1 <= nx - 1;
  if (interior)
    march<S, REDUCE, true>(p, m, y0, acc);
  else
    march<S, REDUCE, false>(p, m, y0, acc);

  if (REDUCE) {
#pragma unroll
    for (int q = 0; q < RED_COUNT; ++q) {
      double v = wave_sum(acc[q]);
      if (lane == 0) partials[(size_t)(seg * n_strips + strip) * RED_COUNT + q] = v;
    }
  }
}

// ------------------------------------------------------------------ aligned strip kernel
//
// The fast kernel.  A wavefront owns 64 aligned columns x0 .. x0+63 (every
// lane a node; a partial last strip, below, fewer), so each row of
// each population is stored as whole aligned 256-byte (FP32) or 512-byte
// (FP64) lines.  Overlapping 62-column strips store rows that straddle cache
// lines shared with the neighbouring strip; measured on gfx950, the march
// moves data markedly slower that way.  The pseudopotential of the columns
// beside the strip (x0-1 for lane 0's stencil, x0+64 for lane 63's) comes from
// a second row of 9 pulled loads in which only lanes 0 and 63 are in range:
// lane 0 pulls column x0-1 and lane 63 column x0+64; the other lanes' offsets
// are out of range, so those loads return 0 without a memory access.

// Loads and stores take their row part as a wavefront-uniform offset and
// their column part per lane; a row that is not loaded or not stored uses an
// empty buffer resource instead of per-lane out-of-range offsets.  On lanes
// other than 0 and 63 the halo loads read the lane's own pulled populations
// again (the same cache lines as the row's main loads); their results are
// not used.
struct AMarch {
  const void* f;
  void* fo;
  unsigned N, nx, bytes;  // nodes, lattice width, bytes of the population array
  ColGeo c;   // the lane's column
  ColGeo h;   // lane 0: column x0-1, lane 63: column x0+64; real where that node exists
  int y1;
  unsigned colB[9];  // byte offsets of the pulled columns (interior strips)
  // The columns beside the strip are pulled one population per lane: lane
  // l <= 8 pulls population l of column x0-1, lane 48+i population i of
  // column x0+64 (one load instruction per row).  Lane constants of that
  // pull: the population's plane and source column (element offsets), the
  // node's own opposite plane and column (bounce-back), its e_y, whether its
  // source column lies beyond a wall, and whether the lane pulls at all.
  unsigned hplane, hcol, hback;
  int hey;
  bool hwall, hon;
  // float storage: the column byte offset of the halo column's reference
  // (the lane's own where there is none)
  unsigned href;
  double* traj;  // replay: rho - rho_ref, j_x, j_y, psi of every stored node, [4][ny][nx]
  // masked lattices: the per-node link words, the psi of the nodes beside
  // moving walls (written by moving_kernel before the march; NULL without
  // moving walls), the population the lane pulls of a column beside the
  // strip, and the column whose link word the lane reads for that column
  // (x0-1 on lanes 0-8, x0+64 on lanes 48-56 and 63, its own elsewhere)
  const uint16_t* links;
  const double* psi_moving;
  unsigned hidx, hlcol;
  // bits ORed into the lane's link word: 0, or on a partial strip's lanes past
  // the last column LINK_NOTOWN (and LINK_SOLID where the column does not exist)
  unsigned lkor;
  bool lockstep;  // every block holds 4 existing strips (they march in lockstep)
  bool owner;     // the lane's node belongs to this strip (false past a partial last strip's end)
};

// Reference offsets of one row (float storage): c at the lane's column (m)
// and, on lanes 0 and 63, at the column beside the strip (h).
struct RefRow {
  float m, h;
};

// Link words (masked lattices) of one row, packed in one register: the lane's
// node (low half) and the column beside the strip (high half; see
// AMarch::hlcol).
struct LinkPair {
  unsigned w;
  __device__ unsigned own() const { return w & 0xFFFFu; }
  __device__ unsigned halo() const { return w >> 16; }
};

template <class S>
struct ASlot {
  S raw[9];  // the lane's 9 pulled populations (stored values)
  S rh;      // lanes 0-8 and 55-63: one population of a column beside the strip
  RefRow r;   // float storage: the reference offsets of this row
  LinkPair lk;  // masked lattices: the link words the row was pulled with
  // masked lattices with moving walls: psi of the lane's node and (lanes 0
  // and 63) of the column beside the strip where that node takes the
  // moving-wall term (moving_kernel computed it; 0 elsewhere)
  double pm, ph;
};

struct ARow {
  double drho, jx, jy, psi;
  // psi of the west and east neighbours (lane l - 1 and l + 1; lane 0's
  // west and lane 63's east are the columns beside the strip): each row's
  // psi is shifted once, for the three collisions that use it
  double pw, pe;
  bool bad;
  RowGeo g;
  RefRow cr;  // float storage: the reference offsets of this row
};

// Link words of row y (masked lattices); rows beyond a non-periodic edge read
// row 0 (they are not pulled).
template <bool RAGGED>
__device__ inline LinkPair aload_links(const StepParams& p, const AMarch& m, int y) {
  const RowGeo g = row_geo(p, y);
  const unsigned row = g.real ? g.own : 0u;
  const __amdgpu_buffer_rsrc_t r = buf_rsrc(m.links, 2u * m.N);
  const unsigned own = (unsigned)__builtin_amdgcn_raw_buffer_load_b16(r, (int)(m.c.own * 2u), (int)(row * 2u), 0);
  const unsigned halo = (unsigned)__builtin_amdgcn_raw_buffer_load_b16(r, (int)(m.hlcol * 2u), (int)(row * 2u), 0);
  LinkPair lk;
  lk.w = (RAGGED ? (own | m.lkor) : own) | (halo << 16);
  return lk;
}

template <class S, bool INTERIOR, bool MASKED, bool MOVING>
__device__ inline void aissue_row(const StepParams& p, const AMarch& m, int y, bool live, ASlot<S>& sl, RowGeo& g,
                                  const LinkPair& lk) {
  g = row_geo(p, y);
  const __amdgpu_buffer_rsrc_t in = buf_rsrc(m.f, live ? m.bytes : 0u);
  if (MASKED) {
    // bounce-back wherever the link word says the pull source is solid or
    // beyond a wall: the node's own opposite population
    sl.lk = lk;
    const unsigned own = state_planes<S>() * g.own + m.c.own;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int exi = ex(i), eyi = ey(i);
      const unsigned row = eyi == 1 ? g.bot : (eyi == -1 ? g.top : g.own);
      const unsigned col = exi == 1 ? m.c.left : (exi == -1 ? m.c.right : m.c.own);
      const bool wall = i > 0 && ((lk.own() >> i) & 1u);
      const unsigned e = wall ? (unsigned)opp(i) * m.nx + own : state_planes<S>() * row + (unsigned)i * m.nx + col;
      sl.raw[i] = BufIO<S>::load(in, g.real ? e * (unsigned)sizeof(S) : m.bytes);
    }
  } else if (INTERIOR) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int eyi = ey(i);
      const unsigned row = eyi == 1 ? g.bot : (eyi == -1 ? g.top : g.own);
      const unsigned rb = (state_planes<S>() * row + (unsigned)i * m.nx) * (unsigned)sizeof(S);
      sl.raw[i] = BufIO<S>::load(in, m.colB[i], rb);
    }
  } else {
    unsigned off[9];
    pull_offsets<S>(g, m.c, m.nx, m.bytes, off);
    load_row<S>(in, off, sl.raw);
  }
  if (MOVING) {
    // psi of nodes beside moving walls (lanes whose node, or on lanes 0 and
    // 63 the column beside the strip, takes the moving-wall term; the other
    // lanes' offsets fall outside the buffer)
    const __amdgpu_buffer_rsrc_t pr = buf_rsrc(m.psi_moving, (live && g.real) ? 8u * m.N : 0u);
    const bool mo = (lk.own() & (LINK_MOVING | LINK_SOLID)) == LINK_MOVING;
    const bool mh = m.h.real && (lk.halo() & (LINK_MOVING | LINK_SOLID)) == LINK_MOVING;
    sl.pm = BufIO<double>::load(pr, mo ? (g.own + m.c.own) * 8u : 8u * m.N);
    sl.ph = BufIO<double>::load(pr, mh ? (g.own + m.h.own) * 8u : 8u * m.N);
  }
  if (MASKED) {
    // the columns beside the strip, one population per lane; the choices
    // between rows and between pull and bounce-back are taken with bit masks
    // (as selects, the compiler may turn the per-lane row choice into a table
    // in scratch memory behind a branch)
    const unsigned mb = 0u - (unsigned)(m.hey == 1), mt = 0u - (unsigned)(m.hey == -1);
    const unsigned row = (g.bot & mb) | (g.top & mt) | (g.own & ~(mb | mt));
    const unsigned mw = 0u - ((lk.halo() >> m.hidx) & (unsigned)(m.hidx > 0u));
    const unsigned e = ((state_planes<S>() * g.own + m.hback) & mw) | ((state_planes<S>() * row + m.hplane + m.hcol) & ~mw);
    sl.rh = BufIO<S>::load(in, (m.hon && g.real) ? e * (unsigned)sizeof(S) : m.bytes);
  } else {
    // the columns beside the strip, one population per lane
    const unsigned row = m.hey == 1 ? g.bot : (m.hey == -1 ? g.top : g.own);
    const bool wall = !INTERIOR && (m.hwall || (m.hey == 1 && g.wall_b) || (m.hey == -1 && g.wall_t));
    const unsigned e =
        wall ? state_planes<S>() * g.own + m.hback : state_planes<S>() * row + m.hplane + m.hcol;
    sl.rh = BufIO<S>::load(in, (m.hon && g.real) ? e * (unsigned)sizeof(S) : m.bytes);
  }
  if constexpr (sizeof(S) == 4) {
    // every population pulled into this row was stored relative to the
    // puller's own offset: one offset per node
    // (the row's tenth run, from byte 4 (10 y + 9) nx)
    const __amdgpu_buffer_rsrc_t rf = buf_rsrc(m.f, (live && g.real) ? m.bytes : 0u);
    const unsigned rrow = 4u * (10u * g.own + 9u * m.nx);
    sl.r.m = load_ref16(rf, m.c.own * 2u, rrow);
    sl.r.h = load_ref16(rf, m.href, rrow);
  }
}

// DPP move of a float: lane l receives lane l-1's v (CTRL 0x138, wave_shr:1)
// or lane l+1's (0x130, wave_shl:1); a lane without a source lane gets `fill`.
template <int CTRL>
__device__ inline float fbits_dpp(float v, float fill) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, fill),
                                                               __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}

// Reference offsets of the nodes that pull row q's post-collision
// populations, from the reference rows q-1 (`rb`), q (`r0`) and q+1 (`rt`):
// cd[i] = c(x + e_i), or c(x) when x + e_i is solid or lies beyond a wall
// (masked lattices: bit opp(i) of the node's link word).  Lane 0's west and
// lane 63's east neighbours are the columns beside the strip.
template <bool INTERIOR, bool MASKED>
__device__ inline void dest_refs_row(const AMarch& m, const RowGeo& g, const RefRow& rb, const RefRow& r0,
                                     const RefRow& rt, unsigned lkown, float cd[9]) {
  // rows q-1, q, q+1 (b, 0, t) at columns x - 1 (w), x, x + 1 (e); lane 0's
  // x - 1 and lane 63's x + 1 are the columns beside the strip (named values,
  // not arrays, so that nothing is indexed at run time)
  const float wb = fbits_dpp<0x138>(rb.m, rb.h), w0 = fbits_dpp<0x138>(r0.m, r0.h), wt = fbits_dpp<0x138>(rt.m, rt.h);
  const float eb = fbits_dpp<0x130>(rb.m, rb.h), e0 = fbits_dpp<0x130>(r0.m, r0.h), et = fbits_dpp<0x130>(rt.m, rt.h);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int exi = ex(i), eyi = ey(i);
    const float cw = eyi == 1 ? wt : (eyi == -1 ? wb : w0);
    const float ce = eyi == 1 ? et : (eyi == -1 ? eb : e0);
    const float cc = eyi == 1 ? rt.m : (eyi == -1 ? rb.m : r0.m);
    const float dst = exi == 1 ? ce : (exi == -1 ? cw : cc);
    if (MASKED) {
      cd[i] = (i > 0 && ((lkown >> opp(i)) & 1u)) ? r0.m : dst;
    } else if (INTERIOR) {
      cd[i] = dst;
    } else {
      const bool wall = (eyi == 1 && g.wall_t) || (eyi == -1 && g.wall_b) || (exi == 1 && m.c.wall_r) ||
                        (exi == -1 && m.c.wall_l);
      cd[i] = wall ? r0.m : dst;
    }
  }
}

// DPP move of a double within rows of 16 lanes (CTRL 0x100 + k: lane l
// receives lane l+k's v); lanes without a source lane read 0.  No lane's
// previous value is kept, so each half is one move.
template <int CTRL>
__device__ inline double row_dpp0(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, true);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// DPP move of a double within rows of 16 lanes (CTRL 0x100 + k: lane l
// receives lane l+k's v; 0x110 + k: lane l-k's); lanes without a source lane
// keep their own v.
template <int CTRL>
__device__ inline double row_dpp(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  int lo = (int)(unsigned)b, hi = (int)(unsigned)(b >> 32);
  lo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Sum of the 9 populations of the columns beside the strip, pulled one per
// lane, in node_sums' order d0 + ((d1 + d3) + (d2 + d4)) + ((d5 + d7) + (d6 + d8)),
// so that psi there is bitwise the one the column's own strip computes.
// Lane l <= 8 holds d_l of column x0-1 and lane 48+i d_i of column x0+64: the
// same shifts within rows of 16 lanes sum the first into lane 0 and the
// second into lane 48, and a last shift (row_shr:15) moves lane 48's sum to
// lane 63 (lane 0, with no source lane, keeps its own).
__device__ inline double halo_sum(double v) {
  const double a1 = v + row_dpp0<0x102>(v);    // lane 1: d1+d3, 2: d2+d4, 5: d5+d7, 6: d6+d8 (48+: the same)
  const double a2 = a1 + row_dpp0<0x101>(a1);  // lane 1: S4, lane 5: S8
  const double a3 = v + row_dpp0<0x101>(a2);   // lane 0: d0 + S4
  const double a4 = a3 + row_dpp0<0x105>(a2);  // lane 0: (d0 + S4) + S8
  return row_dpp<0x11F>(a4);                   // lane 63: lane 48's sum; lane 0 keeps its own
}

// Density, momentum and psi of a pulled row.  Masked lattices: psi_solid on
// solid nodes; a node beside a moving wall (and a column beside the strip
// whose node is one) takes the psi moving_kernel computed for it.
template <class S, bool MASKED, bool MOVING, bool RAGGED>
__device__ inline void arow_state(const StepParams& p, const AMarch& m, const ASlot<S>& sl, ARow& t) {
  double d[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) d[i] = (double)sl.raw[i];
  double cm = 0.0, ch = 0.0;
  if constexpr (sizeof(S) == 4) {
    cm = (double)sl.r.m;
    ch = (double)sl.r.h;
    t.cr = sl.r;
  }
  bool solid = false, hsolid = false, moving = false, hmoving = false;
  if (MASKED) {
    solid = (sl.lk.own() & LINK_SOLID) != 0u;
    hsolid = (sl.lk.halo() & LINK_SOLID) != 0u;
    if (MOVING) {
      moving = !solid && (sl.lk.own() & LINK_MOVING);
      hmoving = !hsolid && (sl.lk.halo() & LINK_MOVING);
    }
  }
  node_sums<S>(d, cm, t.drho, t.jx, t.jy);
  bool bad;
  const double ps = psi_of(p, p.rho_ref + t.drho, bad);
  // a partial strip: the lanes past the lattice's last column that are not
  // a wrapped column take psi_solid (masked lattices: their link words say
  // solid)
  const bool here = t.g.real && (!RAGGED || MASKED || m.c.real);
  t.psi = (here && !solid) ? (moving ? sl.pm : ps) : p.psi_solid;
  t.bad = here && !solid && bad;
  // the halo column's density in the same arithmetic as its own strip uses
  double hr = halo_sum((double)sl.rh);
  if constexpr (sizeof(S) == 4) hr += ch;
  bool badh;
  const double psh = psi_of(p, p.rho_ref + hr, badh);
  const double psih = (t.g.real && m.h.real && !hsolid) ? (hmoving ? sl.ph : psh) : p.psi_solid;
  t.pw = wave_shr1_fill(t.psi, psih);
  t.pe = wave_shl1_fill(t.psi, psih);
}

// Collide and store row y (slot `s0`, state `t0`), with psi of rows y-1 (`tm`)
// and y+1 (`t1`, finished here from slot `s1`); the loads of row y + AHEAD
// go into slot `sn` first.  Masked lattices: `ln` holds the link words of row
// y + AHEAD, and the link words of row y + AHEAD + 1 are loaded into `l0`.
template <class S, bool REDUCE, bool TRAJ, bool INTERIOR, bool MASKED, bool MOVING, bool RAGGED, int AHEAD>
__device__ inline void amarch_row(const AMarch& m, int y, const ASlot<S>& s0, const ASlot<S>& s1, ASlot<S>& sn,
                                  const ARow& tm, const ARow& t0, ARow& t1, ARow& tn, LinkPair& l0,
                                  const LinkPair& ln, double* acc) {
  const StepParams& p = kernarg_params();
  // the block's 4 waves (4 neighbouring strips of one run) start each row
  // together, so that the block's loads of a row are one contiguous stretch
  // of each run of that row; a bare barrier, no wait for memory
  if (m.lockstep) __builtin_amdgcn_s_barrier();
  if (MASKED) l0 = aload_links<RAGGED>(p, m, y + AHEAD + 1);
  aissue_row<S, INTERIOR, MASKED, MOVING>(p, m, y + AHEAD, y + AHEAD <= m.y1, sn, tn.g, ln);
  arow_state<S, MASKED, MOVING, RAGGED>(p, m, s1, t1);
  const double pW = t0.pw, pE = t0.pe;
  const double pSW = tm.pw, pSE = tm.pe;
  const double pNW = t1.pw, pNE = t1.pe;
  double d[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) d[i] = (double)s0.raw[i];
  double cm = 0.0;
  if constexpr (sizeof(S) == 4) cm = (double)t0.cr.m;
  // solid nodes keep their populations; nodes beside moving walls were
  // collided and stored by moving_kernel
  const bool skip = MASKED && ((s0.lk.own() & (LINK_SOLID | LINK_NOTOWN)) || (MOVING && (s0.lk.own() & LINK_MOVING)));
  const bool store = t0.g.real && (!RAGGED || MASKED || m.owner) && !skip;
  double Sx, Sy;
  stencil_sums(pE, t1.psi, pW, tm.psi, pNE, pNW, pSW, pSE, Sx, Sy);
  double dw[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) dw[i] = d[i];
  NodeMacro mac = collide_node<S>(p, d, cm, t0.drho, t0.jx, t0.jy, t0.psi, Sx, Sy);
  float cd[9];
  if constexpr (sizeof(S) == 4) {
    dest_refs_row<INTERIOR, MASKED>(m, t0.g, tm.cr, t0.cr, t1.cr, MASKED ? s0.lk.own() : 0u, cd);
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) cd[i] = 0.0f;
  }
  const __amdgpu_buffer_rsrc_t out = buf_rsrc(m.fo, t0.g.real ? m.bytes : 0u);
  // a lane that does not store: its stores fall outside the buffer
  const unsigned col = ((!MASKED && !RAGGED) || store) ? m.c.own * (unsigned)sizeof(S) : m.bytes;
#pragma unroll
  for (int i = 0; i < 9; ++i)
    BufIO<S>::store(store_value<S>(d[i], wgt(i), (double)cd[i]), out, col,
                    (state_planes<S>() * t0.g.own + (unsigned)i * m.nx) * (unsigned)sizeof(S));
  if (TRAJ) {
    // the replayed step's pulled-state quantities, as the adjoint reads them
    const __amdgpu_buffer_rsrc_t tr = buf_rsrc(m.traj, store ? 4u * m.N * 8u : 0u);
    const double tv[4] = {t0.drho, t0.jx, t0.jy, t0.psi};
#pragma unroll
    for (int q = 0; q < 4; ++q) BufIO<double>::store(tv[q], tr, m.c.own * 8u, ((unsigned)q * m.N + t0.g.own) * 8u);
  }
  if (REDUCE && store) {
    if (!INTERIOR) {
      double wx = 0.0, wy = 0.0;
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        const int exi = ex(i), eyi = ey(i);
        bool wall;
        if (MASKED)
          wall = (s0.lk.own() >> i) & 1u;
        else
          wall = (eyi == 1 && t0.g.wall_b) || (eyi == -1 && t0.g.wall_t) || (exi == 1 && m.c.wall_l) ||
                 (exi == -1 && m.c.wall_r);
        if (wall) {
          // the pulled deviation at a wall link is the node's own opposite
          // population; the wall received -(f_i + fbar_opp) e_i = -2 f_i e_i
          double both = 2.0 * (dw[i] + wgt(i) * (p.rho_ref + cm));
          wx -= exi * both;
          wy -= eyi * both;
        }
      }
      acc[RED_WALLX] += wx;
      acc[RED_WALLY] += wy;
    }
    accumulate_node(p, acc, p.rho_ref + t0.drho, t0.jx, t0.jy, mac, t0.bad);
  }
}

// The march over rows y0 .. y1-1, with three row slots: row y+2 in flight
// while row y collides.  (A fourth slot, rows y+2 and y+3 in flight, measured
// the same or slower for both storages once runs are short.)  Masked
// lattices keep the link words one row further ahead, so that the offsets of
// a row's pulls never wait for its link words.
template <class S, bool REDUCE, bool TRAJ, bool INTERIOR, bool MASKED, bool MOVING, bool RAGGED>
__device__ inline void amarch(const StepParams& p, const AMarch& m, int y0, double* acc) {
  ASlot<S> sa, sb, sc;
  ARow ta, tb, tc;
  // link words of the next row each slot receives (masked lattices)
  LinkPair la{0u}, lb{0u}, lc{0u};
  if (MASKED) {
    lc = aload_links<RAGGED>(p, m, y0 - 1);
    la = aload_links<RAGGED>(p, m, y0);
    lb = aload_links<RAGGED>(p, m, y0 + 1);
  }
  // row r lives in slot (r - y0 + 1) mod 3: y0-1 -> c, y0 -> a, y0+1 -> b
  aissue_row<S, INTERIOR, MASKED, MOVING>(p, m, y0 - 1, true, sc, tc.g, lc);
  aissue_row<S, INTERIOR, MASKED, MOVING>(p, m, y0, true, sa, ta.g, la);
  aissue_row<S, INTERIOR, MASKED, MOVING>(p, m, y0 + 1, true, sb, tb.g, lb);
  if (MASKED) lc = aload_links<RAGGED>(p, m, y0 + 2);
  arow_state<S, MASKED, MOVING, RAGGED>(p, m, sc, tc);
  arow_state<S, MASKED, MOVING, RAGGED>(p, m, sa, ta);
  for (int y = y0; y < m.y1; y += 3) {
    amarch_row<S, REDUCE, TRAJ, INTERIOR, MASKED, MOVING, RAGGED, 2>(m, y, sa, sb, sc, tc, ta, tb, tc, la, lc, acc);
    if (y + 1 >= m.y1) break;
    amarch_row<S, REDUCE, TRAJ, INTERIOR, MASKED, MOVING, RAGGED, 2>(m, y + 1, sb, sc, sa, ta, tb, tc, ta, lb, la, acc);
    if (y + 2 >= m.y1) break;
    amarch_row<S, REDUCE, TRAJ, INTERIOR, MASKED, MOVING, RAGGED, 2>(m, y + 2, sc, sa, sb, tb, tc, ta, tb, lc, lb, acc);
  }
}

// Column geometry of column x (possibly one outside the box).
__device__ inline ColGeo col_geo(const StepParams& p, int x, bool want) {
  ColGeo c;
  const int nx = p.nx;
  int xw = x;
  c.real = want;
  if (x < 0 || x >= nx) {
    if (p.periodic_x)
      xw = x < 0 ? x + nx : x - nx;
    else
      c.real = false, xw = 0;
  }
  if (!want) xw = 0;
  int xl = xw - 1, xr = xw + 1;
  c.wall_l = c.wall_r = false;
  if (xl < 0) {
    if (p.periodic_x) xl += nx;
    else c.wall_l = true, xl = 0;
  }
  if (xr >= nx) {
    if (p.periodic_x) xr -= nx;
    else c.wall_r = true, xr = 0;
  }
  c.own = (unsigned)xw;
  c.left = (unsigned)xl;
  c.right = (unsigned)xr;
  return c;
}

template <class S, bool REDUCE, bool TRAJ, bool MASKED, bool MOVING>
__global__ __launch_bounds__(256) void aligned_kernel(StepParams p, const S* __restrict__ f, S* __restrict__ fo,
                                                      int n_strips, int seg_len, int n_segs, int groups, int per_xcd,
                                                      int interleave, double* __restrict__ partials,
                                                      double* __restrict__ traj, const uint16_t* __restrict__ links,
                                                      const double* __restrict__ psi_moving, int lockstep) {
  // Blocks go to the 8 XCDs round-robin (block b to XCD b mod 8).  Either
  // each XCD takes one contiguous band of runs, neighbouring runs sharing its
  // L2, or (interleave) the XCDs take successive runs in turn, so that all of
  // them stream from the same few DRAM rows at a time.
  const int b = blockIdx.x;
  int seg, group;
  if (interleave) {
    const int i = b >> 3, q = i / groups;
    seg = 8 * q + (b & 7);
    group = i - q * groups;
  } else {
    const int L = (b & 7) * per_xcd + (b >> 3);
    seg = L / groups;
    group = L - seg * groups;
  }
  const int wv = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int strip = group * 4 + wv;
  if (seg >= n_segs || strip >= n_strips) return;  // uniform per wavefront

  AMarch m;
  m.N = (unsigned)p.nx * (unsigned)p.ny;
  m.nx = (unsigned)p.nx;
  m.bytes = (unsigned)state_planes<S>() * m.N * (unsigned)sizeof(S);
  m.f = f;
  m.fo = fo;
  const int x0 = strip * WAVE;
  // A partial last strip (widths that are not a multiple of 64): its lane w
  // takes the column after the lattice's last one (wrapped, or beyond the
  // wall), whose psi the last column needs, and the lanes past it idle;
  // neither stores.  Such a strip has no column beside it on the right.
  const int w = min(WAVE, p.nx - x0);
  const bool ragged = w < WAVE;
  const bool hl = lane == 0 || (lane == WAVE - 1 && !ragged);
  m.owner = true;
  m.lkor = 0u;
  if (!ragged) {
    m.c = col_geo(p, x0 + lane, true);
  } else {
    m.c = col_geo(p, x0 + min(lane, w), lane <= w);
    m.owner = lane < w;
    m.lkor = lane < w ? 0u : (LINK_NOTOWN | (m.c.real ? 0u : LINK_SOLID));
  }
  m.h = col_geo(p, lane == 0 ? x0 - 1 : x0 + WAVE, hl);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int exi = ex(i);
    m.colB[i] = (exi == 1 ? m.c.left : (exi == -1 ? m.c.right : m.c.own)) * (unsigned)sizeof(S);
  }
  {
    // the columns beside the strip, one population per lane
    const bool left = lane <= 8, right = !ragged && lane >= 48 && lane <= 56;
    const int hi = left ? lane : (right ? lane - 48 : 0);
    const ColGeo hg = col_geo(p, left ? x0 - 1 : x0 + WAVE, left || right);
    const int exi = ex(hi);
    m.hplane = (unsigned)hi * m.nx;
    m.hcol = exi == 1 ? hg.left : (exi == -1 ? hg.right : hg.own);
    m.hback = (unsigned)opp(hi) * m.nx + hg.own;
    m.hey = ey(hi);
    m.hwall = (exi == 1 && hg.wall_l) || (exi == -1 && hg.wall_r);
    m.hon = (left || right) && hg.real;
    m.hidx = (unsigned)hi;
    // link word of the column beside the strip: the pulling lanes' column,
    // and lane 63's (which takes that column's psi); the lane's own elsewhere
    const ColGeo hr = col_geo(p, x0 + WAVE, !ragged);
    m.hlcol = (m.hon ? hg.own : ((lane == WAVE - 1 && hr.real) ? hr.own : m.c.own));
  }
  // float storage: byte offset within a row's reference run of the halo
  // column's offset (the lane's own where there is none)
  m.href = (m.h.real ? m.h.own : m.c.own) * 2u;
  m.traj = traj;
  m.links = links;
  m.psi_moving = psi_moving;
  // Lattices that stream from HBM (lockstep set by the host), with every
  // strip group complete: the 4 waves of each block march the same rows of
  // the same run and meet at a barrier before each row (the same number of
  // barriers, whichever path each wave takes).  On the 2048 x 16384 lattice
  // 2.9% faster for double storage, 1% for float; on lattices that sit in the
  // last-level cache, where the march is bound by latency, slower (the masked
  // 1024 x 1024 annulus, FP64: 26.4k -> 24.7k MLUPS).
  m.lockstep = lockstep && (n_strips % 4 == 0);
  const int y0 = seg * seg_len;
  m.y1 = min(y0 + seg_len, p.ny);

  double acc[RED_COUNT];
#pragma unroll
  for (int q = 0; q < RED_COUNT; ++q) acc[q] = 0.0;

  // Interior strips (the pulls of columns x0-1 .. x0+64 stay inside the box
  // without wrapping) of y-periodic lattices take the select-free offsets.
  const bool interior = p.periodic_y && x0 >= 2 && x0 + WAVE + 1 <= p.nx - 1;
  // (a partial strip of an unmasked lattice, at most one per run, takes its
  // own instance of the march, so that whole strips keep theirs unchanged;
  // the masked march marks the lanes past the last column in their link
  // words instead)
  if (MASKED && ragged)
    amarch<S, REDUCE, TRAJ, false, true, MOVING, true>(p, m, y0, acc);
  else if (MASKED)
    amarch<S, REDUCE, TRAJ, false, true, MOVING, false>(p, m, y0, acc);
  else if (interior)
    amarch<S, REDUCE, TRAJ, true, false, false, false>(p, m, y0, acc);
  else if (ragged)
    amarch<S, REDUCE, TRAJ, false, false, false, true>(p, m, y0, acc);
  else
    amarch<S, REDUCE, TRAJ, false, false, false, false>(p, m, y0, acc);

  if (REDUCE) {
#pragma unroll
    for (int q = 0; q < RED_COUNT; ++q) {
      double v = wave_sum(acc[q]);
      if (lane == 0) partials[(size_t)(seg * n_strips + strip) * RED_COUNT + q] = v;
    }
  }
}

// ------------------------------------------------------------------ finalize
// Fixed-order sum of reduction partials.  Up to FIN_SMALL partials (and
// without the extra range): one block sums them.  Otherwise two stages:
// block b of FIN_BLOCKS sums the partials b*256 + t, b*256 + t + 256*FIN_BLOCKS,
// ... of `partials` (then of the `*extra_count` partials at `extra`, the tiles
// of nodes beside moving walls, when extra is non-NULL) into tmp[b], and one
// block sums the FIN_BLOCKS results.  The grouping depends only on the
// counts, so the result is bitwise reproducible.  (One block over the 43,712
// partials of the 2048 x 16384 lattice took 112 us, the two stages 10 us; over
// a few thousand one block is the faster, 6.5 us.)
constexpr int FIN_BLOCKS = kFinalizeBlocks;
constexpr int FIN_SMALL = 4096;

__device__ inline void block_sum_to(double s[RED_COUNT], double* __restrict__ out) {
  __shared__ double lds[RED_COUNT][256];
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < RED_COUNT; ++q) lds[q][t] = s[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
#pragma unroll
      for (int q = 0; q < RED_COUNT; ++q) lds[q][t] += lds[q][t + w];
    }
    __syncthreads();
  }
  if (t < RED_COUNT) out[t] = lds[t][0];
}

__global__ __launch_bounds__(256) void finalize_stage1_kernel(const double* __restrict__ partials, int n_parts,
                                                              const double* __restrict__ extra,
                                                              const int* __restrict__ extra_count,
                                                              double* __restrict__ tmp) {
  const int t = threadIdx.x;
  const int stride = gridDim.x * 256;
  double s[RED_COUNT];
#pragma unroll
  for (int q = 0; q < RED_COUNT; ++q) s[q] = 0.0;
  for (int b = blockIdx.x * 256 + t; b < n_parts; b += stride) {
#pragma unroll
    for (int q = 0; q < RED_COUNT; ++q) s[q] += partials[(size_t)b * RED_COUNT + q];
  }
  if (extra) {
    const int ne = *extra_count;
    for (int b = blockIdx.x * 256 + t; b < ne; b += stride) {
#pragma unroll
      for (int q = 0; q < RED_COUNT; ++q) s[q] += extra[(size_t)b * RED_COUNT + q];
    }
  }
  block_sum_to(s, tmp + (size_t)blockIdx.x * RED_COUNT);
}

__global__ __launch_bounds__(256) void finalize_kernel(const double* __restrict__ tmp, double* __restrict__ out) {
  const int t = threadIdx.x;
  double s[RED_COUNT];
#pragma unroll
  for (int q = 0; q < RED_COUNT; ++q) s[q] = t < FIN_BLOCKS ? tmp[(size_t)t * RED_COUNT + q] : 0.0;
  block_sum_to(s, out);
}

// ------------------------------------------------------------------ launchers
static dim3 node_grid(const StepParams& p, dim3 blk) {
  return dim3((p.nx + blk.x - 1) / blk.x, (p.ny + blk.y - 1) / blk.y);
}

int two_pass_blocks(int nx, int ny) { return ((nx + 63) / 64) * ((ny + 3) / 4); }

void fused_shape(int nx, int ny, int seg_len, bool aligned, int* n_strips, int* n_segs) {
  *n_strips = aligned ? (nx + WAVE - 1) / WAVE : (nx + STRIP - 1) / STRIP;
  *n_segs = (ny + seg_len - 1) / seg_len;
}

template <class S>
hipError_t launch_init(const StepParams& p, const double* rho0, const double* ux0, const double* uy0,
                       const uint8_t* mask, void* fa, void* fb, hipStream_t st) {
  dim3 blk(64, 4);
  hipLaunchKernelGGL(init_kernel<S>, node_grid(p, blk), blk, 0, st, p, rho0, ux0, uy0, mask, (S*)fa, (S*)fb);
  return hipGetLastError();
}

// The 62-column strip kernel: double storage only (float storage keeps a
// per-node reference plane, which the aligned kernel and the general fused
// kernel read).  Returns false when it does not apply.
template <class S>
static bool launch_fast62(const StepParams& p, const StepLaunch& L, hipStream_t st) {
  if constexpr (sizeof(S) != 8) {
    return false;
  } else {
    const S* f = (const S*)L.f_in;
    S* fo = (S*)L.f_out;
    int n_strips, n_segs;
    fused_shape(p.nx, p.ny, L.seg_len, false, &n_strips, &n_segs);
    int groups = (n_strips + 3) / 4;
    int total = groups * n_segs;
    int per_xcd = (total + 7) / 8;
    if (L.reduce)
      hipLaunchKernelGGL((fast_kernel<S, true>), dim3(8 * per_xcd), dim3(256), 0, st, p, f, fo, n_strips, L.seg_len,
                         n_segs, groups, per_xcd, L.partials);
    else
      hipLaunchKernelGGL((fast_kernel<S, false>), dim3(8 * per_xcd), dim3(256), 0, st, p, f, fo, n_strips,
                         L.seg_len, n_segs, groups, per_xcd, L.partials);
    return true;
  }
}

template <class S>
hipError_t launch_step(const StepParams& p, const StepLaunch& L, hipStream_t st) {
  const S* f = (const S*)L.f_in;
  S* fo = (S*)L.f_out;
  // only the aligned strip kernel writes the trajectory
  if (L.traj && !(L.kernel == 0 && L.aligned && !L.masked)) return hipErrorNotSupported;
  if (L.kernel == 1) {
    dim3 blk(64, 4);
    dim3 grd = node_grid(p, blk);
    hipLaunchKernelGGL(psi_kernel<S>, grd, blk, 0, st, p, f, L.mask, L.wall_u, (double*)L.psi);
    if (L.reduce)
      hipLaunchKernelGGL((collide_kernel<S, true>), grd, blk, 0, st, p, f, fo, L.mask, L.wall_u,
                         (const double*)L.psi, L.partials);
    else
      hipLaunchKernelGGL((collide_kernel<S, false>), grd, blk, 0, st, p, f, fo, L.mask, L.wall_u,
                         (const double*)L.psi, L.partials);
  } else if (L.aligned || L.masked) {
    int n_strips, n_segs;
    fused_shape(p.nx, p.ny, L.seg_len, true, &n_strips, &n_segs);
    int groups = (n_strips + 3) / 4;
    int total = groups * n_segs;
    // blocks per XCD: interleaved, every strip group of ceil(n_segs / 8) runs
    int per_xcd = L.interleave ? groups * ((n_segs + 7) / 8) : (total + 7) / 8;
    const int il = L.interleave ? 1 : 0;
    const dim3 grd(8 * per_xcd), blk(256);
    if (L.traj && L.reduce) return hipErrorInvalidValue;
    if (L.masked) {
      if (L.traj || !L.links) return hipErrorInvalidValue;
      double* pm = nullptr;
      if (L.wall_u) {
        // the nodes beside moving walls first, on the tile kernel (their reduction
        // partials follow the march's)
        pm = (double*)L.psi;
        const dim3 tblk(TILE_X, TILE_Y);
        const int tiles_x = (p.nx + TILE_X - 1) / TILE_X;
        const int n_tiles = tiles_x * ((p.ny + TILE_Y - 1) / TILE_Y);
        const dim3 tgrd(std::min(n_tiles, 2048));
        if (L.reduce)
          hipLaunchKernelGGL((moving_tiles_kernel<S, true>), tgrd, tblk, 0, st, p, f, fo, L.mask, L.wall_u, L.links,
                             pm, L.tile_list, L.tile_count, tiles_x, L.moving_partials);
        else
          hipLaunchKernelGGL((moving_tiles_kernel<S, false>), tgrd, tblk, 0, st, p, f, fo, L.mask, L.wall_u,
                             L.links, pm, L.tile_list, L.tile_count, tiles_x, L.moving_partials);
      }
      if (pm && L.reduce)
        hipLaunchKernelGGL((aligned_kernel<S, true, false, true, true>), grd, blk, 0, st, p, f, fo, n_strips,
                           L.seg_len, n_segs, groups, per_xcd, il, L.partials, nullptr, L.links, pm, 0);
      else if (pm)
        hipLaunchKernelGGL((aligned_kernel<S, false, false, true, true>), grd, blk, 0, st, p, f, fo, n_strips,
                           L.seg_len, n_segs, groups, per_xcd, il, L.partials, nullptr, L.links, pm, 0);
      else if (L.reduce)
        hipLaunchKernelGGL((aligned_kernel<S, true, false, true, false>), grd, blk, 0, st, p, f, fo, n_strips,
                           L.seg_len, n_segs, groups, per_xcd, il, L.partials, nullptr, L.links, nullptr, 0);
      else
        hipLaunchKernelGGL((aligned_kernel<S, false, false, true, false>), grd, blk, 0, st, p, f, fo, n_strips,
                           L.seg_len, n_segs, groups, per_xcd, il, L.partials, nullptr, L.links, nullptr, 0);
    } else if (L.traj)
      hipLaunchKernelGGL((aligned_kernel<S, false, true, false, false>), grd, blk, 0, st, p, f, fo, n_strips, L.seg_len,
                         n_segs, groups, per_xcd, il, L.partials, L.traj, nullptr, nullptr, L.lockstep);
    else if (L.reduce)
      hipLaunchKernelGGL((aligned_kernel<S, true, false, false, false>), grd, blk, 0, st, p, f, fo, n_strips, L.seg_len,
                         n_segs, groups, per_xcd, il, L.partials, nullptr, nullptr, nullptr, L.lockstep);
    else
      hipLaunchKernelGGL((aligned_kernel<S, false, false, false, false>), grd, blk, 0, st, p, f, fo, n_strips, L.seg_len,
                         n_segs, groups, per_xcd, il, L.partials, nullptr, nullptr, nullptr, L.lockstep);
  } else if (L.fast && launch_fast62<S>(p, L, st)) {
    // launched: the 62-column strip kernel (double storage, widths not a multiple of 64, cache-resident)
  } else {
    dim3 blk(TILE_X, TILE_Y);
    dim3 grd((p.nx + TILE_X - 1) / TILE_X, (p.ny + TILE_Y - 1) / TILE_Y);
    if (L.reduce)
      hipLaunchKernelGGL((tile_kernel<S, true>), grd, blk, 0, st, p, f, fo, L.mask, L.wall_u, L.partials);
    else
      hipLaunchKernelGGL((tile_kernel<S, false>), grd, blk, 0, st, p, f, fo, L.mask, L.wall_u, L.partials);
  }
  return hipGetLastError();
}

hipError_t launch_links(const StepParams& p, const uint8_t* mask, int moving, uint16_t* links, unsigned* tile_flags,
                        int* tile_list, int* tile_count, hipStream_t st) {
  const dim3 blk(TILE_X, TILE_Y);
  const dim3 grd((p.nx + TILE_X - 1) / TILE_X, (p.ny + TILE_Y - 1) / TILE_Y);
  hipLaunchKernelGGL(links_kernel, grd, blk, 0, st, p, mask, moving, links, tile_flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !moving) return e;
  hipLaunchKernelGGL(compact_tiles_kernel, dim3(1), dim3(1024), 0, st, (int)(grd.x * grd.y), tile_flags, tile_list,
                     tile_count);
  return hipGetLastError();
}

hipError_t launch_reref(const StepParams& p, void* fa, void* fb, const uint8_t* mask, hipStream_t st) {
  dim3 blk(64, 4);
  hipLaunchKernelGGL(reref_new_kernel, node_grid(p, blk), blk, 0, st, p, (const float*)fa, (float*)fb, mask);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reref_shift_kernel, node_grid(p, blk), blk, 0, st, p, (float*)fa, (float*)fb, mask);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reref_copy_kernel, node_grid(p, blk), blk, 0, st, p, (float*)fa, (const float*)fb);
  return hipGetLastError();
}

template <class S>
hipError_t launch_fields(const StepParams& p, const void* f, const uint8_t* mask, const double* wall_u, void* psi,
                         double* rho, double* ux, double* uy, double* fx, double* fy, double* psi_o,
                         double* partials, int reduce, hipStream_t st) {
  dim3 blk(64, 4);
  dim3 grd = node_grid(p, blk);
  hipLaunchKernelGGL(psi_kernel<S>, grd, blk, 0, st, p, (const S*)f, mask, wall_u, (double*)psi);
  hipLaunchKernelGGL(fields_kernel<S>, grd, blk, 0, st, p, (const S*)f, mask, wall_u, (const double*)psi, rho, ux,
                     uy, fx, fy, psi_o, partials, reduce);
  return hipGetLastError();
}

hipError_t launch_finalize(const double* partials, int n_parts, double* out, double* tmp, hipStream_t s,
                           const double* extra, const int* extra_count) {
  if (n_parts <= FIN_SMALL && !extra) {
    hipLaunchKernelGGL(finalize_stage1_kernel, dim3(1), dim3(256), 0, s, partials, n_parts, extra, extra_count, out);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(finalize_stage1_kernel, dim3(FIN_BLOCKS), dim3(256), 0, s, partials, n_parts, extra, extra_count,
                     tmp);
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, s, tmp, out);
  return hipGetLastError();
}

template hipError_t launch_init<float>(const StepParams&, const double*, const double*, const double*,
                                       const uint8_t*, void*, void*, hipStream_t);
template hipError_t launch_init<double>(const StepParams&, const double*, const double*, const double*,
                                        const uint8_t*, void*, void*, hipStream_t);
template hipError_t launch_step<float>(const StepParams&, const StepLaunch&, hipStream_t);
template hipError_t launch_step<double>(const StepParams&, const StepLaunch&, hipStream_t);
template hipError_t launch_fields<float>(const StepParams&, const void*, const uint8_t*, const double*, void*, double*,
                                         double*, double*, double*, double*, double*, double*, int, hipStream_t);
template hipError_t launch_fields<double>(const StepParams&, const void*, const uint8_t*, const double*, void*,
                                          double*, double*, double*, double*, double*, double*, double*, int,
                                          hipStream_t);

}  // namespace pplbm
