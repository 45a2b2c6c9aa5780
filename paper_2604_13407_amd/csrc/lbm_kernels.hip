// HIP kernels of one pseudopotential MRT step for gfx950 (CDNA4, wave64).
//
// Two step implementations share the node arithmetic of lbm_node.h:
//  * the fused strip kernel: one wavefront owns a 62-column strip (plus one
//    halo column on each side) over a run of rows and marches up the rows.
//    Each row is pulled once; its density and pseudopotential are computed
//    in registers; the force stencil reads the three live rows of psi through
//    cross-lane shuffles; the collision of the middle row is stored.  One
//    kernel per step, populations read and written once (plus the halo).
//  * the two-pass kernels: a psi pass writes the pseudopotential field, then
//    a collide pass pulls again, reads psi of the 8 neighbours and collides.
//    Simple, one node per thread; the reference for the fused kernel.
// Reductions (every reduce_every steps) are FP64 per-wave partial sums
// finished by a fixed-order kernel, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

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
                            const double* __restrict__ uy0, S* __restrict__ fa, S* __restrict__ fb) {
  int x = blockIdx.x * blockDim.x + threadIdx.x;
  int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= p.nx || y >= p.ny) return;
  size_t k = (size_t)y * p.nx + x;
  size_t plane = (size_t)p.nx * p.ny;
  double r = rho0[k];
  double u = ux0 ? ux0[k] : 0.0;
  double v = uy0 ? uy0[k] : 0.0;
  double usq = u * u + v * v;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    double eu = ex(i) * u + ey(i) * v;
    // f_eq - w rho_ref = w [(rho - rho_ref) + rho (3 e.u + 9/2 (e.u)^2 - 3/2 u^2)]
    double dv = wgt(i) * ((r - p.rho_ref) + r * (3.0 * eu + 4.5 * eu * eu - 1.5 * usq));
    fa[(size_t)i * plane + k] = (S)dv;
    fb[(size_t)i * plane + k] = (S)dv;
  }
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
  double d[9];
  pull_node<S>(p, f, mask, wall_u, x, y, d, nullptr);
  double drho, jx, jy;
  node_sums(d, drho, jx, jy);
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
  const int lane = threadIdx.x % WAVE;
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
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
    pull_node<S>(p, f, mask, wall_u, x, y, d, REDUCE ? wall : nullptr);
    double drho, jx, jy;
    node_sums(d, drho, jx, jy);
    double Sx, Sy;
    stencil_sums(psi_at(p, psi, mask, x + 1, y), psi_at(p, psi, mask, x, y + 1), psi_at(p, psi, mask, x - 1, y),
                 psi_at(p, psi, mask, x, y - 1), psi_at(p, psi, mask, x + 1, y + 1), psi_at(p, psi, mask, x - 1, y + 1),
                 psi_at(p, psi, mask, x - 1, y - 1), psi_at(p, psi, mask, x + 1, y - 1), Sx, Sy);
    NodeMacro mac = collide_node(p, d, drho, jx, jy, psi[k], Sx, Sy);
    const size_t plane = (size_t)p.nx * p.ny;
#pragma unroll
    for (int i = 0; i < 9; ++i) fo[(size_t)i * plane + k] = (S)d[i];
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
      pull_node<S>(p, f, mask, wall_u, x, y, d, reduce ? wall : nullptr);
      double drho, jx, jy;
      node_sums(d, drho, jx, jy);
      r = p.rho_ref + drho;
      double Sx, Sy;
      stencil_sums(psi_at(p, psi, mask, x + 1, y), psi_at(p, psi, mask, x, y + 1), psi_at(p, psi, mask, x - 1, y),
                   psi_at(p, psi, mask, x, y - 1), psi_at(p, psi, mask, x + 1, y + 1),
                   psi_at(p, psi, mask, x - 1, y + 1), psi_at(p, psi, mask, x - 1, y - 1),
                   psi_at(p, psi, mask, x + 1, y - 1), Sx, Sy);
      NodeMacro mac = collide_node(p, d, drho, jx, jy, ps, Sx, Sy);
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

// ------------------------------------------------------------------ fused strip kernel
//
// Lane l of a wavefront holds column x = x0 - 1 + l; lanes 1..62 are the
// strip's own columns, lanes 0 and 63 are halo columns that only supply psi.
// The wave computes rows y0..y1-1 and also pulls rows y0-1 and y1 (halo rows)
// for their psi.  Row pipeline: row r is pulled, summed and given psi; once
// psi of row r+1 exists, row r collides and is stored.
template <class S>
__device__ inline void strip_row_pull(const StepParams& p, const S* __restrict__ f, const uint8_t* __restrict__ mask,
                                      const double* __restrict__ wall_u, int x, int y, bool lane_in, double d[9],
                                      double& drho, double& jx, double& jy, double& psi, bool& fluid, bool& bad,
                                      double* wall) {
  // classify (x, y): outside the box across a wall, masked solid, or fluid
  int xw = 0, yw = 0;
  bool inside;
  bool sol = !lane_in || solid_at(p, mask, x, y, xw, yw, inside);
  fluid = !sol;
  bad = false;
  if (fluid) {
    pull_node<S>(p, f, mask, wall_u, xw, yw, d, wall);
    node_sums(d, drho, jx, jy);
    psi = psi_of(p, p.rho_ref + drho, bad);
  } else {
    psi = p.psi_solid;
    drho = jx = jy = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) d[i] = 0.0;
  }
}

template <class S, bool REDUCE>
__global__ __launch_bounds__(256) void fused_kernel(StepParams p, const S* __restrict__ f, S* __restrict__ fo,
                                                    const uint8_t* __restrict__ mask,
                                                    const double* __restrict__ wall_u, int n_strips, int seg_len,
                                                    int n_segs, double* __restrict__ partials) {
  const int lane = threadIdx.x % WAVE;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  if (wave >= n_strips * n_segs) return;  // whole wave exits together
  const int strip = wave % n_strips;
  const int seg = wave / n_strips;
  const int x0 = strip * STRIP;
  const int x = x0 - 1 + lane;
  const int y0 = seg * seg_len;
  const int y1 = min(y0 + seg_len, p.ny);
  // a lane is a real column (or the periodic/wall column just outside) if x <= nx
  const bool lane_in = (x <= p.nx);
  const bool owner = (lane >= 1 && lane <= STRIP && x < p.nx);
  const size_t plane = (size_t)p.nx * p.ny;

  double acc[RED_COUNT];
#pragma unroll
  for (int q = 0; q < RED_COUNT; ++q) acc[q] = 0.0;

  double dc[9], dn[9];
  double drc, jxc, jyc, drn, jxn, jyn;
  double psm, psc, psn;
  bool flc, fln, badc, badn;
  double wallc[2] = {0.0, 0.0}, walln[2] = {0.0, 0.0};

  // prologue: halo row y0-1 (psi only) and row y0
  {
    double dtmp[9], a, b, c;
    bool ftmp, btmp;
    strip_row_pull<S>(p, f, mask, wall_u, x, y0 - 1, lane_in, dtmp, a, b, c, psm, ftmp, btmp, nullptr);
  }
  strip_row_pull<S>(p, f, mask, wall_u, x, y0, lane_in, dc, drc, jxc, jyc, psc, flc, badc, REDUCE ? wallc : nullptr);

  for (int y = y0; y < y1; ++y) {
    walln[0] = walln[1] = 0.0;
    strip_row_pull<S>(p, f, mask, wall_u, x, y + 1, lane_in, dn, drn, jxn, jyn, psn, fln, badn,
                      (REDUCE && y + 1 < y1) ? walln : nullptr);
    // neighbours' psi through the wavefront (lanes 0 and 63 never collide)
    double pW = shfl_up1(psc), pE = shfl_down1(psc);
    double pSW = shfl_up1(psm), pSE = shfl_down1(psm);
    double pNW = shfl_up1(psn), pNE = shfl_down1(psn);
    if (owner && flc) {
      double Sx, Sy;
      stencil_sums(pE, psn, pW, psm, pNE, pNW, pSW, pSE, Sx, Sy);
      NodeMacro mac = collide_node(p, dc, drc, jxc, jyc, psc, Sx, Sy);
      const size_t k = (size_t)y * p.nx + x;
#pragma unroll
      for (int i = 0; i < 9; ++i) fo[(size_t)i * plane + k] = (S)dc[i];
      if (REDUCE) {
        acc[RED_WALLX] += wallc[0];
        acc[RED_WALLY] += wallc[1];
        accumulate_node(p, acc, p.rho_ref + drc, jxc, jyc, mac, badc);
      }
    }
    // rotate the row pipeline
    psm = psc;
    psc = psn;
#pragma unroll
    for (int i = 0; i < 9; ++i) dc[i] = dn[i];
    drc = drn;
    jxc = jxn;
    jyc = jyn;
    flc = fln;
    badc = badn;
    wallc[0] = walln[0];
    wallc[1] = walln[1];
  }
  if (REDUCE) {
#pragma unroll
    for (int q = 0; q < RED_COUNT; ++q) {
      double v = wave_sum(acc[q]);
      if (lane == 0) partials[(size_t)wave * RED_COUNT + q] = v;
    }
  }
}

// ------------------------------------------------------------------ finalize
__global__ void finalize_kernel(const double* __restrict__ partials, int n_parts, double* __restrict__ out) {
  __shared__ double lds[RED_COUNT][256];
  const int t = threadIdx.x;
  double s[RED_COUNT];
#pragma unroll
  for (int q = 0; q < RED_COUNT; ++q) s[q] = 0.0;
  for (int b = t; b < n_parts; b += 256) {
#pragma unroll
    for (int q = 0; q < RED_COUNT; ++q) s[q] += partials[(size_t)b * RED_COUNT + q];
  }
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

// ------------------------------------------------------------------ launchers
static dim3 node_grid(const StepParams& p, dim3 blk) {
  return dim3((p.nx + blk.x - 1) / blk.x, (p.ny + blk.y - 1) / blk.y);
}

int two_pass_blocks(int nx, int ny) { return ((nx + 63) / 64) * ((ny + 3) / 4); }

void fused_shape(int nx, int ny, int seg_len, int* n_strips, int* n_segs) {
  *n_strips = (nx + STRIP - 1) / STRIP;
  *n_segs = (ny + seg_len - 1) / seg_len;
}

template <class S>
hipError_t launch_init(const StepParams& p, const double* rho0, const double* ux0, const double* uy0, void* fa,
                       void* fb, hipStream_t st) {
  dim3 blk(64, 4);
  hipLaunchKernelGGL(init_kernel<S>, node_grid(p, blk), blk, 0, st, p, rho0, ux0, uy0, (S*)fa, (S*)fb);
  return hipGetLastError();
}

template <class S>
hipError_t launch_step(const StepParams& p, const StepLaunch& L, hipStream_t st) {
  const S* f = (const S*)L.f_in;
  S* fo = (S*)L.f_out;
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
  } else {
    int n_strips, n_segs;
    fused_shape(p.nx, p.ny, L.seg_len, &n_strips, &n_segs);
    int waves = n_strips * n_segs;
    int blocks = (waves + 3) / 4;
    if (L.reduce)
      hipLaunchKernelGGL((fused_kernel<S, true>), dim3(blocks), dim3(256), 0, st, p, f, fo, L.mask, L.wall_u,
                         n_strips, L.seg_len, n_segs, L.partials);
    else
      hipLaunchKernelGGL((fused_kernel<S, false>), dim3(blocks), dim3(256), 0, st, p, f, fo, L.mask, L.wall_u,
                         n_strips, L.seg_len, n_segs, L.partials);
  }
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

hipError_t launch_finalize(const double* partials, int n_parts, double* out, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, s, partials, n_parts, out);
  return hipGetLastError();
}

template hipError_t launch_init<float>(const StepParams&, const double*, const double*, const double*, void*, void*,
                                       hipStream_t);
template hipError_t launch_init<double>(const StepParams&, const double*, const double*, const double*, void*, void*,
                                        hipStream_t);
template hipError_t launch_step<float>(const StepParams&, const StepLaunch&, hipStream_t);
template hipError_t launch_step<double>(const StepParams&, const StepLaunch&, hipStream_t);
template hipError_t launch_fields<float>(const StepParams&, const void*, const uint8_t*, const double*, void*, double*,
                                         double*, double*, double*, double*, double*, double*, int, hipStream_t);
template hipError_t launch_fields<double>(const StepParams&, const void*, const uint8_t*, const double*, void*,
                                          double*, double*, double*, double*, double*, double*, double*, int,
                                          hipStream_t);

}  // namespace pplbm
