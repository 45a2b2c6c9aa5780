// Adjoint (reverse-mode) kernels of the step, and the trajectory replay that
// feeds them.
//
// Notation for step n (1-based): A = fbar^{n-1} (post-collision state before
// the step), B = fbar^n.  lambda^n = dL/dB.  For each step the backward sweep
// runs
//   traj_kernel    (replay)  rho - rho_ref, j and psi of step n's pulled state,
//   collide_kernel (replay)  the ordinary step from A to B (psi read from traj),
// and, in reverse step order,
//   adj_local_kernel   lambda^n(x) by transposing the pull of step n+1:
//                        lambda_i(x) = P_i(x + e_i) if x + e_i is fluid,
//                                      P_opp(i)(x)  otherwise (bounce-back),
//                      with P = D^{n+1} + R^{n+1} the adjoint of step n+1's
//                      pulled populations; then the reverse of x's collision
//                      (plus the loss's direct sensitivities at step n), giving
//                      D^n (9 values), dL/dpsi_c and dL/dS of x, and the
//                      node's share of dL/dG and dL/d|F_ext|;
//   adj_psi_kernel     dL/dpsi(x) = dL/dpsi_c(x) + sum_k w_k e_k . dL/dS(x - e_k)
//                      and R^n(x) = psi'(rho(x)) dL/dpsi(x).
// At the end, dL/drho0(x) = sum_i w_i lambda^0_i(x) (fbar^0 = w_i rho0 at rest).
#include <hip/hip_runtime.h>

#include "lbm_adjoint_node.h"

namespace pplbm {

constexpr int AWAVE = 64;

__device__ inline double awave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, AWAVE);
  return v;
}

// Block (64 x 4) reduction of n <= 4 values, added to acc[block][0..n).
__device__ inline void block_add(const double* v, int n, double* __restrict__ acc, int block_id, int stride) {
  __shared__ double lds[4][4];
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int lane = tid % AWAVE, wid = tid / AWAVE;
  for (int q = 0; q < n; ++q) {
    double s = awave_sum(v[q]);
    if (lane == 0) lds[q][wid] = s;
  }
  __syncthreads();
  if (tid < n) {
    double s = ((lds[tid][0] + lds[tid][1]) + (lds[tid][2] + lds[tid][3]));
    acc[(size_t)block_id * stride + tid] += s;
  }
}

// Node of this thread: a one-dimensional grid of 64 x 4 tiles (tiles of a
// tile row consecutive).  Measured faster than 256 x 1, 128 x 2 or 32 x 8
// rows for these gather-heavy kernels.
__device__ inline void node_xy(const StepParams& p, int& x, int& y) {
  const unsigned nbx = (unsigned)(p.nx + 63) / 64;
  const unsigned by = blockIdx.x / nbx;
  const unsigned bx = blockIdx.x - by * nbx;
  x = (int)(bx * 64 + (threadIdx.x & 63));
  y = (int)(by * 4 + (threadIdx.x >> 6));
}

// ------------------------------------------------------------------ kernels (one node per lane)
template <class S>
__global__ void traj_kernel(StepParams p, const S* __restrict__ f, const uint8_t* __restrict__ mask,
                            double* __restrict__ traj) {
  int x, y;
  node_xy(p, x, y);
  if (x >= p.nx || y >= p.ny) return;
  adj_traj_node<S>(p, f, mask, traj, x, y);
}

template <class L>
__global__ void adj_local_kernel(StepParams p, AdjStepArgs a) {
  int x, y;
  node_xy(p, x, y);
  double part[2] = {0.0, 0.0};
  if (x < p.nx && y < p.ny) adj_local_node<L>(p, a, x, y, part);
  block_add(part, 2, a.param_acc, blockIdx.x, 2);
}

template <class L>
__global__ void adj_psi_kernel(StepParams p, AdjStepArgs a) {
  int x, y;
  node_xy(p, x, y);
  if (x >= p.nx || y >= p.ny) return;
  adj_psi_node<L>(p, a, x, y);
}

template <class L>
__global__ void adj_rho0_kernel(StepParams p, AdjStepArgs a, double* __restrict__ grad_rho0) {
  int x, y;
  node_xy(p, x, y);
  if (x >= p.nx || y >= p.ny) return;
  grad_rho0[(size_t)y * p.nx + x] = adj_rho0_node<L>(p, a, x, y);
}

// ------------------------------------------------------------------ velocity-error loss
__global__ void uerr_kernel(StepParams p, const uint8_t* __restrict__ mask, const double* __restrict__ ux,
                            const double* __restrict__ ut, double* __restrict__ partials) {
  int x, y;
  node_xy(p, x, y);
  double v[2] = {0.0, 0.0};
  if (x < p.nx && y < p.ny) {
    const size_t k = (size_t)y * p.nx + x;
    if (!(mask && mask[k])) {
      const double d = ux[k] - ut[k];
      v[0] = d * d;
      v[1] = ut[k] * ut[k];
    }
  }
  __shared__ double lds[2][4];
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int lane = tid % AWAVE, wid = tid / AWAVE;
  for (int q = 0; q < 2; ++q) {
    double s = awave_sum(v[q]);
    if (lane == 0) lds[q][wid] = s;
  }
  __syncthreads();
  if (tid < 2) partials[(size_t)(blockIdx.x) * 2 + tid] =
      (lds[tid][0] + lds[tid][1]) + (lds[tid][2] + lds[tid][3]);
}

// Fixed-order sum of n pairs (one block).
__global__ void pair_sum_kernel(const double* __restrict__ partials, int n, double* __restrict__ out) {
  __shared__ double lds[2][256];
  const int t = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int i = t; i < n; i += 256) {
    a += partials[(size_t)i * 2];
    b += partials[(size_t)i * 2 + 1];
  }
  lds[0][t] = a;
  lds[1][t] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      lds[0][t] += lds[0][t + w];
      lds[1][t] += lds[1][t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = lds[0][0];
    out[1] = lds[1][0];
  }
}

__global__ void zero_kernel(double* __restrict__ p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0.0;
}

// ------------------------------------------------------------------ launchers
static const dim3 ABLOCK(256, 1);
static dim3 agrid(const StepParams& p) { return dim3((unsigned)(((p.nx + 63) / 64) * ((p.ny + 3) / 4))); }

int adj_blocks(int nx, int ny) { return ((nx + 63) / 64) * ((ny + 3) / 4); }

template <class S>
hipError_t launch_traj(const StepParams& p, const void* f, const uint8_t* mask, double* traj, hipStream_t st) {
  hipLaunchKernelGGL(traj_kernel<S>, agrid(p), ABLOCK, 0, st, p, (const S*)f, mask, traj);
  return hipGetLastError();
}

template <class L>
hipError_t launch_adj_step(const StepParams& p, const AdjStepArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(adj_local_kernel<L>, agrid(p), ABLOCK, 0, st, p, a);
  hipLaunchKernelGGL(adj_psi_kernel<L>, agrid(p), ABLOCK, 0, st, p, a);
  return hipGetLastError();
}

template <class L>
hipError_t launch_adj_rho0(const StepParams& p, const AdjStepArgs& a, double* grad_rho0, hipStream_t st) {
  hipLaunchKernelGGL(adj_rho0_kernel<L>, agrid(p), ABLOCK, 0, st, p, a, grad_rho0);
  return hipGetLastError();
}

hipError_t launch_uerr(const StepParams& p, const uint8_t* mask, const double* ux, const double* ut,
                       double* partials, double* out, hipStream_t st) {
  hipLaunchKernelGGL(uerr_kernel, agrid(p), ABLOCK, 0, st, p, mask, ux, ut, partials);
  hipLaunchKernelGGL(pair_sum_kernel, dim3(1), dim3(256), 0, st, partials, adj_blocks(p.nx, p.ny), out);
  return hipGetLastError();
}

hipError_t launch_pair_sum(const double* partials, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(pair_sum_kernel, dim3(1), dim3(256), 0, st, partials, n, out);
  return hipGetLastError();
}

hipError_t launch_zero(double* ptr, size_t n, hipStream_t st) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, ptr, n);
  return hipGetLastError();
}

template hipError_t launch_adj_step<float>(const StepParams&, const AdjStepArgs&, hipStream_t);
template hipError_t launch_adj_step<double>(const StepParams&, const AdjStepArgs&, hipStream_t);
template hipError_t launch_adj_rho0<float>(const StepParams&, const AdjStepArgs&, double*, hipStream_t);
template hipError_t launch_adj_rho0<double>(const StepParams&, const AdjStepArgs&, double*, hipStream_t);
template hipError_t launch_traj<float>(const StepParams&, const void*, const uint8_t*, double*, hipStream_t);
template hipError_t launch_traj<double>(const StepParams&, const void*, const uint8_t*, double*, hipStream_t);

}  // namespace pplbm
