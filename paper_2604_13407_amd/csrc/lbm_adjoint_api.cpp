// Host side of the discrete adjoint: lbm_adjoint_workspace_bytes,
// lbm_adjoint_forward and lbm_adjoint_backward of include/pplbm.h.
//
// Forward: initialise at rest, run N steps on the handle's population arrays,
// copying the state into checkpoint slot c before step cK + 1, and reduce the
// loss's observables.  Backward: for each segment, last first, copy its
// checkpoint into two replay arrays, replay the segment storing every step's
// trajectory (rho - rho_ref, j, psi of the pulled state), then run the reverse
// steps of the segment from its last step to its first.  All buffers live in
// the caller's adjoint workspace; nothing is allocated here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pplbm.h"
#include "lbm_adjoint_internal.h"
#include "lbm_handle.h"
#include "lbm_internal.h"

using namespace pplbm_host;
using pplbm::RED_COUNT;

namespace {

struct AdjLayout {
  size_t n;             // nodes
  int64_t n_ckpt;       // saved states
  int64_t seg;          // trajectory slots (min(K, N))
  int64_t n_log;        // reduction records of the forward pass
  size_t state_bytes;   // one population array, 256-aligned
  size_t ckpt, rep0, rep1, traj, D0, D1, R0, R1, T, acc, pair, log, ux, upart, uout, total;
};

bool adj_cfg_ok(const lbm_adjoint_cfg* a, std::string& why) {
  if (!a) {
    why = "adjoint config is NULL";
    return false;
  }
  if (a->n_steps < 1) {
    why = "n_steps must be >= 1";
    return false;
  }
  if (a->checkpoint_every < 1) {
    why = "checkpoint_every must be >= 1";
    return false;
  }
  if (a->loss == LBM_LOSS_DRAG) {
    if (a->window < 2 || a->window > a->n_steps) {
      why = "drag loss needs 2 <= window <= n_steps";
      return false;
    }
  } else if (a->loss == LBM_LOSS_UERR) {
    if (!a->u_target_dev) {
      why = "velocity-error loss needs u_target_dev";
      return false;
    }
  } else {
    why = "unknown loss";
    return false;
  }
  return true;
}

AdjLayout adj_layout(const lbm_config* c, const lbm_adjoint_cfg* a) {
  AdjLayout L;
  L.n = (size_t)c->nx * c->ny;
  const int64_t N = a->n_steps, K = a->checkpoint_every;
  L.n_ckpt = (N + K - 1) / K;
  L.seg = std::min<int64_t>(K, N);
  L.n_log = (a->loss == LBM_LOSS_DRAG) ? a->window : 1;
  L.state_bytes = align256(state_bytes_of(c));
  const size_t nd = L.n * sizeof(double);
  const size_t blocks = (size_t)pplbm::adj_blocks(c->nx, c->ny);
  size_t off = 0;
  L.ckpt = off;
  off += (size_t)L.n_ckpt * L.state_bytes;
  L.rep0 = off;
  off += L.state_bytes;
  L.rep1 = off;
  off += L.state_bytes;
  L.traj = off;
  off = align256(off + (size_t)L.seg * 4 * nd);
  // D: float for float storage, double for double storage
  const size_t nl = L.n * elem_size(c);
  L.D0 = off;
  off = align256(off + 9 * nl);
  L.D1 = off;
  off = align256(off + 9 * nl);
  L.R0 = off;
  off = align256(off + nd);
  L.R1 = off;
  off = align256(off + nd);
  L.T = off;
  off = align256(off + 3 * nd);
  L.acc = off;
  off = align256(off + blocks * 2 * sizeof(double));
  L.pair = off;
  off = align256(off + 2 * sizeof(double));
  L.log = off;
  off = align256(off + (size_t)L.n_log * RED_COUNT * sizeof(double));
  L.ux = off;
  off = align256(off + (a->loss == LBM_LOSS_UERR ? nd : 0));
  L.upart = off;
  off = align256(off + blocks * 2 * sizeof(double));
  L.uout = off;
  off = align256(off + 2 * sizeof(double));
  L.total = off;
  return L;
}

template <class T>
T* at(char* ws, size_t off) {
  return reinterpret_cast<T*>(ws + off);
}

}  // namespace

extern "C" {

int lbm_adjoint_workspace_bytes(const lbm_config* cfg, const lbm_adjoint_cfg* a, size_t* bytes) {
  g_create_error.clear();
  std::string why;
  if (!bytes) return fail_query(LBM_ERR_INVALID_ARG, "bytes is NULL");
  if (!config_ok(cfg, why) || !adj_cfg_ok(a, why)) return fail_query(LBM_ERR_INVALID_ARG, why);
  *bytes = adj_layout(cfg, a).total;
  return LBM_OK;
}

int lbm_adjoint_forward(lbm_lattice* h, const lbm_adjoint_cfg* a, const double* rho0, void* workspace,
                        size_t workspace_bytes, double* loss_host) {
  if (!h) return LBM_ERR_INVALID_ARG;
  h->adj.ready = false;
  std::string why;
  if (!adj_cfg_ok(a, why)) return fail(h, LBM_ERR_INVALID_ARG, why);
  if (!rho0 || !workspace) return fail(h, LBM_ERR_INVALID_ARG, "rho0 and workspace must be non-NULL");
  if (((uintptr_t)workspace & 255u) != 0) return fail(h, LBM_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (h->buf.wall_u) return fail(h, LBM_ERR_UNSUPPORTED, "the adjoint does not support moving walls");
  begin_stepping(h);
  const AdjLayout L = adj_layout(&h->cfg, a);
  if (workspace_bytes < L.total) return fail(h, LBM_ERR_INVALID_ARG, "adjoint workspace too small");
  char* ws = (char*)workspace;
  const bool fp64 = h->cfg.precision == LBM_FP64;
  const int64_t N = a->n_steps, K = a->checkpoint_every;
  const int64_t first_logged = (a->loss == LBM_LOSS_DRAG) ? N - a->window + 1 : N;

  const uint8_t* mask = h->buf.mask;
  hipError_t e = fp64 ? pplbm::launch_init<double>(h->prm, rho0, nullptr, nullptr, mask, h->buf.f_a, h->buf.f_b,
                                                   h->stream)
                      : pplbm::launch_init<float>(h->prm, rho0, nullptr, nullptr, mask, h->buf.f_a, h->buf.f_b,
                                                  h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "init launch");
  h->cur = 0;
  h->steps = 0;
  h->initialized = true;
  const size_t sbytes = state_bytes_of(&h->cfg);
  double* log = at<double>(ws, L.log);
  for (int64_t t = 1; t <= N; ++t) {
    if ((t - 1) % K == 0) {
      e = hipMemcpyAsync(ws + L.ckpt + (size_t)((t - 1) / K) * L.state_bytes, state_ptr(h, h->cur), sbytes,
                         hipMemcpyDeviceToDevice, h->stream);
      if (e != hipSuccess) return hip_fail(h, e, "checkpoint copy");
    }
    if (a->loss == LBM_LOSS_UERR && t == N) {
      double* ux = at<double>(ws, L.ux);
      const void* f = state_ptr(h, h->cur);
      e = fp64 ? pplbm::launch_fields<double>(h->prm, f, h->buf.mask, nullptr, h->psi, nullptr, ux, nullptr, nullptr,
                                              nullptr, nullptr, h->partials, 0, h->stream)
               : pplbm::launch_fields<float>(h->prm, f, h->buf.mask, nullptr, h->psi, nullptr, ux, nullptr, nullptr,
                                             nullptr, nullptr, h->partials, 0, h->stream);
      if (e != hipSuccess) return hip_fail(h, e, "fields launch");
      e = pplbm::launch_uerr(h->prm, h->buf.mask, ux, a->u_target_dev, at<double>(ws, L.upart),
                             at<double>(ws, L.uout), h->stream);
      if (e != hipSuccess) return hip_fail(h, e, "velocity error launch");
    }
    const int reduce = t >= first_logged ? 1 : 0;
    e = step_between(h, state_ptr(h, h->cur), state_ptr(h, 1 - h->cur), reduce);
    if (e != hipSuccess) return hip_fail(h, e, "step launch");
    if (reduce) {
      e = pplbm::launch_finalize(h->partials, n_parts_of(h), log + (size_t)(t - first_logged) * RED_COUNT,
                                 h->fin_tmp, h->stream);
      if (e != hipSuccess) return hip_fail(h, e, "reduction launch");
    }
    h->cur = 1 - h->cur;
    h->steps = t;
  }
  std::vector<double> host((size_t)L.n_log * RED_COUNT);
  double uo[2] = {0.0, 0.0};
  e = hipMemcpyAsync(host.data(), log, host.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "reduction copy");
  if (a->loss == LBM_LOSS_UERR) {
    e = hipMemcpyAsync(uo, at<double>(ws, L.uout), sizeof uo, hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "reduction copy");
  }
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "stream synchronize");

  double Lval;
  double inv_den = 0.0;
  if (a->loss == LBM_LOSS_DRAG) {
    const int64_t W = a->window;
    double sb = 0.0;
    for (int64_t r = 0; r < W; ++r) sb += host[(size_t)r * RED_COUNT + pplbm::RED_BUOY];
    const double p_first = host[pplbm::RED_PPHI];
    const double p_last = host[(size_t)(W - 1) * RED_COUNT + pplbm::RED_PPHI];
    Lval = sb / (double)W - (p_last - p_first) / (double)(W - 1);
  } else {
    if (!(uo[1] > 0.0)) return fail(h, LBM_ERR_INVALID_ARG, "u_target is zero on every fluid node");
    inv_den = 1.0 / uo[1];
    Lval = uo[0] * inv_den;
  }
  if (loss_host) *loss_host = Lval;
  for (int64_t r = 0; r < L.n_log; ++r) {
    lbm_reduction rec;
    fill_record(&host[(size_t)r * RED_COUNT], first_logged + r, &rec);
    int st = fault_status(h, rec);
    if (st != LBM_OK) return st;
  }
  h->adj.ready = true;
  h->adj.cfg = *a;
  h->adj.ws = ws;
  h->adj.ws_bytes = workspace_bytes;
  h->adj.inv_den = inv_den;
  return LBM_OK;
}

int lbm_adjoint_backward(lbm_lattice* h, double* grad_rho0, double* grad_force, double* grad_G) {
  if (!h) return LBM_ERR_INVALID_ARG;
  if (!h->adj.ready) return fail(h, LBM_ERR_STATE, "lbm_adjoint_backward without a matching lbm_adjoint_forward");
  begin_stepping(h);
  const lbm_adjoint_cfg& a = h->adj.cfg;
  const AdjLayout L = adj_layout(&h->cfg, &a);
  char* ws = h->adj.ws;
  const bool fp64 = h->cfg.precision == LBM_FP64;
  const int64_t N = a.n_steps, K = a.checkpoint_every;
  const size_t n = L.n;
  const size_t sbytes = state_bytes_of(&h->cfg);
  const int blocks = pplbm::adj_blocks(h->cfg.nx, h->cfg.ny);
  void* D[2] = {ws + L.D0, ws + L.D1};
  double* R[2] = {at<double>(ws, L.R0), at<double>(ws, L.R1)};
  double* acc = at<double>(ws, L.acc);
  double* traj = at<double>(ws, L.traj);
  hipError_t e = pplbm::launch_zero(acc, (size_t)blocks * 2, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "zero launch");

  pplbm::AdjStepArgs s;
  std::memset(&s, 0, sizeof s);
  s.mask = h->buf.mask;
  s.T = at<double>(ws, L.T);
  s.param_acc = acc;
  s.u_target = a.u_target_dev;
  s.loss_kind = a.loss;
  const double W = (double)a.window;
  int cur = 0;  // D[cur], R[cur] receive step n; D[1 - cur], R[1 - cur] hold step n + 1
  for (int64_t c = L.n_ckpt - 1; c >= 0; --c) {
    const int64_t s0 = c * K, s1 = std::min<int64_t>(s0 + K, N);
    void* A = ws + L.rep0;
    void* B = ws + L.rep1;
    const void* ck = ws + L.ckpt + (size_t)c * L.state_bytes;
    e = hipMemcpyAsync(A, ck, sbytes, hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(B, ck, sbytes, hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "checkpoint copy");
    const bool fused = replay_writes_traj(h);
    for (int64_t t = s0 + 1; t <= s1; ++t) {
      double* slot = traj + (size_t)(t - s0 - 1) * 4 * n;
      if (fused) {
        // the replayed step writes step t's trajectory itself (the last
        // step's populations are not used)
        e = step_between(h, A, B, 0, slot);
        if (e != hipSuccess) return hip_fail(h, e, "replay step launch");
        std::swap(A, B);
        continue;
      }
      e = fp64 ? pplbm::launch_traj<double>(h->prm, A, h->buf.mask, slot, h->stream)
               : pplbm::launch_traj<float>(h->prm, A, h->buf.mask, slot, h->stream);
      if (e != hipSuccess) return hip_fail(h, e, "replay launch");
      if (t < s1) {
        e = step_between(h, A, B, 0);
        if (e != hipSuccess) return hip_fail(h, e, "replay step launch");
        std::swap(A, B);
      }
    }
    for (int64_t t = s1; t > s0; --t) {
      s.traj = traj + (size_t)(t - s0 - 1) * 4 * n;
      s.D_next = D[1 - cur];
      s.R_next = R[1 - cur];
      s.D = D[cur];
      s.R = R[cur];
      s.have_next = t < N ? 1 : 0;
      s.cB = s.cP = s.cU = 0.0;
      if (a.loss == LBM_LOSS_DRAG) {
        if (t > N - a.window) s.cB = 1.0 / W;
        if (t == N - a.window + 1) s.cP = 1.0 / (W - 1.0);
        if (t == N) s.cP = -1.0 / (W - 1.0);
      } else if (t == N) {
        s.cU = h->adj.inv_den;
      }
      e = fp64 ? pplbm::launch_adj_step<double>(h->prm, s, h->stream)
               : pplbm::launch_adj_step<float>(h->prm, s, h->stream);
      if (e != hipSuccess) return hip_fail(h, e, "adjoint step launch");
      cur = 1 - cur;
    }
  }
  if (grad_rho0) {
    s.D_next = D[1 - cur];
    s.R_next = R[1 - cur];
    s.have_next = 1;
    e = fp64 ? pplbm::launch_adj_rho0<double>(h->prm, s, grad_rho0, h->stream)
             : pplbm::launch_adj_rho0<float>(h->prm, s, grad_rho0, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "initial-state gradient launch");
  }
  double* pair = at<double>(ws, L.pair);
  e = pplbm::launch_pair_sum(acc, blocks, pair, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "parameter gradient launch");
  double hp[2];
  e = hipMemcpyAsync(hp, pair, sizeof hp, hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "gradient copy");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "stream synchronize");
  if (grad_G) *grad_G = hp[0];
  if (grad_force) *grad_force = hp[1];
  return LBM_OK;
}

}  // extern "C"
