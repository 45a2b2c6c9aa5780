/* A client of liblbm.so written in plain C (no Python, no torch): it allocates
 * the device buffers with the HIP runtime, steps a small falling-droplet
 * channel in both precisions through the C-ABI of include/pplbm.h, and checks
 * what does not depend on the arithmetic: no faults, the mass of a walled
 * channel conserved, finite read-out fields.  Prints one line per precision
 * and exits non-zero on any failure.  Run by tests/test_gpu_c_client.py. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "pplbm.h"

#define NX 192
#define NY 128
#define STEPS 200
#define EVERY 50

/* Compensated (Kahan) sum: a plain running sum of 24,576 densities drifts by
 * ~1e-13 of the total, more than the FP64 step changes the mass. */
static double ksum(const double* v, int n) {
  double s = 0.0, c = 0.0;
  for (int i = 0; i < n; ++i) {
    const double y = v[i] - c, t = s + y;
    c = (t - s) - y;
    s = t;
  }
  return s;
}

static int fail(const char* what, int rc, const lbm_lattice* h) {
  fprintf(stderr, "lbm_c_client: %s failed (%d): %s\n", what, rc, lbm_last_error(h));
  return 1;
}

#define HIP(call)                                                                 \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      fprintf(stderr, "lbm_c_client: %s: %s\n", #call, hipGetErrorString(e_));   \
      return 1;                                                                   \
    }                                                                             \
  } while (0)

#define LBM(call, h)                                   \
  do {                                                 \
    int rc_ = (call);                                  \
    if (rc_ != LBM_OK) return fail(#call, rc_, (h));   \
  } while (0)

static int run(int32_t precision) {
  /* Carnahan-Starling at 0.7 T_c with eps = 1.895: the coexistence densities of
   * the mechanical-stability condition (Eq. 1) */
  const double rho_g = 0.010692540759551266, rho_l = 0.3583420128243473, T = 0.0660275;
  const double s[9] = {1.0, 1.1, 1.1, 1.0, 1.1, 1.0, 1.1, 1.25, 1.25};
  /* x walls, y periodic; float storage stores deviations from rho_g */
  lbm_config cfg = {NX, NY, 0, 1, precision, LBM_KERNEL_FUSED, precision == LBM_FP32_DEV ? rho_g : 0.0, 16, 0};
  size_t state_bytes = 0, ws_bytes = 0;
  LBM(lbm_state_bytes(&cfg, &state_bytes), NULL);
  LBM(lbm_workspace_bytes(&cfg, &ws_bytes), NULL);

  /* a droplet of radius 20 in the middle of the channel, at rest */
  double* rho0 = malloc(sizeof(double) * NX * NY);
  double* rho = malloc(sizeof(double) * NX * NY);
  if (!rho0 || !rho) return 1;
  for (int y = 0; y < NY; ++y)
    for (int x = 0; x < NX; ++x) {
      const double dx = x - (NX / 2 - 0.5), dy = y - (NY / 2 - 0.5);
      const double r = sqrt(dx * dx + dy * dy);
      rho0[y * NX + x] = 0.5 * (rho_l + rho_g) - 0.5 * (rho_l - rho_g) * tanh(r - 20.0);
    }
  const double mass0 = ksum(rho0, NX * NY);

  void *fa = NULL, *fb = NULL, *ws = NULL, *rho0_dev = NULL, *rho_dev = NULL;
  hipStream_t stream;
  HIP(hipStreamCreate(&stream));
  HIP(hipMalloc(&fa, state_bytes));
  HIP(hipMalloc(&fb, state_bytes));
  HIP(hipMalloc(&ws, ws_bytes));
  HIP(hipMalloc(&rho0_dev, sizeof(double) * NX * NY));
  HIP(hipMalloc(&rho_dev, sizeof(double) * NX * NY));
  HIP(hipMemcpy(rho0_dev, rho0, sizeof(double) * NX * NY, hipMemcpyHostToDevice));

  lbm_buffers buf = {fa, fb, ws, NULL, NULL};
  lbm_lattice* h = NULL;
  LBM(lbm_create(&cfg, &buf, (void*)stream, &h), NULL);
  LBM(lbm_set_eos(h, LBM_EOS_CS, 1.0, 4.0, 1.0, T, 1.0), h);
  LBM(lbm_set_G(h, -1.0), h);
  LBM(lbm_set_relaxation(h, s), h);
  LBM(lbm_set_scheme(h, LBM_SCHEME_IMPROVED, 1.895, NAN, NAN, LBM_Q2_DEFAULT), h);
  LBM(lbm_set_body_force(h, LBM_FORCE_BUOYANT, 0.0, -1e-6), h);
  LBM(lbm_set_phase_densities(h, rho_g, rho_l), h);
  LBM(lbm_set_walls(h, rho_g), h);
  LBM(lbm_init_equilibrium(h, (const double*)rho0_dev, NULL, NULL), h);

  lbm_reduction rec[STEPS / EVERY];
  LBM(lbm_step(h, STEPS, EVERY, rec, STEPS / EVERY), h);
  LBM(lbm_read_fields(h, (double*)rho_dev, NULL, NULL, NULL, NULL, NULL), h);
  HIP(hipStreamSynchronize(stream));
  HIP(hipMemcpy(rho, rho_dev, sizeof(double) * NX * NY, hipMemcpyDeviceToHost));
  int64_t steps = 0;
  LBM(lbm_step_count(h, &steps), h);

  /* FP64: 1e-16 of the mass per step (the closed-form back-transform rounds a
   * node's nine populations the same way every step); float storage: the
   * rounding of the stored values */
  const double tol = precision == LBM_FP64 ? 1e-16 * STEPS : 1e-6;
  int bad = steps != STEPS;
  double worst = 0.0;
  for (int k = 0; k < STEPS / EVERY; ++k) {
    const double e = fabs(rec[k].mass - mass0) / mass0;
    if (e > worst) worst = e;
    bad |= rec[k].faults != 0.0 || rec[k].step != (int64_t)(k + 1) * EVERY;
  }
  for (int i = 0; i < NX * NY; ++i) bad |= !isfinite(rho[i]) || rho[i] <= 0.0;
  const double mass = ksum(rho, NX * NY);
  const double e_read = fabs(mass - mass0) / mass0;
  if (e_read > worst) worst = e_read;
  bad |= worst > tol;
  const double uc = rec[STEPS / EVERY - 1].uc_num / rec[STEPS / EVERY - 1].uc_den;
  printf("{\"precision\": \"%s\", \"steps\": %lld, \"mass_rel_err\": %.3e, \"bar\": %.1e, \"U_c\": %.6e, "
         "\"mass_rel_err_by_record\": [%.3e, %.3e, %.3e, %.3e], \"ok\": %s}\n",
         precision == LBM_FP64 ? "fp64" : "fp32", (long long)steps, worst, tol, uc,
         (rec[0].mass - mass0) / mass0, (rec[1].mass - mass0) / mass0, (rec[2].mass - mass0) / mass0,
         (rec[3].mass - mass0) / mass0, bad ? "false" : "true");

  LBM(lbm_destroy(h), NULL);
  HIP(hipFree(fa));
  HIP(hipFree(fb));
  HIP(hipFree(ws));
  HIP(hipFree(rho0_dev));
  HIP(hipFree(rho_dev));
  HIP(hipStreamDestroy(stream));
  free(rho0);
  free(rho);
  return bad;
}

int main(void) {
  if (lbm_abi_version() != LBM_ABI_VERSION) {
    fprintf(stderr, "lbm_c_client: library ABI %d, header %d\n", lbm_abi_version(), LBM_ABI_VERSION);
    return 1;
  }
  int bad = run(LBM_FP64);
  bad |= run(LBM_FP32_DEV);
  return bad ? 1 : 0;
}
