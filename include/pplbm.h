/*
 * pplbm.h — C-ABI of the MI355X (gfx950) pseudopotential MRT lattice Boltzmann
 * library liblbm.so.
 *
 * Model: R. Huang, J. Huang & Q. Li, "Improved third-order scheme in
 * pseudopotential lattice Boltzmann model for multiphase flows" (2026).
 * One time step is: pull streaming with halfway bounce-back (Eq. 2b), density
 * and momentum (Eq. 3), pseudopotential from the equation of state (Eq. 5
 * inverted), Shan-Chen force (Eq. 4), MRT collision in moment space with the
 * third-order source term (Eq. 2a with Eqs. 6-8 and Eq. 11 or Eqs. 13 + 42).
 *
 * Conventions
 *  - Lattice units dx = dt = c = 1, c_s^2 = 1/3.  D2Q9 velocities
 *    e0..e8 = (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1).
 *  - Arrays are row-major with x fastest.  Scalar fields are [y][x]; vector
 *    fields [2][y][x].  A population array holds rows of planes,
 *    f[y][p][x]: row y is P runs of nx elements, the row's values of the 9
 *    populations (p = i) and, for LBM_FP32_DEV, a tenth run with the row's
 *    reference offsets (below).  Population i of node (x, y) is element
 *    (y * P + i) * nx + x, P = 9 (LBM_FP64) or 10 (LBM_FP32_DEV).
 *  - The stored state is the post-collision field.  A step streams then
 *    collides.  "Macroscopic fields of the current state" are the pre-collision
 *    fields the next step would use.
 *  - Precision LBM_FP64 stores f in double.  LBM_FP32_DEV stores, in float,
 *    each post-collision population relative to the reference density of the
 *    node that will pull it: s_i(x) = f_i(x) - w_i * rhat(x + e_i) (rhat(x)
 *    when x + e_i is solid or beyond a wall), with rhat = rho_ref + c and the
 *    offsets c kept as 16-bit floats in the first half of each row's tenth
 *    run (16-bit element 2 (10 y + 9) nx + x; set from the initial density,
 *    see lbm_rereference; the run's second half is zero).  The stored deviations stay small in
 *    liquid and vapour alike, so their rounding stays small where a uniform
 *    reference would not.  Both precisions compute the step in double (each
 *    population is rounded once when stored) and reduce in double.
 *  - Ownership: the caller allocates and frees every device buffer (the
 *    population arrays, the workspace, the mask, the wall velocities and all
 *    outputs).  The library never allocates or frees device memory; it keeps
 *    pointers and a parameter block.  Pointers named *_dev are device pointers,
 *    *_host are host pointers.
 *  - Streams: every kernel is enqueued on the hipStream_t given to lbm_create.
 *    Functions that return host values synchronise that stream (stated per
 *    function); the others only enqueue work.
 *  - Errors: every function returns LBM_OK (0) or a negative LBM_ERR_* code and
 *    records a message readable with lbm_last_error.  No C++ exception crosses
 *    the ABI.  A handle must not be used from two threads at once.
 */
#ifndef PPLBM_H
#define PPLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 4

enum lbm_status {
  LBM_OK = 0,
  LBM_ERR_INVALID_ARG = -1, /* a size, pointer or parameter is out of range */
  LBM_ERR_HIP = -2,         /* a HIP runtime call failed */
  LBM_ERR_NONFINITE = -3,   /* a reduction found non-finite values */
  LBM_ERR_EOS_DOMAIN = -4,  /* a reduction found rho <= 0 or a negative psi^2 */
  LBM_ERR_UNSUPPORTED = -5, /* the request is valid but not implemented */
  LBM_ERR_STATE = -6        /* call out of order (e.g. step before init) */
};

enum lbm_precision { LBM_FP64 = 0, LBM_FP32_DEV = 1 };
enum lbm_kernel { LBM_KERNEL_FUSED = 0, LBM_KERNEL_TWO_PASS = 1 };
enum lbm_eos { LBM_EOS_VDW = 0, LBM_EOS_CS = 1 };
enum lbm_scheme { LBM_SCHEME_ORIGINAL = 0, LBM_SCHEME_IMPROVED = 1 };
enum lbm_q2 { LBM_Q2_DEFAULT = 0, LBM_Q2_NEG_Q1 = 1, LBM_Q2_NEG_HALF_Q1 = 2 };
enum lbm_force { LBM_FORCE_CONST = 0, LBM_FORCE_BUOYANT = 1 };

/* Lattice description, fixed for the life of a handle. */
typedef struct lbm_config {
  int32_t nx, ny;          /* lattice size, 1 <= nx, ny and 9*nx*ny < 2^31 */
  int32_t periodic_x;      /* 1: periodic in x; 0: bounce-back walls at x = -1/2 and nx - 1/2 */
  int32_t periodic_y;      /* same for y */
  int32_t precision;       /* enum lbm_precision */
  int32_t kernel;          /* enum lbm_kernel: fused single kernel per step or two passes */
  double rho_ref;          /* LBM_FP32_DEV: base of the per-node reference densities (any value
                              near the densities; the offsets are stored relative to it) */
  int32_t log_capacity;    /* reduction records lbm_step may collect in one call (>= 1) */
  int32_t reserved;
} lbm_config;

/* Caller-owned device buffers. */
typedef struct lbm_buffers {
  void* f_a;               /* population array of lbm_state_bytes: [ny][9][nx] double, or
                              [ny][10][nx] float (9 populations + the reference offsets) */
  void* f_b;               /* second population array of the same size (ping-pong) */
  void* workspace;         /* lbm_workspace_bytes() bytes, 256-byte aligned */
  const uint8_t* mask;     /* [ny][nx], 1 = solid node, 0 = fluid; NULL = no solid nodes inside */
  const double* wall_u;    /* [2][ny][nx] velocity of solid nodes (moving walls); NULL = static */
} lbm_buffers;

/* Observables of the pre-collision state of one step, summed over fluid nodes
 * (FP64, fixed-order deterministic reduction). */
typedef struct lbm_reduction {
  double mass;     /* sum rho */
  double mom_x;    /* sum rho u_x (u of Eq. 3, including half the force) */
  double mom_y;
  double wall_x;   /* momentum handed to walls by bounce-back links in this step */
  double wall_y;
  double uc_num;   /* sum rho u_y over nodes with rho > (rho_l + rho_g)/2 (Eq. 47 numerator) */
  double uc_den;   /* sum rho over the same nodes (Eq. 47 denominator) */
  double buoy;     /* sum phi (rho - rho_g) |g|, phi = (rho - rho_g)/(rho_l - rho_g) */
  double pphi;     /* sum phi rho u . g/|g| */
  double faults;   /* nodes with rho <= 0, negative psi^2, or non-finite rho/u */
  int64_t step;    /* index of the step these observables belong to (1 = first step) */
} lbm_reduction;

typedef struct lbm_lattice lbm_lattice;

/* ABI version of the loaded library (LBM_ABI_VERSION). */
int lbm_abi_version(void);

/* Bytes of one population array (f_a or f_b) for this configuration: 9 planes
 * of double, or 10 planes of float (the populations and the reference offsets). */
int lbm_state_bytes(const lbm_config* cfg, size_t* bytes);

/* Bytes of the workspace (reduction partials, reduction log, two-pass
 * pseudopotential field, read-out scratch, the link words of masked
 * lattices).  Pure host computation. */
int lbm_workspace_bytes(const lbm_config* cfg, size_t* bytes);

/* Creates a handle on the current HIP device.  Validates the configuration and
 * the buffer pointers (non-NULL f_a, f_b, workspace), stores them, and
 * installs the default parameters: Carnahan-Starling a = 1, b = 4, R = 1 with
 * T = 0.7 T_c, G = -1, all rates 1, improved scheme with eps = 0, no force,
 * rho_s = rho_g = 0, rho_l = 1.  Enqueues nothing.  *out is NULL on error. */
int lbm_create(const lbm_config* cfg, const lbm_buffers* buf, void* hip_stream, lbm_lattice** out);

/* Bytes of the library-owned workspace of lbm_create_static handles (32 MiB). */
#define LBM_STATIC_WORKSPACE_BYTES ((size_t)32 << 20)

/* lbm_create for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same handle, but its workspace is a library-owned static device array of
 * LBM_STATIC_WORKSPACE_BYTES on the current device instead of a caller
 * buffer.  buf->workspace must be NULL; the caller still owns f_a, f_b, mask,
 * wall_u and every output.  Configurations whose lbm_workspace_bytes exceeds
 * LBM_STATIC_WORKSPACE_BYTES (about 2.8 million nodes) are rejected with
 * LBM_ERR_INVALID_ARG.  Allocates nothing: the array exists on every device
 * the library runs on until the process ends; its address is resolved the
 * first time this is called on a device.  Every handle made this way on one
 * device shares that array, and a call leaves its contents for the next: calls
 * on such handles that overlap in time (other host threads, other streams)
 * race.  Results are those of lbm_create's handle. */
int lbm_create_static(const lbm_config* cfg, const lbm_buffers* buf, void* hip_stream, lbm_lattice** out);

/* Releases the handle (not the caller's buffers).  NULL is accepted. */
int lbm_destroy(lbm_lattice* h);

/* Message of the last error on this handle ("" if none); with h = NULL, that
 * of the last call made without a handle (lbm_create, lbm_create_static,
 * lbm_state_bytes, lbm_workspace_bytes, lbm_adjoint_workspace_bytes; each
 * clears it first).  The pointer stays valid until the next such call. */
const char* lbm_last_error(const lbm_lattice* h);

/* Equation of state p_EOS(rho).  kind LBM_EOS_VDW: Eq. (43),
 * p = k_eos (rho R T/(1 - b rho) - a rho^2).  LBM_EOS_CS: Carnahan-Starling,
 * p = k_eos (rho R T (1 + eta + eta^2 - eta^3)/(1 - eta)^3 - a rho^2), eta = b rho/4.
 * The pseudopotential is psi = sqrt(2 (rho/3 - p_EOS)) (Eq. 5 with G_eos = -1). */
int lbm_set_eos(lbm_lattice* h, int32_t kind, double a, double b, double R, double T, double k_eos);

/* Interaction strength G of Eq. (4); it also enters G psi^2 in Q_m.  G = -1 is
 * the paper's model. */
int lbm_set_G(lbm_lattice* h, double G);

/* Diagonal collision matrix of Eq. (6), s[0..8] =
 * (s_0, s_e, s_eps, s_j, s_q, s_j, s_q, s_p, s_p); each in [0, 2]. */
int lbm_set_relaxation(lbm_lattice* h, const double* s_host);

/* Source term.  scheme LBM_SCHEME_ORIGINAL: Eq. (11).  LBM_SCHEME_IMPROVED:
 * Eq. (13) with Q_{m,4}, Q_{m,6} from Eq. (42).  k1, k2 NaN mean -eps/16
 * (Sec. 3).  q2_policy LBM_Q2_DEFAULT gives -Q_{m,1} (original) or
 * -Q_{m,1}/2 (improved, Sec. 2.2). */
int lbm_set_scheme(lbm_lattice* h, int32_t scheme, double eps, double k1, double k2, int32_t q2_policy);

/* External force.  LBM_FORCE_CONST: F_ext = (fx, fy) (the driving force of
 * Sec. 2.1).  LBM_FORCE_BUOYANT: F_ext = (rho - rho_g)(fx, fy) with (fx, fy)
 * the gravity vector (Sec. 3.3). */
int lbm_set_body_force(lbm_lattice* h, int32_t mode, double fx, double fy);

/* Coexistence densities used by the buoyant force and the observables
 * (0 < rho_g < rho_l). */
int lbm_set_phase_densities(lbm_lattice* h, double rho_g, double rho_l);

/* Virtual density of solid nodes: their pseudopotential is psi(rho_s) (the
 * virtual-density wall of Sec. 3). */
int lbm_set_walls(lbm_lattice* h, double rho_s);

/* fbar := M^-1 m^eq(rho0, u0) (Eq. 7) at every node and resets the step
 * counter.  rho0_dev: [ny][nx] double, device; ux0_dev, uy0_dev: [ny][nx]
 * double or NULL (= 0).  Enqueues one kernel. */
int lbm_init_equilibrium(lbm_lattice* h, const double* rho0_dev, const double* ux0_dev, const double* uy0_dev);

/* Advances n >= 0 steps.  If reduce_every > 0, the observables of every step
 * whose index is a multiple of reduce_every are recorded (at most
 * cfg.log_capacity per call, else LBM_ERR_INVALID_ARG before any work).  If
 * out_host is non-NULL, min(records, n_out) records are copied to it and the
 * stream is synchronised; a record with faults > 0 then makes the call return
 * LBM_ERR_EOS_DOMAIN or LBM_ERR_NONFINITE after the copy.  With out_host NULL
 * the call only enqueues kernels on the handle's stream (no allocation, copy,
 * memset or synchronisation), so a caller may capture it into a HIP graph; the
 * handle's step counter (and with it the steps that reduce and re-reference)
 * advances when the call is made, not when the graph replays, and an even n
 * leaves the state in the array it started from. */
int lbm_step(lbm_lattice* h, int64_t n, int32_t reduce_every, lbm_reduction* out_host, int64_t n_out);

/* Launch tuning of the fused strip kernels (unmasked lattices, and masked
 * ones on the masked strip march): rows each wavefront marches through
 * (1 <= rows <= 4096; 0 restores the default chosen from the lattice size and
 * precision).  The tile kernel does not use it.
 * The state does not depend on it; reductions may differ in the last bits,
 * since their partial sums are grouped by run. */
int lbm_set_rows_per_wave(lbm_lattice* h, int32_t rows);

/* Kernel of the fused step on lattices with a solid mask or moving walls (of
 * any width with float storage; double storage: widths that are a multiple of
 * 64, or lattices whose two population arrays exceed 256 MB): 1 (default) the
 * masked strip march (wavefronts march aligned 64-column strips, the last one
 * partial where the width is not a multiple of 64, bounce-back chosen per link from a 16-bit
 * link word per node that the library writes into the workspace before the
 * first step), 0 the tile kernel (one node per thread, psi of a tile in LDS).
 * Both compute the same node arithmetic (float storage: the same state
 * bitwise; double storage: to a few ulp, where the compiler contracts a
 * product and a sum differently).  Also resets the rows per wave to the
 * default.  on not 0 or 1: LBM_ERR_INVALID_ARG. */
int lbm_set_masked_strips(lbm_lattice* h, int32_t on);

/* Steps taken since lbm_init_equilibrium / lbm_set_state. */
int lbm_step_count(const lbm_lattice* h, int64_t* steps);

/* Pre-collision fields of the current state (what the next step uses):
 * rho, u of Eq. (3), the interaction force of Eq. (4), psi.  All outputs are
 * [ny][nx] double device arrays and may be NULL; values at solid nodes are 0
 * (psi: psi(rho_s)).  Enqueues two kernels. */
int lbm_read_fields(lbm_lattice* h, double* rho_dev, double* ux_dev, double* uy_dev, double* fintx_dev,
                    double* finty_dev, double* psi_dev);

/* Observables of the current state (those the next step would record).
 * Synchronises the stream.  Returns LBM_ERR_EOS_DOMAIN / LBM_ERR_NONFINITE
 * when faults > 0 (out is still filled). */
int lbm_reduce(lbm_lattice* h, lbm_reduction* out_host);

/* Device pointer of the population array that holds the current state. */
int lbm_state_ptr(const lbm_lattice* h, void** f_dev);

/* Checkpoint / resume: copy the current state (populations, and for
 * LBM_FP32_DEV the reference offsets) to / from a caller buffer of
 * lbm_state_bytes (device, enqueued device-to-device copy).  lbm_set_state
 * also sets the step counter. */
int lbm_get_state(lbm_lattice* h, void* dst_dev);
int lbm_set_state(lbm_lattice* h, const void* src_dev, int64_t step);

/* LBM_FP32_DEV: make every node's reference density its current density (the
 * sum of its post-collision populations) and re-express the stored
 * populations against it (one more rounding each); for long runs in which
 * the density moves far from where it started.  No-op for LBM_FP64.  Enqueues
 * three kernels; invalidates a recorded adjoint forward pass. */
int lbm_rereference(lbm_lattice* h);

/* LBM_FP32_DEV: lbm_step re-references (as lbm_rereference, after the step,
 * so the step's reductions are unaffected) after every step whose count is a
 * multiple of k; k = 0 never.  Default 1000: without it the references of a
 * moving interface go stale and the rounding of the stored deviations
 * accumulates over long runs.  The adjoint's forward pass and replay do not
 * re-reference.  No effect for LBM_FP64.  k < 0: LBM_ERR_INVALID_ARG. */
int lbm_set_rereference_every(lbm_lattice* h, int64_t k);

/* ---------------------------------------------------------------------------
 * Discrete adjoint (reverse-mode gradients of a loss of a run).
 *
 * A run is fbar^0 = f^eq(rho0, 0) (Eq. 7 at rest) followed by n_steps steps.
 * The observables of step n are those of its pre-collision state (see
 * lbm_reduction).  Losses:
 *  LBM_LOSS_DRAG  time-averaged droplet drag over the last W steps (the
 *                 falling droplet of Sec. 3.3; the paper defines no drag
 *                 formula, this one is the buoyant weight minus the droplet
 *                 region's momentum rate):
 *                   L = (1/W) sum_{n=N-W+1..N} buoy(n) - (pphi(N) - pphi(N-W+1)) / (W - 1)
 *  LBM_LOSS_UERR  relative squared velocity error of step N (the error norm
 *                 of Sec. 3.1 without the root):
 *                   L = sum_fluid (u_x - u_target)^2 / sum_fluid u_target^2
 * Gradients are those of the discrete run (the adjoint of every step's
 * streaming, bounce-back, pseudopotential stencil and collision), with respect
 * to the initial density field, the magnitude |F_ext| of the body force or
 * gravity (direction held fixed) and the interaction strength G.  They are
 * computed in double for both precisions; for LBM_FP32_DEV they are those of
 * the run as stored (the linearisation point is the FP32 trajectory) and the
 * per-step adjoint scratch (of the pulled populations, of psi and of the
 * stencil sums) is stored in float.
 * Memory: the forward pass saves fbar every checkpoint_every steps; the
 * backward pass replays each segment from its checkpoint, keeping
 * rho - rho_ref, j and psi of every step of the segment (32 bytes per node and
 * step), then runs the reverse steps.  Static solid nodes (mask) are
 * supported, moving walls (wall_u) are not (LBM_ERR_UNSUPPORTED).
 * ------------------------------------------------------------------------- */

enum lbm_loss { LBM_LOSS_DRAG = 0, LBM_LOSS_UERR = 1 };

typedef struct lbm_adjoint_cfg {
  int64_t n_steps;               /* N >= 1 */
  int64_t window;                /* LBM_LOSS_DRAG: W, 2 <= W <= N (ignored otherwise) */
  int32_t loss;                  /* enum lbm_loss */
  int32_t checkpoint_every;      /* K >= 1: steps between saved states */
  const double* u_target_dev;    /* LBM_LOSS_UERR: [ny][nx] double, device (ignored otherwise) */
} lbm_adjoint_cfg;

/* Bytes of the adjoint workspace for this lattice and run:
 * ceil(N/K) + 2 population arrays, min(K, N) * 4 * nx * ny doubles of
 * trajectory, 18 * nx * ny values of the storage type and 5 * nx * ny doubles
 * of adjoint fields (one more double for LBM_LOSS_UERR), plus small reduction
 * buffers.
 * Pure host computation. */
int lbm_adjoint_workspace_bytes(const lbm_config* cfg, const lbm_adjoint_cfg* a, size_t* bytes);

/* Forward pass: initialises the lattice at rest with density rho0_dev
 * ([ny][nx] double, device), runs a->n_steps steps (the handle then holds the
 * state after step N, as after lbm_step), saves the checkpoints into
 * workspace_dev (caller-owned, 256-byte aligned, >= lbm_adjoint_workspace_bytes)
 * and returns the loss in *loss_host.  Keeps a and the workspace pointer for
 * lbm_adjoint_backward; the caller must keep both (and u_target_dev) alive and
 * unchanged until then.  Synchronises the stream.  Returns LBM_ERR_EOS_DOMAIN /
 * LBM_ERR_NONFINITE if a step in the loss window recorded faults (the loss is
 * still written). */
int lbm_adjoint_forward(lbm_lattice* h, const lbm_adjoint_cfg* a, const double* rho0_dev, void* workspace_dev,
                        size_t workspace_bytes, double* loss_host);

/* Reverse pass of the last lbm_adjoint_forward on this handle (LBM_ERR_STATE
 * if there is none, or if a parameter setter was called since).  Writes
 * dL/drho0 to grad_rho0_dev ([ny][nx] double, device; 0 at solid nodes) and
 * dL/d|F_ext|, dL/dG to the host doubles; any output may be NULL.  Does not
 * change the lattice state; may be called again.  Synchronises the stream. */
int lbm_adjoint_backward(lbm_lattice* h, double* grad_rho0_dev, double* grad_force_host, double* grad_G_host);

#ifdef __cplusplus
}
#endif

#endif /* PPLBM_H */
