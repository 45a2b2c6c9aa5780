// Node-level device arithmetic of one D2Q9 pseudopotential MRT step.
//
// Arithmetic convention: the step works on deviations d_i = f_i - w_i R with
// a uniform R (rho_ref; 0 for double storage, so d_i = f_i).  Since
// M (w_i R) = R (1, -2, 1, 0, 0, 0, 0, 0, 0), the collision acts on deviation
// moments with m^eq shifted by the same vector; all other terms are unchanged.
// Float storage pulls deviations from a per-node density R + c instead; the
// same identity moves their moments to the uniform R (rho + c, e - 2c,
// eps + c), and the collision's output is again relative to R.
//
// Storage convention: double storage keeps d_i.  Float storage keeps each
// post-collision population relative to the reference density of the node
// that will pull it: s_i(x) = fbar_i(x) - w_i rhat(x + e_i), or - w_i rhat(x)
// when x + e_i is solid or beyond a wall (the population then returns to x by
// bounce-back).  The per-node reference density rhat = R + c has its offset c
// held in a tenth plane of the population array (the initial density, unless
// re-referenced; see ref_plane).  A pull at x therefore adds the same w_i c(x) to
// every population it gathers, and the store at x subtracts the offsets of
// its 8 neighbours.  The stored values stay small in liquid and vapour alike
// (at an interface they are of the order of the density step between two
// neighbours), so the one rounding per stored population is small.
//
// Arithmetic is double for both storage types: loads are widened, the step is
// computed in double and each population is rounded once when stored.  In
// float arithmetic the per-step force increment (e.g. 1e-7 against a momentum
// of 1e-3) keeps only ~10 significant bits, and its rounding, identical from
// step to step near a steady state, biases the flow (and the 1/6, 1/9 of the
// inverse transform scale mass and momentum by a fixed factor per step).  On
// gfx950 a double FMA issues at the same rate as an unpacked float FMA, so the
// wider type costs registers, not throughput.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_params.h"

namespace pplbm {

// D2Q9 velocities in the order (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1).
__host__ __device__ constexpr int ex(int i) { return (i == 1 || i == 5 || i == 8) ? 1 : (i == 3 || i == 6 || i == 7) ? -1 : 0; }
__host__ __device__ constexpr int ey(int i) { return (i == 2 || i == 5 || i == 6) ? 1 : (i == 4 || i == 7 || i == 8) ? -1 : 0; }
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : (i <= 4 ? ((i + 1) % 4) + 1 : ((i - 3) % 4) + 5); }
__host__ __device__ constexpr double wgt(int i) { return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0); }

static_assert(opp(1) == 3 && opp(2) == 4 && opp(3) == 1 && opp(4) == 2, "opposites");
static_assert(opp(5) == 7 && opp(6) == 8 && opp(7) == 5 && opp(8) == 6, "opposites");

// 1/a to within about one ulp: the hardware reciprocal estimate refined by two
// Newton-Raphson steps (e <- 1 - a r, r <- r + r e).
__host__ __device__ inline double recip(double a) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(a);
  double e = __builtin_fma(-a, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-a, r, 1.0);
  return __builtin_fma(r, e, r);
#else
  return 1.0 / a;
#endif
}

// sqrt(q), 0 for q <= 0: the reciprocal-square-root estimate y, then one
// coupled Newton step on g = q y ~ sqrt(q) and h = y/2 ~ 1/(2 sqrt(q))
// (Goldschmidt's iteration) and a final residual correction g + (q - g^2) h.
__host__ __device__ inline double root(double q) {
#if defined(__HIP_DEVICE_COMPILE__)
  double qq = q > 0.0 ? q : 1.0;
  double y = __builtin_amdgcn_rsq(qq);
  double g = qq * y;
  double h = 0.5 * y;
  double r = __builtin_fma(-g, h, 0.5);
  g = __builtin_fma(g, r, g);
  h = __builtin_fma(h, r, h);
  r = __builtin_fma(-g, g, qq);
  g = __builtin_fma(r, h, g);
  return q > 0.0 ? g : 0.0;
#else
  return q > 0.0 ? sqrt(q) : 0.0;
#endif
}

// psi^2 = 2 (rho c_s^2 - p_EOS), evaluated in double (the difference cancels
// strongly in the vapour).  Van der Waals (Eq. 43) or Carnahan-Starling.
__device__ __host__ inline double psi_squared(const StepParams& p, double r) {
  double pe;
  if (p.eos_kind == 0) {
    pe = p.k_eos * (r * p.RT * recip(1.0 - p.b * r) - p.a * r * r);
  } else {
    double eta = 0.25 * p.b * r;
    double om = 1.0 - eta;
    pe = p.k_eos * (r * p.RT * (1.0 + eta * (1.0 + eta * (1.0 - eta))) * recip(om * om * om) - p.a * r * r);
  }
  return 2.0 * (r * (1.0 / 3.0) - pe);
}

// Returns psi; a negative psi^2 is clamped to 0 and reported through `bad`.
__host__ __device__ inline double psi_of(const StepParams& p, double r, bool& bad) {
  double q = psi_squared(p, r);
  bad = !(q >= 0.0) || !(r > 0.0);
  return root(q);
}

// Whether lattice position (x, y) (possibly one step outside the box) is
// solid, and its wrapped in-box index when it is inside.
__host__ __device__ inline bool solid_at(const StepParams& p, const uint8_t* __restrict__ mask, int x, int y,
                                int& xw, int& yw, bool& inside) {
  inside = true;
  if (x < 0) {
    if (!p.periodic_x) inside = false;
    x += p.nx;
  } else if (x >= p.nx) {
    if (!p.periodic_x) inside = false;
    x -= p.nx;
  }
  if (y < 0) {
    if (!p.periodic_y) inside = false;
    y += p.ny;
  } else if (y >= p.ny) {
    if (!p.periodic_y) inside = false;
    y -= p.ny;
  }
  xw = x;
  yw = y;
  if (!inside) return true;
  return mask ? (mask[(unsigned)y * (unsigned)p.nx + (unsigned)x] != 0) : false;  // nx ny < 2^31
}

// Layout of a population array: rows of planes.  Row y holds P runs of nx
// elements, P = state_planes<S>(): the row's values of the 9 populations
// (f[y][i][x]: population i of node (x, y) is element (y P + i) nx + x), and
// for float storage a tenth run whose first half holds the row's reference
// offsets c as 16-bit floats (second half zero; any representable c serves as
// a reference, 11 significant bits keep the stored deviations small, and the
// offsets cost 2 bytes per node to read).  A wavefront pulling one row thus
// reads the 9 populations from three neighbouring P-run blocks instead of 9
// planes a whole lattice apart (measured: 5% faster for float storage).
template <class S>
__host__ __device__ constexpr int state_planes() {
  return sizeof(S) == 4 ? 10 : 9;
}

// Element index of population i of node (x, y).  Lattices have 9 nx ny <
// 2^31 (checked at creation), so with at most 10 planes every element index
// fits 32 bits; 32-bit products are cheaper than 64-bit ones.
template <class S>
__host__ __device__ inline size_t pop_at(int nx, int y, int i, int x) {
  return (size_t)(((unsigned)y * (unsigned)state_planes<S>() + (unsigned)i) * (unsigned)nx + (unsigned)x);
}

typedef _Float16 RefT;

// Index, in 16-bit units of a float population array, of node (x, y)'s
// reference offset.
__host__ __device__ inline size_t ref_at(int nx, int y, int x) {
  // the float element index of the row's tenth run fits 32 bits; doubled, it may not
  return 2 * (size_t)(((unsigned)y * 10u + 9u) * (unsigned)nx) + (size_t)x;
}

template <class S>
__host__ __device__ inline RefT* ref_base(S* f) {
  return (RefT*)f;
}
template <class S>
__host__ __device__ inline const RefT* ref_base(const S* f) {
  return (const RefT*)f;
}

// The reference offset c of node (x, y) (0 for double storage).
template <class S>
__host__ __device__ inline double ref_offset(const S* __restrict__ f, int nx, int y, int x) {
  if constexpr (sizeof(S) == 4) {
    return (double)ref_base(f)[ref_at(nx, y, x)];
  } else {
    return 0.0;
  }
}

// Stored value of a post-collision deviation d whose puller has offset c.
template <class S>
__host__ __device__ inline S store_value(double d, double w, double c) {
  if constexpr (sizeof(S) == 4) {
    return (S)(d - w * c);
  } else {
    return (S)d;
  }
}

// Reference offsets (float storage) of the nodes that pull node (x, y)'s
// post-collision populations: c[i] = c(x + e_i), or c(x) when x + e_i is solid
// or beyond a wall.  Zero for double storage.
template <class S>
__host__ __device__ inline void dest_refs(const StepParams& p, const S* __restrict__ f, const uint8_t* __restrict__ mask,
                                          int x, int y, double c[9]) {
  if constexpr (sizeof(S) == 4) {
    const double c_self = ref_offset<S>(f, p.nx, y, x);
    c[0] = c_self;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      int xd, yd;
      bool inside;
      const bool sol = solid_at(p, mask, x + ex(i), y + ey(i), xd, yd, inside);
      c[i] = sol ? c_self : ref_offset<S>(f, p.nx, yd, xd);
    }
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) c[i] = 0.0;
  }
}

// Pull streaming (Eq. 2b) with halfway bounce-back: d[i] = dbar_i(x - e_i), or
// dbar_opp(i)(x) (+ the moving-wall term) when x - e_i is solid, as
// deviations from w_i (R + c) with c the node's reference offset (returned;
// 0 for double storage).  When `wall` is non-null, accumulates the momentum
// handed to the walls.  When `cdst` is non-null (float storage), also
// returns the offsets of the nodes that will pull this node's post-collision
// populations (the node x + e_i is the source of direction opp(i)).  When
// `sbits` is non-null, bit i of it is set when x - e_i is solid or beyond a
// wall.
template <class S>
__host__ __device__ inline void pull_node(const StepParams& p, const S* __restrict__ f, const uint8_t* __restrict__ mask,
                                          const double* __restrict__ wall_u, int x, int y, double d[9], double* wall,
                                          double& c, float* cdst = nullptr, unsigned* sbits = nullptr) {
  const int nx = p.nx;
  const size_t plane = (size_t)nx * p.ny;  // of the wall-velocity field
  // every population gathered here was stored relative to this node's offset
  const double c_self = ref_offset<S>(f, nx, y, x);
  c = c_self;
  bool sol[9], ins[9];
  int xs[9], ys[9];
  sol[0] = false;
  ins[0] = true;
  xs[0] = x;
  ys[0] = y;
#pragma unroll
  for (int i = 1; i < 9; ++i) sol[i] = solid_at(p, mask, x - ex(i), y - ey(i), xs[i], ys[i], ins[i]);
  if (sbits) {
    unsigned b = 0;
#pragma unroll
    for (int i = 1; i < 9; ++i) b |= sol[i] ? (1u << i) : 0u;
    *sbits = b;
  }
  // offsets of the pullers: every position is in the box (solid_at wraps
  // even across a non-periodic edge), so the loads are unconditional
  double cd[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) cd[i] = 0.0;
  if constexpr (sizeof(S) == 4) {
    if (cdst) {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const int j = opp(i);
        const double cj = ref_offset<S>(f, nx, ys[j], xs[j]);
        cd[i] = sol[j] ? c_self : cj;
        cdst[i] = (float)cd[i];
      }
    }
  }
  d[0] = (double)f[pop_at<S>(nx, y, 0, x)];
  double rho_w = 0.0;
  bool have_rho_w = false;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    // the pulled population, or the node's own opposite one across a wall
    const size_t src = sol[i] ? pop_at<S>(nx, y, opp(i), x) : pop_at<S>(nx, ys[i], i, xs[i]);
    double v = (double)f[src];
    if (sol[i]) {
      double mw = 0.0;
      if (wall_u && ins[i]) {
        if (!have_rho_w) {
          // density of this node at the previous step: sum of its own fbar
          if constexpr (sizeof(S) == 4) {
            if (!cdst) {
#pragma unroll
              for (int q = 0; q < 9; ++q)
                cd[q] = sol[opp(q)] ? c_self : ref_offset<S>(f, nx, ys[opp(q)], xs[opp(q)]);
            }
          }
          double s = 0.0;
#pragma unroll
          for (int q = 0; q < 9; ++q) s += (double)f[pop_at<S>(nx, y, q, x)] + wgt(q) * cd[q];
          rho_w = p.rho_ref + s;
          have_rho_w = true;
        }
        const size_t ks = (unsigned)ys[i] * (unsigned)nx + (unsigned)xs[i];
        double eu = ex(i) * wall_u[ks] + ey(i) * wall_u[plane + ks];
        mw = 6.0 * wgt(i) * rho_w * eu;
        v += mw;
      }
      if (wall) {
        // the wall received -(f_i + fbar_opp) e_i, with f_i = fbar_opp + mw
        double fi = v + wgt(i) * (p.rho_ref + c_self);
        double both = 2.0 * fi - mw;
        wall[0] -= ex(i) * both;
        wall[1] -= ey(i) * both;
      }
    }
    d[i] = v;
  }
}

// Density deviation (from R) and lattice momentum of pulled deviations d
// relative to R + c, in a fixed summation order.
template <class S>
__host__ __device__ inline void node_sums(const double d[9], double c, double& drho, double& jx, double& jy) {
  double s13 = d[1] - d[3];
  double s24 = d[2] - d[4];
  double c57 = d[5] - d[7];
  double c86 = d[8] - d[6];
  jx = s13 + (c57 + c86);
  jy = s24 + (c57 - c86);
  drho = d[0] + ((d[1] + d[3]) + (d[2] + d[4])) + ((d[5] + d[7]) + (d[6] + d[8]));
  if constexpr (sizeof(S) == 4) drho += c;
}

// Stencil sums S = sum_k w_k psi(x + e_k) e_k of Eq. (4) (w = 1/3, 1/12),
// taken pairwise so that fields invariant along x or y give exactly zero.
__host__ __device__ inline void stencil_sums(double pE, double pN, double pW, double pS, double pNE, double pNW,
                                             double pSW, double pSE, double& Sx, double& Sy) {
  const double w1 = 1.0 / 3.0, w2 = 1.0 / 12.0;
  Sx = w1 * (pE - pW) + w2 * ((pNE - pNW) + (pSE - pSW));
  Sy = w1 * (pN - pS) + w2 * ((pNE - pSE) + (pNW - pSW));
}

struct NodeMacro {
  double ux, uy, Fx, Fy;
};

// Collision in moment space (Eq. 2a) with Eqs. (6)-(8), the force of Eq. (4)
// and the source term of Eq. (11) or Eqs. (13) + (42).  d holds the pulled
// deviations on entry (from R + c; float storage only, c = 0 otherwise) and
// the post-collision deviations from R on exit.
//   drho  : rho - rho_ref, jx, jy : momentum
//   psi_c : psi of this node, Sx, Sy : stencil sums of its neighbours
// Q_m uses P_ab = F_a F_b / (G psi^2) = G S_a S_b, which is the same quantity
// without the division (F_int = -G psi S).
// Returns u (Eq. 3) and the total force.  The caller rounds d to the storage
// type once per population.
template <class S>
__host__ __device__ inline NodeMacro collide_node(const StepParams& p, double d[9], double c, double drho, double jx,
                                                  double jy, double psi_c, double Sx, double Sy) {
  NodeMacro out;
  const double G = p.G;
  const double Fix = -G * psi_c * Sx;
  const double Fiy = -G * psi_c * Sy;
  const double r = p.rho_ref + drho;
  double Fx, Fy;
  if (p.force_mode == 1) {
    double dr = r - p.rho_g;
    Fx = Fix + dr * p.fx;
    Fy = Fiy + dr * p.fy;
  } else {
    Fx = Fix + p.fx;
    Fy = Fiy + p.fy;
  }
  const double inv_r = recip(r);
  const double ux = (jx + 0.5 * Fx) * inv_r;
  const double uy = (jy + 0.5 * Fy) * inv_r;

  // moments of the pulled deviations
  const double d0 = d[0];
  const double s4 = (d[1] + d[3]) + (d[2] + d[4]);
  const double s8 = (d[5] + d[7]) + (d[6] + d[8]);
  const double s13 = d[1] - d[3];
  const double s24 = d[2] - d[4];
  const double c57 = d[5] - d[7];
  const double c86 = d[8] - d[6];
  double m1 = 2.0 * s8 - s4 - 4.0 * d0;
  double m2 = 4.0 * d0 - 2.0 * s4 + s8;
  if constexpr (sizeof(S) == 4) {
    // from the node's reference R + c to R: M (w_i c) = c (1, -2, 1, 0, ...)
    m1 -= 2.0 * c;
    m2 += c;
  }
  const double m4 = (c57 + c86) - 2.0 * s13;
  const double m6 = (c57 - c86) - 2.0 * s24;
  const double m7 = (d[1] + d[3]) - (d[2] + d[4]);
  const double m8 = (d[5] + d[7]) - (d[6] + d[8]);

  // equilibrium deviation moments (Eq. 7 minus rho_ref (1,-2,1,0,...))
  const double ru2 = r * (ux * ux + uy * uy);
  const double e1 = -2.0 * drho + 3.0 * ru2;
  const double e2 = drho - 3.0 * ru2;
  const double e4 = -r * ux;
  const double e6 = -r * uy;
  const double e7 = r * (ux * ux - uy * uy);
  const double e8 = r * ux * uy;

  // force moments (Eq. 8)
  const double Fu = Fx * ux + Fy * uy;
  const double F1 = 6.0 * Fu;
  const double F7 = 2.0 * (Fx * ux - Fy * uy);
  const double F8 = Fx * uy + Fy * ux;

  // source moments
  const double Pxx = G * Sx * Sx;
  const double Pyy = G * Sy * Sy;
  const double Pxy = G * Sx * Sy;
  const double Q1 = p.q1 * (Pxx + Pyy);
  const double Q2 = p.q2 * Q1;
  const double Q4 = (p.qa * Pxx - p.qb * Pyy) * ux;
  const double Q6 = (p.qa * Pyy - p.qb * Pxx) * uy;
  const double Q7 = p.q7 * (Pxx - Pyy);
  const double Q8 = p.q7 * Pxy;

  // relaxation: mbar = m - s (m - meq) + (1 - s/2) F_m + s Q
  const double b1 = m1 - p.s[1] * (m1 - e1) + p.h[1] * F1 + p.s[1] * Q1;
  const double b2 = m2 - p.s[2] * (m2 - e2) - p.h[2] * F1 + p.s[2] * Q2;
  const double b4 = m4 - p.s[4] * (m4 - e4) - p.h[4] * Fx + p.s[4] * Q4;
  const double b6 = m6 - p.s[6] * (m6 - e6) - p.h[6] * Fy + p.s[6] * Q6;
  const double b7 = m7 - p.s[7] * (m7 - e7) + p.h[7] * F7 + p.s[7] * Q7;
  const double b8 = m8 - p.s[8] * (m8 - e8) + p.h[8] * F8 + p.s[8] * Q8;
  const double b3 = jx + Fx;  // conserved moment plus the force, for any s_j
  const double b5 = jy + Fy;

  // back-transform fbar = M^T D^-1 mbar
  const double A = drho * (1.0 / 9.0);
  const double B = b1 * (1.0 / 36.0);
  const double C = b2 * (1.0 / 36.0);
  const double base1 = A - B - 2.0 * C;
  const double base2 = A + 2.0 * B + C;
  const double X = (b3 - b4) * (1.0 / 6.0);
  const double Y = (b5 - b6) * (1.0 / 6.0);
  const double Pp = b3 * (1.0 / 6.0) + b4 * (1.0 / 12.0);
  const double Qp = b5 * (1.0 / 6.0) + b6 * (1.0 / 12.0);
  const double m7q = b7 * 0.25;
  const double m8q = b8 * 0.25;
  d[0] = A - 4.0 * B + 4.0 * C;
  d[1] = base1 + X + m7q;
  d[3] = base1 - X + m7q;
  d[2] = base1 + Y - m7q;
  d[4] = base1 - Y - m7q;
  d[5] = base2 + Pp + Qp + m8q;
  d[6] = base2 - Pp + Qp - m8q;
  d[7] = base2 - Pp - Qp + m8q;
  d[8] = base2 + Pp - Qp - m8q;

  out.ux = ux;
  out.uy = uy;
  out.Fx = Fx;
  out.Fy = Fy;
  return out;
}

// Adds this fluid node's observables to acc[RED_COUNT].
__host__ __device__ inline void accumulate_node(const StepParams& p, double* acc, double rho, double jx, double jy,
                                                const NodeMacro& m, bool bad) {
  double px = jx + 0.5 * m.Fx;  // rho u_x
  double py = jy + 0.5 * m.Fy;
  acc[RED_MASS] += rho;
  acc[RED_MOMX] += px;
  acc[RED_MOMY] += py;
  if (rho > 0.5 * (p.rho_l + p.rho_g)) {
    acc[RED_UC_NUM] += py;
    acc[RED_UC_DEN] += rho;
  }
  double dr = rho - p.rho_g;
  double phi = dr / (p.rho_l - p.rho_g);
  acc[RED_BUOY] += phi * dr * p.gmag;
  acc[RED_PPHI] += phi * (px * p.ghx + py * p.ghy);
  bool finite = isfinite(rho) && isfinite(m.ux) && isfinite(m.uy);
  if (bad || !finite) acc[RED_FAULTS] += 1.0;
}

}  // namespace pplbm
