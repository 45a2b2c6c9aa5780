// TEST INFRASTRUCTURE ONLY — the FP64 CPU oracle.
//
// A plain, slow, node-by-node implementation of one time step of the MRT
// pseudopotential lattice Boltzmann model with the third-order source term of
// R. Huang, J. Huang & Q. Li, "Improved third-order scheme in pseudopotential
// lattice Boltzmann model for multiphase flows" (2026).  Only the tests, the
// smoke check and the benchmark's CPU-baseline leg load this library.  It
// shares no code, header, table or helper with the GPU library.
//
// Conventions (all taken from the paper's Sec. 2 and Sec. 3 unless noted):
//   * D2Q9, lattice units dx = dt = c = 1, c_s^2 = 1/3 (Sec. 3 sets dx = dt = 1;
//     c_s^2 = 1/3 is the value implied by the equilibrium moments, Eq. (7)).
//   * Velocities e0..e8 = (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1).
//   * M is the orthogonal Lallemand-Luo matrix (cited in Sec. 2), applied as a
//     dense 9x9 matrix-vector product; M^-1 = M^T D^-1 with D = M M^T.
//   * The stored state is the post-collision field fbar[i][y][x]; one step is
//     pull streaming (Eq. 2b) followed by the collision (Eq. 2a).
//   * Walls are halfway bounce-back (not in the paper; the paper uses a
//     non-equilibrium extrapolation wall that it does not describe).  Solid
//     nodes carry the pseudopotential of a virtual density rho_s (Sec. 3).
//   * psi = sqrt(2 (p_EOS - rho c_s^2) / G_eos) with G_eos = -1 fixed (Eq. 5
//     inverted); the user's G multiplies Eq. (4) and the G psi^2 of Eqs. (11),
//     (13), (42).  With G = -1 this is exactly the paper's model.
//
// The scalar type is a template parameter: T = double for ordinary runs,
// T = std::complex<double> for complex-step derivatives, and T = Rv, a
// reverse-mode scalar that records every operation on a tape, for the
// oracle's own discrete adjoint (the transpose of the same arithmetic,
// obtained mechanically by sweeping the tape backwards).  Every branch tests
// the real part, so all three follow the same path.
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -fopenmp -shared -fPIC
// (no fast-math; IEEE binary64 round-to-nearest everywhere).

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using cplx = std::complex<double>;

inline double re(double v) { return v; }
inline double re(const cplx& v) { return v.real(); }
inline double im(double) { return 0.0; }
inline double im(const cplx& v) { return v.imag(); }
inline bool finite_value(double v) { return std::isfinite(v); }
inline bool finite_value(const cplx& v) { return std::isfinite(v.real()) && std::isfinite(v.imag()); }

// ---------------------------------------------------------------- reverse mode
// The tape: node t was produced from operands a[t], b[t] (-1: none) with
// partial derivatives da[t], db[t].  Inputs are nodes without operands.
struct Tape {
  std::vector<int64_t> a, b;
  std::vector<double> da, db;
  int64_t push(int64_t ia, double pa, int64_t ib, double pb) {
    a.push_back(ia);
    da.push_back(pa);
    b.push_back(ib);
    db.push_back(pb);
    return (int64_t)a.size() - 1;
  }
  // Adjoints of every node given a seed of 1 at `out`.
  std::vector<double> reverse(int64_t out) const {
    std::vector<double> adj(a.size(), 0.0);
    if (out < 0) return adj;
    adj[out] = 1.0;
    for (int64_t t = out; t >= 0; --t) {
      const double g = adj[t];
      if (g == 0.0) continue;
      if (a[t] >= 0) adj[a[t]] += da[t] * g;
      if (b[t] >= 0) adj[b[t]] += db[t] * g;
    }
    return adj;
  }
};

Tape* g_tape = nullptr;  // the tape being recorded (one at a time, single-threaded)

// A value and its tape node (-1 for a constant, which records nothing).
struct Rv {
  double v = 0.0;
  int64_t id = -1;
  Rv() = default;
  Rv(double x) : v(x), id(-1) {}
  static Rv input(double x) {
    Rv r(x);
    r.id = g_tape->push(-1, 0.0, -1, 0.0);
    return r;
  }
  static Rv node(double val, int64_t ia, double pa, int64_t ib, double pb) {
    Rv r(val);
    if (ia >= 0 || ib >= 0) r.id = g_tape->push(ia, pa, ib, pb);
    return r;
  }
  Rv& operator+=(const Rv& o);
  Rv& operator-=(const Rv& o);
};
inline Rv operator+(const Rv& x, const Rv& y) { return Rv::node(x.v + y.v, x.id, 1.0, y.id, 1.0); }
inline Rv operator-(const Rv& x, const Rv& y) { return Rv::node(x.v - y.v, x.id, 1.0, y.id, -1.0); }
inline Rv operator*(const Rv& x, const Rv& y) { return Rv::node(x.v * y.v, x.id, y.v, y.id, x.v); }
inline Rv operator/(const Rv& x, const Rv& y) {
  const double q = x.v / y.v;
  return Rv::node(q, x.id, 1.0 / y.v, y.id, -q / y.v);
}
inline Rv operator-(const Rv& x) { return Rv::node(-x.v, x.id, -1.0, -1, 0.0); }
inline Rv operator+(const Rv& x, double y) { return x + Rv(y); }
inline Rv operator+(double x, const Rv& y) { return Rv(x) + y; }
inline Rv operator-(const Rv& x, double y) { return x - Rv(y); }
inline Rv operator-(double x, const Rv& y) { return Rv(x) - y; }
inline Rv operator*(const Rv& x, double y) { return x * Rv(y); }
inline Rv operator*(double x, const Rv& y) { return Rv(x) * y; }
inline Rv operator/(const Rv& x, double y) { return x / Rv(y); }
inline Rv operator/(double x, const Rv& y) { return Rv(x) / y; }
inline Rv& Rv::operator+=(const Rv& o) { return *this = *this + o; }
inline Rv& Rv::operator-=(const Rv& o) { return *this = *this - o; }
// d sqrt(q) = dq / (2 sqrt(q)); taken as 0 at q = 0 (a clamped pseudopotential).
inline Rv sqrt(const Rv& q) {
  const double r = std::sqrt(q.v);
  return Rv::node(r, q.id, r > 0.0 ? 0.5 / r : 0.0, -1, 0.0);
}
inline double re(const Rv& v) { return v.v; }
inline bool finite_value(const Rv& v) { return std::isfinite(v.v); }

// D2Q9 lattice (Sec. 2; velocity order as listed in the header comment).
const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
const double WGT[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                       1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

// Orthogonal transformation matrix: rows are the moments
// (rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy).
const double MMAT[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
};

// Interaction weights of Eq. (4): w(1) = 1/3, w(2) = 1/12.  The paper does not
// print them; these are the values that make Eq. (39) hold for both stencils.
const double OMEGA[9] = {0.0,        1.0 / 3.0,  1.0 / 3.0,  1.0 / 3.0, 1.0 / 3.0,
                         1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0};

}  // namespace

extern "C" {

// Mirrored field by field by the Python ctypes binding in oracle/oracle.py.
struct OracleParams {
  int32_t nx, ny;
  int32_t periodic_x, periodic_y;  // 1 = periodic axis, 0 = bounce-back walls at -1/2 and n-1/2
  int32_t eos_kind;                // 0 = van der Waals (Eq. 43), 1 = Carnahan-Starling
  int32_t scheme;                  // 0 = original (Eq. 11), 1 = improved (Eqs. 13, 42)
  int32_t q2_policy;               // 0 = scheme default, 1 = Q2 = -Q1, 2 = Q2 = -Q1/2
  int32_t force_mode;              // 0 = constant force (fx, fy); 1 = buoyant (rho - rho_g)(fx, fy)
  double a, b, R, T, k_eos;        // EOS constants
  double G;                        // interaction strength in Eq. (4)
  double s[9];                     // diagonal of the collision matrix, Eq. (6)
  double eps, k1, k2;              // Eq. (11) and Eq. (42)
  double fx, fy;                   // body force, or gravity vector in buoyant mode
  double rho_g, rho_l;             // coexistence densities (buoyancy, loss weights)
  double rho_s;                    // virtual density of solid nodes
};

// Per-step observables of the pre-collision macroscopic state, summed over
// fluid nodes.
enum {
  RED_MASS = 0,      // sum rho
  RED_MOMX,          // sum (j + F/2)_x = sum rho u_x
  RED_MOMY,          // sum rho u_y
  RED_WALLX,         // momentum handed to walls by bounce-back links, x
  RED_WALLY,         // same, y
  RED_UC_NUM,        // sum rho u_y over nodes with rho > (rho_l + rho_g)/2
  RED_UC_DEN,        // sum rho over the same nodes
  RED_BUOY,          // sum phi (rho - rho_g) |g|,  phi = (rho - rho_g)/(rho_l - rho_g)
  RED_PPHI,          // sum phi rho u . g/|g|
  RED_FAULTS,        // nodes with rho <= 0, negative psi^2, or non-finite values
  RED_COUNT
};

struct OracleLoss {
  int32_t kind;            // 0 = drag window L_D, 1 = velocity error L_u at the last step
  int32_t window;          // L_D: number of final steps averaged (>= 2)
  const double* u_target;  // L_u: target u_x per node (ny*nx), ignored for L_D
};

}  // extern "C"

namespace {

template <class T>
struct Sim {
  const OracleParams& p;
  int nx, ny;
  size_t n;
  const uint8_t* mask;   // 1 = solid, may be null
  const double* wall_u;  // [2][ny][nx] velocity of solid nodes, may be null
  T G, fx, fy;           // the parameters a complex-step run may perturb
  std::vector<T> f;      // post-collision populations f[(i*ny + y)*nx + x]

  // Per-step work arrays (pre-collision state of the current step).
  std::vector<T> fpre, rho, jx, jy, psi, fintx, finty, ftotx, ftoty, ux, uy;
  std::vector<uint8_t> solid;

  Sim(const OracleParams& prm, const uint8_t* m, const double* wu)
      : p(prm), nx(prm.nx), ny(prm.ny), n((size_t)prm.nx * prm.ny), mask(m), wall_u(wu),
        G(prm.G), fx(prm.fx), fy(prm.fy) {
    f.assign(9 * n, T(0));
    fpre.assign(9 * n, T(0));
    rho.assign(n, T(0));
    jx.assign(n, T(0));
    jy.assign(n, T(0));
    psi.assign(n, T(0));
    fintx.assign(n, T(0));
    finty.assign(n, T(0));
    ftotx.assign(n, T(0));
    ftoty.assign(n, T(0));
    ux.assign(n, T(0));
    uy.assign(n, T(0));
    solid.assign(n, 0);
    for (size_t k = 0; k < n; ++k) solid[k] = (mask && mask[k]) ? 1 : 0;
  }

  size_t idx(int x, int y) const { return (size_t)y * nx + x; }
  size_t fidx(int i, int x, int y) const { return ((size_t)i * ny + y) * nx + x; }

  // Resolves a neighbour position.  Returns false when it lies outside the
  // domain across a non-periodic axis (that is, inside an analytic wall).
  bool resolve(int x, int y, int& xo, int& yo) const {
    if (x < 0 || x >= nx) {
      if (!p.periodic_x) return false;
      x = (x % nx + nx) % nx;
    }
    if (y < 0 || y >= ny) {
      if (!p.periodic_y) return false;
      y = (y % ny + ny) % ny;
    }
    xo = x;
    yo = y;
    return true;
  }
  bool is_solid_at(int x, int y) const {
    int xo, yo;
    if (!resolve(x, y, xo, yo)) return true;
    return solid[idx(xo, yo)] != 0;
  }

  // Equation of state.  Van der Waals: Eq. (43).  Carnahan-Starling: the
  // textbook form p = rho R T (1 + eta + eta^2 - eta^3)/(1 - eta)^3 - a rho^2,
  // eta = b rho / 4 (named in Sec. 2 among the usable EOSs).
  T p_eos(const T& r) const {
    if (p.eos_kind == 0) {
      return p.k_eos * (r * p.R * p.T / (1.0 - p.b * r) - p.a * r * r);
    }
    T eta = p.b * r / 4.0;
    T num = 1.0 + eta + eta * eta - eta * eta * eta;
    T den = (1.0 - eta) * (1.0 - eta) * (1.0 - eta);
    return p.k_eos * (r * p.R * p.T * num / den - p.a * r * r);
  }

  // psi = sqrt(2 (p_EOS - rho c_s^2) / (G_eos dx^2)), G_eos = -1 (Eq. 5 solved
  // for psi).  A negative radicand is clamped to zero and counted as a fault.
  T psi_of(const T& r, int& fault) const {
    const double G_eos = -1.0;
    T psi2 = 2.0 * (p_eos(r) - r / 3.0) / G_eos;
    if (re(psi2) < 0.0) {
      fault = 1;
      psi2 = T(0);
    }
    using std::sqrt;
    return sqrt(psi2);
  }

  void init_equilibrium(const T* rho0, const double* ux0, const double* uy0) {
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        size_t k = idx(x, y);
        T r = rho0[k];
        T u = ux0 ? T(ux0[k]) : T(0);
        T v = uy0 ? T(uy0[k]) : T(0);
        T meq[9];
        equilibrium_moments(r, u, v, meq);
        T fb[9];
        from_moments(meq, fb);
        for (int i = 0; i < 9; ++i) f[fidx(i, x, y)] = fb[i];
      }
  }

  // Equilibrium moments, Eq. (7).
  static void equilibrium_moments(const T& r, const T& u, const T& v, T meq[9]) {
    T usq = u * u + v * v;
    meq[0] = r;
    meq[1] = -2.0 * r + 3.0 * r * usq;
    meq[2] = r - 3.0 * r * usq;
    meq[3] = r * u;
    meq[4] = -r * u;
    meq[5] = r * v;
    meq[6] = -r * v;
    meq[7] = r * u * u - r * v * v;
    meq[8] = r * u * v;
  }

  static void to_moments(const T fi[9], T m[9]) {
    for (int k = 0; k < 9; ++k) {
      T acc = T(0);
      for (int i = 0; i < 9; ++i) acc += MMAT[k][i] * fi[i];
      m[k] = acc;
    }
  }

  // f = M^-1 m with M^-1 = M^T D^-1, D_k = sum_i M[k][i]^2.
  static void from_moments(const T m[9], T fi[9]) {
    double D[9];
    for (int k = 0; k < 9; ++k) {
      double d = 0.0;
      for (int i = 0; i < 9; ++i) d += MMAT[k][i] * MMAT[k][i];
      D[k] = d;
    }
    for (int i = 0; i < 9; ++i) {
      T acc = T(0);
      for (int k = 0; k < 9; ++k) acc += MMAT[k][i] * m[k] / D[k];
      fi[i] = acc;
    }
  }

  // Discrete source term Q_m: the original scheme, Eq. (11), or the improved
  // scheme, Eq. (13) with Q_{m,4}, Q_{m,6} from Eq. (42) and Q_{m,2} = -Q_{m,1}/2
  // (the choice stated in Sec. 2.2).  k1 and k2 enter only the second-order
  // moments; eps enters the improved third-order moments.
  void source_moments(const T& Fix, const T& Fiy, const T& ps, const T& u, const T& v, T Q[9]) const {
    const double c = 1.0;
    T den = G * ps * ps * c * c;
    T phixx = Fix * Fix / den;
    T phiyy = Fiy * Fiy / den;
    T phixy = Fix * Fiy / den;
    for (int k = 0; k < 9; ++k) Q[k] = T(0);
    Q[1] = 3.0 * (p.k1 + 2.0 * p.k2) * (phixx + phiyy);
    Q[7] = p.k1 * (phixx - phiyy);
    Q[8] = p.k1 * phixy;
    int q2 = p.q2_policy;
    if (q2 == 0) q2 = (p.scheme == 1) ? 2 : 1;
    Q[2] = (q2 == 1) ? T(-Q[1]) : T(-Q[1] / 2.0);
    if (p.scheme == 1) {
      Q[4] = ((30.0 * p.eps - 15.0) / 16.0 * phixx - (3.0 * p.eps / 8.0) * phiyy) * (u / c);
      Q[6] = ((30.0 * p.eps - 15.0) / 16.0 * phiyy - (3.0 * p.eps / 8.0) * phixx) * (v / c);
    }
  }

  // Collision in moment space, Eq. (2a), with m^eq from Eq. (7) and F_m from
  // Eq. (8).  u is the velocity of Eq. (3) (it includes half the force).
  void collide(const T fi[9], const T& r, const T& u, const T& v, const T& Fx, const T& Fy,
               const T& Fix, const T& Fiy, const T& ps, T fout[9]) const {
    T m[9], meq[9], Fm[9], Q[9], mbar[9];
    to_moments(fi, m);
    equilibrium_moments(r, u, v, meq);
    T Fu = Fx * u + Fy * v;
    Fm[0] = T(0);
    Fm[1] = 6.0 * Fu;
    Fm[2] = -6.0 * Fu;
    Fm[3] = Fx;
    Fm[4] = -Fx;
    Fm[5] = Fy;
    Fm[6] = -Fy;
    Fm[7] = 2.0 * Fx * u - 2.0 * Fy * v;
    Fm[8] = Fx * v + Fy * u;
    source_moments(Fix, Fiy, ps, u, v, Q);
    for (int k = 0; k < 9; ++k)
      mbar[k] = m[k] + Fm[k] - p.s[k] * (m[k] - meq[k] + Fm[k] / 2.0) + p.s[k] * Q[k];
    from_moments(mbar, fout);
  }

  // Pre-collision state of the next step from the stored post-collision field:
  // pull streaming with halfway bounce-back (S1), moments (S2), pseudopotential
  // (S3), forces and velocity (S4).  Fills the work arrays; returns the number
  // of fault nodes.
  int macroscopic(T* red /* RED_COUNT or null */) {
    int faults = 0;
    psi_solid_value = T(0);
    {
      int fl = 0;
      psi_solid_value = psi_of(T(p.rho_s), fl);
    }
#pragma omp parallel for schedule(static) reduction(+ : faults) if (kParallel)
    for (int y = 0; y < ny; ++y) {
      for (int x = 0; x < nx; ++x) {
        size_t k = idx(x, y);
        if (solid[k]) continue;
        // S1: pull streaming, Eq. (2b); halfway bounce-back at solid links.
        for (int i = 0; i < 9; ++i) {
          int xs, ys;
          bool inside = resolve(x - EX[i], y - EY[i], xs, ys);
          if (inside && !solid[idx(xs, ys)]) {
            fpre[fidx(i, x, y)] = f[fidx(i, xs, ys)];
          } else {
            T val = f[fidx(OPP[i], x, y)];
            if (wall_u && inside) {
              // Moving wall: + 2 w_i rho_w (e_i . u_w) / c_s^2, rho_w the local
              // density of the previous step (sum of this node's fbar).
              T rw = T(0);
              for (int q = 0; q < 9; ++q) rw += f[fidx(q, x, y)];
              size_t ks = idx(xs, ys);
              double eu = EX[i] * wall_u[ks] + EY[i] * wall_u[n + ks];
              val += 2.0 * WGT[i] * rw * eu * 3.0;
            }
            fpre[fidx(i, x, y)] = val;
          }
        }
        // S2: density and lattice momentum, Eq. (3).
        T r = T(0), mx = T(0), my = T(0);
        for (int i = 0; i < 9; ++i) {
          T fv = fpre[fidx(i, x, y)];
          r += fv;
          mx += double(EX[i]) * fv;
          my += double(EY[i]) * fv;
        }
        rho[k] = r;
        jx[k] = mx;
        jy[k] = my;
        // S3: pseudopotential of the fluid node.
        int fl = 0;
        if (re(r) <= 0.0) fl = 1;
        psi[k] = psi_of(r, fl);
        faults += fl;
      }
    }
    for (size_t k = 0; k < n; ++k)
      if (solid[k]) psi[k] = psi_solid_value;

    // S4: interaction force, Eq. (4), total force and velocity, Eq. (3).
#pragma omp parallel for schedule(static) if (kParallel)
    for (int y = 0; y < ny; ++y) {
      for (int x = 0; x < nx; ++x) {
        size_t k = idx(x, y);
        if (solid[k]) continue;
        T sx = T(0), sy = T(0);
        for (int i = 1; i < 9; ++i) {
          int xn, yn;
          T pn = resolve(x + EX[i], y + EY[i], xn, yn) ? psi[idx(xn, yn)] : psi_solid_value;
          sx += OMEGA[i] * pn * double(EX[i]);
          sy += OMEGA[i] * pn * double(EY[i]);
        }
        fintx[k] = -G * psi[k] * sx;
        finty[k] = -G * psi[k] * sy;
        T ex, ey;
        if (p.force_mode == 1) {
          ex = (rho[k] - p.rho_g) * fx;
          ey = (rho[k] - p.rho_g) * fy;
        } else {
          ex = fx;
          ey = fy;
        }
        ftotx[k] = fintx[k] + ex;
        ftoty[k] = finty[k] + ey;
        ux[k] = (jx[k] + ftotx[k] / 2.0) / rho[k];
        uy[k] = (jy[k] + ftoty[k] / 2.0) / rho[k];
      }
    }

    if (red) reductions(red, faults);
    return faults;
  }

  void reductions(T* red, int faults) {
    for (int q = 0; q < RED_COUNT; ++q) red[q] = T(0);
    using std::sqrt;
    T gmag = sqrt(fx * fx + fy * fy);
    T ghx = T(0), ghy = T(0);
    if (re(gmag) > 0.0) {
      ghx = fx / gmag;
      ghy = fy / gmag;
    }
    double rho_mid = 0.5 * (p.rho_l + p.rho_g);
    double drho = p.rho_l - p.rho_g;
    int nonfinite = 0;
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        size_t k = idx(x, y);
        if (solid[k]) continue;
        T r = rho[k];
        red[RED_MASS] += r;
        red[RED_MOMX] += r * ux[k];
        red[RED_MOMY] += r * uy[k];
        for (int i = 1; i < 9; ++i) {
          if (!is_solid_at(x - EX[i], y - EY[i])) continue;
          // Bounce-back link: fbar_opp(x) left towards the wall and came back
          // as f_i(x); the wall received -(f_i + fbar_opp) e_i.
          T both = fpre[fidx(i, x, y)] + f[fidx(OPP[i], x, y)];
          red[RED_WALLX] -= double(EX[i]) * both;
          red[RED_WALLY] -= double(EY[i]) * both;
        }
        if (re(r) > rho_mid) {
          red[RED_UC_NUM] += r * uy[k];
          red[RED_UC_DEN] += r;
        }
        T phi = (r - p.rho_g) / drho;
        red[RED_BUOY] += phi * (r - p.rho_g) * gmag;
        red[RED_PPHI] += phi * r * (ux[k] * ghx + uy[k] * ghy);
        if (!finite_value(r) || !finite_value(ux[k]) || !finite_value(uy[k])) nonfinite++;
      }
    red[RED_FAULTS] = T(double(faults + nonfinite));
  }

  // One full step: S1-S4 then the collision S5 and back-transform S6.
  int step(T* red) {
    int faults = macroscopic(red);
    std::vector<T> fnew(f);
#pragma omp parallel for schedule(static) if (kParallel)
    for (int y = 0; y < ny; ++y) {
      for (int x = 0; x < nx; ++x) {
        size_t k = idx(x, y);
        if (solid[k]) continue;
        T fi[9], fo[9];
        for (int i = 0; i < 9; ++i) fi[i] = fpre[fidx(i, x, y)];
        collide(fi, rho[k], ux[k], uy[k], ftotx[k], ftoty[k], fintx[k], finty[k], psi[k], fo);
        for (int i = 0; i < 9; ++i) fnew[fidx(i, x, y)] = fo[i];
      }
    }
    f.swap(fnew);
    return faults;
  }

  T psi_solid_value = T(0);
  // Recording a tape is sequential.
  static constexpr bool kParallel = !std::is_same<T, Rv>::value;
};

// The loss of a run of nsteps from the current state (see oracle_loss).
template <class T>
T run_loss(Sim<T>& s, const OracleLoss* loss, int64_t nsteps) {
  std::vector<T> red(RED_COUNT);
  T L(0.0);
  T p_first(0.0), p_last(0.0);
  for (int64_t t = 1; t <= nsteps; ++t) {
    bool last = (t == nsteps);
    bool in_window = (loss->kind == 0) && (t > nsteps - loss->window);
    if (in_window || (loss->kind == 1 && last)) {
      s.macroscopic(red.data());
      if (loss->kind == 0) {
        L += red[RED_BUOY] / double(loss->window);
        if (t == nsteps - loss->window + 1) p_first = red[RED_PPHI];
        if (last) p_last = red[RED_PPHI];
      } else {
        T num(0.0), den(0.0);
        for (size_t k = 0; k < s.n; ++k) {
          if (s.solid[k]) continue;
          T d = s.ux[k] - loss->u_target[k];
          num += d * d;
          den += loss->u_target[k] * loss->u_target[k];
        }
        L = num / den;
      }
    }
    s.step(nullptr);
  }
  if (loss->kind == 0) L -= (p_last - p_first) / double(loss->window - 1);
  return L;
}

int set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
  return omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

bool params_ok(const OracleParams* p) {
  return p && p->nx > 0 && p->ny > 0 && (long long)p->nx * p->ny < (1LL << 40);
}

}  // namespace

extern "C" {

int oracle_abi_version(void) { return 1; }

int oracle_threads(int nthreads) { return set_threads(nthreads); }

int oracle_red_count(void) { return RED_COUNT; }

// fbar := M^-1 m^eq(rho0, u0) at every node (u pointers may be null = 0).
int oracle_init(const OracleParams* p, const uint8_t* mask, const double* rho0, const double* ux0,
                const double* uy0, double* f_out) {
  if (!params_ok(p) || !rho0 || !f_out) return -1;
  Sim<double> s(*p, mask, nullptr);
  s.init_equilibrium(rho0, ux0, uy0);
  std::memcpy(f_out, s.f.data(), sizeof(double) * 9 * s.n);
  return 0;
}

// Advances fbar (in place) by nsteps.  red_out, if non-null, receives
// RED_COUNT doubles per step (pre-collision observables of that step).
// Returns the total fault count over the run (>= 0) or -1 on bad arguments.
long long oracle_step(const OracleParams* p, const uint8_t* mask, const double* wall_u, double* f,
                      int64_t nsteps, double* red_out, int nthreads) {
  if (!params_ok(p) || !f || nsteps < 0) return -1;
  set_threads(nthreads);
  Sim<double> s(*p, mask, wall_u);
  std::memcpy(s.f.data(), f, sizeof(double) * 9 * s.n);
  long long faults = 0;
  for (int64_t t = 0; t < nsteps; ++t) faults += s.step(red_out ? red_out + t * RED_COUNT : nullptr);
  std::memcpy(f, s.f.data(), sizeof(double) * 9 * s.n);
  return faults;
}

// Pre-collision macroscopic fields that the next step would use (S1-S4 on
// the stored fbar): rho, u (Eq. 3), F_int (Eq. 4), psi, and pulled f.
// Any output pointer may be null.  red (RED_COUNT doubles) may be null.
int oracle_macros(const OracleParams* p, const uint8_t* mask, const double* wall_u, const double* f,
                  double* rho, double* ux, double* uy, double* fintx, double* finty, double* psi,
                  double* fpre, double* red, int nthreads) {
  if (!params_ok(p) || !f) return -1;
  set_threads(nthreads);
  Sim<double> s(*p, mask, wall_u);
  std::memcpy(s.f.data(), f, sizeof(double) * 9 * s.n);
  int faults = s.macroscopic(red);
  size_t bytes = sizeof(double) * s.n;
  if (rho) std::memcpy(rho, s.rho.data(), bytes);
  if (ux) std::memcpy(ux, s.ux.data(), bytes);
  if (uy) std::memcpy(uy, s.uy.data(), bytes);
  if (fintx) std::memcpy(fintx, s.fintx.data(), bytes);
  if (finty) std::memcpy(finty, s.finty.data(), bytes);
  if (psi) std::memcpy(psi, s.psi.data(), bytes);
  if (fpre) std::memcpy(fpre, s.fpre.data(), 9 * bytes);
  return faults;
}

// Node-level pieces, exposed for unit pins.
void oracle_moments(const double* fi, double* m) { Sim<double>::to_moments(fi, m); }
void oracle_from_moments(const double* m, double* fi) { Sim<double>::from_moments(m, fi); }
void oracle_equilibrium_moments(double r, double u, double v, double* meq) {
  Sim<double>::equilibrium_moments(r, u, v, meq);
}
int oracle_source(const OracleParams* p, double Fix, double Fiy, double psi, double u, double v, double* Q) {
  if (!p) return -1;
  Sim<double> s(*p, nullptr, nullptr);
  s.source_moments(Fix, Fiy, psi, u, v, Q);
  return 0;
}
int oracle_collide(const OracleParams* p, const double* fi, double r, double u, double v, double Fx,
                   double Fy, double Fix, double Fiy, double psi, double* fout) {
  if (!p) return -1;
  Sim<double> s(*p, nullptr, nullptr);
  s.collide(fi, r, u, v, Fx, Fy, Fix, Fiy, psi, fout);
  return 0;
}
double oracle_p_eos(const OracleParams* p, double r) {
  Sim<double> s(*p, nullptr, nullptr);
  return s.p_eos(r);
}
double oracle_psi(const OracleParams* p, double r) {
  Sim<double> s(*p, nullptr, nullptr);
  int fl = 0;
  return s.psi_of(r, fl);
}

// Loss of a run of nsteps from fbar = f^eq(rho0, 0), and optionally its
// complex-step derivative along one input direction:
//   perturb = 0: none;  1: body-force / gravity magnitude (fx, fy) += i h (fx, fy)/|f|;
//   2: G += i h;  3: rho0 += i h v  (v has ny*nx entries).
// Loss kinds (observables of the pre-collision state of each step n = 1..N):
//   L_D = mean_{window} BUOY(n) - (PPHI(N) - PPHI(N-window+1)) / (window - 1)
//   L_u = sum_fluid (u_x(N) - u_target)^2 / sum_fluid u_target^2
// dL = Im L(x + i h v) / h, exact to rounding for analytic steps.
int oracle_loss(const OracleParams* p, const uint8_t* mask, const double* wall_u, const double* rho0,
                int64_t nsteps, const OracleLoss* loss, int32_t perturb, const double* v, double h,
                double* L_out, double* dL_out, int nthreads) {
  if (!params_ok(p) || !rho0 || !loss || nsteps < 1) return -1;
  if (loss->kind == 0 && (loss->window < 2 || loss->window > nsteps)) return -1;
  if (loss->kind == 1 && !loss->u_target) return -1;
  if (perturb == 3 && !v) return -1;
  set_threads(nthreads);
  Sim<cplx> s(*p, mask, wall_u);
  const cplx ih(0.0, h);
  if (perturb == 1) {
    double mag = std::sqrt(p->fx * p->fx + p->fy * p->fy);
    if (mag > 0) {
      s.fx = cplx(p->fx) + ih * (p->fx / mag);
      s.fy = cplx(p->fy) + ih * (p->fy / mag);
    }
  } else if (perturb == 2) {
    s.G = cplx(p->G) + ih;
  }
  std::vector<cplx> r0(s.n);
  for (size_t k = 0; k < s.n; ++k) r0[k] = cplx(rho0[k]) + ((perturb == 3) ? ih * v[k] : cplx(0.0));
  s.init_equilibrium(r0.data(), nullptr, nullptr);

  cplx L = run_loss(s, loss, nsteps);
  if (L_out) *L_out = re(L);
  if (dL_out) *dL_out = (perturb != 0 && h != 0.0) ? im(L) / h : 0.0;
  return 0;
}

// The oracle's own discrete adjoint of the same loss: the run is recorded on a
// tape in the reverse-mode scalar and swept backwards once.  Outputs (any may
// be null): the loss, dL/drho0 at every node (ny*nx; 0 at solid nodes), dL/dG
// and dL/d|F| (body force or gravity magnitude, direction fixed).  Runs on one
// thread; the tape holds roughly 1,000 entries (32 bytes each) per node and
// step, so it is meant for small lattices.  Returns -1 on bad arguments, -2
// when the tape would exceed max_tape entries.
int oracle_adjoint(const OracleParams* p, const uint8_t* mask, const double* wall_u, const double* rho0,
                   int64_t nsteps, const OracleLoss* loss, int64_t max_tape, double* L_out, double* grad_rho0,
                   double* dG_out, double* dF_out) {
  if (!params_ok(p) || !rho0 || !loss || nsteps < 1) return -1;
  if (loss->kind == 0 && (loss->window < 2 || loss->window > nsteps)) return -1;
  if (loss->kind == 1 && !loss->u_target) return -1;
  const size_t n = (size_t)p->nx * p->ny;
  if ((double)n * (double)nsteps * 1000.0 > (double)max_tape) return -2;
  Tape tape;
  g_tape = &tape;
  Sim<Rv> s(*p, mask, wall_u);
  s.G = Rv::input(p->G);
  const double mag = std::sqrt(p->fx * p->fx + p->fy * p->fy);
  Rv F = Rv::input(mag);
  if (mag > 0.0) {
    s.fx = F * (p->fx / mag);
    s.fy = F * (p->fy / mag);
  }
  std::vector<Rv> r0(n);
  for (size_t k = 0; k < n; ++k) r0[k] = Rv::input(rho0[k]);
  s.init_equilibrium(r0.data(), nullptr, nullptr);
  Rv L = run_loss(s, loss, nsteps);
  g_tape = nullptr;
  std::vector<double> adj = tape.reverse(L.id);
  if (L_out) *L_out = L.v;
  if (grad_rho0)
    for (size_t k = 0; k < n; ++k) grad_rho0[k] = s.solid[k] ? 0.0 : adj[r0[k].id];
  if (dG_out) *dG_out = adj[s.G.id];
  if (dF_out) *dF_out = adj[F.id];
  return 0;
}

}  // extern "C"
