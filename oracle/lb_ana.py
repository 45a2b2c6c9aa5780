"""TEST INFRASTRUCTURE ONLY: "LB-ana", the steady velocity profile that the
lattice Boltzmann equation itself predicts for two-phase Poiseuille flow.

Sec. 2.1 of R. Huang, J. Huang & Q. Li, "Improved third-order scheme in
pseudopotential lattice Boltzmann model for multiphase flows" (2026) reduces
the steady LB equation of a flow that varies only across the channel to a few
relations per lattice line; Sec. 3.1 solves them for a given converged density
profile ("LB-ana") and compares with the simulation and with the continuum
profile of Eq. (44).  This module does the same, in plain numpy, sharing no code
with the GPU library or the oracle's C++ step:

* grid-aligned channel (Sec. 2.1.1): per node i across the channel the
  unknowns are the flow velocity u^i and the two population differences that
  stream across it, a^i = f_{5-8}^i (towards +i) and b^i = f_{6-7}^i (towards
  -i).  Eq. (19) ties them to u at every node; Eqs. (17) and (18) give their
  post-collision values, which streaming hands to the neighbouring node.
  Eliminating a and b in the interior gives Eq. (22).  At the two nodes beside
  the walls halfway bounce-back returns the post-collision value of the other
  difference with its sign flipped (a population leaving towards the wall
  comes back along the opposite direction), which closes the system;
* grid-oblique channel (Sec. 2.1.2): the same with the 45-degree lines as
  nodes, Eq. (35) in place of Eq. (19), Eqs. (33), (34) for the streamed
  differences f_{1-4} (towards +i) and f_{2-3} (towards -i), the 7-point force
  stencil of Eq. (39), and the third-order source Q_{m,4+6} of Eq. (40);
* the continuum profile of Eq. (44) integrated with the same density;
* the error norm of Sec. 3.1 (Err, the equation after Eq. (44));
* the fit of K in Eq. (40): the K whose oblique LB-ana profile is closest
  (in Err) to the continuum profile, i.e. that suppresses the spurious
  velocity oscillations.

Conventions: lattice units (dx = dt = c = 1, c_s^2 = 1/3), G = -1, so
psi_hat = psi (Eq. 5).  Every function takes the fluid nodes (or lines) of
one channel cross-section, index 0 next to the lower wall.
"""
from __future__ import annotations

import math
from typing import Callable, Optional

import numpy as np

ORIGINAL, IMPROVED = 0, 1


def force_aligned(psi: np.ndarray, psi_wall: float) -> np.ndarray:
    """Eq. (39), grid-aligned: F^i = psi^i (psi^{i+1} - psi^{i-1}) / 2, with the
    solid nodes beyond the walls at psi_wall."""
    p = np.concatenate(([psi_wall], psi, [psi_wall]))
    return psi * (p[2:] - p[:-2]) / 2.0


def force_oblique(psi: np.ndarray, psi_wall: float) -> np.ndarray:
    """Eq. (39), grid-oblique: F_x^i = psi^i (psi^{i+2} + 4 psi^{i+1} - 4 psi^{i-1} - psi^{i-2}) / 12,
    with two solid lines beyond each wall at psi_wall."""
    p = np.concatenate(([psi_wall] * 2, psi, [psi_wall] * 2))
    return psi * (p[4:] + 4.0 * p[3:-1] - 4.0 * p[1:-3] - p[:-4]) / 12.0


def _solve(n, rho_u, post_a, post_b, mom, rhs_mom, rhs_post):
    """Assembles and solves the 3n system of one channel cross-section.

    Unknown vector [u (n), a (n), b (n)].  For each line i the callables give
    the u-coefficients of: mom(i) in  a + b - mom(i) u = rhs_mom, and
    post_a(i), post_b(i) in the post-collision values
        A^i = (1 - s_p) a^i + post_a(i) u^i + rhs_post,
        B^i = (1 - s_p) b^i + post_b(i) u^i + rhs_post
    (rho_u carries 1 - s_p).  Streaming: a^{i+1} = A^i, b^{i-1} = B^i;
    bounce-back: a^0 = -B^0, b^{n-1} = -A^{n-1}."""
    keep = rho_u
    M = np.zeros((3 * n, 3 * n))
    r = np.zeros(3 * n)
    U, A, B = 0, n, 2 * n
    for i in range(n):
        # momentum of line i
        M[i, A + i] = 1.0
        M[i, B + i] = 1.0
        M[i, U + i] = -mom(i)
        r[i] = rhs_mom
        # a^i: streamed from line i-1, or bounced back at the lower wall
        k = n + i
        M[k, A + i] = 1.0
        if i > 0:
            M[k, A + i - 1] = -keep
            M[k, U + i - 1] = -post_a(i - 1)
            r[k] = rhs_post
        else:
            M[k, B + 0] = keep
            M[k, U + 0] = post_b(0)
            r[k] = -rhs_post
        # b^i: streamed from line i+1, or bounced back at the upper wall
        k = 2 * n + i
        M[k, B + i] = 1.0
        if i < n - 1:
            M[k, B + i + 1] = -keep
            M[k, U + i + 1] = -post_b(i + 1)
            r[k] = rhs_post
        else:
            M[k, A + n - 1] = keep
            M[k, U + n - 1] = post_a(n - 1)
            r[k] = -rhs_post
    x = np.linalg.solve(M, r)
    return x[:n], x[n:2 * n], x[2 * n:]


def aligned_profile(rho, psi, psi_wall, F_dri, s_p, s_q, eps, scheme=IMPROVED, q6: Optional[np.ndarray] = None):
    """LB-ana of the grid-aligned channel: the flow velocity at each fluid node.

    rho, psi: density and pseudopotential of the fluid nodes across the channel
    (index 0 beside the lower wall); psi_wall: pseudopotential of the solid
    nodes; F_dri: driving force along the flow.  The third-order source is
    Q_{m,6} = q6^i u^i: Eq. (28), q6 = (3 eps / 8) F^2 / psi^2, for the
    improved scheme, 0 for the original one (or the given coefficients).
    Returns (u, a, b, F) with a = f_{5-8}, b = f_{6-7} and F the interaction
    force of Eq. (39)."""
    rho = np.asarray(rho, float)
    psi = np.asarray(psi, float)
    n = len(rho)
    F = force_aligned(psi, psi_wall)
    if q6 is None:
        q6 = (3.0 * eps / 8.0) * F * F / (psi * psi) if scheme == IMPROVED else np.zeros(n)
    c2 = (6.0 * s_q - 4.0 * s_p - s_p * s_q) / (12.0 * s_q)   # Eqs. (17), (18)
    c3 = (4.0 + s_q) / (6.0 * s_q)                          # Eq. (19)
    h = (2.0 - s_p) / 4.0
    u, a, b = _solve(
        n, 1.0 - s_p,
        post_a=lambda i: s_p / 6.0 * rho[i] + h * F[i] + s_p / 6.0 * q6[i],   # Eq. (17)
        post_b=lambda i: s_p / 6.0 * rho[i] - h * F[i] + s_p / 6.0 * q6[i],   # Eq. (18)
        mom=lambda i: rho[i] / 3.0 + q6[i] / 3.0,                              # Eq. (19)
        rhs_mom=-c3 * F_dri, rhs_post=c2 * F_dri)
    return u, a, b, F


def aligned_fd_residual(rho, F, q6, u, F_dri, nu):
    """Residual of Eq. (22) at the interior nodes 1 .. n-2."""
    Q = q6 * u
    i = np.arange(1, len(rho) - 1)
    return ((rho[i - 1] + 1.5 * F[i - 1]) * u[i - 1] + (rho[i + 1] - 1.5 * F[i + 1]) * u[i + 1] - 2.0 * rho[i] * u[i]
            + (Q[i - 1] + Q[i + 1] - 2.0 * Q[i]) + F_dri / nu)


def oblique_profile(rho, psi, psi_wall, F_dri, s_p, s_q, K: Optional[float] = None):
    """LB-ana of the grid-oblique channel: the flow velocity u_beta on each fluid
    45-degree line (index 0 beside the lower wall, increasing with x - y).

    K: the factor of Eq. (40), Q_{m,4+6} = -2 K F_x^2/psi^2 (u_x + u_y) =
    -2 sqrt(2) K F_x^2/psi^2 u_beta; None for the original scheme
    (Q_{m,4+6} = 0).  The improved scheme has K = (24 eps - 15)/32.
    Returns (u_beta, a, b, F_x) with a = f_{1-4}, b = f_{2-3}."""
    rho = np.asarray(rho, float)
    psi = np.asarray(psi, float)
    n = len(rho)
    Fx = force_oblique(psi, psi_wall)
    r2 = math.sqrt(2.0)
    q46 = np.zeros(n) if K is None else -2.0 * r2 * K * Fx * Fx / (psi * psi)
    c2 = (3.0 * s_q - s_p - s_p * s_q) / (6.0 * s_q)   # Eqs. (33), (34)
    c3 = (1.0 + s_q) / (3.0 * s_q)                    # Eq. (35)
    h = (2.0 - s_p) / 2.0
    Fa = r2 * Fx                                      # F_alpha = sqrt(2) F_x
    u, a, b = _solve(
        n, 1.0 - s_p,
        post_a=lambda i: r2 * s_p / 3.0 * rho[i] + h * Fa[i] - s_p / 6.0 * q46[i],    # Eq. (33)
        post_b=lambda i: r2 * s_p / 3.0 * rho[i] - h * Fa[i] - s_p / 6.0 * q46[i],    # Eq. (34)
        mom=lambda i: r2 * 2.0 / 3.0 * rho[i] - q46[i] / 3.0,                          # Eq. (35)
        rhs_mom=-r2 * c3 * F_dri, rhs_post=r2 * c2 * F_dri)
    return u, a, b, Fx


def theory_profile(rho, F_dri, nu, spacing=1.0, refine=200):
    """Eq. (44), (rho nu u')' = -F_dri, integrated across the channel with the
    node densities rho (linear between nodes, constant from the outermost node
    to its wall), no slip at the two walls half a spacing beyond the outermost
    nodes.  Returns u at the nodes."""
    rho = np.asarray(rho, float)
    n = len(rho)
    x_nodes = (np.arange(n) + 0.5) * spacing           # walls at 0 and n * spacing
    L = n * spacing
    xs = np.linspace(0.0, L, n * refine + 1)
    r = np.interp(xs, x_nodes, rho)
    # rho nu u' = -F (x - c) + C1; u = int_0^x (-F (s - c) + C1)/(rho nu) ds; C1 from u(L) = 0
    g0 = 1.0 / (r * nu)
    g1 = -F_dri * xs / (r * nu)

    def cumtrapz(y):
        out = np.zeros_like(y)
        out[1:] = np.cumsum(0.5 * (y[1:] + y[:-1]) * np.diff(xs))
        return out

    I0, I1 = cumtrapz(g0), cumtrapz(g1)
    C1 = -I1[-1] / I0[-1]
    u = I1 + C1 * I0
    return np.interp(x_nodes, xs, u)


def err(u, u_ref):
    """The relative error of Sec. 3.1: sqrt(sum (u - u_ref)^2 / sum u_ref^2)."""
    u, u_ref = np.asarray(u, float), np.asarray(u_ref, float)
    return math.sqrt(np.sum((u - u_ref) ** 2) / np.sum(u_ref ** 2))


def golden_min(f: Callable[[float], float], lo: float, hi: float, tol: float = 1e-10) -> float:
    """Minimiser of a unimodal f on [lo, hi] by golden-section search."""
    g = (math.sqrt(5.0) - 1.0) / 2.0
    a, b = lo, hi
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = f(c), f(d)
    while b - a > tol:
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = f(d)
    return 0.5 * (a + b)


def fit_K(rho, psi, psi_wall, F_dri, s_p, s_q, lo=-3.0, hi=3.0):
    """The K of Eq. (40) that makes the oblique LB-ana profile closest to the
    continuum profile of Eq. (44) (normal spacing 1/sqrt 2), i.e. suppresses
    the spurious oscillations.  Returns (K, Err at K)."""
    nu = (1.0 / s_p - 0.5) / 3.0
    ut = theory_profile(rho, F_dri, nu, spacing=1.0 / math.sqrt(2.0))
    f = lambda K: err(oblique_profile(rho, psi, psi_wall, F_dri, s_p, s_q, K)[0], ut)
    K = golden_min(f, lo, hi)
    return K, f(K)
