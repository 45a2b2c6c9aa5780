"""Pins of the oracle's node-level arithmetic against what the paper fixes.

* The transformation matrix applied to the textbook D2Q9 equilibrium
  w_i rho (1 + 3 e.u + 9/2 (e.u)^2 - 3/2 u^2) must give the equilibrium moments
  printed in Eq. (7); applied to Guo's velocity-space force term
  w_i [3 (e_i - u) + 9 (e_i.u) e_i] . F it must give the force moments of Eq. (8).
* Collision invariants of Eq. (2a): density conserved, lattice momentum
  increased by exactly F, the full-relaxation limit returns the equilibrium.
* The improved source term, Eq. (42), reduces to Eq. (28) in the grid-aligned
  configuration and to Eq. (41) in the grid-oblique one; it vanishes with the
  velocity, so at u = 0 the improved and original schemes differ only through
  Q_{m,2} (Sec. 2.2).
"""
import numpy as np
import pytest

from oracle import oracle as O

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def textbook_feq(r, u, v):
    eu = EX * u + EY * v
    return W * r * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * (u * u + v * v))


def guo_force(u, v, Fx, Fy):
    eu = EX * u + EY * v
    return W * ((3 * (EX - u) + 9 * eu * EX) * Fx + (3 * (EY - v) + 9 * eu * EY) * Fy)


def paper_meq(r, u, v):
    # Eq. (7), c = 1
    q = u * u + v * v
    return np.array([r, -2 * r + 3 * r * q, r - 3 * r * q, r * u, -r * u, r * v, -r * v, r * (u * u - v * v), r * u * v])


def paper_Fm(u, v, Fx, Fy):
    # Eq. (8), c = 1
    Fu = Fx * u + Fy * v
    return np.array([0, 6 * Fu, -6 * Fu, Fx, -Fx, Fy, -Fy, 2 * Fx * u - 2 * Fy * v, Fx * v + Fy * u])


def params(**kw):
    base = dict(nx=1, ny=1, eos_kind=O.EOS_CS, T=0.07, eps=1.895)
    base.update(kw)
    return O.Params(**base)


RNG = np.random.default_rng(1234)
SAMPLES = [(RNG.uniform(0.01, 8.0), RNG.uniform(-0.2, 0.2), RNG.uniform(-0.2, 0.2)) for _ in range(20)]


def matrix():
    return np.stack([O.moments(np.eye(9)[i]) for i in range(9)], axis=1)


def test_matrix_is_orthogonal_with_lallemand_luo_norms():
    M = matrix()
    G = M @ M.T
    assert np.array_equal(G, np.diag([9.0, 36, 36, 6, 12, 6, 12, 4, 4]))
    # rows are integer vectors
    assert np.array_equal(M, np.round(M))


@pytest.mark.parametrize("r,u,v", SAMPLES)
def test_moments_of_textbook_equilibrium_are_eq7(r, u, v):
    m = O.moments(textbook_feq(r, u, v))
    np.testing.assert_allclose(m, paper_meq(r, u, v), rtol=0, atol=1e-14 * max(1.0, r))
    np.testing.assert_allclose(O.equilibrium_moments(r, u, v), m, rtol=0, atol=1e-14 * max(1.0, r))


@pytest.mark.parametrize("r,u,v", SAMPLES[:8])
def test_moments_of_guo_force_are_eq8(r, u, v):
    Fx, Fy = RNG.uniform(-1e-2, 1e-2, 2)
    np.testing.assert_allclose(O.moments(guo_force(u, v, Fx, Fy)), paper_Fm(u, v, Fx, Fy), rtol=0, atol=1e-16)


def test_moment_round_trip_and_inverse():
    M = matrix()
    Minv = np.linalg.inv(M)
    for _ in range(50):
        f = RNG.uniform(-1, 1, 9)
        back = O.from_moments(O.moments(f))
        np.testing.assert_allclose(back, f, rtol=0, atol=4 * np.finfo(float).eps)
        m = RNG.uniform(-1, 1, 9)
        np.testing.assert_allclose(O.from_moments(m), Minv @ m, rtol=0, atol=8 * np.finfo(float).eps)


def test_collision_force_term_is_eq8_when_nothing_relaxes():
    # s = 0: mbar = m + F_m, so M (fbar - f) recovers F_m of Eq. (8), while
    # velocity-space Guo forcing is its preimage.
    p = params(s=(0.0,) * 9, eps=0.0)
    for r, u, v in SAMPLES[:6]:
        f = textbook_feq(r, u, v) + RNG.uniform(-1e-3, 1e-3, 9)
        Fx, Fy = RNG.uniform(-1e-3, 1e-3, 2)
        out = O.collide(p, f, r, u, v, Fx, Fy, 0.0, 0.0, 1.0)
        tol = 8 * np.finfo(float).eps * max(1.0, r)  # rounding of fbar - f at the scale of f
        np.testing.assert_allclose(O.moments(out - f), paper_Fm(u, v, Fx, Fy), rtol=0, atol=4 * tol)
        np.testing.assert_allclose(out - f, guo_force(u, v, Fx, Fy), rtol=0, atol=tol)


def test_collision_conserves_mass_and_adds_force_to_momentum():
    for r, u0, v0 in SAMPLES[:10]:
        s = tuple(RNG.uniform(0.5, 1.9, 9))
        p = params(s=s, eps=1.7, scheme=O.SCHEME_IMPROVED)
        f = textbook_feq(r, u0, v0) + RNG.uniform(-1e-3, 1e-3, 9) * r
        Fx, Fy = RNG.uniform(-1e-3, 1e-3, 2)
        Fix, Fiy = 0.7 * Fx, 0.4 * Fy
        jx, jy = EX @ f, EY @ f
        rr = f.sum()
        u, v = (jx + Fx / 2) / rr, (jy + Fy / 2) / rr
        out = O.collide(p, f, rr, u, v, Fx, Fy, Fix, Fiy, 0.3)
        assert abs(out.sum() - rr) <= 1e-15 * 9 * max(1, rr)
        assert abs(EX @ out - (jx + Fx)) <= 1e-16 * 9 * max(1, rr)
        assert abs(EY @ out - (jy + Fy)) <= 1e-16 * 9 * max(1, rr)


def test_full_relaxation_without_force_returns_equilibrium():
    p = params(s=(1.0,) * 9, eps=0.0)
    for r, u, v in SAMPLES[:6]:
        f = textbook_feq(r, u, v) + RNG.uniform(-1e-3, 1e-3, 9) * np.array([0, 1, -1, 1, -1, 1, -1, 1, -1])
        rr = f.sum()
        uu, vv = EX @ f / rr, EY @ f / rr
        out = O.collide(p, f, rr, uu, vv, 0.0, 0.0, 0.0, 0.0, 1.0)
        np.testing.assert_allclose(out, textbook_feq(rr, uu, vv), rtol=0, atol=1e-15 * max(1, rr))


@pytest.mark.parametrize("eps", [0.0, 1.0, 1.895, 2.0])
def test_improved_source_reduces_to_eq28_grid_aligned(eps):
    # Grid-aligned case of Sec. 2.1.1: interface normal x, flow along y,
    # F_int,y = 0, u_x = 0.  Eq. (28): Q_{m,6} = (3 eps / 8) F^2 / psi_hat^2 u_y,
    # with psi_hat = sqrt(-G) psi and G = -1.
    p = params(eps=eps, scheme=O.SCHEME_IMPROVED)
    for _ in range(10):
        Fx, psi, v = RNG.uniform(-1e-2, 1e-2), RNG.uniform(0.05, 1.0), RNG.uniform(-0.1, 0.1)
        Q = O.source(p, Fx, 0.0, psi, 0.0, v)
        np.testing.assert_allclose(Q[6], 3 * eps / 8 * Fx * Fx / psi ** 2 * v, rtol=1e-14, atol=1e-300)
        assert Q[4] == 0.0 and Q[0] == Q[3] == Q[5] == 0.0


@pytest.mark.parametrize("eps", [0.0, 1.0, 1.895, 2.0])
def test_improved_source_reduces_to_eq41_grid_oblique(eps):
    # Grid-oblique case of Sec. 2.1.2: F_int,x = -F_int,y, u_x = u_y.
    # Eq. (41): Q_{m,4} = (15 - 24 eps)/16 F_x^2/psi_hat^2 u_x, and likewise Q_{m,6}.
    p = params(eps=eps, scheme=O.SCHEME_IMPROVED)
    for _ in range(10):
        F, psi, u = RNG.uniform(-1e-2, 1e-2), RNG.uniform(0.05, 1.0), RNG.uniform(-0.1, 0.1)
        Q = O.source(p, F, -F, psi, u, u)
        want = (15 - 24 * eps) / 16 * F * F / psi ** 2 * u
        np.testing.assert_allclose(Q[4], want, rtol=1e-13, atol=1e-300)
        np.testing.assert_allclose(Q[6], want, rtol=1e-13, atol=1e-300)
        # Eq. (40): Q_{m,4+6} = -2 K F_x^2/psi_hat^2 (u_x + u_y), K = (24 eps - 15)/32
        K = (24 * eps - 15) / 32
        np.testing.assert_allclose(Q[4] + Q[6], -2 * K * F * F / psi ** 2 * (2 * u), rtol=1e-13, atol=1e-300)


def test_schemes_share_second_order_terms_and_differ_in_q2():
    # Eq. (13) keeps Q_{m,1}, Q_{m,7}, Q_{m,8} of Eq. (11); Sec. 2.2 sets Q_{m,2} = -Q_{m,1}/2
    # where the original sets -Q_{m,1} (Sec. 2).
    po = params(eps=1.3, scheme=O.SCHEME_ORIGINAL)
    pi = params(eps=1.3, scheme=O.SCHEME_IMPROVED)
    for _ in range(10):
        Fx, Fy, psi, u, v = RNG.uniform(-1e-2, 1e-2), RNG.uniform(-1e-2, 1e-2), RNG.uniform(0.05, 1), \
            RNG.uniform(-0.1, 0.1), RNG.uniform(-0.1, 0.1)
        Qo, Qi = O.source(po, Fx, Fy, psi, u, v), O.source(pi, Fx, Fy, psi, u, v)
        for k in (0, 1, 3, 5, 7, 8):
            assert Qo[k] == Qi[k]
        assert Qo[2] == -Qo[1]
        assert Qi[2] == -Qi[1] / 2
        assert Qo[4] == Qo[6] == 0.0
        # eps = -8 (k1 + k2) with k1 = k2 = -eps/16 (Sec. 2, Sec. 3): the trace term
        # Q_{m,1} = 3 (k1 + 2 k2) |F|^2 / (G psi^2) = (9 eps / 16) |F|^2 / psi_hat^2.
        np.testing.assert_allclose(Qo[1], 9 * 1.3 / 16 * (Fx * Fx + Fy * Fy) / psi ** 2, rtol=1e-14)


def test_improved_equals_original_at_rest_with_same_q2_policy():
    # Sec. 2.2: the improved terms vanish at u = 0, so with one Q_{m,2} choice the
    # two schemes collide a resting node bitwise identically; with each scheme's
    # own Q_{m,2} they differ exactly by s_eps * Q_{m,1}/2 along moment 2.
    s = (1.0, 1.25, 1.25, 1.0, 9 / 7, 1.0, 9 / 7, 1.25, 1.25)
    M = matrix()
    for q2 in (O.Q2_NEG_Q1, O.Q2_NEG_HALF_Q1):
        po = params(s=s, eps=1.895, scheme=O.SCHEME_ORIGINAL, q2_policy=q2)
        pi = params(s=s, eps=1.895, scheme=O.SCHEME_IMPROVED, q2_policy=q2)
        for r, _, _ in SAMPLES[:8]:
            f = textbook_feq(r, 0, 0) + RNG.uniform(-1e-3, 1e-3, 9) * r
            Fix, Fiy = RNG.uniform(-1e-3, 1e-3, 2)
            a = O.collide(po, f, r, 0.0, 0.0, Fix, Fiy, Fix, Fiy, 0.4)
            b = O.collide(pi, f, r, 0.0, 0.0, Fix, Fiy, Fix, Fiy, 0.4)
            assert np.array_equal(a, b)
    po = params(s=s, eps=1.895, scheme=O.SCHEME_ORIGINAL)
    pi = params(s=s, eps=1.895, scheme=O.SCHEME_IMPROVED)
    r = 0.3
    f = textbook_feq(r, 0, 0)
    Fix, Fiy = 2e-3, -1e-3
    a = O.collide(po, f, r, 0.0, 0.0, Fix, Fiy, Fix, Fiy, 0.4)
    b = O.collide(pi, f, r, 0.0, 0.0, Fix, Fiy, Fix, Fiy, 0.4)
    Q1 = O.source(po, Fix, Fiy, 0.4, 0, 0)[1]
    want = s[2] * (Q1 / 2) * M[2] / 36.0
    np.testing.assert_allclose(b - a, want, rtol=1e-9, atol=1e-18)
    tol = 4 * np.finfo(float).eps * r  # rounding at the scale of f
    assert abs((b - a).sum()) < tol and abs(EX @ (b - a)) < tol and abs(EY @ (b - a)) < tol


def source_tensor(Q):
    """The second-order source elements as the symmetric tensor that Eq. (10)
    differentiates: [[Q1/6 + Q7/2, Q8], [Q8, Q1/6 - Q7/2]] (c = 1)."""
    return np.array([[Q[1] / 6 + Q[7] / 2, Q[8]], [Q[8], Q[1] / 6 - Q[7] / 2]])


@pytest.mark.parametrize("scheme", [O.SCHEME_ORIGINAL, O.SCHEME_IMPROVED])
@pytest.mark.parametrize("k1,k2", [(None, None), (-0.07, 0.02), (0.05, -0.11)])
def test_second_order_source_rotates_with_the_force(scheme, k1, k2):
    # Eq. (10): Q_{m,1}, Q_{m,7}, Q_{m,8} enter the pressure tensor through one
    # symmetric tensor built from F_int alone, so it must rotate with the force:
    # T(R F) = R T(F) R^T for every rotation R.  Under a 45-degree turn the
    # traceless part moves from the p_xx moment (Q_{m,7}) into the p_xy moment
    # (Q_{m,8}), which fixes Q_{m,8} against Q_{m,7} and Q_{m,1}.
    p = params(eps=1.895, scheme=scheme, k1=k1, k2=k2)
    for _ in range(6):
        F = RNG.uniform(-1e-2, 1e-2, 2)
        psi, u, v = RNG.uniform(0.05, 1.0), RNG.uniform(-0.1, 0.1), RNG.uniform(-0.1, 0.1)
        T0 = source_tensor(O.source(p, F[0], F[1], psi, u, v))
        for ang in (np.pi / 4, np.pi / 6, 1.1, 2.5, -0.7):
            R = np.array([[np.cos(ang), -np.sin(ang)], [np.sin(ang), np.cos(ang)]])
            Fr = R @ F
            T1 = source_tensor(O.source(p, Fr[0], Fr[1], psi, u, v))
            np.testing.assert_allclose(T1, R @ T0 @ R.T, rtol=0, atol=1e-13 * np.abs(T0).max())
        # the tensor is symmetric in its construction; its isotropic part carries
        # eps = -8 (k1 + k2) (Sec. 2): trace = (k1 + 2 k2) |F|^2 / (G psi^2)
        kk1 = -1.895 / 16 if k1 is None else k1
        kk2 = -1.895 / 16 if k2 is None else k2
        np.testing.assert_allclose(np.trace(T0), -(kk1 + 2 * kk2) * (F @ F) / psi ** 2, rtol=1e-13)
        # a force along x alone leaves no p_xy source, a force along the diagonal no p_xx source
        Qx = O.source(p, F[0], 0.0, psi, u, v)
        Qd = O.source(p, F[0], F[0], psi, u, v)
        assert Qx[8] == 0.0 and Qd[7] == 0.0
