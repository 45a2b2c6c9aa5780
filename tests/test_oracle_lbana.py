"""LB-ana (oracle/lb_ana.py): the paper's finite-difference velocity equations
solved for a given density profile, checked against the oracle and against
the values of the paper's Table 1.

* Grid-aligned (Sec. 2.1.1): Eqs. (16)-(19) with halfway bounce-back at the
  two walls reproduce the converged oracle profile to rounding, for both
  schemes and several eps and tau; eliminated, they are Eq. (22).
* Grid-oblique (Sec. 2.1.2): Eqs. (32)-(35) reproduce it to the few 1e-4 that
  the analysis's assumption u_alpha = 0 leaves out.
* Eq. (40): the K that suppresses the oblique oscillations, fitted on the
  converged 45-degree channels of Table 1's setups, follows (24 eps - 15)/32.
* Table 1 (Sec. 3.1), in the paper's setups (van der Waals, K_EOS = 1/16,
  W = 128 sqrt 2, F = 2e-7) on the oracle's converged density profiles
  (tests/golden/table1_profiles.json): the original scheme's Err is the
  paper's to 2% (aligned, eps = 1, 2) and 5% (oblique, every eps); the
  improved scheme's oblique Err is the paper's tau = 1.5 column to 7%.  In the
  aligned channels the improved scheme's Err and the eps = 0 Err, both near
  1e-3, depend on the wall treatment (the paper's is a non-equilibrium
  extrapolation, this one halfway bounce-back): there only the ratios are
  pinned (more than 10x at eps = 1, 2, equal at eps = 0, independent of tau).
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import coexistence as X
from oracle import lb_ana as A
from oracle import oracle as O
from tests.test_oracle_steady import CASES, aligned, converge, oblique

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
F_DRI = 2e-7  # Sec. 3.1
TABLE1 = [(0.0, 0.72), (1.0, 0.65), (2.0, 0.54)]


def psi_of(eos, r):
    """psi = sqrt(2 (rho/3 - p_EOS)) (Eq. 5 with G = -1), from the Python EOS."""
    r = np.asarray(r, float)
    return np.sqrt(np.maximum(2.0 * (r / 3.0 - eos.p(r)), 0.0))


def rates(tau):
    sp = 1.0 / tau
    return sp, 1.0 / (0.5 + (1.0 / 12.0) / (tau - 0.5))


@pytest.mark.parametrize("case", CASES)
def test_aligned_lb_ana_is_the_converged_oracle_profile(case):
    scheme, eps, tau = case
    o, p = aligned(scheme, eps, tau, fx=1e-7)
    m, _ = converge(o)
    eos = X.cs(0.8)
    rho = m["rho"][:, 0]
    psi = psi_of(eos, rho)
    u, a, b, F = A.aligned_profile(rho, psi, psi_of(eos, p.rho_s), p.fx, p.s[7], p.s[4], eps,
                                   A.IMPROVED if scheme == O.SCHEME_IMPROVED else A.ORIGINAL)
    us = m["ux"][:, 0]
    np.testing.assert_allclose(F, m["finty"][:, 0], rtol=0, atol=1e-13 * np.max(np.abs(F)) + 1e-20)
    assert np.max(np.abs(u - us)) <= 1e-9 * np.max(np.abs(us))
    # the relations it solves, eliminated in the interior, are Eq. (22)
    nu = (1.0 / p.s[7] - 0.5) / 3.0
    q6 = (3 * eps / 8) * F * F / (psi * psi) if scheme == O.SCHEME_IMPROVED else np.zeros_like(F)
    assert np.max(np.abs(A.aligned_fd_residual(rho, F, q6, u, p.fx, nu))) <= 1e-11 * p.fx / nu


def test_aligned_lb_ana_single_phase_is_the_slip_parabola():
    # Uniform density: Eq. (22) is the second-order difference form of the
    # Navier-Stokes equation; with (1/s_q - 1/2)(1/s_p - 1/2) = 3/16 halfway
    # bounce-back puts the no-slip planes exactly half a node out.
    n, rho0, F, tau = 16, 0.2, 1e-6, 0.8
    sp = 1 / tau
    sq = 1 / (0.5 + (3 / 16) / (tau - 0.5))
    u, *_ = A.aligned_profile(np.full(n, rho0), np.full(n, 0.3), 0.3, F, sp, sq, 0.0, A.ORIGINAL)
    y = np.arange(n)
    nu = (tau - 0.5) / 3
    np.testing.assert_allclose(u, F / (2 * rho0 * nu) * (y + 0.5) * (n - 0.5 - y), rtol=1e-12)
    np.testing.assert_allclose(A.theory_profile(np.full(n, rho0), F, nu), u, rtol=1e-9)


@pytest.mark.parametrize("scheme", [O.SCHEME_ORIGINAL, O.SCHEME_IMPROVED])
def test_oblique_lb_ana_approximates_the_converged_oracle_profile(scheme):
    N, eps, Fdri = 32, 1.895, 1e-6
    o, p = oblique(scheme, eps, 1.5, Fdri, N=N)
    m, _ = converge(o)
    eos = X.cs(0.8)
    r = m["rho"][0][2:]
    ub = ((m["ux"][0] + m["uy"][0]) / math.sqrt(2.0))[2:]
    K = (24 * eps - 15) / 32 if scheme == O.SCHEME_IMPROVED else None
    u, a, b, Fx = A.oblique_profile(r, psi_of(eos, r), psi_of(eos, p.rho_s), Fdri, p.s[7], p.s[4], K)
    np.testing.assert_allclose(Fx, m["fintx"][0][2:], rtol=0, atol=1e-13 * np.max(np.abs(Fx)))
    # the analysis assumes u_alpha = 0; the converged discrete state carries ~1e-4
    assert np.max(np.abs(u - ub)) <= 1e-3 * np.max(np.abs(ub))
    # the lines beside the walls, where the bounce-back rows act, agree more closely
    assert np.max(np.abs(u - ub)[[0, 1, -2, -1]]) <= 1e-4 * np.max(np.abs(ub))


@pytest.fixture(scope="module")
def profiles():
    with open(os.path.join(GOLDEN, "table1_profiles.json")) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def paper():
    with open(os.path.join(GOLDEN, "paper_numbers.json")) as fh:
        return json.load(fh)["table1_err"]


def test_K_fit_follows_eq40(profiles):
    # Eq. (40): K is found by solving Eq. (38) for a two-phase density profile so
    # that the spurious oscillations vanish; here, the K whose LB-ana profile is
    # closest (Err) to Eq. (44) on the converged 45-degree channel of each
    # (eps, T_r) of Table 1.
    Ks = []
    for eps, T_r in TABLE1:
        eos = X.vdw_paper(T_r)
        rg, _, _ = X.mechanical_stability(eos, eps)
        r = np.array(profiles["oblique"][str(eps)])
        for tau in (0.8, 1.5):
            sp, sq = rates(tau)
            K, e = A.fit_K(r, psi_of(eos, r), float(psi_of(eos, rg)), F_DRI, sp, sq)
            print(f"[K fit] eps={eps} tau={tau}: K = {K:.4f}, Eq. (40) {(24 * eps - 15) / 32:.4f}, Err {e:.2e}")
            assert abs(K - (24 * eps - 15) / 32) < 0.06
        Ks.append(K)
    slope, icpt = np.polyfit([c[0] for c in TABLE1], Ks, 1)
    print(f"[K fit] K = {slope:.4f} eps {icpt:+.4f}; Eq. (40): 0.75 eps - 0.46875")
    assert abs(slope - 0.75) < 0.05 * 0.75
    assert abs(icpt - (-15 / 32)) < 0.06


def lb_ana_aligned_err(r, eos, eps, tau, scheme, rg):
    """LB-ana velocity profile of the aligned channel (181 rows) at the density r,
    and its Err against Eq. (44)."""
    sp, sq = rates(tau)
    nu = (1 / sp - 0.5) / 3
    ut = A.theory_profile(r, F_DRI, nu)
    ua, *_ = A.aligned_profile(r, psi_of(eos, r), float(psi_of(eos, rg)), F_DRI, sp, sq, eps,
                               A.IMPROVED if scheme == O.SCHEME_IMPROVED else A.ORIGINAL)
    return ua, ut, A.err(ua, ut)


def test_table1_aligned_with_lb_ana(profiles, paper):
    # The aligned channels of Table 1 with LB-ana on the oracle's converged
    # densities (LB-ana is the oracle's steady state to rounding: tested above on
    # small channels, and on these by test_table1_aligned_lb_ana_is_the_oracles_steady_state).
    errs = {}
    for eps, T_r in TABLE1:
        eos = X.vdw_paper(T_r)
        rg, _, _ = X.mechanical_stability(eos, eps)
        r = np.array(profiles["aligned"][str(eps)])
        row = paper[f"eps{int(eps)}_aligned"]
        for scheme in (O.SCHEME_ORIGINAL, O.SCHEME_IMPROVED):
            for k, tau in enumerate((0.8, 1.5)):
                errs[(eps, scheme, tau)] = e = lb_ana_aligned_err(r, eos, eps, tau, scheme, rg)[2]
                col = k + (2 if scheme == O.SCHEME_IMPROVED else 0)
                print(f"[Table 1] aligned eps={eps} scheme={scheme} tau={tau}: Err {e:.4e} (paper {row[col]:.4e})")
                if scheme == O.SCHEME_ORIGINAL and eps > 0:
                    # the error the original scheme's Q_m,6 leaves (Eq. 28) dominates: the
                    # paper's values, 5.22e-2 and 12.92e-2, to 2%
                    assert abs(e - row[col]) <= 0.02 * row[col]
    for eps, _ in TABLE1:
        for tau in (0.8, 1.5):
            o, i = errs[(eps, O.SCHEME_ORIGINAL, tau)], errs[(eps, O.SCHEME_IMPROVED, tau)]
            if eps == 0.0:
                # Eq. (28) vanishes with eps: the schemes coincide (Table 1, first row)
                assert abs(o - i) <= 1e-9 * o
            else:
                # Table 1: 5.221e-2 / 0.415e-2 = 12.6 at eps = 1, 12.922e-2 / 0.389e-2 = 33 at eps = 2
                assert o / i > 10.0, (eps, tau, o / i)
        # Err does not depend on tau (Table 1's columns agree to 3 digits)
        for scheme in (O.SCHEME_ORIGINAL, O.SCHEME_IMPROVED):
            a, b = errs[(eps, scheme, 0.8)], errs[(eps, scheme, 1.5)]
            assert abs(a - b) <= 1e-3 * a
    # and the original scheme's error grows with eps (Table 1)
    assert errs[(2.0, O.SCHEME_ORIGINAL, 0.8)] > errs[(1.0, O.SCHEME_ORIGINAL, 0.8)]


@pytest.mark.slow
def test_table1_aligned_lb_ana_is_the_oracles_steady_state(profiles):
    # The oracle, started from the LB-ana velocity profile of each aligned channel
    # of Table 1, stays on it.  Converging these channels from rest is out of
    # reach: the liquid slab, about 60 times denser than the gas layers that
    # couple it to the walls, relaxes on a time scale of millions of steps, and at
    # eps = 2 the centred slab drifts slowly towards a wall.  Started on the
    # steady state, only the fast modes that the equilibrium initial populations
    # excite remain; after 20,000 steps they are below 2e-3 of the peak velocity.
    for eps, T_r in TABLE1:
        eos = X.vdw_paper(T_r)
        rg, _, _ = X.mechanical_stability(eos, eps)
        r = np.array(profiles["aligned"][str(eps)])
        for scheme in (O.SCHEME_ORIGINAL, O.SCHEME_IMPROVED):
            for tau in (0.8, 1.5):
                ua, ut, e_ana = lb_ana_aligned_err(r, eos, eps, tau, scheme, rg)
                sp, sq = rates(tau)
                p = O.Params(nx=1, ny=len(r), periodic_x=True, periodic_y=False, eos_kind=O.EOS_VDW, a=eos.a, b=eos.b,
                             R=eos.R, T=eos.T, k_eos=eos.k_eos, eps=eps, s=(1, sp, sp, 1, sq, 1, sq, sp, sp),
                             scheme=scheme, fx=F_DRI, rho_g=rg, rho_l=float(r.max()), rho_s=rg)
                o = O.Oracle(p, threads=1).init(r[:, None], ux0=ua[:, None])
                o.step(20000)
                us = o.macros()["ux"][:, 0]
                d = np.max(np.abs(us - ua)) / np.max(np.abs(ua))
                e_sim = A.err(us, ut)
                print(f"[Table 1] aligned eps={eps} scheme={scheme} tau={tau}: oracle after 20,000 steps "
                      f"{d:.1e} from LB-ana, Err {e_sim:.4e} (LB-ana {e_ana:.4e})", flush=True)
                assert d < 2e-3
                if scheme == O.SCHEME_ORIGINAL and eps > 0:
                    assert abs(e_sim - e_ana) <= 0.01 * e_ana


def test_table1_oblique_with_lb_ana(profiles, paper):
    # The 45-degree channel of the same setups (254 fluid lines of the 256 x 256
    # lattice), with LB-ana on the oracle's converged densities.  The original
    # scheme gives Table 1's values to 5% in both tau columns; the improved scheme
    # those of its tau = 1.5 column to 7% (LB-ana's Err does not depend on tau,
    # the paper's simulations vary by up to 36% between the columns), several
    # times smaller at every eps.
    for eps, T_r in TABLE1:
        eos = X.vdw_paper(T_r)
        rg, _, _ = X.mechanical_stability(eos, eps)
        r = np.array(profiles["oblique"][str(eps)])
        row = paper[f"eps{int(eps)}_oblique"]
        for k, tau in enumerate((0.8, 1.5)):
            sp, sq = rates(tau)
            nu = (1 / sp - 0.5) / 3
            ut = A.theory_profile(r, F_DRI, nu, spacing=1 / math.sqrt(2))
            psi, psiw = psi_of(eos, r), float(psi_of(eos, rg))
            e_o = A.err(A.oblique_profile(r, psi, psiw, F_DRI, sp, sq, None)[0], ut)
            e_i = A.err(A.oblique_profile(r, psi, psiw, F_DRI, sp, sq, (24 * eps - 15) / 32)[0], ut)
            print(f"[Table 1] oblique eps={eps} tau={tau}: original {e_o:.3e} (paper {row[k]:.3e}), "
                  f"improved {e_i:.3e} (paper {row[2 + k]:.3e})")
            assert abs(e_o - row[k]) <= 0.05 * row[k]
            if tau == 1.5:
                assert abs(e_i - row[3]) <= 0.07 * row[3]
            assert e_o / e_i > 4.0
