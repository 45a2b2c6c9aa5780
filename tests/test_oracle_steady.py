"""Pins of the oracle at steady state: the paper's discrete-level relations.

The discrete analysis of Sec. 2.1 derives exact relations that a converged
two-phase Poiseuille flow (or a static flat interface) must satisfy node by
node.  The lattice here is oriented with the flow along x and the interface
normal along y, so the paper's (x, y) become (y, x): its directions 2, 4 become
1, 3, its 1+5+8 become 2+5+6, its Q_{m,6} becomes Q_{m,4}.

* Eq. (16): f_1 - f_3 = 2/3 rho u_x + (2 - s_q)/(3 s_q) F_dri - Q_{m,4}/3 at every node.
* Eq. (22): the finite-difference velocity equation across the interface.
* Eq. (38): its grid-oblique counterpart along the 45-degree line index.
* Eqs. (23), (24), (26): the static relations at s_e = s_p, which contain the
  second-order source terms through eps only.
* Sec. 2.2: the improved scheme leaves a static interface unchanged.
* Eq. (1): a converged flat interface sits near the eps-mechanical-stability
  coexistence densities (the coexistence-curve check of Sec. 3.1); at Sec.
  3.2's setting (eps = 1.895, T_r = 0.5) on the Maxwell densities, ratio 113.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import coexistence as X
from oracle import oracle as O
from paper_2604_13407_amd import workloads as WL
from tests.helpers import oracle_for

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def converge(o, chunk=2000, max_steps=400000, tol=1e-12, static=False):
    prev = o.macros()
    steps = 0
    while steps < max_steps:
        o.step(chunk)
        steps += chunk
        cur = o.macros()
        if static:
            d = max(np.max(np.abs(cur["rho"] - prev["rho"])), np.max(np.abs(cur["ux"] - prev["ux"])),
                    np.max(np.abs(cur["uy"] - prev["uy"])))
            if d < tol:
                return cur, steps
        else:
            d = np.max(np.abs(cur["ux"] - prev["ux"])) / max(np.max(np.abs(cur["ux"])), 1e-300)
            if d < tol:
                return cur, steps
        prev = cur
    raise AssertionError(f"not converged after {steps} steps (change {d:.3e})")


def rates(tau, se=None):
    sp = 1 / tau
    sq = 1 / (0.5 + (1 / 12) / (tau - 0.5))
    se = sp if se is None else se
    return (1, se, se, 1, sq, 1, sq, sp, sp)


def aligned(scheme, eps, tau, fx, ny=25, y0=7, y1=18, T_r=0.8):
    # An odd channel width, symmetric about its centre line, keeps the
    # staggered momentum sum_y (-1)^(y+t) j_y at zero: streaming and halfway
    # bounce-back conserve it exactly, so once excited it never decays, and the
    # mirror symmetry of this layout forbids it.
    eos = X.cs(T_r)
    rg, rl, _ = X.mechanical_stability(eos, eps)
    y = np.arange(ny)[:, None] * np.ones((1, 2))
    rho = rg + 0.5 * (rl - rg) * (np.tanh(y - (y0 - 0.5)) - np.tanh(y - (y1 - 0.5)))
    p = O.Params(nx=2, ny=ny, periodic_x=True, periodic_y=False, eos_kind=O.EOS_CS, T=eos.T, eps=eps,
                 s=rates(tau), scheme=scheme, fx=fx, rho_g=rg, rho_l=rl, rho_s=rg)
    return O.Oracle(p).init(rho), p


CASES = [(O.SCHEME_ORIGINAL, 1.895, 1.5), (O.SCHEME_IMPROVED, 1.895, 1.5), (O.SCHEME_IMPROVED, 1.0, 0.8),
         (O.SCHEME_ORIGINAL, 1.0, 0.8), (O.SCHEME_ORIGINAL, 0.0, 1.5)]


@pytest.fixture(scope="module")
def converged_aligned():
    out = {}
    for scheme, eps, tau in CASES:
        o, p = aligned(scheme, eps, tau, fx=1e-7)
        m, _ = converge(o)
        out[(scheme, eps, tau)] = (o, p, m)
    return out


def q4_field(p, m):
    Q = np.array([O.source(p, m["fintx"][i, 0], m["finty"][i, 0], m["psi"][i, 0], m["ux"][i, 0], m["uy"][i, 0])
                  for i in range(p.ny)])
    return Q[:, 4]


@pytest.mark.parametrize("case", CASES)
def test_eq16_one_node_relation(converged_aligned, case):
    o, p, m = converged_aligned[case]
    sq = p.s[4]
    f = m["fpre"][:, :, 0]
    lhs = f[1] - f[3]
    rhs = 2 / 3 * m["rho"][:, 0] * m["ux"][:, 0] + (2 - sq) / (3 * sq) * p.fx - q4_field(p, m) / 3
    scale = np.max(np.abs(2 / 3 * m["rho"][:, 0] * m["ux"][:, 0]))
    assert np.max(np.abs(lhs - rhs)) <= 1e-9 * scale


@pytest.mark.parametrize("case", CASES)
def test_eq22_finite_difference_velocity_equation(converged_aligned, case):
    o, p, m = converged_aligned[case]
    nu = (1 / p.s[7] - 0.5) / 3
    r, u, F = m["rho"][:, 0], m["ux"][:, 0], m["finty"][:, 0]
    Q = q4_field(p, m)
    i = np.arange(1, p.ny - 1)
    res = ((r[i - 1] + 1.5 * F[i - 1]) * u[i - 1] + (r[i + 1] - 1.5 * F[i + 1]) * u[i + 1] - 2 * r[i] * u[i]
           + (Q[i - 1] + Q[i + 1] - 2 * Q[i]) + p.fx / nu)
    assert np.max(np.abs(res)) <= 1e-8 * p.fx / nu


def test_eq22_fails_for_a_wrong_q4_sign(converged_aligned):
    # The relation is sharp enough to reject a flipped third-order term.
    o, p, m = converged_aligned[(O.SCHEME_IMPROVED, 1.895, 1.5)]
    nu = (1 / p.s[7] - 0.5) / 3
    r, u, F = m["rho"][:, 0], m["ux"][:, 0], m["finty"][:, 0]
    Q = -q4_field(p, m)
    i = np.arange(1, p.ny - 1)
    res = ((r[i - 1] + 1.5 * F[i - 1]) * u[i - 1] + (r[i + 1] - 1.5 * F[i + 1]) * u[i + 1] - 2 * r[i] * u[i]
           + (Q[i - 1] + Q[i + 1] - 2 * Q[i]) + p.fx / nu)
    assert np.max(np.abs(res)) > 1e-3 * p.fx / nu


def test_improved_scheme_removes_the_interface_oscillation_term(converged_aligned):
    # Sec. 2.1.1: with Eq. (28) the eps-term of Eq. (27) is cancelled, so the
    # improved profile satisfies (rho + 3 eps F^2/(8 psi^2)) d2u + 3/2 F du = -F_dri/nu
    # (the smooth, theory-like equation), while the original one does not.
    def smooth_residual(key):
        o, p, m = converged_aligned[key]
        nu = (1 / p.s[7] - 0.5) / 3
        r, u, F, ps = m["rho"][:, 0], m["ux"][:, 0], m["finty"][:, 0], m["psi"][:, 0]
        i = np.arange(1, p.ny - 1)
        eq = r[i] + 3 * p.eps / 8 * F[i] ** 2 / ps[i] ** 2
        res = eq * (u[i - 1] + u[i + 1] - 2 * u[i]) + 1.5 * F[i] * (u[i + 1] - u[i - 1]) + p.fx / nu
        return np.max(np.abs(res)) / (p.fx / nu)
    assert smooth_residual((O.SCHEME_IMPROVED, 1.895, 1.5)) < 1e-8
    assert smooth_residual((O.SCHEME_ORIGINAL, 1.895, 1.5)) > 1e-2


@pytest.fixture(scope="module")
def static_profiles():
    out = {}
    for scheme in (O.SCHEME_ORIGINAL, O.SCHEME_IMPROVED):
        o, p = aligned(scheme, 1.895, 0.8, fx=0.0)
        m, _ = converge(o, static=True, tol=1e-15)
        out[scheme] = (o, p, m)
    return out


def test_eq23_eq24_eq26_static_relations(static_profiles):
    o, p, m = static_profiles[O.SCHEME_ORIGINAL]
    eps = p.eps
    r, F, ps = m["rho"][:, 0], m["finty"][:, 0], m["psi"][:, 0]
    f = m["fpre"][:, :, 0]
    ratio = F ** 2 / ps ** 2
    # Eq. (23): f_{0+1+3} = 2/3 rho - eps/8 F^2/psi^2
    np.testing.assert_allclose(f[0] + f[1] + f[3], 2 / 3 * r - eps / 8 * ratio, rtol=0, atol=1e-13)
    # Eq. (24): f_{2+5+6} = rho/6 - F/4 + eps/16 F^2/psi^2 ; f_{4+7+8} = rho/6 + F/4 + eps/16 F^2/psi^2
    np.testing.assert_allclose(f[2] + f[5] + f[6], r / 6 - F / 4 + eps / 16 * ratio, rtol=0, atol=1e-13)
    np.testing.assert_allclose(f[4] + f[7] + f[8], r / 6 + F / 4 + eps / 16 * ratio, rtol=0, atol=1e-13)
    # Eq. (26): rho^{i+1} - 3/2 F^{i+1} = rho^i + 3/2 F^i + 3eps/8 (F^2/psi^2)^i - 3eps/8 (F^2/psi^2)^{i+1}
    i = np.arange(0, p.ny - 1)
    lhs = r[i + 1] - 1.5 * F[i + 1]
    rhs = r[i] + 1.5 * F[i] + 3 * eps / 8 * ratio[i] - 3 * eps / 8 * ratio[i + 1]
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-13)
    assert np.max(np.abs(m["ux"])) < 1e-14 and np.max(np.abs(m["uy"])) < 1e-14


def test_improved_scheme_reduces_to_original_for_a_static_interface(static_profiles):
    a = static_profiles[O.SCHEME_ORIGINAL][2]["rho"]
    b = static_profiles[O.SCHEME_IMPROVED][2]["rho"]
    np.testing.assert_allclose(b, a, rtol=0, atol=1e-13)


def test_flat_interface_reaches_mechanical_stability_densities():
    # Paper's vdW setting (K_EOS = 1/16, eps = 1, T_r = 0.65): Eq. (1) predicts
    # rho_g, rho_l with a ratio close to 60 (Sec. 3.1).  A converged flat interface
    # reproduces them up to the discretisation of the wide interface, and lies far
    # from the Maxwell densities, which belong to a different eps.
    eos = X.vdw_paper(0.65)
    rg, rl, _ = X.mechanical_stability(eos, 1.0)
    mg, ml, _ = X.maxwell(eos)
    ny = 96
    y = np.arange(ny)[:, None] * np.ones((1, 2))
    rho = rg + 0.5 * (rl - rg) * (np.tanh((y - 23.5) / 4) - np.tanh((y - 71.5) / 4))
    p = O.Params(nx=2, ny=ny, periodic_x=True, periodic_y=True, eos_kind=O.EOS_VDW, a=eos.a, b=eos.b, R=eos.R,
                 T=eos.T, k_eos=eos.k_eos, eps=1.0, s=rates(1.0), scheme=O.SCHEME_IMPROVED, rho_g=rg, rho_l=rl)
    o = O.Oracle(p).init(rho)
    o.step(30000)
    r = o.macros()["rho"][:, 0]
    assert abs(r[47] / rl - 1) < 1e-4
    assert abs(r[0] / rg - 1) < 2e-2
    assert abs(r[0] / mg - 1) > 0.5
    assert 55 < r[47] / r[0] < 65


def test_flat_interface_at_the_annular_setting_is_thermodynamically_consistent():
    # Sec. 3.2's van der Waals setting (T_r = 0.5, eps = 1.895): eps is chosen
    # there so that the coexistence densities are the thermodynamic ones, with a
    # density ratio of about 113.  A converged flat interface of the full step
    # (Q_m with k1 = k2 = -eps/16) must land on the Maxwell equal-area densities
    # (an independent closed form of the EOS) and on the paper's ratio; Eq. (1)'s
    # continuum gas density at this eps lies 4% away, so the check separates the two.
    g = GOLDEN["annular_density_ratio"]
    eos = X.vdw_paper(g["T_r"])
    mg, ml, _ = X.maxwell(eos)
    rg, rl, _ = X.mechanical_stability(eos, g["eps"])
    for scheme in (O.SCHEME_ORIGINAL, O.SCHEME_IMPROVED):
        w = WL.vdw_layer(nx=2, ny=96, scheme=scheme)
        assert w.T == eos.T and w.eps == g["eps"] and w.k_eos == eos.k_eos
        o = oracle_for(w)
        o.step(30000)
        r = o.macros()["rho"][:, 0]
        liq, gas = r[48], r[0]
        print(f"[Sec. 3.2] scheme {scheme}: rho_l {liq:.6f} (Maxwell {ml:.6f}), rho_g {gas:.6f} "
              f"(Maxwell {mg:.6f}, Eq. (1) {rg:.6f}), ratio {liq / gas:.3f} (paper {g['ratio']})")
        assert abs(liq / ml - 1) < 1e-5 and abs(liq / rl - 1) < 1e-4
        assert abs(gas / mg - 1) < 1e-3
        assert abs(gas / rg - 1) > 0.03
        assert abs(liq / gas - g["ratio"]) < 0.5


def oblique(scheme, eps, tau, F, N=32, T_r=0.8):
    eos = X.cs(T_r)
    rg, rl, _ = X.mechanical_stability(eos, eps)
    x = np.arange(N)[None, :]
    y = np.arange(N)[:, None]
    d = np.mod(x - y, N).astype(float)
    mask = ((d == 0) | (d == 1)).astype(np.uint8)
    s2 = math.sqrt(2)
    lo, hi = 9.5, 24.5
    rho = rg + 0.5 * (rl - rg) * (np.tanh((d - lo) / s2) - np.tanh((d - hi) / s2))
    f = F / s2
    p = O.Params(nx=N, ny=N, eos_kind=O.EOS_CS, T=eos.T, eps=eps, s=rates(tau), scheme=scheme, fx=f, fy=f,
                 rho_g=rg, rho_l=rl, rho_s=rg)
    return O.Oracle(p, mask=mask).init(rho), p


@pytest.mark.parametrize("scheme", [O.SCHEME_ORIGINAL, O.SCHEME_IMPROVED])
def test_eq32_eq35_exact_and_eq38_approximate_grid_oblique(scheme):
    # Reading: Eq. (30) assumes u_alpha = 0 exactly.  The converged discrete
    # state of a 45-degree interface carries a small steady normal velocity
    # (about 1e-4 here, present with no driving force at all), so the one-node
    # relations Eqs. (32) and (35), which do not involve u_alpha, hold to
    # round-off while the three-line equation Eq. (38) holds to a few per cent
    # of F_dri/nu at the interface.
    N = 32
    s2 = math.sqrt(2)
    o, p = oblique(scheme, 1.895, 1.5, 1e-6, N=N)
    m, _ = converge(o)
    nu = (1 / p.s[7] - 0.5) / 3
    sq = p.s[4]
    Fdri = 1e-6
    # Fields on line i = (x - y) mod N, read on row y = 0 (x = i).
    f = m["fpre"][:, 0, :]
    r = m["rho"][0]
    ub = (m["ux"][0] + m["uy"][0]) / s2
    Fx = m["fintx"][0]
    Q = np.array([O.source(p, m["fintx"][0, i], m["finty"][0, i], m["psi"][0, i], m["ux"][0, i], m["uy"][0, i])
                  for i in range(N)])
    Q46 = Q[:, 4] + Q[:, 6]
    scale = np.max(np.abs(r * ub))
    fl = np.arange(2, N)
    eq32 = f[5] - f[7] - (s2 / 6 * r * ub + s2 * (2 - sq) / (12 * sq) * Fdri + Q46 / 6)
    assert np.max(np.abs(eq32[fl])) <= 1e-11 * scale
    eq35 = (f[1] - f[4]) + (f[2] - f[3]) - (s2 * 2 / 3 * r * ub - s2 * (1 + sq) / (3 * sq) * Fdri - Q46 / 3)
    assert np.max(np.abs(eq35[fl])) <= 1e-11 * scale
    # Eq. (38) uses streaming from lines i-2..i+2, so all of them must be fluid: i in 4..N-3
    i = np.arange(4, N - 2)
    res = ((r[i - 1] + 1.5 * Fx[i - 1]) * ub[i - 1] + (r[i + 1] - 1.5 * Fx[i + 1]) * ub[i + 1] - 2 * r[i] * ub[i]
           - s2 / 4 * (Q46[i - 1] + Q46[i + 1] - 2 * Q46[i]) + Fdri / nu / 2)
    assert np.max(np.abs(res)) <= 0.1 * Fdri / nu
    # a wrong sign of the third-order term breaks it by far more
    bad = ((r[i - 1] + 1.5 * Fx[i - 1]) * ub[i - 1] + (r[i + 1] - 1.5 * Fx[i + 1]) * ub[i + 1] - 2 * r[i] * ub[i]
           + s2 / 4 * (Q46[i - 1] + Q46[i + 1] - 2 * Q46[i]) + Fdri / nu / 2)
    if scheme == O.SCHEME_IMPROVED:
        assert np.max(np.abs(bad)) > 0.3 * Fdri / nu
    # all fields depend on the line index only
    for yy in range(1, N, 7):
        np.testing.assert_allclose(np.roll(m["ux"][yy], -yy), m["ux"][0], rtol=1e-9, atol=1e-20)


def test_static_oblique_interface_carries_a_steady_normal_velocity():
    # The observation behind the reading above: no driving force, converged,
    # yet (j + F/2)/rho normal to the interface is about 1e-4 and steady.
    o, p = oblique(O.SCHEME_ORIGINAL, 1.895, 1.5, 0.0, N=32)
    o.step(60000)
    m0 = o.macros()
    o.step(1)
    m1 = o.macros()
    ua = (m0["ux"] - m0["uy"]) / math.sqrt(2)
    assert 1e-5 < np.max(np.abs(ua)) < 1e-3
    assert np.max(np.abs(m1["ux"] - m0["ux"])) < 1e-14
