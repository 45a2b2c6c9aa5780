"""Lattice-level pins of the oracle: stencil, EOS, conservation, symmetry,
and the single-phase Poiseuille closed form.

* Eq. (39): for a pseudopotential field that varies along one lattice line
  family, the force of Eq. (4) reduces to a 5-point (grid-aligned) or 7-point
  (grid-oblique) one-dimensional stencil.  This fixes the interaction weights
  w(1) = 1/3, w(2) = 1/12, the sign and the normalisation.
* psi = sqrt(2 (rho/3 - p_EOS)) (Eq. 5 with G = -1), checked against an
  independent Python EOS.
* Streaming, halfway bounce-back and collision conserve mass; in a periodic box
  the total momentum grows by exactly N F_ext per step because the pairwise
  force sums to zero.
* Symmetric inputs stay symmetric (bitwise for translation invariance).
* Single-phase Poiseuille flow: Eq. (22) with rho = const and F_int = 0 is the
  second-order difference form of the Navier-Stokes equation, so the converged
  profile has exact curvature -F/(rho nu), nu = (1/s_p - 1/2)/3; with
  (1/s_q - 1/2)(1/s_p - 1/2) = 3/16 halfway bounce-back makes it the exact
  parabola with walls half a node outside the fluid.
"""
import math

import numpy as np
import pytest

from oracle import coexistence as X
from oracle import oracle as O

W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def params(**kw):
    base = dict(eos_kind=O.EOS_CS, T=X.cs(0.8).T, eps=1.895, rho_g=0.0232, rho_l=0.3075, rho_s=0.0232)
    base.update(kw)
    return O.Params(**base)


def field_from_density(rho):
    """fbar = w_i rho (a resting equilibrium)."""
    return np.ascontiguousarray(W9[:, None, None] * rho[None, :, :])


def test_stencil_grid_aligned_eq39():
    y = np.arange(32)[:, None] * np.ones((1, 4))
    rho = 0.15 + 0.12 * np.tanh((y - 10.3) / 2.0) - 0.1 * np.tanh((y - 22.7) / 3.0)
    o = O.Oracle(params(nx=4, ny=32))
    o.f = field_from_density(rho)
    m = o.macros()
    psi = m["psi"][:, 0]
    want = psi * (np.roll(psi, -1) - np.roll(psi, 1)) / 2.0   # psi^i (psi^{i+1} - psi^{i-1}) / 2
    np.testing.assert_allclose(m["finty"][:, 0], want, rtol=1e-13, atol=1e-17)
    assert np.all(m["fintx"] == 0.0)
    for col in range(1, 4):
        assert np.array_equal(m["finty"][:, col], m["finty"][:, 0])


def test_stencil_grid_oblique_eq39():
    N = 40
    x = np.arange(N)[None, :]
    y = np.arange(N)[:, None]
    d = np.mod(x - y, N).astype(float)
    rho = 0.15 + 0.1 * np.sin(2 * math.pi * d / N) + 0.03 * np.cos(6 * math.pi * d / N)
    o = O.Oracle(params(nx=N, ny=N))
    o.f = field_from_density(rho)
    m = o.macros()
    # line index i = x - y (increasing along alpha = (x - y)/sqrt(2))
    line = np.array([m["psi"][0, k] for k in range(N)])  # row y = 0: i = x
    for yy in range(N):
        for xx in range(N):
            assert m["psi"][yy, xx] == line[(xx - yy) % N]
    want = line * (np.roll(line, -2) + 4 * np.roll(line, -1) - 4 * np.roll(line, 1) - np.roll(line, 2)) / 12.0
    np.testing.assert_allclose(m["fintx"][0, :], want, rtol=1e-12, atol=1e-17)
    # F_int,x = -F_int,y for a field depending on x - y only (Sec. 2.1.2)
    np.testing.assert_allclose(m["finty"], -m["fintx"], rtol=1e-13, atol=1e-18)


@pytest.mark.parametrize("kind,T_r", [("cs", 0.7), ("cs", 0.8), ("vdw", 0.5), ("vdw", 0.65)])
def test_psi_and_eos_match_independent_python_eos(kind, T_r):
    eos = X.eos_for(kind, T_r)
    p = params(eos_kind=O.EOS_CS if kind == "cs" else O.EOS_VDW, a=eos.a, b=eos.b, R=eos.R, T=eos.T,
               k_eos=eos.k_eos, nx=1, ny=1)
    top = 0.45 if kind == "cs" else 9.0
    for r in np.linspace(top * 1e-3, top, 57):
        assert abs(O.p_eos(p, r) - eos.p(r)) <= 1e-15 * max(1.0, abs(eos.p(r))) * 4
        np.testing.assert_allclose(O.psi(p, r), math.sqrt(2 * (r / 3 - eos.p(r))), rtol=1e-14)


def _random_lattice(nx, ny, seed, periodic=(True, True), mask=None, **kw):
    rng = np.random.default_rng(seed)
    rho = 0.1 + 0.15 * rng.random((ny, nx))
    if mask is not None:
        rho = np.where(mask == 1, 0.05, rho)
    o = O.Oracle(params(nx=nx, ny=ny, periodic_x=periodic[0], periodic_y=periodic[1], **kw), mask=mask)
    o.init(rho)
    return o


@pytest.mark.parametrize("scheme", [O.SCHEME_ORIGINAL, O.SCHEME_IMPROVED])
def test_mass_is_conserved_with_walls_and_mask(scheme):
    nx, ny = 23, 17
    rng = np.random.default_rng(3)
    mask = (rng.random((ny, nx)) < 0.08).astype(np.uint8)
    o = _random_lattice(nx, ny, 5, periodic=(False, True), mask=mask, scheme=scheme, fx=1e-5, fy=-2e-5)
    red = o.step(300, reductions=True)
    mass = red[:, 0]
    assert red[:, -1].sum() == 0
    assert np.max(np.abs(mass - mass[0])) <= 1e-13 * mass[0]


def test_momentum_grows_by_the_external_force_in_a_periodic_box():
    nx, ny = 19, 13
    F = (3e-6, -7e-6)
    o = _random_lattice(nx, ny, 7, fx=F[0], fy=F[1])
    red = o.step(200, reductions=True)
    dmx = np.diff(red[:, 1])
    dmy = np.diff(red[:, 2])
    np.testing.assert_allclose(dmx, nx * ny * F[0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(dmy, nx * ny * F[1], rtol=0, atol=1e-15)


def test_buoyant_force_momentum_balance_in_periodic_box():
    # F_ext = (rho - rho_g) g: momentum grows by sum_x (rho - rho_g) g per step.
    nx, ny = 16, 21
    o = _random_lattice(nx, ny, 11, force_mode=O.FORCE_BUOYANT, fx=0.0, fy=-1e-5, rho_g=0.05)
    red = o.step(50, reductions=True)
    mass = red[0, 0]
    want = (mass - nx * ny * 0.05) * -1e-5
    # summation round-off of ~N terms of size rho u
    np.testing.assert_allclose(np.diff(red[:, 2]), want, rtol=0, atol=1e-14)
    np.testing.assert_allclose(np.diff(red[:, 1]), 0.0, rtol=0, atol=1e-14)


def _aligned_channel(nx=4, ny=40, y0=10, y1=30, tau=0.8, eps=1.895, scheme=O.SCHEME_IMPROVED, fx=1e-6,
                     T_r=0.8, s=None):
    co = X.mechanical_stability(X.cs(T_r), eps)
    rg, rl = co[0], co[1]
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    rho = rg + 0.5 * (rl - rg) * (np.tanh(y - (y0 - 0.5)) - np.tanh(y - (y1 - 0.5)))
    sp = 1 / tau
    sq = 1 / (0.5 + (1 / 12) / (tau - 0.5))
    rates = s if s is not None else (1, sp, sp, 1, sq, 1, sq, sp, sp)
    p = params(nx=nx, ny=ny, periodic_x=True, periodic_y=False, T=X.cs(T_r).T, eps=eps, s=rates,
               scheme=scheme, fx=fx, rho_g=rg, rho_l=rl, rho_s=rg)
    return O.Oracle(p).init(rho)


def test_translation_invariance_is_bitwise():
    o = _aligned_channel()
    o.step(700)
    m = o.macros()
    for col in range(1, 4):
        for k in ("rho", "ux", "uy", "psi", "finty"):
            assert np.array_equal(m[k][:, col], m[k][:, 0])
        assert np.array_equal(o.f[:, :, col], o.f[:, :, 0])
    assert np.all(m["fintx"] == 0.0)


def test_mirror_symmetry_about_channel_centre():
    o = _aligned_channel(fx=0.0)
    o.step(500)
    m = o.macros()
    np.testing.assert_allclose(m["rho"][::-1], m["rho"], rtol=1e-13, atol=0)
    np.testing.assert_allclose(m["finty"][::-1], -m["finty"], rtol=0, atol=1e-15)


def _single_phase(tau=0.8, sq=None, ny=16, F=1e-6, steps=60000):
    rho0 = 0.2
    sp = 1 / tau
    if sq is None:
        sq = 1 / (0.5 + (1 / 12) / (tau - 0.5))
    # supercritical temperature: a uniform density is a stable single phase
    p = params(nx=2, ny=ny, periodic_x=True, periodic_y=False, s=(1, sp, sp, 1, sq, 1, sq, sp, sp), fx=F,
               rho_s=rho0, eps=1.895, T=X.cs(1.5).T)
    o = O.Oracle(p).init(np.full((ny, 2), rho0))
    o.step(steps)
    return o, p, rho0


def test_single_phase_curvature_is_exact():
    # Eq. (22) with rho uniform and F_int = Q = 0: u^{i-1} + u^{i+1} - 2 u^i = -F / (rho nu).
    tau = 0.8
    o, p, rho0 = _single_phase(tau=tau)
    m = o.macros()
    # uniform density up to round-off: the interaction force is negligible next to F
    assert np.max(np.abs(m["fintx"])) < 1e-10 * p.fx and np.max(np.abs(m["finty"])) < 1e-10 * p.fx
    u = m["ux"][:, 0]
    nu = (tau - 0.5) / 3
    curv = u[:-2] + u[2:] - 2 * u[1:-1]
    np.testing.assert_allclose(curv, -p.fx / (rho0 * nu), rtol=1e-10)


def test_single_phase_magic_rates_give_the_exact_parabola():
    # Halfway bounce-back with Lambda = (1/s_q - 1/2)(1/s_p - 1/2) = 3/16 puts the
    # no-slip plane exactly half a node outside the fluid: u(y) = F/(2 rho nu) (y + 1/2)(H - 1/2 - y).
    tau = 0.8
    sq = 1 / (0.5 + (3 / 16) / (tau - 0.5))
    ny = 16
    o, p, rho0 = _single_phase(tau=tau, sq=sq, ny=ny)
    u = o.macros()["ux"][:, 0]
    y = np.arange(ny)
    nu = (tau - 0.5) / 3
    exact = p.fx / (2 * rho0 * nu) * (y + 0.5) * (ny - 0.5 - y)
    np.testing.assert_allclose(u, exact, rtol=1e-10)
    # and with the paper's rates (Lambda = 1/12) the profile carries a slip
    o2, _, _ = _single_phase(tau=tau, ny=ny)
    u2 = o2.macros()["ux"][:, 0]
    assert np.max(np.abs(u2 - exact)) > 1e-4 * exact.max()
