"""Pins of the oracle's walls and observables: the moving-wall term of halfway
bounce-back, the momentum handed to walls, and the droplet velocity U_c.

* Isolated fluid nodes (every neighbour solid) reflect all nine populations,
  so their pulled state is known in closed form from the initial equilibrium:
  the density is unchanged and the lattice momentum is mirrored about the
  momentum of the wall, j = 2 rho u_w - rho u0 (an elastic reflection off a
  moving wall); the wall receives 2 rho (u0 - u_w).  U_c of Eq. (47) sums over
  the liquid region rho > (rho_l + rho_g)/2 only.  Every observable of such a
  lattice is written out by hand from these facts.
* Plane Couette flow: one flat halfway wall moving tangentially drives a
  single-phase channel to the exact linear profile with the no-slip planes
  half a node outside the fluid (Eq. (22) with F = 0 has zero curvature; the
  walls fix the two constants).
* Cylindrical Couette flow: Eq. (46) with F = 0 and uniform density gives
  u_theta = A r + B / r between a turning inner wall and a resting outer wall.
  Staircase walls hold it to first order in the lattice spacing: the error
  halves when the radii double.
* Momentum balance in a walled channel: between two steps the total momentum
  sum (j + F/2) changes by N F_ext minus the momentum the walls received.
"""
import numpy as np
import pytest

from oracle import coexistence as X
from oracle import oracle as O
from paper_2604_13407_amd import workloads as WL

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
RHO1 = 0.2          # single-phase density for the Couette cases
T_SUPER = X.cs(1.5).T  # supercritical: a uniform density is a stable single phase


def isolated_lattice(values, wall=(0.0, 0.0), g=(3e-6, -1e-5), rho_g=0.02, rho_l=0.32):
    """Fluid nodes at (2k, 0) of a 2n x 2 periodic lattice, every other node solid;
    values = [(rho0, ux0, uy0), ...]; the solid nodes move with velocity `wall`."""
    n = len(values)
    nx, ny = 2 * n, 2
    mask = np.ones((ny, nx), np.uint8)
    mask[0, 0::2] = 0
    rho0 = np.full((ny, nx), 0.05)
    ux0, uy0 = np.zeros((ny, nx)), np.zeros((ny, nx))
    for k, (r, u, v) in enumerate(values):
        rho0[0, 2 * k], ux0[0, 2 * k], uy0[0, 2 * k] = r, u, v
    wall_u = np.zeros((2, ny, nx))
    wall_u[0][mask == 1] = wall[0]
    wall_u[1][mask == 1] = wall[1]
    p = O.Params(nx=nx, ny=ny, eos_kind=O.EOS_CS, T=X.cs(0.7).T, eps=1.895, rho_g=rho_g, rho_l=rho_l,
                 rho_s=rho_g, force_mode=O.FORCE_BUOYANT, fx=g[0], fy=g[1])
    o = O.Oracle(p, mask=mask, wall_u=wall_u if any(wall) else None).init(rho0, ux0, uy0)
    return o, p


VALUES = [(0.021, 1e-3, -2e-3), (0.12, -3e-3, 5e-3), (0.30, 2e-3, -4e-3), (0.33, -1e-3, 7e-3)]


@pytest.mark.parametrize("wall", [(0.0, 0.0), (4e-3, -1.5e-3)])
def test_isolated_nodes_observables_by_hand(wall):
    o, p = isolated_lattice(VALUES, wall=wall)
    m = o.macros()
    red = m["red"]
    r = np.array([v[0] for v in VALUES])
    u0 = np.array([v[1] for v in VALUES])
    v0 = np.array([v[2] for v in VALUES])
    gx, gy = p.fx, p.fy
    gmag = np.hypot(gx, gy)
    # reflection: density kept, lattice momentum mirrored about the wall's
    jx = 2 * r * wall[0] - r * u0
    jy = 2 * r * wall[1] - r * v0
    # no interaction force between a node and a uniform solid ring; buoyancy only
    Fx, Fy = (r - p.rho_g) * gx, (r - p.rho_g) * gy
    ux, uy = (jx + Fx / 2) / r, (jy + Fy / 2) / r
    np.testing.assert_allclose(m["rho"][0, 0::2], r, rtol=1e-15)
    np.testing.assert_allclose(m["ux"][0, 0::2], ux, rtol=1e-12, atol=1e-17)
    np.testing.assert_allclose(m["uy"][0, 0::2], uy, rtol=1e-12, atol=1e-17)
    assert np.all(m["fintx"] == 0.0) and np.all(m["finty"] == 0.0)
    tol = 1e-15
    assert red["mass"] == pytest.approx(r.sum(), rel=tol)
    assert red["momx"] == pytest.approx((jx + Fx / 2).sum(), rel=1e-12)
    assert red["momy"] == pytest.approx((jy + Fy / 2).sum(), rel=1e-12)
    # the walls received the momentum the nodes lost: 2 rho (u0 - u_w)
    assert red["wallx"] == pytest.approx((2 * r * (u0 - wall[0])).sum(), rel=1e-12)
    assert red["wally"] == pytest.approx((2 * r * (v0 - wall[1])).sum(), rel=1e-12)
    # Eq. (47) over the liquid region rho > (rho_l + rho_g)/2 = 0.17: the last two nodes
    liquid = r > 0.5 * (p.rho_l + p.rho_g)
    assert liquid.tolist() == [False, False, True, True]
    assert red["uc_den"] == pytest.approx(r[liquid].sum(), rel=tol)
    assert red["uc_num"] == pytest.approx((r * uy)[liquid].sum(), rel=1e-12)
    # droplet-drag terms: phi = (rho - rho_g)/(rho_l - rho_g), momentum along g/|g|
    phi = (r - p.rho_g) / (p.rho_l - p.rho_g)
    assert red["buoy"] == pytest.approx((phi * (r - p.rho_g) * gmag).sum(), rel=1e-13)
    assert red["pphi"] == pytest.approx((phi * r * (ux * gx + uy * gy) / gmag).sum(), rel=1e-12)
    assert red["faults"] == 0


def test_isolated_node_at_rest_against_a_moving_wall_is_dragged_along():
    # A resting node whose ring moves at u_w leaves the pull with velocity 2 u_w.
    o, _ = isolated_lattice([(0.25, 0.0, 0.0)], wall=(3e-3, 1e-3), g=(0.0, 0.0))
    m = o.macros()
    assert m["ux"][0, 0] == pytest.approx(6e-3, rel=1e-12)
    assert m["uy"][0, 0] == pytest.approx(2e-3, rel=1e-12)
    assert m["rho"][0, 0] == pytest.approx(0.25, rel=1e-15)


def couette(ny=18, U=0.01, tau=0.8, steps=20000, top=True):
    """Single-phase channel: solid rows 0 and ny-1, x periodic; one wall row moves along x."""
    nx = 2
    mask = np.zeros((ny, nx), np.uint8)
    mask[0] = mask[-1] = 1
    wall_u = np.zeros((2, ny, nx))
    wall_u[0, -1 if top else 0] = U
    p = O.Params(nx=nx, ny=ny, eos_kind=O.EOS_CS, T=T_SUPER, eps=1.895, s=WL.rates_from_tau(tau),
                 rho_g=RHO1, rho_l=0.3, rho_s=RHO1)
    o = O.Oracle(p, mask=mask, wall_u=wall_u).init(np.full((ny, nx), RHO1))
    red = o.step(steps, reductions=True)
    return o, red


@pytest.mark.parametrize("tau,top", [(0.8, True), (0.8, False), (1.5, True)])
def test_plane_couette_is_the_exact_linear_profile(tau, top):
    ny, U = 18, 0.01
    o, red = couette(ny=ny, U=U, tau=tau, top=top)
    m = o.macros()
    y = np.arange(1, ny - 1)
    H = ny - 2  # no-slip planes at y = 1/2 and y = ny - 3/2
    exact = U * (y - 0.5) / H if top else U * (ny - 1.5 - y) / H
    np.testing.assert_allclose(m["ux"][1:-1, 0], exact, rtol=0, atol=1e-11 * U)
    assert np.abs(m["uy"]).max() < 1e-14
    # a flat wall moving along itself adds no mass
    assert abs(red[-1, 0] - red[0, 0]) <= 1e-14 * red[0, 0]


def cylindrical_couette(N, r_in, r_out, U=0.01, steps=20000):
    w = WL.annular_shear().with_size(N, N, init_args={"centre": ((N - 1) / 2, (N - 1) / 2), "r_in": r_in,
                                                      "r_out": r_out, "u_wall": U, "r_liq_in": 0.0,
                                                      "r_liq_out": 0.0})
    p = O.Params(nx=N, ny=N, eos_kind=O.EOS_CS, T=T_SUPER, eps=1.895, s=WL.rates_from_tau(0.8), rho_g=RHO1,
                 rho_l=0.3, rho_s=RHO1)
    mask = w.mask()
    o = O.Oracle(p, mask=mask, wall_u=w.wall_velocity()).init(np.full((N, N), RHO1))
    o.step(steps)
    m = o.macros()
    c = (N - 1) / 2
    x = np.arange(N)[None, :] - c
    y = np.arange(N)[:, None] - c
    r = np.sqrt(x * x + y * y)
    fluid = mask == 0
    ut = (-y * m["ux"] + x * m["uy"]) / np.where(fluid, r, 1.0)
    # Eq. (46) with F = 0 and uniform rho: u = A r + B / r, u(r_in) = U, u(r_out) = 0
    A = -U * r_in / (r_out ** 2 - r_in ** 2)
    B = U * r_in * r_out ** 2 / (r_out ** 2 - r_in ** 2)
    err = np.abs(ut - (A * r + B / r))[fluid].max() / U
    return err


@pytest.mark.slow
def test_cylindrical_couette_converges_to_eq46_at_first_order():
    e1 = cylindrical_couette(64, 8.0, 28.0, steps=12000)
    e2 = cylindrical_couette(128, 16.0, 56.0, steps=25000)
    # staircase walls: a few per cent at these radii, first order in the spacing
    assert e1 < 0.07 and e2 < 0.035
    assert 1.6 < e1 / e2 < 2.4


@pytest.mark.parametrize("walls_in", ["y", "x"])
def test_walled_channel_momentum_balance(walls_in):
    # Between the pre-collision states of steps n and n+1: sum(j + F/2) changes by
    # sum F_ext (the interaction force sums to zero along flat walls) minus the
    # momentum handed to the walls by the bounce-back links of step n+1.
    nx, ny = (12, 10) if walls_in == "y" else (10, 12)
    rng = np.random.default_rng(21)
    rho = 0.12 + 0.1 * rng.random((ny, nx))
    F = 2e-5
    fx, fy = (F, 0.0) if walls_in == "y" else (0.0, F)
    p = O.Params(nx=nx, ny=ny, periodic_x=walls_in == "y", periodic_y=walls_in == "x", eos_kind=O.EOS_CS,
                 T=X.cs(0.8).T, eps=1.895, fx=fx, fy=fy, rho_g=0.0232, rho_l=0.3075, rho_s=0.0232)
    o = O.Oracle(p).init(rho)
    red = o.step(400, reductions=True)
    k_mom, k_wall = (1, 3) if walls_in == "y" else (2, 4)
    d_mom = np.diff(red[:, k_mom])
    want = nx * ny * F - red[1:, k_wall]
    assert np.abs(red[1:, k_wall]).max() > 1e-3 * nx * ny * F  # the walls take a real share
    np.testing.assert_allclose(d_mom, want, rtol=0, atol=1e-15)
