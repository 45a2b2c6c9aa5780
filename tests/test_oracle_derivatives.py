"""The oracle's derivatives (complex step) against central finite differences.

Complex step evaluates the loss with one input carrying an imaginary part
i h v; Im L / h is the exact directional derivative of the discrete map up to
rounding.  It is pinned here against central differences of real runs, which
share only the forward arithmetic with it.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2604_13407_amd import workloads as WL
from tests.helpers import oracle_params


def small_case(scheme=O.SCHEME_IMPROVED):
    w = WL.small_droplet(nx=20, ny=28, radius=5.0, scheme=scheme, g=2e-6, perturb=1e-4)
    return w, oracle_params(w)


def fd(fun, x0, h):
    return (fun(x0 + h) - fun(x0 - h)) / (2 * h)


@pytest.mark.parametrize("scheme", [O.SCHEME_ORIGINAL, O.SCHEME_IMPROVED])
def test_drag_loss_gradients_match_central_differences(scheme):
    w, p = small_case(scheme)
    rho0 = w.rho0()
    n, win = 30, 10
    L0, dLg = O.loss(p, rho0, n, O.LOSS_DRAG, window=win, perturb=O.PERTURB_FORCE, h=1e-30)
    _, dLG = O.loss(p, rho0, n, O.LOSS_DRAG, window=win, perturb=O.PERTURB_G, h=1e-30)

    def L_of_g(g):
        q = oracle_params(w, fy=-g)
        return O.loss(q, rho0, n, O.LOSS_DRAG, window=win)[0]

    def L_of_G(G):
        q = oracle_params(w, G=G)
        return O.loss(q, rho0, n, O.LOSS_DRAG, window=win)[0]

    g0 = -w.fy
    assert dLg == pytest.approx(fd(L_of_g, g0, 1e-3 * g0), rel=1e-6)
    assert dLG == pytest.approx(fd(L_of_G, -1.0, 1e-5), rel=1e-6)

    rng = np.random.default_rng(5)
    v = rng.standard_normal(rho0.shape)
    _, dLr = O.loss(p, rho0, n, O.LOSS_DRAG, window=win, perturb=O.PERTURB_RHO0, v=v, h=1e-30)
    h = 1e-7
    Lp = O.loss(p, rho0 + h * v, n, O.LOSS_DRAG, window=win)[0]
    Lm = O.loss(p, rho0 - h * v, n, O.LOSS_DRAG, window=win)[0]
    assert dLr == pytest.approx((Lp - Lm) / (2 * h), rel=1e-5)


def test_velocity_error_loss_gradient_matches_central_differences():
    w = WL.poiseuille_aligned().with_size(4, 40, init_args={"y0": 10, "y1": 30})
    p = oracle_params(w)
    rho0 = w.rho0()
    target = np.full(rho0.shape, 1e-6)
    n = 50
    L0, dLF = O.loss(p, rho0, n, O.LOSS_UERR, u_target=target, perturb=O.PERTURB_FORCE, h=1e-30)
    assert L0 > 0

    def L_of_F(F):
        return O.loss(oracle_params(w, fx=F), rho0, n, O.LOSS_UERR, u_target=target)[0]

    assert dLF == pytest.approx(fd(L_of_F, w.fx, 1e-3 * w.fx), rel=1e-6)


def test_complex_step_leaves_the_real_part_unchanged():
    w, p = small_case()
    rho0 = w.rho0()
    a = O.loss(p, rho0, 12, O.LOSS_DRAG, window=4)[0]
    b = O.loss(p, rho0, 12, O.LOSS_DRAG, window=4, perturb=O.PERTURB_G, h=1e-30)[0]
    assert a == b
    # and the real-valued loss equals the observables of a plain run
    o = O.Oracle(p).init(rho0)
    red = o.step(12, reductions=True)
    names = O.RED_NAMES
    buoy, pphi = red[:, names.index("buoy")], red[:, names.index("pphi")]
    want = buoy[-4:].mean() - (pphi[-1] - pphi[-4]) / 3
    assert a == pytest.approx(want, rel=1e-13)


# ---------------------------------------------------------------- the oracle's own adjoint

def tiny_case(name):
    """12 x 16 droplet channel, and variants with a solid block, periodic x, the original
    scheme, van der Waals EOS and a moving wall."""
    w = WL.small_droplet(nx=12, ny=16, radius=3.0, g=1e-5)
    mask = wall_u = None
    if name in ("masked", "moving"):
        from dataclasses import replace
        w = replace(w, periodic_x=True, scheme=O.SCHEME_ORIGINAL)
        mask = np.zeros((w.ny, w.nx), np.uint8)
        mask[6:9, 2:4] = 1
        mask[0, 9:11] = 1
        if name == "moving":
            wall_u = np.zeros((2, w.ny, w.nx))
            wall_u[0][mask == 1] = 0.01
    if name == "vdw":
        # the paper's van der Waals constants (a = 9/49, b = 2/21, R = 1) at T = 0.5 T_c: a
        # vapour (the eps = 1.895 mechanical-stability density 0.07311) with a denser vapour bump
        from dataclasses import replace
        a, b = 9.0 / 49.0, 2.0 / 21.0
        w = replace(w, eos_kind=O.EOS_VDW, a=a, b=b, R=1.0, T=0.5 * 8 * a / (27 * b), rho_g=0.07311,
                    rho_l=0.12, rho_s=0.07311)
    return w, mask, wall_u


@pytest.mark.parametrize("name", ["droplet", "masked", "moving", "vdw"])
@pytest.mark.parametrize("kind", [O.LOSS_DRAG, O.LOSS_UERR])
def test_oracle_adjoint_matches_its_complex_step(name, kind):
    """The taped reverse sweep is the transpose of the same arithmetic the complex step
    differentiates forward: <dL/drho0, v> and dL/dG, dL/d|F| agree to rounding."""
    w, mask, wall_u = tiny_case(name)
    p = oracle_params(w)
    rho0 = w.rho0()
    n, win = 12, 5
    ut = np.random.default_rng(2).normal(size=rho0.shape) * 1e-4
    kw = dict(window=win, u_target=ut, mask=mask, wall_u=wall_u)
    L, g, dG, dF = O.adjoint(p, rho0, n, kind, **kw)
    Lc, dGc = O.loss(p, rho0, n, kind, perturb=O.PERTURB_G, **kw)
    _, dFc = O.loss(p, rho0, n, kind, perturb=O.PERTURB_FORCE, **kw)
    assert L == Lc
    assert dG == pytest.approx(dGc, rel=1e-10, abs=1e-13 * abs(L))
    assert dF == pytest.approx(dFc, rel=1e-10)
    for seed in (3, 4):
        v = np.random.default_rng(seed).uniform(-1, 1, rho0.shape)
        _, dv = O.loss(p, rho0, n, kind, perturb=O.PERTURB_RHO0, v=v, **kw)
        assert float((g * v).sum()) == pytest.approx(dv, rel=1e-10)
    if mask is not None:
        assert np.all(g[mask == 1] == 0.0)


def test_oracle_adjoint_is_the_gradient_node_by_node():
    """Single-node directions: each component of dL/drho0 equals the complex-step
    derivative along that node's unit vector."""
    w, mask, wall_u = tiny_case("droplet")
    p = oracle_params(w)
    rho0 = w.rho0()
    n, win = 8, 3
    _, g, _, _ = O.adjoint(p, rho0, n, O.LOSS_DRAG, window=win)
    for (y, x) in ((0, 0), (7, 5), (8, 6), (15, 11), (3, 9)):
        v = np.zeros(rho0.shape)
        v[y, x] = 1.0
        _, d = O.loss(p, rho0, n, O.LOSS_DRAG, window=win, perturb=O.PERTURB_RHO0, v=v)
        assert g[y, x] == pytest.approx(d, rel=1e-10, abs=1e-14 * np.abs(g).max())
