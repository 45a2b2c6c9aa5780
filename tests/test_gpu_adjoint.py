"""GPU discrete adjoint (through the C-ABI) against the FP64 oracle.

The oracle's derivatives are complex-step tangents of its own run (exact to
rounding for these analytic steps) and its own discrete adjoint (a reverse
sweep of its recorded run, which gives the whole dL/drho0 field).  Bars: the FP64 GPU gradients within
1e-9 relative of them, the FP32-storage gradients within 1e-3.  At the full
falling-droplet adjoint size (512 x 2048, 20,000 steps, checkpoints every 500)
the oracle is too slow; there the GPU gradients are checked against central
finite differences of the FP64 GPU run, which is itself pinned to the oracle
by the forward parity tests.
"""
import numpy as np
import pytest
import torch
from dataclasses import replace

from oracle import oracle as O
from paper_2604_13407_amd import adjoint as AD
from paper_2604_13407_amd import lattice as LT
from paper_2604_13407_amd import workloads as WL
from tests.helpers import oracle_params

pytestmark = pytest.mark.gpu

N_SMALL, W_SMALL, K_SMALL = 30, 10, 7


def lattice_for(w, precision=LT.FP64, kernel=LT.KERNEL_FUSED, mask=None):
    rho_ref = w.rho_g if precision == LT.FP32_DEV else 0.0
    lat = LT.Lattice(w.nx, w.ny, w.periodic_x, w.periodic_y, precision, kernel, rho_ref,
                     mask=w.mask() if mask is None else mask)
    lat.set_eos(w.eos_kind, w.a, w.b, w.R, w.T, w.k_eos)
    lat.set_G(w.G)
    lat.set_relaxation(w.s)
    lat.set_scheme(w.scheme, w.eps, w.k1, w.k2)
    lat.set_body_force(w.force_mode, w.fx, w.fy)
    lat.set_phase_densities(w.rho_g, w.rho_l)
    lat.set_walls(w.rho_s)
    return lat


def small_case(name):
    """(workload, mask, loss kind, u_target) of a small case the oracle runs in seconds."""
    w = WL.small_droplet(nx=24, ny=32, radius=6.0, g=1e-5)
    mask = None
    if name.startswith("masked"):
        # periodic in x, the original scheme, two solid blocks (one touching the bottom wall row)
        w = replace(w, periodic_x=True, scheme=WL.SCHEME_ORIGINAL)
        mask = np.zeros((w.ny, w.nx), np.uint8)
        mask[12:16, 3:7] = 1
        mask[0:2, 20:22] = 1
    kind = LT.LOSS_UERR if name.endswith("uerr") else LT.LOSS_DRAG
    ut = np.random.default_rng(1).normal(size=(w.ny, w.nx)) * 1e-4 if kind == LT.LOSS_UERR else None
    return w, mask, kind, ut


def directions(w, n=2):
    return [np.random.default_rng(10 + i).uniform(-1.0, 1.0, (w.ny, w.nx)) for i in range(n)]


def oracle_derivatives(w, mask, kind, ut, n, window, vs):
    p = oracle_params(w)
    rho0 = w.rho0()
    L, dG = O.loss(p, rho0, n, kind, window=window, u_target=ut, mask=mask, perturb=O.PERTURB_G)
    _, dg = O.loss(p, rho0, n, kind, window=window, u_target=ut, mask=mask, perturb=O.PERTURB_FORCE)
    dv = [O.loss(p, rho0, n, kind, window=window, u_target=ut, mask=mask, perturb=O.PERTURB_RHO0, v=v)[1]
          for v in vs]
    return L, dG, dg, dv


def gpu_gradients(w, mask, kind, ut, n, window, k, precision=LT.FP64, kernel=LT.KERNEL_FUSED):
    lat = lattice_for(w, precision, kernel, mask)
    L = lat.adjoint_forward(w.rho0(), n, loss=kind, window=window, checkpoint_every=k, u_target=ut)
    g, gf, gG = lat.adjoint_backward()
    torch.cuda.synchronize()
    return L, gG, gf, g.cpu().numpy(), lat


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


SMALL = ("drag", "uerr", "masked_drag", "masked_uerr")


@pytest.fixture(scope="module")
def oracle_small():
    out = {}
    for name in SMALL:
        w, mask, kind, ut = small_case(name)
        out[name] = oracle_derivatives(w, mask, kind, ut, N_SMALL, W_SMALL, directions(w))
    return out


@pytest.mark.parametrize("name", SMALL)
def test_fp64_adjoint_matches_oracle_complex_step(name, oracle_small):
    w, mask, kind, ut = small_case(name)
    Lo, dGo, dgo, dvo = oracle_small[name]
    L, gG, gf, g, _ = gpu_gradients(w, mask, kind, ut, N_SMALL, W_SMALL, K_SMALL)
    print(f"{name}: L {L:.6e} dG {gG:.6e} (oracle {dGo:.6e}) dg {gf:.6e} (oracle {dgo:.6e})", flush=True)
    assert rel(L, Lo) <= 1e-11, (L, Lo)
    assert rel(gG, dGo) <= 1e-9, (gG, dGo)
    assert rel(gf, dgo) <= 1e-9, (gf, dgo)
    for v, d in zip(directions(w), dvo):
        assert rel(float((g * v).sum()), d) <= 1e-9, (float((g * v).sum()), d)
    if mask is not None:
        assert np.all(g[mask == 1] == 0.0)


@pytest.mark.parametrize("name", ("drag", "masked_uerr"))
@pytest.mark.parametrize("precision", (LT.FP64, LT.FP32_DEV))
def test_gradient_field_matches_the_oracle_adjoint(name, precision):
    """dL/drho0 node by node, dL/dG and dL/d|F| against the oracle's own discrete adjoint
    (a reverse sweep of its recorded run)."""
    w, mask, kind, ut = small_case(name)
    Lo, go, dGo, dFo = O.adjoint(oracle_params(w), w.rho0(), N_SMALL, kind, window=W_SMALL, u_target=ut, mask=mask)
    L, gG, gf, g, _ = gpu_gradients(w, mask, kind, ut, N_SMALL, W_SMALL, K_SMALL, precision=precision)
    tol = 1e-9 if precision == LT.FP64 else 1e-3
    err = np.max(np.abs(g - go)) / np.max(np.abs(go))
    print(f"{name} {precision}: field err {err:.2e} dG {rel(gG, dGo):.2e} dF {rel(gf, dFo):.2e}", flush=True)
    assert err <= tol
    assert rel(gG, dGo) <= tol and rel(gf, dFo) <= tol


@pytest.mark.parametrize("name", ("drag", "uerr", "masked_drag"))
def test_fp32_adjoint_within_bar(name, oracle_small):
    w, mask, kind, ut = small_case(name)
    Lo, dGo, dgo, dvo = oracle_small[name]
    L, gG, gf, g, _ = gpu_gradients(w, mask, kind, ut, N_SMALL, W_SMALL, K_SMALL, precision=LT.FP32_DEV)
    print(f"{name} fp32: L rel {rel(L, Lo):.2e} dG rel {rel(gG, dGo):.2e} dg rel {rel(gf, dgo):.2e}", flush=True)
    # the drag loss is a difference of sums (buoyant weight minus a momentum rate) that cancel to
    # about 1/20 of either; it gets the gradients' bar
    assert rel(L, Lo) <= 1e-3
    assert rel(gG, dGo) <= 1e-3 and rel(gf, dgo) <= 1e-3
    for v, d in zip(directions(w), dvo):
        assert rel(float((g * v).sum()), d) <= 1e-3


@pytest.mark.parametrize("precision", (LT.FP64, LT.FP32_DEV))
def test_checkpoint_interval_does_not_change_the_gradients(precision):
    w, mask, kind, ut = small_case("drag")
    ref = gpu_gradients(w, mask, kind, ut, N_SMALL, W_SMALL, N_SMALL, precision=precision)
    for k in (1, 4, K_SMALL, 1000):
        out = gpu_gradients(w, mask, kind, ut, N_SMALL, W_SMALL, k, precision=precision)
        assert out[0] == ref[0] and out[1] == ref[1] and out[2] == ref[2], k
        assert np.array_equal(out[3], ref[3]), k


@pytest.mark.parametrize("precision", (LT.FP64, LT.FP32_DEV))
def test_two_pass_and_fused_forward_give_the_same_gradients(precision):
    w, mask, kind, ut = small_case("masked_drag")
    a = gpu_gradients(w, mask, kind, ut, N_SMALL, W_SMALL, K_SMALL, precision, LT.KERNEL_FUSED)
    b = gpu_gradients(w, mask, kind, ut, N_SMALL, W_SMALL, K_SMALL, precision, LT.KERNEL_TWO_PASS)
    tol = 1e-11 if precision == LT.FP64 else 0.0
    assert rel(a[1], b[1]) <= tol and rel(a[2], b[2]) <= tol
    assert np.max(np.abs(a[3] - b[3])) <= tol * np.max(np.abs(b[3]))


def test_backward_is_repeatable_and_leaves_the_run_state():
    w, mask, kind, ut = small_case("drag")
    L, gG, gf, g, lat = gpu_gradients(w, mask, kind, ut, N_SMALL, W_SMALL, K_SMALL)
    state = lat.state().clone()
    assert lat.step_count == N_SMALL
    g2, gf2, gG2 = lat.adjoint_backward()
    assert np.array_equal(g2.cpu().numpy(), g) and gf2 == gf and gG2 == gG
    assert torch.equal(lat.state(), state)
    # the run is the ordinary stepping from rest
    ref = lattice_for(w)
    ref.init_equilibrium(w.rho0())
    ref.step(N_SMALL)
    assert torch.equal(ref.state(), state)
    # a parameter change invalidates the recorded forward pass
    lat.set_G(w.G)
    with pytest.raises(LT.LbmError) as e:
        lat.adjoint_backward()
    assert e.value.code == -6


def test_autograd_function_chains_the_adjoint():
    w, mask, kind, ut = small_case("drag")
    lat = lattice_for(w)
    dev = lat.device
    gmag = float(np.hypot(w.fx, w.fy))
    f = torch.tensor(gmag, dtype=torch.float64, device=dev, requires_grad=True)
    G = torch.tensor(w.G, dtype=torch.float64, device=dev, requires_grad=True)
    rho0 = torch.tensor(w.rho0(), dtype=torch.float64, device=dev, requires_grad=True)
    L = AD.lbm_loss(f, G, rho0, lat, n_steps=N_SMALL, loss=LT.LOSS_DRAG, window=W_SMALL,
                    checkpoint_every=K_SMALL)
    (3.0 * L).backward()
    Lr, gG, gf, g, _ = gpu_gradients(w, mask, kind, ut, N_SMALL, W_SMALL, K_SMALL)
    assert float(L.detach()) == Lr
    assert float(f.grad) == 3.0 * gf and float(G.grad) == 3.0 * gG
    assert np.array_equal(rho0.grad.cpu().numpy(), 3.0 * g)


# ------------------------------------------------------------------ grid-aligned Poiseuille, velocity error

def poiseuille_target(w):
    """u_x of (rho nu u')' = -F across the channel with the initial density profile and
    no slip at the halfway walls (uniform kinematic viscosity nu = (1/s_nu - 1/2)/3)."""
    nu = (1.0 / w.s[7] - 0.5) / 3.0
    rho = w.rho0()[:, 0]
    y = np.arange(w.ny, dtype=np.float64)
    yc = 0.5 * (w.ny - 1)
    fine = np.linspace(-0.5, w.ny - 0.5, 20 * w.ny + 1)
    rf = np.interp(fine, y, rho)
    du = -w.fx * (fine - yc) / (nu * rf)
    u = np.concatenate(([0.0], np.cumsum(0.5 * (du[1:] + du[:-1]) * np.diff(fine))))
    u -= np.interp(w.ny - 0.5, fine, u) * (fine + 0.5) / w.ny  # exact zero at both walls
    prof = np.interp(y, fine, u)
    return np.ascontiguousarray(np.broadcast_to(prof[:, None], (w.ny, w.nx)))


@pytest.mark.parametrize("precision", (LT.FP64, LT.FP32_DEV))
def test_aligned_poiseuille_velocity_error_gradients(precision):
    """Grid-aligned two-phase Poiseuille (4 x 100, walls in y): gradients of the
    velocity error after 2,000 steps against the oracle's complex step."""
    w = WL.poiseuille_aligned()
    n, k = 2000, 300
    ut = poiseuille_target(w)
    vs = directions(w, 1)
    Lo, dGo, dgo, dvo = oracle_derivatives(w, None, LT.LOSS_UERR, ut, n, 2, vs)
    L, gG, gf, g, _ = gpu_gradients(w, None, LT.LOSS_UERR, ut, n, 2, k, precision=precision)
    tol = 1e-9 if precision == LT.FP64 else 1e-3
    print(f"poiseuille {precision}: L {L:.6e} ({Lo:.6e}) dG {rel(gG, dGo):.2e} dg {rel(gf, dgo):.2e}", flush=True)
    assert rel(L, Lo) <= (1e-11 if precision == LT.FP64 else 1e-3)
    assert rel(gG, dGo) <= tol and rel(gf, dgo) <= tol
    assert rel(float((g * vs[0]).sum()), dvo[0]) <= tol


# ------------------------------------------------------------------ full size: falling droplet adjoint

def run_loss(w, precision, gmag=None, G=None, rho0=None, n=None, window=5000):
    lat = lattice_for(w, precision)
    if gmag is not None:
        lat.set_force_magnitude(gmag)
    if G is not None:
        lat.set_G(G)
    L = lat.adjoint_forward(w.rho0() if rho0 is None else rho0, n or w.steps, loss=LT.LOSS_DRAG, window=window,
                            checkpoint_every=500)
    return L, lat


@pytest.mark.parametrize("precision", (LT.FP32_DEV, LT.FP64))
def test_full_size_droplet_adjoint_against_central_differences(precision):
    """Central differences with h = 1e-4 (relative for |g|, absolute along a +-1 field for
    rho0).  For G the loss is curved on that scale (the droplet's shape oscillation shifts
    with G: the h = 1e-4 quotient is 3% below its limit), so G takes h = 3e-6, where the
    quotients have converged; the h = 1e-4 quotient must still be farther from the adjoint."""
    w = WL.droplet_adjoint()
    gmag = float(np.hypot(w.fx, w.fy))
    h, hG = 1e-4, 3e-6
    L, lat = run_loss(w, precision)
    g, gf, gG = lat.adjoint_backward()
    v = np.random.default_rng(99).choice([-1.0, 1.0], size=(w.ny, w.nx))
    gv = float((g.cpu().numpy() * v).sum())
    del lat
    torch.cuda.empty_cache()
    # central differences of the FP64 run
    fd_g = (run_loss(w, LT.FP64, gmag=gmag * (1 + h))[0] - run_loss(w, LT.FP64, gmag=gmag * (1 - h))[0]) / (
        2 * h * gmag)
    fd_G = (run_loss(w, LT.FP64, G=w.G * (1 + hG))[0] - run_loss(w, LT.FP64, G=w.G * (1 - hG))[0]) / (2 * hG * w.G)
    fd_G_coarse = (run_loss(w, LT.FP64, G=w.G * (1 + h))[0] - run_loss(w, LT.FP64, G=w.G * (1 - h))[0]) / (
        2 * h * w.G)
    r0 = w.rho0()
    fd_v = (run_loss(w, LT.FP64, rho0=r0 + h * v)[0] - run_loss(w, LT.FP64, rho0=r0 - h * v)[0]) / (2 * h)
    print(f"droplet adjoint {precision}: L {L:.8e} dL/dg {gf:.6e} (FD {fd_g:.6e}) dL/dG {gG:.6e} (FD {fd_G:.6e}, "
          f"h=1e-4: {fd_G_coarse:.6e}) dL/drho0.v {gv:.6e} (FD {fd_v:.6e})", flush=True)
    assert rel(gf, fd_g) <= 1e-3
    assert rel(gG, fd_G) <= 1e-3
    assert abs(gG - fd_G) < abs(gG - fd_G_coarse)
    assert rel(gv, fd_v) <= 1e-3


def test_longer_horizon_droplet_against_the_oracle():
    """64 x 128 droplet channel, 2,000 steps, drag over the last 500: GPU FP64 adjoint
    against the oracle's complex step."""
    w = WL.small_droplet(nx=64, ny=128, radius=16.0, g=1e-6)
    n = 2000
    vs = directions(w, 1)
    Lo, dGo, dgo, dvo = oracle_derivatives(w, None, LT.LOSS_DRAG, None, n, n // 4, vs)
    L, gG, gf, g, _ = gpu_gradients(w, None, LT.LOSS_DRAG, None, n, n // 4, 100)
    assert rel(L, Lo) <= 1e-11
    assert rel(gG, dGo) <= 1e-9 and rel(gf, dgo) <= 1e-9
    assert rel(float((g * vs[0]).sum()), dvo[0]) <= 1e-9


def aligned_masked_case():
    """A masked lattice of width 64 (one strip: the forward and replay steps run on
    the masked strip march), periodic in x, the original scheme."""
    w = WL.small_droplet(nx=64, ny=32, radius=7.0, g=1e-5)
    w = replace(w, periodic_x=True, scheme=WL.SCHEME_ORIGINAL)
    mask = np.zeros((w.ny, w.nx), np.uint8)
    mask[12:16, 3:7] = 1
    mask[0:2, 50:53] = 1
    mask[25, 63] = 1
    return w, mask


@pytest.mark.parametrize("precision", [LT.FP64, LT.FP32_DEV])
def test_adjoint_on_the_masked_strip_march(precision):
    # The adjoint's forward run and its replays take the masked strip march on
    # this lattice: the gradients equal the tile kernel's (to the rounding of
    # sums grouped differently) and, in FP64, the oracle's complex-step
    # derivatives.
    w, mask = aligned_masked_case()
    kind = LT.LOSS_DRAG
    outs = []
    for masked in (True, False):
        lat = lattice_for(w, precision, LT.KERNEL_FUSED, mask)
        lat.set_masked_strips(masked)
        L = lat.adjoint_forward(w.rho0(), N_SMALL, loss=kind, window=W_SMALL, checkpoint_every=K_SMALL)
        g, gf, gG = lat.adjoint_backward()
        torch.cuda.synchronize()
        outs.append((L, gG, gf, g.cpu().numpy()))
    (La, gGa, gfa, ga), (Lb, gGb, gfb, gb) = outs
    if precision == LT.FP32_DEV:
        # the replayed states are bitwise equal; the loss and the parameter
        # gradients are sums grouped by the kernels' runs or tiles
        assert rel(La, Lb) <= 1e-12 and rel(gGa, gGb) <= 1e-12 and rel(gfa, gfb) <= 1e-12
        assert np.max(np.abs(ga - gb)) <= 1e-12 * np.max(np.abs(gb))
    else:
        assert rel(La, Lb) <= 1e-12 and rel(gGa, gGb) <= 1e-11 and rel(gfa, gfb) <= 1e-11
        assert np.max(np.abs(ga - gb)) <= 1e-11 * np.max(np.abs(gb))
        Lo, dGo, dgo, dvo = oracle_derivatives(w, mask, kind, None, N_SMALL, W_SMALL, directions(w, 1))
        print(f"masked march adjoint: L {La:.6e} (oracle {Lo:.6e}) dG {gGa:.6e} ({dGo:.6e}) "
              f"dg {gfa:.6e} ({dgo:.6e})", flush=True)
        assert rel(La, Lo) <= 1e-11, (La, Lo)
        assert rel(gGa, dGo) <= 1e-9 and rel(gfa, dgo) <= 1e-9
        v = directions(w, 1)[0]
        assert rel(float(np.sum(ga * v)), dvo[0]) <= 1e-9
    assert np.all(ga[mask == 1] == 0.0)
