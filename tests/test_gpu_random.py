"""Seeded random configurations of the step, through the C-ABI, against the
oracle.

Each case draws, from its own seed, a lattice size (widths below, at and
above multiples of 64, one-row and one-column lattices), periodic or walled
axes, no mask, scattered solid nodes or solid blobs, resting or moving walls,
the scheme, a constant or buoyant force, the precision, the fused or the
two-pass kernel, the rows per wavefront and a reduction interval.  The initial
densities are random (0.05-0.25), so every term of the step is far from zero.
The bars are those of the parity tests: FP64 within 1e-12 of each field's
scale (velocities: of max(peak, 1e-2), as for the edge shapes, whose random
densities drive their own currents), float storage within 1e-5 of the density
and 1e-4 of max(peak speed, 1e-3); the reduction records to rounding.  The
floor matters on the tiniest periodic lattices, where the random densities
even out within a few steps and only the body force moves the fluid (peak
~1e-5): float storage then rounds deviations from references the initial
densities left stale by up to a third, ~1e-9 in u.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2604_13407_amd import lattice as LT
from paper_2604_13407_amd import workloads as WL
from tests.helpers import fp64_bar
from tests.test_gpu_parity import FIELDS, field_scale, gpu_fields

pytestmark = pytest.mark.gpu

N_CASES = 200


def blobs(nx, ny, rng):
    m = np.zeros((ny, nx), np.uint8)
    yy, xx = np.mgrid[0:ny, 0:nx]
    for _ in range(max(1, nx * ny // 200)):
        cx, cy, r = rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(1.0, 3.5)
        m[(xx - cx) ** 2 + (yy - cy) ** 2 < r * r] = 1
    return m


def draw(seed):
    rng = np.random.default_rng(1000 + seed)
    c = dict(
        # half the widths a multiple of 64 (the strip marches), half not
        nx=int(64 * rng.integers(1, 5)) if rng.random() < 0.5 else int(rng.choice([1, 2, 3, 17, 62, 63, 65, 127,
                                                                                    129, 200])),
        ny=int(rng.choice([1, 2, 3, 5, 8, 13, 24, 40, 67, 100])),
        px=bool(rng.random() < 0.6), py=bool(rng.random() < 0.6),
        scheme=int(rng.integers(0, 2)), buoyant=bool(rng.random() < 0.5),
        precision=LT.FP64 if rng.random() < 0.5 else LT.FP32_DEV,
        kernel=LT.KERNEL_TWO_PASS if rng.random() < 0.25 else LT.KERNEL_FUSED,
        steps=int(rng.integers(3, 12)), reduce_every=int(rng.choice([0, 1, 2, 3])),
        rows=int(rng.choice([0, 0, 1, 2, 5])))
    kind = str(rng.choice(["none", "scatter", "blobs"])) if c["nx"] * c["ny"] > 50 else "none"
    mask = None
    if kind == "scatter":
        mask = (rng.random((c["ny"], c["nx"])) < 0.1).astype(np.uint8)
    elif kind == "blobs":
        mask = blobs(c["nx"], c["ny"], rng)
    wall_u = None
    if mask is not None and rng.random() < 0.4:
        wall_u = np.zeros((2, c["ny"], c["nx"]))
        wall_u[:, mask == 1] = rng.uniform(-0.02, 0.02, (2, int(mask.sum())))
    c.update(mask=mask, wall_u=wall_u, kind=kind, moving=wall_u is not None,
             rho0=0.05 + 0.2 * rng.random((c["ny"], c["nx"])))
    return c


@pytest.mark.parametrize("seed", range(N_CASES))
def test_random_configuration_matches_oracle(seed):
    c = draw(seed)
    nx, ny = c["nx"], c["ny"]
    print(f"[random] seed={seed} {nx}x{ny} px={c['px']} py={c['py']} mask={c['kind']} moving={c['moving']} "
          f"scheme={c['scheme']} buoyant={c['buoyant']} precision={c['precision']} kernel={c['kernel']} "
          f"steps={c['steps']} reduce_every={c['reduce_every']} rows={c['rows']}", flush=True)
    w = WL.small_droplet()
    fmode = LT.FORCE_BUOYANT if c["buoyant"] else LT.FORCE_CONST
    fx, fy = (1e-6, -2e-6) if c["buoyant"] else (2e-6, 1e-6)
    lat = LT.Lattice(nx, ny, c["px"], c["py"], c["precision"], c["kernel"], mask=c["mask"], wall_u=c["wall_u"])
    lat.set_eos(w.eos_kind, w.a, w.b, w.R, w.T, w.k_eos)
    lat.set_relaxation(w.s)
    lat.set_scheme(c["scheme"], w.eps)
    lat.set_body_force(fmode, fx, fy)
    lat.set_phase_densities(w.rho_g, w.rho_l)
    lat.set_walls(w.rho_s)
    if c["rows"]:
        lat.set_rows_per_wave(c["rows"])
    lat.init_equilibrium(c["rho0"])
    recs = lat.step(c["steps"], reduce_every=c["reduce_every"])
    g = gpu_fields(lat)

    p = O.Params(nx=nx, ny=ny, periodic_x=c["px"], periodic_y=c["py"], eos_kind=w.eos_kind, a=w.a, b=w.b, R=w.R,
                 T=w.T, k_eos=w.k_eos, eps=w.eps, s=w.s, scheme=c["scheme"],
                 force_mode=O.FORCE_BUOYANT if c["buoyant"] else O.FORCE_CONST, fx=fx, fy=fy,
                 rho_g=w.rho_g, rho_l=w.rho_l, rho_s=w.rho_s)
    o = O.Oracle(p, mask=c["mask"], wall_u=c["wall_u"]).init(c["rho0"])
    red = o.step(c["steps"], reductions=True)
    om = o.macros()
    fl = np.ones((ny, nx), bool) if c["mask"] is None else c["mask"] == 0
    if not fl.any():
        return
    umax = max(np.max(np.abs(om["ux"][fl])), np.max(np.abs(om["uy"][fl])), 1e-300)
    if c["precision"] == LT.FP64:
        psi_max = np.max(np.abs(om["psi"]))
        for k in FIELDS:
            err = np.max(np.abs(g[k][fl] - om[k][fl])) / field_scale(k, om[k][fl], psi_max)
            assert err <= fp64_bar(c["steps"]), (seed, k, err)
        f = lat.state().cpu().numpy()
        err = np.max(np.abs(f[:, fl] - o.f[:, fl])) / np.max(np.abs(o.f[:, fl]))
        assert err <= fp64_bar(c["steps"]), (seed, "f", err)
    else:
        rerr = np.max(np.abs(g["rho"][fl] - om["rho"][fl]) / om["rho"][fl])
        du = max(np.max(np.abs(g["ux"][fl] - om["ux"][fl])), np.max(np.abs(g["uy"][fl] - om["uy"][fl])))
        assert rerr <= 1e-5, (seed, "rho", rerr)
        assert du <= 1e-4 * max(umax, 1e-3), (seed, "u", du, umax)

    # reduction records: the steps asked for, each against the oracle's observables of that step
    k = c["reduce_every"]
    expect = [s for s in range(1, c["steps"] + 1) if k and s % k == 0]
    assert [r["step"] for r in recs] == expect
    names = O.RED_NAMES
    tol = 1e-11 if c["precision"] == LT.FP64 else 1e-4
    for r in recs:
        ref = dict(zip(names, red[r["step"] - 1]))
        mass = ref["mass"]
        # momentum-like sums are bounded by mass x peak speed (the peak of this run)
        mom_scale = mass * max(umax, 1e-3)
        for kg, ko, scale in (("mass", "mass", mass), ("uc_den", "uc_den", mass), ("buoy", "buoy", mass * 1e-6),
                              ("mom_x", "momx", mom_scale), ("mom_y", "momy", mom_scale),
                              ("wall_x", "wallx", mom_scale), ("wall_y", "wally", mom_scale),
                              ("uc_num", "uc_num", mom_scale), ("pphi", "pphi", mom_scale)):
            assert abs(r[kg] - ref[ko]) <= tol * max(abs(ref[ko]), scale), (seed, kg, r[kg], ref[ko])
        assert r["faults"] == ref["faults"] == 0


N_ADJ = 24


def draw_adjoint(seed):
    """A small random adjoint case (node-steps kept within the oracle's tape)."""
    rng = np.random.default_rng(5000 + seed)
    nx = int(rng.choice([8, 13, 24, 64, 65, 128]))
    ny = int(rng.choice([6, 9, 16, 24]))
    n = int(rng.integers(4, 21))
    while nx * ny * n > 25000:
        n -= 1
    c = dict(nx=nx, ny=ny, n=n, px=bool(rng.random() < 0.6), py=bool(rng.random() < 0.6),
             scheme=int(rng.integers(0, 2)), precision=LT.FP64 if rng.random() < 0.5 else LT.FP32_DEV,
             kernel=LT.KERNEL_TWO_PASS if rng.random() < 0.25 else LT.KERNEL_FUSED,
             loss=LT.LOSS_UERR if rng.random() < 0.5 else LT.LOSS_DRAG,
             window=int(rng.integers(2, n + 1)), k=int(rng.integers(1, n + 4)))
    # the drag loss weighs the buoyant force; the velocity error takes either force
    c["buoyant"] = c["loss"] == LT.LOSS_DRAG or bool(rng.random() < 0.5)
    kind = str(rng.choice(["none", "scatter", "blobs"]))
    mask = None
    if kind == "scatter":
        mask = (rng.random((ny, nx)) < 0.1).astype(np.uint8)
    elif kind == "blobs":
        mask = blobs(nx, ny, rng)
    c.update(mask=mask, kind=kind, rho0=0.05 + 0.2 * rng.random((ny, nx)),
             ut=rng.normal(size=(ny, nx)) * 1e-3 if c["loss"] == LT.LOSS_UERR else None)
    return c


@pytest.mark.parametrize("seed", range(N_ADJ))
def test_random_adjoint_matches_the_oracle_adjoint(seed):
    """dL/drho0 node by node, dL/dG and dL/d|F| of a random small case against the
    oracle's own discrete adjoint: FP64 within 1e-9, float storage within 1e-3."""
    c = draw_adjoint(seed)
    nx, ny = c["nx"], c["ny"]
    print(f"[random adjoint] seed={seed} {nx}x{ny} n={c['n']} px={c['px']} py={c['py']} mask={c['kind']} "
          f"scheme={c['scheme']} buoyant={c['buoyant']} precision={c['precision']} kernel={c['kernel']} "
          f"loss={c['loss']} window={c['window']} k={c['k']}", flush=True)
    w = WL.small_droplet()
    fmode = LT.FORCE_BUOYANT if c["buoyant"] else LT.FORCE_CONST
    fx, fy = (0.0, -1e-5) if c["buoyant"] else (2e-6, 1e-6)
    rho_ref = w.rho_g if c["precision"] == LT.FP32_DEV else 0.0
    lat = LT.Lattice(nx, ny, c["px"], c["py"], c["precision"], c["kernel"], rho_ref, mask=c["mask"])
    lat.set_eos(w.eos_kind, w.a, w.b, w.R, w.T, w.k_eos)
    lat.set_relaxation(w.s)
    lat.set_scheme(c["scheme"], w.eps)
    lat.set_body_force(fmode, fx, fy)
    lat.set_phase_densities(w.rho_g, w.rho_l)
    lat.set_walls(w.rho_s)
    L = lat.adjoint_forward(c["rho0"], c["n"], loss=c["loss"], window=c["window"], checkpoint_every=c["k"],
                            u_target=c["ut"])
    g, gF, gG = lat.adjoint_backward()
    torch.cuda.synchronize()
    g = g.cpu().numpy()

    p = O.Params(nx=nx, ny=ny, periodic_x=c["px"], periodic_y=c["py"], eos_kind=w.eos_kind, a=w.a, b=w.b, R=w.R,
                 T=w.T, k_eos=w.k_eos, eps=w.eps, s=w.s, scheme=c["scheme"],
                 force_mode=O.FORCE_BUOYANT if c["buoyant"] else O.FORCE_CONST, fx=fx, fy=fy,
                 rho_g=w.rho_g, rho_l=w.rho_l, rho_s=w.rho_s)
    Lo, go, dGo, dFo = O.adjoint(p, c["rho0"], c["n"], c["loss"], window=c["window"], u_target=c["ut"],
                                 mask=c["mask"])
    tol = 1e-9 if c["precision"] == LT.FP64 else 1e-3
    err = np.max(np.abs(g - go)) / np.max(np.abs(go))
    rl = abs(L - Lo) / abs(Lo)
    rG = abs(gG - dGo) / max(abs(dGo), 1e-300)
    rF = abs(gF - dFo) / max(abs(dFo), 1e-300)
    print(f"[random adjoint] L {rl:.2e} field {err:.2e} dG {rG:.2e} dF {rF:.2e}", flush=True)
    assert rl <= (1e-11 if c["precision"] == LT.FP64 else 1e-3), (seed, "L", rl)
    assert err <= tol, (seed, "field", err)
    assert rG <= tol and rF <= tol, (seed, rG, rF)
    if c["mask"] is not None:
        assert np.all(g[c["mask"] == 1] == 0.0)
