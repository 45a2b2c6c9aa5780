"""Seeded synthetic workloads: lattice geometry, parameters and initial fields.

This module is the one place both the GPU library's callers and the CPU oracle's
tests take their inputs from.  It holds none of the method's arithmetic: only
shapes, masks, tanh initial profiles, seeded perturbations and parameter sets.

Workloads (one per benchmark configuration; sizes as stated):

* ``poiseuille_aligned``  4 x 100, x periodic, bounce-back walls at y = -1/2 and
  99.5, Carnahan-Starling EOS at 0.8 T_c, liquid layer y in [25, 75), force 1e-7
  along x (the grid-aligned two-phase Poiseuille flow of Sec. 3.1).
* ``poiseuille_oblique``  256 x 256 periodic, a two-line-thick 45-degree solid
  band (x - y) mod 256 in {0, 1}, CS at 0.7 T_c, liquid in the middle 128 of the
  254 fluid diagonals, force 1e-7 along (1, 1)/sqrt(2), seeded +-1e-6 density
  perturbation (the grid-oblique case of Sec. 3.1).
* ``annular_shear``  1024 x 1024, solid for r < 100 and r > 480 around
  (511.5, 511.5), the inner wall turning counter-clockwise at 0.01, liquid
  annulus r in [200, 320], CS at 0.75 T_c (Sec. 3.2, wall-driven).
* ``droplet``  2048 x 16384, walls at x = -1/2 and 2047.5, y periodic, a liquid
  droplet of radius 256 centred at (1023.5, 8191.5), CS at 0.7 T_c, buoyant
  gravity (rho - rho_g)(0, -1e-7) (Sec. 3.3).
* ``droplet_adjoint``  512 x 2048, same boundaries and physics, radius 64,
  seeded +-1e-4 density perturbation; the gradient workload.

The coexistence densities come from ``coexistence.json`` (mechanical stability
condition of Eq. (1) with eps = 1.895), written by the oracle's coexistence
script.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(_HERE, "coexistence.json")) as _fh:
    COEXISTENCE = json.load(_fh)

EOS_VDW, EOS_CS = 0, 1
SCHEME_ORIGINAL, SCHEME_IMPROVED = 0, 1
FORCE_CONST, FORCE_BUOYANT = 0, 1


def rates_from_tau(tau: float) -> Tuple[float, ...]:
    """Collision rates of Sec. 3: s_0 = s_j = 1, s_e = s_eps = s_p = 1/tau and
    (1/s_q - 1/2)(1/s_p - 1/2) = 1/12.  Order (s_0, s_e, s_eps, s_j, s_q, s_j, s_q, s_p, s_p)."""
    sp = 1.0 / tau
    sq = 1.0 / (0.5 + (1.0 / 12.0) / (tau - 0.5))
    return (1.0, sp, sp, 1.0, sq, 1.0, sq, sp, sp)


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    periodic_x: bool
    periodic_y: bool
    eos_kind: int
    a: float
    b: float
    R: float
    T: float
    k_eos: float
    eps: float
    s: Tuple[float, ...]
    force_mode: int
    fx: float
    fy: float
    rho_g: float
    rho_l: float
    rho_s: float
    steps: int
    scheme: int = SCHEME_IMPROVED
    G: float = -1.0
    k1: Optional[float] = None       # None: -eps/16 (Sec. 3)
    k2: Optional[float] = None
    reduce_every: int = 0
    geometry: str = "none"           # none | oblique_band | annulus | analytic walls only
    init: str = "none"               # layer_y | oblique_layers | annulus | droplet
    init_args: dict = field(default_factory=dict)
    perturb: float = 0.0
    seed: int = 0

    @property
    def nodes(self) -> int:
        return self.nx * self.ny

    def with_size(self, nx: int, ny: int, **kw) -> "Workload":
        """A copy on a different lattice with geometry parameters scaled to fit."""
        return replace(self, nx=nx, ny=ny, **kw)

    # ------------------------------------------------------------ inputs
    def mask(self) -> Optional[np.ndarray]:
        """uint8 [ny, nx], 1 = solid, or None when the only walls are the analytic
        ones across non-periodic axes."""
        if self.geometry == "oblique_band":
            x = np.arange(self.nx)[None, :]
            y = np.arange(self.ny)[:, None]
            d = np.mod(x - y, self.nx)
            return np.ascontiguousarray(((d == 0) | (d == 1)).astype(np.uint8))
        if self.geometry == "annulus":
            r = self._radius()
            a = self.init_args
            return np.ascontiguousarray(((r < a["r_in"]) | (r > a["r_out"])).astype(np.uint8))
        return None

    def wall_velocity(self) -> Optional[np.ndarray]:
        """float64 [2, ny, nx] velocity of solid nodes, or None for static walls.
        Annulus: rigid counter-clockwise rotation of the inner wall with surface
        speed u_w at r_in, evaluated at each solid node; the outer wall is at rest."""
        if self.geometry != "annulus" or not self.init_args.get("u_wall"):
            return None
        a = self.init_args
        xc, yc = a["centre"]
        x = np.arange(self.nx)[None, :] - xc
        y = np.arange(self.ny)[:, None] - yc
        omega = a["u_wall"] / a["r_in"]
        inner = (self._radius() < a["r_in"])
        wu = np.zeros((2, self.ny, self.nx))
        wu[0] = np.where(inner, -omega * y * np.ones_like(x), 0.0)
        wu[1] = np.where(inner, omega * x * np.ones_like(y), 0.0)
        return np.ascontiguousarray(wu)

    def _radius(self):
        xc, yc = self.init_args["centre"]
        x = np.arange(self.nx)[None, :] - xc
        y = np.arange(self.ny)[:, None] - yc
        return np.sqrt(x * x + y * y)

    def rho0(self) -> np.ndarray:
        """float64 [ny, nx] initial density (tanh profiles of width 2), plus the
        seeded uniform perturbation of amplitude ``perturb``."""
        rg, rl = self.rho_g, self.rho_l
        mid, half = 0.5 * (rl + rg), 0.5 * (rl - rg)
        a = self.init_args
        shape = (self.ny, self.nx)
        if self.init == "layer_y":
            y = np.arange(self.ny, dtype=np.float64)[:, None] * np.ones((1, self.nx))
            lo, hi = a["y0"] - 0.5, a["y1"] - 0.5
            rho = rg + half * (np.tanh(y - lo) - np.tanh(y - hi))
        elif self.init == "oblique_layers":
            x = np.arange(self.nx)[None, :]
            y = np.arange(self.ny)[:, None]
            d = np.mod(x - y, self.nx).astype(np.float64)
            s2 = math.sqrt(2.0)
            lo, hi = a["d0"] - 0.5, a["d1"] - 0.5
            rho = rg + half * (np.tanh((d - lo) / s2) - np.tanh((d - hi) / s2))
        elif self.init == "annulus":
            r = self._radius()
            rho = rg + half * (np.tanh(r - a["r_liq_in"]) - np.tanh(r - a["r_liq_out"]))
        elif self.init == "droplet":
            xc, yc = a["centre"]
            x = np.arange(self.nx, dtype=np.float64)[None, :] - xc
            y = np.arange(self.ny, dtype=np.float64)[:, None] - yc
            r = np.sqrt(x * x + y * y)
            rho = mid - half * np.tanh(r - a["radius"])
        else:
            rho = np.full(shape, rg)
        rho = np.ascontiguousarray(np.broadcast_to(rho, shape), dtype=np.float64).copy()
        if self.perturb:
            rng = np.random.default_rng(self.seed)
            rho += rng.uniform(-self.perturb, self.perturb, size=shape)
        return rho

    def fluid_fraction(self) -> float:
        m = self.mask()
        return 1.0 if m is None else float(1.0 - m.mean())


def _coex(key: str):
    c = COEXISTENCE[key]
    return c["T"], c["rho_g"], c["rho_l"]


def poiseuille_aligned(eps: float = 1.895, tau: float = 0.8, scheme: int = SCHEME_IMPROVED) -> Workload:
    T, rg, rl = _coex("cs_0.80_eps1.895")
    return Workload("poiseuille_aligned", 4, 100, True, False, EOS_CS, 1.0, 4.0, 1.0, T, 1.0, eps,
                    rates_from_tau(tau), FORCE_CONST, 1e-7, 0.0, rg, rl, rg, 20000, scheme=scheme,
                    init="layer_y", init_args={"y0": 25, "y1": 75})


def poiseuille_oblique(eps: float = 1.895, tau: float = 0.8, scheme: int = SCHEME_IMPROVED) -> Workload:
    T, rg, rl = _coex("cs_0.70_eps1.895")
    f = 1e-7 / math.sqrt(2.0)
    return Workload("poiseuille_oblique", 256, 256, True, True, EOS_CS, 1.0, 4.0, 1.0, T, 1.0, eps,
                    rates_from_tau(tau), FORCE_CONST, f, f, rg, rl, rg, 50000, scheme=scheme,
                    geometry="oblique_band", init="oblique_layers", init_args={"d0": 65, "d1": 193},
                    perturb=1e-6, seed=0)


def annular_shear(scheme: int = SCHEME_IMPROVED) -> Workload:
    T, rg, rl = _coex("cs_0.75_eps1.895")
    return Workload("annular_shear", 1024, 1024, True, True, EOS_CS, 1.0, 4.0, 1.0, T, 1.0, 1.895,
                    rates_from_tau(0.8), FORCE_CONST, 0.0, 0.0, rg, rl, rg, 100000, scheme=scheme,
                    geometry="annulus", init="annulus",
                    init_args={"centre": (511.5, 511.5), "r_in": 100.0, "r_out": 480.0, "u_wall": 0.01,
                               "r_liq_in": 200.0, "r_liq_out": 320.0})


DROPLET_RATES = (1.0, 1.1, 1.1, 1.0, 1.1, 1.0, 1.1, 1.25, 1.25)


def droplet(scheme: int = SCHEME_IMPROVED, g: float = 1e-7) -> Workload:
    T, rg, rl = _coex("cs_0.70_eps1.895")
    return Workload("droplet", 2048, 16384, False, True, EOS_CS, 1.0, 4.0, 1.0, T, 1.0, 1.895,
                    DROPLET_RATES, FORCE_BUOYANT, 0.0, -g, rg, rl, rg, 200000, scheme=scheme,
                    reduce_every=100, init="droplet",
                    init_args={"centre": (1023.5, 8191.5), "radius": 256.0})


def droplet_adjoint(scheme: int = SCHEME_IMPROVED, g: float = 1e-7) -> Workload:
    T, rg, rl = _coex("cs_0.70_eps1.895")
    return Workload("droplet_adjoint", 512, 2048, False, True, EOS_CS, 1.0, 4.0, 1.0, T, 1.0, 1.895,
                    DROPLET_RATES, FORCE_BUOYANT, 0.0, -g, rg, rl, rg, 20000, scheme=scheme,
                    init="droplet", init_args={"centre": (255.5, 1023.5), "radius": 64.0},
                    perturb=1e-4, seed=0)


def small_droplet(nx: int = 48, ny: int = 64, radius: float = 10.0, scheme: int = SCHEME_IMPROVED,
                  g: float = 1e-6, perturb: float = 1e-4) -> Workload:
    """A reduced droplet channel (same physics) small enough for the oracle."""
    w = droplet_adjoint(scheme=scheme, g=g)
    return replace(w, name="droplet_small", nx=nx, ny=ny, steps=200,
                   init_args={"centre": (nx / 2 - 0.5, ny / 2 - 0.5), "radius": radius}, perturb=perturb)


def vdw_layer(nx: int = 64, ny: int = 96, key: str = "vdw_0.50_eps1.895", tau: float = 1.0, fx: float = 0.0,
              periodic_y: bool = True, scheme: int = SCHEME_IMPROVED) -> Workload:
    """A flat liquid layer, y in [ny/4, 3ny/4), in the van der Waals fluid of
    Sec. 3 (a = 9/49, b = 2/21, R = 1, K = 1/16) at one of its coexistence
    cases.  The default is the setting of Sec. 3.2 (T_r = 0.5, eps = 1.895,
    density ratio about 113) in a box periodic in x and y; with
    ``periodic_y=False`` and a force ``fx`` it is the aligned two-phase channel
    of Sec. 3.1 (keys ``vdw_0.72_eps0``, ``vdw_0.65_eps1``, ``vdw_0.54_eps2``)."""
    c = COEXISTENCE[key]
    rg, rl = c["rho_g"], c["rho_l"]
    return Workload(f"vdw_layer_{key}", nx, ny, True, periodic_y, EOS_VDW, 9.0 / 49.0, 2.0 / 21.0, 1.0, c["T"],
                    1.0 / 16.0, c["eps"], rates_from_tau(tau), FORCE_CONST, fx, 0.0, rg, rl, rg, 0,
                    scheme=scheme, init="layer_y", init_args={"y0": ny // 4, "y1": 3 * ny // 4})


ALL = {
    "poiseuille_aligned": poiseuille_aligned,
    "poiseuille_oblique": poiseuille_oblique,
    "annular_shear": annular_shear,
    "droplet": droplet,
    "droplet_adjoint": droplet_adjoint,
}
