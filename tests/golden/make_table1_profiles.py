"""Writes table1_profiles.json: converged static density profiles of the
two-phase channels of Table 1 (Sec. 3.1), computed by the CPU oracle only.

Setups (Sec. 3.1, with this repository's walls, halfway bounce-back, and the
readings of the paper it documents): van der Waals EOS of Eq. (43) with
a = 9/49, b = 2/21, R = 1, K_EOS = 1/16; (eps, T_r) = (0, 0.72), (1, 0.65),
(2, 0.54); k1 = k2 = -eps/16; channel width W = 128 sqrt 2 with gas layers of
W/4 at the walls and liquid in the middle W/2:
* grid-aligned: 181 fluid rows (128 sqrt 2 = 181.02 nodes) between walls at
  y = -1/2 and 180.5, one column (fields depend on y only);
* grid-oblique: the 256 x 256 periodic lattice with the two-line solid band
  (x - y) mod 256 in {0, 1}, 254 fluid 45-degree lines (normal spacing
  1/sqrt 2, width 127 sqrt 2 between the halfway walls).
Each starts from tanh layers at the mechanical-stability densities of Eq. (1)
and runs without driving force, with tau = 1 and the original scheme (a static
interface is the same for both schemes at s_e = s_p), until the density
changes by less than 1e-10 (about 1e-11 of the liquid density) over 1,000
steps.  The profiles are inputs of the
LB-ana tests (the flow is then driven); nothing here comes from the GPU path.

    python tests/golden/make_table1_profiles.py
"""
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import coexistence as X  # noqa: E402
from oracle import oracle as O  # noqa: E402

CASES = [(0.0, 0.72), (1.0, 0.65), (2.0, 0.54)]


def params(eos, eps, nx, ny, periodic_y, rg, rl):
    sp = 1.0  # tau = 1
    sq = 1.0 / (0.5 + (1.0 / 12.0) / (1.0 - 0.5))
    return O.Params(nx=nx, ny=ny, periodic_x=True, periodic_y=periodic_y, eos_kind=O.EOS_VDW, a=eos.a, b=eos.b,
                    R=eos.R, T=eos.T, k_eos=eos.k_eos, eps=eps, s=(1, sp, sp, 1, sq, 1, sq, sp, sp),
                    scheme=O.SCHEME_ORIGINAL, rho_g=rg, rho_l=rl, rho_s=rg)


def converge(o, pick, chunk=1000, tol=3e-10, max_steps=400000):
    prev = pick(o.macros())
    steps = 0
    while steps < max_steps:
        o.step(chunk)
        steps += chunk
        cur = pick(o.macros())
        d = float(np.max(np.abs(cur - prev)))
        if d < tol:
            return cur, steps, d
        prev = cur
    raise RuntimeError(f"not converged after {steps} steps (change {d:.2e})")


def load():
    path = os.path.join(HERE, "table1_profiles.json")
    if os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    return {"aligned": {}, "oblique": {}, "steps": {}}


def save(out):
    with open(os.path.join(HERE, "table1_profiles.json"), "w") as fh:
        json.dump(out, fh)


def main():
    out = load()
    for eps, T_r in CASES:
        eos = X.vdw_paper(T_r)
        rg, rl, _ = X.mechanical_stability(eos, eps)
        # grid-aligned: rows 0..180, walls at -1/2 and 180.5; liquid W/4 .. 3W/4 from the lower wall
        if str(eps) in out["aligned"] and str(eps) in out["oblique"]:
            continue
        ny = 181
        y = np.arange(ny)[:, None] + 0.5  # distance from the lower wall
        rho = rg + 0.5 * (rl - rg) * (np.tanh((y - ny / 4) / 3) - np.tanh((y - 3 * ny / 4) / 3))
        o = O.Oracle(params(eos, eps, 1, ny, False, rg, rl)).init(np.ascontiguousarray(rho))
        r, steps, d = converge(o, lambda m: m["rho"][:, 0].copy())
        r = 0.5 * (r + r[::-1])
        out["aligned"][str(eps)] = r.tolist()
        out["steps"][f"aligned_{eps}"] = steps
        print(f"aligned eps={eps}: {steps} steps, change {d:.1e}, ratio {r.max() / r.min():.1f}", flush=True)
        # grid-oblique: lines d = (x - y) mod 256, fluid d = 2..255
        N = 256
        x = np.arange(N)[None, :]
        yy = np.arange(N)[:, None]
        dd = np.mod(x - yy, N).astype(float)
        mask = ((dd == 0) | (dd == 1)).astype(np.uint8)
        lines = dd - 1.5  # distance from the lower wall in line spacings (254 fluid lines)
        rho = rg + 0.5 * (rl - rg) * (np.tanh((lines - 254 / 4) / 4) - np.tanh((lines - 3 * 254 / 4) / 4))
        o = O.Oracle(params(eos, eps, N, N, True, rg, rl), mask=mask).init(np.ascontiguousarray(rho))
        r, steps, d = converge(o, lambda m: m["rho"][0].copy())
        r = r[2:]
        r = 0.5 * (r + r[::-1])  # lines 2..255 mirror about the channel's centre line
        out["oblique"][str(eps)] = r.tolist()
        out["steps"][f"oblique_{eps}"] = steps
        print(f"oblique eps={eps}: {steps} steps, change {d:.1e}, ratio {r.max() / r.min():.1f}", flush=True)
        save(out)
    save(out)


if __name__ == "__main__":
    main()
