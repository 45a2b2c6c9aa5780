"""The masked strip march (lattices with solid masks or moving walls) against the
tile kernel, through the C-ABI; and the strip march over widths that are not a
multiple of 64, whose last strip is partial.

Both run the same node arithmetic; what differs is the data movement
(bounce-back chosen from per-node link words, psi of neighbours through lane
shifts and registers instead of an LDS tile).  Float storage must agree
bitwise; double storage to a few ulp (the compiler may contract a product and
a sum into an FMA differently in each kernel).  Reduction records are sums in
a different grouping: they agree to rounding.  The masked march's parity
with the oracle is in test_gpu_parity.py (the oblique channel and the
aligned annulus run on it).
"""
from dataclasses import replace

import numpy as np
import pytest
import torch

from paper_2604_13407_amd import lattice as LT
from paper_2604_13407_amd import workloads as WL

pytestmark = pytest.mark.gpu


def annulus_aligned():
    # width 192: three strips; the inner wall moves, the outer one rests
    w = WL.annular_shear()
    return w.with_size(192, 192, init_args={"centre": (95.5, 95.5), "r_in": 25.0, "r_out": 88.0, "u_wall": 0.01,
                                            "r_liq_in": 40.0, "r_liq_out": 65.0})


def blobs(nx, ny, seed, frac=0.08):
    """A seeded mask of solid blobs (and isolated solid nodes).  Each blob is
    drawn in its bounding box (the same mask as testing every node)."""
    rng = np.random.default_rng(seed)
    m = np.zeros((ny, nx), np.uint8)
    for _ in range(max(1, int(frac * nx * ny / 30))):
        cx, cy, r = rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(1.0, 4.0)
        x0, x1 = max(0, int(cx - r) - 1), min(nx, int(cx + r) + 2)
        y0, y1 = max(0, int(cy - r) - 1), min(ny, int(cy + r) + 2)
        yy, xx = np.mgrid[y0:y1, x0:x1]
        m[y0:y1, x0:x1][(xx - cx) ** 2 + (yy - cy) ** 2 < r * r] = 1
    m[rng.random((ny, nx)) < 0.01] = 1
    return m


class Masked:
    """A droplet workload with an explicit mask and, optionally, wall velocities
    on its solid nodes."""

    def __init__(self, base, mask, wall_u=None):
        self.base, self._mask, self._wall_u = base, mask, wall_u

    def __getattr__(self, k):
        return getattr(self.base, k)

    def mask(self):
        return self._mask

    def wall_velocity(self):
        return self._wall_u


def droplet_blobs(nx=128, ny=96, periodic_x=True, periodic_y=False, moving=False, seed=1):
    w = WL.small_droplet(nx=nx, ny=ny, radius=14.0, g=1e-5)
    w = replace(w, name=f"droplet_blobs_{nx}x{ny}", periodic_x=periodic_x, periodic_y=periodic_y)
    m = blobs(nx, ny, seed)
    # keep the droplet's centre fluid
    yy, xx = np.mgrid[0:ny, 0:nx]
    cx, cy = w.init_args["centre"]
    m[(xx - cx) ** 2 + (yy - cy) ** 2 < 16 ** 2] = 0
    wu = None
    if moving:
        rng = np.random.default_rng(seed + 100)
        wu = np.zeros((2, ny, nx))
        wu[:, m == 1] = rng.uniform(-0.01, 0.01, (2, int(m.sum())))
    return Masked(w, np.ascontiguousarray(m), wu)


def channel_wall_u(nx=64, ny=40):
    # moving walls given, no mask: only the planes beyond the y edges are solid,
    # and they are outside the box (no moving-wall term); one 64-column strip
    w = WL.poiseuille_aligned()
    w = w.with_size(nx, ny, init_args={"y0": 10, "y1": 30})
    return Masked(w, None, np.zeros((2, ny, nx)))


def annulus_ragged():
    # width 150: two full strips and one of 22 columns (float storage takes the
    # masked march at any width)
    w = WL.annular_shear()
    return w.with_size(150, 150, init_args={"centre": (74.5, 74.5), "r_in": 20.0, "r_out": 70.0, "u_wall": 0.01,
                                            "r_liq_in": 35.0, "r_liq_out": 55.0})


CASES = [
    ("oblique", lambda: WL.poiseuille_oblique(), 30),
    ("annulus_ragged_150", annulus_ragged, 40),
    ("blobs_ragged_periodic_x", lambda: droplet_blobs(nx=150, ny=96, seed=7), 40),
    ("blobs_ragged_walled_moving", lambda: droplet_blobs(nx=100, ny=70, periodic_x=False, periodic_y=False,
                                                         moving=True, seed=8), 40),
    ("blobs_one_partial_strip", lambda: droplet_blobs(nx=40, ny=48, periodic_x=True, periodic_y=True, seed=9), 40),
    ("annulus", annulus_aligned, 40),
    ("blobs_periodic_x", lambda: droplet_blobs(), 40),
    ("blobs_walled_x", lambda: droplet_blobs(periodic_x=False, periodic_y=True, seed=2), 40),
    ("blobs_closed_moving", lambda: droplet_blobs(nx=192, ny=70, periodic_x=False, periodic_y=False, moving=True,
                                                  seed=3), 40),
    ("blobs_one_strip_periodic", lambda: droplet_blobs(nx=64, ny=64, periodic_x=True, periodic_y=True, seed=4), 40),
    ("channel_wall_u", channel_wall_u, 60),
]


def make_pair(w, precision):
    a = LT.Lattice.from_workload(w, precision=precision)
    b = LT.Lattice.from_workload(w, precision=precision)
    b.set_masked_strips(False)
    return a, b


def fluid_mask(w, device):
    m = w.mask()
    fl = np.ones((w.ny, w.nx), bool) if m is None else (m == 0)
    return torch.from_numpy(fl).to(device)


def compare_states(w, a, b, precision):
    fl = fluid_mask(w, a.device)
    sa, sb = a.state()[:9][:, fl], b.state()[:9][:, fl]
    if precision == LT.FP32_DEV:
        assert torch.equal(sa, sb), (w.name, (sa - sb).abs().max().item())
        # the reference offsets are untouched by a step
        assert torch.equal(a.state()[9], b.state()[9])
    else:
        err = ((sa - sb).abs().max() / sa.abs().max()).item()
        assert err <= 1e-14, (w.name, err)


@pytest.mark.parametrize("precision", [LT.FP64, LT.FP32_DEV])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_masked_march_matches_tile_kernel(case, precision):
    name, make, steps = CASES[case]
    w = make()
    print(f"[masked] {name} {w.nx}x{w.ny} steps={steps} precision={precision}", flush=True)
    a, b = make_pair(w, precision)
    ra = a.step(steps, reduce_every=10)
    rb = b.step(steps, reduce_every=10)
    torch.cuda.synchronize()
    compare_states(w, a, b, precision)
    for x, y in zip(ra, rb):
        for k in ("mass", "mom_x", "mom_y", "wall_x", "wall_y", "uc_num", "uc_den", "buoy", "pphi"):
            scale = max(abs(y[k]), abs(y["mass"]) * 1e-6)
            assert abs(x[k] - y[k]) <= 1e-11 * scale, (name, k, x[k], y[k])
        assert x["faults"] == y["faults"] == 0


@pytest.mark.parametrize("precision", [LT.FP64, LT.FP32_DEV])
def test_masked_march_state_does_not_depend_on_rows_per_wave(precision):
    # each run recomputes psi of the rows beside it in the same arithmetic, so
    # the state is bitwise the same for any run length
    w = annulus_aligned()
    ref = LT.Lattice.from_workload(w, precision=precision)
    ref.step(25)
    for rows in (1, 2, 4, 5, 7, 16, 200):
        lat = LT.Lattice.from_workload(w, precision=precision)
        lat.set_rows_per_wave(rows)
        lat.step(25)
        torch.cuda.synchronize()
        assert torch.equal(lat.state(), ref.state()), rows


@pytest.mark.parametrize("nx", [128, 150])
@pytest.mark.parametrize("precision", [LT.FP64, LT.FP32_DEV])
def test_masked_march_rereference_and_resume(precision, nx):
    # float storage re-references with the mask; a resumed run is bitwise the
    # uninterrupted one (also with a partial last strip)
    w = droplet_blobs(nx=nx, moving=True, periodic_y=True, seed=5)
    a = LT.Lattice.from_workload(w, precision=precision)
    a.set_rereference_every(7)
    a.step(20)
    snap = a.get_state()
    a.step(20)
    b = LT.Lattice.from_workload(w, precision=precision)
    b.set_rereference_every(7)
    b.set_state(snap, step=20)
    b.step(20)
    torch.cuda.synchronize()
    assert torch.equal(a.state(), b.state())


@pytest.mark.parametrize("precision", [LT.FP64, LT.FP32_DEV])
def test_static_workspace_handles_share_it_with_masks(precision):
    # two handles on the library's static workspace, both masked with moving
    # walls, step in turn: each call writes its link words and tile list again,
    # so both runs are bitwise those of handles with their own workspaces
    ws = [annulus_aligned(), droplet_blobs(moving=True, periodic_y=True, seed=6)]
    shared = [LT.Lattice.from_workload(w, precision=precision, static_workspace=True) for w in ws]
    own = [LT.Lattice.from_workload(w, precision=precision) for w in ws]
    recs_s, recs_o = [[], []], [[], []]
    for _ in range(3):
        for i in range(2):
            recs_s[i] += shared[i].step(5, reduce_every=5)
            recs_o[i] += own[i].step(5, reduce_every=5)
    torch.cuda.synchronize()
    for i in range(2):
        assert torch.equal(shared[i].state(), own[i].state()), ws[i].name
        assert recs_s[i] == recs_o[i]


def hbm_ragged(mask):
    # 2000 x 1100 (31 full strips and one of 16 columns), x walls, y periodic:
    # its two double-storage arrays (317 MB) exceed the last-level cache, so
    # double storage also takes the strip march with a partial last strip
    w = WL.small_droplet(nx=2000, ny=1100, radius=120.0, g=1e-5)
    return Masked(w, mask, None)


@pytest.mark.parametrize("precision", [LT.FP64, LT.FP32_DEV])
def test_partial_last_strip_at_a_size_that_streams_from_hbm(precision):
    """The unmasked strip march, the masked strip march (a mask with a few solid
    blobs) and the tile kernel on the same 2000-column lattice: masked march and
    tile kernel agree as in the masked cases; the unmasked march agrees with the
    tile kernel on the same lattice with an all-fluid mask."""
    w0 = hbm_ragged(None)
    steps = 12
    print(f"[masked] partial last strip 2000x1100 precision={precision}", flush=True)
    free = np.zeros((w0.ny, w0.nx), np.uint8)
    a = LT.Lattice.from_workload(w0, precision=precision)                      # unmasked strip march
    b = LT.Lattice.from_workload(hbm_ragged(free), precision=precision)        # all-fluid mask, tile kernel
    b.set_masked_strips(False)
    m = blobs(w0.nx, w0.ny, 11)
    m[:, :2] = 0
    c = LT.Lattice.from_workload(hbm_ragged(m), precision=precision)           # masked strip march
    d = LT.Lattice.from_workload(hbm_ragged(m), precision=precision)           # masked, tile kernel
    d.set_masked_strips(False)
    for lat in (a, b, c, d):
        lat.step(steps)
    torch.cuda.synchronize()
    compare_states(hbm_ragged(free), a, b, precision)
    compare_states(hbm_ragged(m), c, d, precision)
