"""The largest lattices the library takes, stepped a few times and checked
against the oracle on sampled windows (light-cone crops, as in the full-size
tests), with the step records' mass against the initial state's.

* The strip march addresses each population array with 32-bit byte offsets
  and takes lattices whose arrays hold fewer than 4,294,967,040 bytes.  The
  largest 2048-wide ones: 2048 x 52428 with float storage (10 runs of 4 B per
  node and row, 4,294,901,760 B) and 2048 x 29127 with double storage (9 runs
  of 8 B, 4,294,950,912 B); the offsets of their last rows come within 66 KB
  of 2^32.
* The library accepts lattices with 9 nx ny < 2^31: the largest 16384-wide one
  is 16384 x 14563 (238.6 M nodes, 17.2 GB per double population array), whose
  arrays exceed 32-bit offsets, so the tile kernel steps it (unsigned element
  indices, 64-bit byte offsets).  One row more is refused (a CPU test).
* A tall, narrow channel, 64 x 270,000, whose row-tiled launches (the
  initialisation, the two-pass kernels, the field read-out) have more than
  65,536 blocks along y.
"""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2604_13407_amd import lattice as LT
from paper_2604_13407_amd import workloads as WL
from tests.helpers import fp64_bar
from tests.test_gpu_fullsize import check, crop_oracle

pytestmark = pytest.mark.gpu

FIELDS = ("rho", "ux", "uy", "fintx", "finty", "psi")


class Seeded:
    """A workload whose initial density is computed once (hundreds of millions
    of nodes) and shared by the lattice and the oracle's crops."""

    def __init__(self, w):
        self.w = w
        self._rho0 = w.rho0()

    def __getattr__(self, k):
        return getattr(self.w, k)

    def rho0(self):
        return self._rho0


def grid_limits():
    """The device's grid limits along x and y (hipDeviceAttributeMaxGridDimX and
    ...Y, enum values 29 and 30 of hip_runtime_api.h)."""
    hip = C.CDLL("libamdhip64.so")
    out = []
    for code in (29, 30):
        v = C.c_int(0)
        assert hip.hipDeviceGetAttribute(C.byref(v), code, 0) == 0
        out.append(v.value)
    return out


def windows_of(lat, windows):
    """The fields of each window (host copies), and the peak speed over the lattice."""
    d = lat.read_fields()
    peak = max(float(d["ux"].abs().max()), float(d["uy"].abs().max()))
    out = [{k: d[k][y0:y1, x0:x1].cpu().numpy() for k in FIELDS} for (x0, x1, y0, y1) in windows]
    del d
    return out, peak


def run_and_check(w, precision, steps, windows, kernel=LT.KERNEL_FUSED, every=3):
    sw = Seeded(w)
    mass0 = float(np.sum(sw.rho0()))
    print(f"[maxsize] {w.nx}x{w.ny} precision={precision} kernel={kernel} steps={steps}", flush=True)
    lat = LT.Lattice.from_workload(sw, precision=precision, kernel=kernel)
    recs = lat.step(steps, reduce_every=every)
    got, peak = windows_of(lat, windows)
    torch.cuda.synchronize()
    del lat
    torch.cuda.empty_cache()
    assert [r["step"] for r in recs] == list(range(every, steps + 1, every))
    # mass is conserved (walls and a periodic axis); float storage rounds each
    # node's stored deviations once (about 1e-7 of the density)
    tol = 1e-12 if precision == LT.FP64 else 1e-6
    for r in recs:
        assert r["faults"] == 0
        assert abs(r["mass"] - mass0) <= tol * mass0, (r["step"], r["mass"], mass0)
    for g, (x0, x1, y0, y1) in zip(got, windows):
        print(f"[maxsize] oracle window x[{x0},{x1}) y[{y0},{y1})", flush=True)
        o = crop_oracle(sw, steps, x0, x1, y0, y1)
        check(sw, g, o, 0, x1 - x0, 0, y1 - y0, precision, peak, tol64=fp64_bar(steps))


def edge_windows(nx, ny):
    """The lattice's first and last rows and columns (the largest offsets, the
    walls in x, the periodic seam in y) and the droplet's interface."""
    return [(0, 64, 0, 40), (nx - 64, nx, ny - 40, ny), (nx // 2 - 96, nx // 2 - 32, ny // 2 - 20, ny // 2 + 20)]


@pytest.mark.parametrize("precision,ny", [(LT.FP32_DEV, 52428), (LT.FP64, 29127)], ids=["fp32", "fp64"])
def test_largest_strip_march_lattices(precision, ny):
    planes, size = (10, 4) if precision == LT.FP32_DEV else (9, 8)
    assert planes * size * 2048 * ny < 4294967040 <= planes * size * 2048 * (ny + 1)
    w = WL.small_droplet(nx=2048, ny=ny, radius=64.0, g=1e-6)
    run_and_check(w, precision, 6, edge_windows(w.nx, w.ny))


@pytest.mark.parametrize("precision", [LT.FP32_DEV, LT.FP64], ids=["fp32", "fp64"])
def test_largest_lattice_the_library_accepts(precision):
    nx, ny = 16384, 14563
    assert 9 * nx * ny < 2**31 - 1 <= 9 * nx * (ny + 1)
    w = WL.small_droplet(nx=nx, ny=ny, radius=64.0, g=1e-6)
    run_and_check(w, precision, 4, edge_windows(nx, ny), every=2)


@pytest.mark.parametrize("kernel", [LT.KERNEL_FUSED, LT.KERNEL_TWO_PASS], ids=["fused", "two_pass"])
@pytest.mark.parametrize("precision", [LT.FP32_DEV, LT.FP64], ids=["fp32", "fp64"])
def test_tall_narrow_channel(precision, kernel):
    print(f"[maxsize] device grid limits (x, y): {grid_limits()}", flush=True)
    w = WL.small_droplet(nx=64, ny=270000, radius=20.0, g=1e-6)
    assert (w.ny + 3) // 4 > 65536
    run_and_check(w, precision, 6, [(0, 64, 0, 40), (0, 64, w.ny - 40, w.ny), (0, 64, w.ny // 2 - 30, w.ny // 2 + 30),
                                    (0, 64, 262140, 262160)], kernel=kernel)
