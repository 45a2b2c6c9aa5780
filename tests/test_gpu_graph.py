"""lbm_step captured into a HIP graph (through torch.cuda.graph on the lattice's
stream) and replayed: a step without reductions only enqueues kernels on the
handle's stream (no allocation, no copy, no synchronisation, no memset), so the
graph replays exactly the eager steps.

Every replay is checked against an eager run of the same number of steps, with
eager work and synchronisations between the replays.  The graph holds an even
number of steps, so each replay starts and ends on the same population array;
the handle's own step counter advances at capture, not at replay, so the
captured steps must not reach a re-reference (every 1,000 steps by default).
"""
import pytest
import torch

from paper_2604_13407_amd import lattice as LT
from tests.test_gpu_masked import annulus_aligned, droplet_blobs
from tests.test_gpu_parity import droplet_aligned, droplet_small

pytestmark = pytest.mark.gpu

CASES = [("droplet_aligned", droplet_aligned), ("droplet_130_partial_strip", droplet_small),
         ("annulus_moving_walls", annulus_aligned), ("blobs_150", lambda: droplet_blobs(nx=150, ny=96, seed=12))]


@pytest.mark.parametrize("precision", [LT.FP64, LT.FP32_DEV])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_steps_replay_from_a_captured_graph(case, precision):
    name, make = CASES[case]
    w = make()
    per_replay, replays = 10, 3
    print(f"[graph] {name} {w.nx}x{w.ny} precision={precision}", flush=True)
    s = torch.cuda.Stream()
    eager = LT.Lattice.from_workload(w, precision=precision, stream=s)
    lat = LT.Lattice.from_workload(w, precision=precision, stream=s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        lat.step(per_replay)
    for r in range(replays):
        g.replay()
        eager.step(per_replay)
        torch.cuda.synchronize()
        assert torch.equal(lat.state(), eager.state()), (name, r)
        # eager work between the replays
        _ = (eager.state().float().sum()).item()
