"""The library from a plain-C program (tests/c_client/lbm_c_client.c, built by
build()): HIP runtime allocations, the C-ABI of include/pplbm.h, no Python or
torch in the process.  Both precisions: no faults, the mass of the walled
droplet channel conserved (FP64 1e-16 of it per step, float storage 1e-6;
host sums compensated), finite fields."""
import json
import os
import subprocess

import pytest

from paper_2604_13407_amd import build as B

pytestmark = pytest.mark.gpu


def test_plain_c_client_steps_both_precisions():
    assert os.path.exists(B.C_CLIENT), "the C client is built by __graft_entry__.build()"
    print(f"[c client] {B.C_CLIENT}", flush=True)
    r = subprocess.run([B.C_CLIENT], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stderr
    lines = [json.loads(l) for l in r.stdout.splitlines() if l.startswith("{")]
    assert [l["precision"] for l in lines] == ["fp64", "fp32"]
    for l in lines:
        assert l["ok"] and l["steps"] == 200 and l["mass_rel_err"] <= l["bar"], l
