"""Host-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and validates arguments without touching a GPU."""
import ctypes as C
import math
import os
import re

import pytest

from paper_2604_13407_amd import lattice as LT

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "pplbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[A-Za-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = LT.lib()
    names = declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(LT.EXPORTS)
    with open(os.path.join(ROOT, "include", "pplbm.h")) as fh:
        abi = int(re.search(r"#define LBM_ABI_VERSION (\d+)", fh.read()).group(1))
    assert L.lbm_abi_version() == abi == 4


def cfg(**kw):
    base = dict(nx=64, ny=32, periodic_x=1, periodic_y=0, precision=LT.FP32_DEV, kernel=LT.KERNEL_FUSED,
                rho_ref=0.1, log_capacity=16, reserved=0)
    base.update(kw)
    return LT.Config(**base)


def test_sizes_and_config_validation():
    L = LT.lib()
    b = C.c_size_t(0)
    # float storage: 9 population planes and the per-node reference plane
    assert L.lbm_state_bytes(C.byref(cfg()), C.byref(b)) == 0 and b.value == 10 * 64 * 32 * 4
    assert L.lbm_state_bytes(C.byref(cfg(precision=LT.FP64)), C.byref(b)) == 0 and b.value == 9 * 64 * 32 * 8
    assert L.lbm_workspace_bytes(C.byref(cfg()), C.byref(b)) == 0 and b.value % 256 == 0 and b.value > 64 * 32 * 4
    for bad in (dict(nx=0), dict(ny=-3), dict(precision=7), dict(kernel=5), dict(log_capacity=0),
                dict(nx=100000, ny=100000), dict(rho_ref=math.inf)):
        assert L.lbm_state_bytes(C.byref(cfg(**bad)), C.byref(b)) == -1, bad
        # a call without a handle leaves its message for lbm_last_error(NULL)
        assert L.lbm_last_error(None).decode(), bad
        assert L.lbm_workspace_bytes(C.byref(cfg(**bad)), C.byref(b)) == -1, bad
        assert L.lbm_last_error(None).decode(), bad
    # the largest lattice accepted (9 nx ny < 2^31) and one row more
    big = dict(nx=16384, ny=14563, precision=LT.FP64)
    assert L.lbm_state_bytes(C.byref(cfg(**big)), C.byref(b)) == 0 and b.value == 9 * 8 * 16384 * 14563
    assert L.lbm_workspace_bytes(C.byref(cfg(**big)), C.byref(b)) == 0
    assert L.lbm_state_bytes(C.byref(cfg(**dict(big, ny=14564))), C.byref(b)) == -1
    assert "2^31" in L.lbm_last_error(None).decode()
    assert L.lbm_workspace_bytes(C.byref(cfg()), None) == -1
    assert "NULL" in L.lbm_last_error(None).decode()
    # and a successful one clears it
    assert L.lbm_workspace_bytes(C.byref(cfg()), C.byref(b)) == 0 and L.lbm_last_error(None).decode() == ""


def fake_handle():
    """A handle around fake pointers: valid for host-only calls, never for launches."""
    L = LT.lib()
    c = cfg()
    buf = LT.Buffers(0x10000, 0x20000, 0x30000, None, None)
    h = C.c_void_p(0)
    assert L.lbm_create(C.byref(c), C.byref(buf), None, C.byref(h)) == 0
    return L, h


def test_create_rejects_bad_buffers():
    L = LT.lib()
    h = C.c_void_p(0)
    for buf in (LT.Buffers(0, 0x2000, 0x3000, None, None), LT.Buffers(0x1000, 0x1000, 0x3000, None, None),
                LT.Buffers(0x1000, 0x2000, 0x3001, None, None)):
        assert L.lbm_create(C.byref(cfg()), C.byref(buf), None, C.byref(h)) == -1
        assert L.lbm_last_error(None)
    assert L.lbm_create(C.byref(cfg(nx=0)), C.byref(LT.Buffers(0x1000, 0x2000, 0x3000, None, None)), None,
                        C.byref(h)) == -1


def test_setters_validate_and_state_errors_without_a_gpu():
    L, h = fake_handle()
    try:
        assert L.lbm_set_eos(h, 3, 1, 4, 1, 0.07, 1) == -1
        assert L.lbm_set_eos(h, 1, 1, -4, 1, 0.07, 1) == -1
        assert L.lbm_set_eos(h, 1, 1, 4, 1, 0.07, 1) == 0
        assert L.lbm_set_G(h, 0.0) == -1 and L.lbm_set_G(h, math.nan) == -1 and L.lbm_set_G(h, -1.0) == 0
        good = (C.c_double * 9)(1, 1.25, 1.25, 1, 1.2, 1, 1.2, 1.25, 1.25)
        bad = (C.c_double * 9)(1, 2.5, 1.25, 1, 1.2, 1, 1.2, 1.25, 1.25)
        assert L.lbm_set_relaxation(h, good) == 0 and L.lbm_set_relaxation(h, bad) == -1
        assert L.lbm_set_scheme(h, 2, 1.0, math.nan, math.nan, 0) == -1
        assert L.lbm_set_scheme(h, 1, 1.0, math.nan, math.nan, 9) == -1
        assert L.lbm_set_scheme(h, 1, math.inf, math.nan, math.nan, 0) == -1
        assert L.lbm_set_scheme(h, 0, 1.895, math.nan, math.nan, 0) == 0
        assert L.lbm_set_body_force(h, 3, 0, 0) == -1 and L.lbm_set_body_force(h, 1, 0, -1e-7) == 0
        assert L.lbm_set_phase_densities(h, 0.3, 0.1) == -1 and L.lbm_set_phase_densities(h, 0.01, 0.3) == 0
        assert L.lbm_set_walls(h, -1.0) == -1 and L.lbm_set_walls(h, 0.01) == 0
        # stepping or reading before initialisation is a state error (checked before any launch)
        assert L.lbm_step(h, 1, 0, None, 0) == -6
        assert L.lbm_read_fields(h, None, None, None, None, None, None) == -6
        r = LT.Reduction()
        assert L.lbm_reduce(h, C.byref(r)) == -6
        assert L.lbm_get_state(h, C.c_void_p(0x5000)) == -6
        assert L.lbm_rereference(h) == -6
        assert L.lbm_set_rereference_every(h, -1) == -1 and L.lbm_set_rereference_every(h, 0) == 0
        assert L.lbm_set_rereference_every(h, 1000) == 0
        assert L.lbm_init_equilibrium(h, None, None, None) == -1
        assert "NULL" in L.lbm_last_error(h).decode()
        n = C.c_int64(-1)
        assert L.lbm_step_count(h, C.byref(n)) == 0 and n.value == 0
    finally:
        L.lbm_destroy(h)


def test_no_cpu_fallback_without_a_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        LT.Lattice(8, 8)


def acfg(**kw):
    base = dict(n_steps=100, window=10, loss=LT.LOSS_DRAG, checkpoint_every=30, u_target_dev=None)
    base.update(kw)
    return LT.AdjointConfig(**base)


def test_adjoint_workspace_size_and_validation():
    L = LT.lib()
    b = C.c_size_t(0)
    c = cfg()
    n = 64 * 32
    assert L.lbm_adjoint_workspace_bytes(C.byref(c), C.byref(acfg()), C.byref(b)) == 0
    # 4 checkpoints (steps 0, 30, 60, 90) + 2 replay arrays of FP32 states (10 planes), 30
    # trajectory slots of 4 doubles, adjoint fields of 18 floats and 5 doubles per node
    assert b.value >= (4 + 2) * 10 * n * 4 + 30 * 4 * n * 8 + (18 * 4 + 5 * 8) * n
    assert b.value % 256 == 0
    small = b.value
    assert L.lbm_adjoint_workspace_bytes(C.byref(c), C.byref(acfg(checkpoint_every=10)), C.byref(b)) == 0
    assert b.value < small  # fewer trajectory slots outweigh the extra checkpoints here
    assert L.lbm_adjoint_workspace_bytes(C.byref(c), C.byref(acfg(checkpoint_every=1000)), C.byref(b)) == 0
    assert b.value >= 100 * 4 * n * 8  # trajectory slots are capped at n_steps
    for bad in (dict(n_steps=0), dict(checkpoint_every=0), dict(window=1), dict(window=101), dict(loss=7),
                dict(loss=LT.LOSS_UERR)):
        assert L.lbm_adjoint_workspace_bytes(C.byref(c), C.byref(acfg(**bad)), C.byref(b)) == -1, bad
        assert L.lbm_last_error(None).decode(), bad
    assert L.lbm_adjoint_workspace_bytes(C.byref(c), C.byref(acfg(window=1)), C.byref(b)) == -1
    assert "window" in L.lbm_last_error(None).decode()
    assert L.lbm_adjoint_workspace_bytes(C.byref(c), C.byref(acfg(loss=LT.LOSS_UERR, u_target_dev=0x1000)),
                                         C.byref(b)) == 0


def test_adjoint_argument_and_state_errors_without_a_gpu():
    L, h = fake_handle()
    try:
        gf, gG = C.c_double(0), C.c_double(0)
        assert L.lbm_adjoint_backward(h, None, C.byref(gf), C.byref(gG)) == -6
        out = C.c_double(0)
        a = acfg(window=1)
        assert L.lbm_adjoint_forward(h, C.byref(a), C.c_void_p(0x4000), C.c_void_p(0x8000), 1 << 30,
                                     C.byref(out)) == -1
        a = acfg()
        assert L.lbm_adjoint_forward(h, C.byref(a), None, C.c_void_p(0x8000), 1 << 30, C.byref(out)) == -1
        assert L.lbm_adjoint_forward(h, C.byref(a), C.c_void_p(0x4000), C.c_void_p(0x8001), 1 << 30,
                                     C.byref(out)) == -1
        assert L.lbm_adjoint_forward(h, C.byref(a), C.c_void_p(0x4000), C.c_void_p(0x8000), 256,
                                     C.byref(out)) == -1
        assert "too small" in L.lbm_last_error(h).decode()
        assert L.lbm_adjoint_backward(h, None, None, None) == -6
    finally:
        L.lbm_destroy(h)
    # moving walls are not supported by the adjoint
    c = cfg()
    buf = LT.Buffers(0x10000, 0x20000, 0x30000, None, 0x40000)
    h = C.c_void_p(0)
    assert L.lbm_create(C.byref(c), C.byref(buf), None, C.byref(h)) == 0
    try:
        out = C.c_double(0)
        assert L.lbm_adjoint_forward(h, C.byref(acfg()), C.c_void_p(0x4000), C.c_void_p(0x8000), 1 << 30,
                                     C.byref(out)) == -5
    finally:
        L.lbm_destroy(h)


def test_static_workspace_rejects_lattices_beyond_its_size():
    # lbm_create_static checks the workspace size on the host, before any device call
    L = LT.lib()
    big = LT.Config(2048, 2048, 1, 1, LT.FP64, LT.KERNEL_FUSED, 0.0, 16, 0)
    buf = LT.Buffers(None, None, None, None, None)
    h = C.c_void_p(0)
    rc = L.lbm_create_static(C.byref(big), C.byref(buf), None, C.byref(h))
    assert rc == -1 and not h.value
    msg = L.lbm_last_error(None).decode()
    assert "static workspace holds" in msg, msg
    # a caller workspace is refused: the static variant owns it
    small = LT.Config(64, 64, 1, 1, LT.FP64, LT.KERNEL_FUSED, 0.0, 16, 0)
    buf2 = LT.Buffers(None, None, 256, None, None)
    assert L.lbm_create_static(C.byref(small), C.byref(buf2), None, C.byref(h)) == -1
