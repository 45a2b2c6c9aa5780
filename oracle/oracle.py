"""TEST INFRASTRUCTURE ONLY: ctypes binding of the FP64 CPU oracle.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module.  It loads ``oracle/liboracle.so`` (built from ``lbm_oracle.cpp``
with g++) and never touches the GPU library.

The parameter struct mirrors ``OracleParams`` in ``lbm_oracle.cpp`` field by
field.  All arrays are numpy float64 / uint8, C-contiguous, row-major with x
fastest: scalar fields are ``[ny, nx]``, populations ``[9, ny, nx]``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

# Indices of the per-step observables (RED_* in lbm_oracle.cpp).
RED_NAMES = ("mass", "momx", "momy", "wallx", "wally", "uc_num", "uc_den", "buoy", "pphi", "faults")

EOS_VDW, EOS_CS = 0, 1
SCHEME_ORIGINAL, SCHEME_IMPROVED = 0, 1
Q2_DEFAULT, Q2_NEG_Q1, Q2_NEG_HALF_Q1 = 0, 1, 2
FORCE_CONST, FORCE_BUOYANT = 0, 1


def build(force: bool = True) -> str:
    """Compiles the oracle with g++ (IEEE binary64, no FP contraction)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-shared", "-fPIC", "-o", LIB + ".tmp", SRC]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
        ("eos_kind", C.c_int32), ("scheme", C.c_int32),
        ("q2_policy", C.c_int32), ("force_mode", C.c_int32),
        ("a", C.c_double), ("b", C.c_double), ("R", C.c_double), ("T", C.c_double),
        ("k_eos", C.c_double),
        ("G", C.c_double),
        ("s", C.c_double * 9),
        ("eps", C.c_double), ("k1", C.c_double), ("k2", C.c_double),
        ("fx", C.c_double), ("fy", C.c_double),
        ("rho_g", C.c_double), ("rho_l", C.c_double),
        ("rho_s", C.c_double),
    ]


class _Loss(C.Structure):
    _fields_ = [("kind", C.c_int32), ("window", C.c_int32), ("u_target", C.POINTER(C.c_double))]


@dataclass
class Params:
    """Physical and lattice parameters of one run (oracle side)."""
    nx: int
    ny: int
    periodic_x: bool = True
    periodic_y: bool = True
    eos_kind: int = EOS_CS
    a: float = 1.0
    b: float = 4.0
    R: float = 1.0
    T: float = 0.0
    k_eos: float = 1.0
    G: float = -1.0
    s: tuple = (1.0, 1.25, 1.25, 1.0, 9.0 / 7.0, 1.0, 9.0 / 7.0, 1.25, 1.25)
    scheme: int = SCHEME_IMPROVED
    q2_policy: int = Q2_DEFAULT
    eps: float = 0.0
    k1: Optional[float] = None   # None: -eps/16 (Sec. 3)
    k2: Optional[float] = None
    force_mode: int = FORCE_CONST
    fx: float = 0.0
    fy: float = 0.0
    rho_g: float = 0.0
    rho_l: float = 1.0
    rho_s: float = 0.0

    def to_c(self) -> _Params:
        p = _Params()
        p.nx, p.ny = self.nx, self.ny
        p.periodic_x, p.periodic_y = int(self.periodic_x), int(self.periodic_y)
        p.eos_kind, p.scheme, p.q2_policy, p.force_mode = self.eos_kind, self.scheme, self.q2_policy, self.force_mode
        p.a, p.b, p.R, p.T, p.k_eos = self.a, self.b, self.R, self.T, self.k_eos
        p.G = self.G
        for i in range(9):
            p.s[i] = float(self.s[i])
        p.eps = self.eps
        p.k1 = -self.eps / 16.0 if self.k1 is None else self.k1
        p.k2 = -self.eps / 16.0 if self.k2 is None else self.k2
        p.fx, p.fy = self.fx, self.fy
        p.rho_g, p.rho_l, p.rho_s = self.rho_g, self.rho_l, self.rho_s
        return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        u8 = C.POINTER(C.c_uint8)
        pp = C.POINTER(_Params)
        L.oracle_init.argtypes = [pp, u8, dp, dp, dp, dp]
        L.oracle_step.argtypes = [pp, u8, dp, dp, C.c_int64, dp, C.c_int]
        L.oracle_step.restype = C.c_longlong
        L.oracle_macros.argtypes = [pp, u8, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, C.c_int]
        L.oracle_moments.argtypes = [dp, dp]
        L.oracle_from_moments.argtypes = [dp, dp]
        L.oracle_equilibrium_moments.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        L.oracle_source.argtypes = [pp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, dp]
        L.oracle_collide.argtypes = [pp, dp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                     C.c_double, C.c_double, C.c_double, dp]
        L.oracle_p_eos.argtypes = [pp, C.c_double]
        L.oracle_p_eos.restype = C.c_double
        L.oracle_psi.argtypes = [pp, C.c_double]
        L.oracle_psi.restype = C.c_double
        L.oracle_loss.argtypes = [pp, u8, dp, dp, C.c_int64, C.POINTER(_Loss), C.c_int32, dp, C.c_double,
                                  dp, dp, C.c_int]
        L.oracle_adjoint.argtypes = [pp, u8, dp, dp, C.c_int64, C.POINTER(_Loss), C.c_int64, dp, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _u8(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_uint8))


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        assert a.shape == shape, (a.shape, shape)
    return a


def _mask(m, shape):
    if m is None:
        return None
    m = np.ascontiguousarray(m, dtype=np.uint8)
    assert m.shape == shape
    return m


@dataclass
class Oracle:
    """A lattice advanced by the oracle: holds the post-collision field."""
    params: Params
    mask: Optional[np.ndarray] = None
    wall_u: Optional[np.ndarray] = None  # [2, ny, nx]
    threads: int = 0
    f: np.ndarray = field(default=None, repr=False)
    step_count: int = 0

    def __post_init__(self):
        shp = (self.params.ny, self.params.nx)
        self.mask = _mask(self.mask, shp)
        self.wall_u = _f64(self.wall_u, (2,) + shp)
        self._p = self.params.to_c()

    @property
    def shape(self):
        return (self.params.ny, self.params.nx)

    def init(self, rho0, ux0=None, uy0=None):
        shp = self.shape
        rho0 = _f64(rho0, shp)
        ux0, uy0 = _f64(ux0, shp), _f64(uy0, shp)
        self.f = np.zeros((9,) + shp)
        rc = lib().oracle_init(C.byref(self._p), _u8(self.mask), _dp(rho0), _dp(ux0), _dp(uy0), _dp(self.f))
        assert rc == 0
        self.step_count = 0
        return self

    def step(self, n: int, reductions: bool = False):
        red = np.zeros((n, len(RED_NAMES))) if reductions else None
        faults = lib().oracle_step(C.byref(self._p), _u8(self.mask), _dp(self.wall_u), _dp(self.f),
                                   int(n), _dp(red), int(self.threads))
        assert faults >= 0
        self.step_count += n
        self.last_faults = int(faults)
        return red

    def macros(self):
        """Pre-collision fields the next step would use (rho, ux, uy, Fint, psi, pulled f, observables)."""
        shp = self.shape
        out = {k: np.zeros(shp) for k in ("rho", "ux", "uy", "fintx", "finty", "psi")}
        out["fpre"] = np.zeros((9,) + shp)
        red = np.zeros(len(RED_NAMES))
        lib().oracle_macros(C.byref(self._p), _u8(self.mask), _dp(self.wall_u), _dp(self.f),
                            _dp(out["rho"]), _dp(out["ux"]), _dp(out["uy"]), _dp(out["fintx"]),
                            _dp(out["finty"]), _dp(out["psi"]), _dp(out["fpre"]), _dp(red), int(self.threads))
        out["red"] = dict(zip(RED_NAMES, red))
        return out


# ---------------------------------------------------------------- node level

def moments(fi):
    fi = _f64(fi)
    m = np.zeros(9)
    lib().oracle_moments(_dp(fi), _dp(m))
    return m


def from_moments(m):
    m = _f64(m)
    fi = np.zeros(9)
    lib().oracle_from_moments(_dp(m), _dp(fi))
    return fi


def equilibrium_moments(r, u, v):
    out = np.zeros(9)
    lib().oracle_equilibrium_moments(r, u, v, _dp(out))
    return out


def source(params: Params, Fix, Fiy, psi, u, v):
    out = np.zeros(9)
    p = params.to_c()
    lib().oracle_source(C.byref(p), Fix, Fiy, psi, u, v, _dp(out))
    return out


def collide(params: Params, fi, r, u, v, Fx, Fy, Fix, Fiy, psi):
    fi = _f64(fi)
    out = np.zeros(9)
    p = params.to_c()
    lib().oracle_collide(C.byref(p), _dp(fi), r, u, v, Fx, Fy, Fix, Fiy, psi, _dp(out))
    return out


def p_eos(params: Params, r):
    p = params.to_c()
    return lib().oracle_p_eos(C.byref(p), float(r))


def psi(params: Params, r):
    p = params.to_c()
    return lib().oracle_psi(C.byref(p), float(r))


# ---------------------------------------------------------------- loss / derivatives

LOSS_DRAG, LOSS_UERR = 0, 1
PERTURB_NONE, PERTURB_FORCE, PERTURB_G, PERTURB_RHO0 = 0, 1, 2, 3


def loss(params: Params, rho0, nsteps: int, kind: int, window: int = 2, u_target=None,
         mask=None, wall_u=None, perturb: int = PERTURB_NONE, v=None, h: float = 1e-30, threads: int = 0):
    """Returns (L, dL) with dL the complex-step derivative along the perturbation."""
    shp = (params.ny, params.nx)
    rho0 = _f64(rho0, shp)
    mask = _mask(mask, shp)
    wall_u = _f64(wall_u, (2,) + shp)
    ut = _f64(u_target, shp)
    v = _f64(v, shp)
    spec = _Loss()
    spec.kind = kind
    spec.window = window
    spec.u_target = _dp(ut)
    L = C.c_double(0.0)
    dL = C.c_double(0.0)
    p = params.to_c()
    rc = lib().oracle_loss(C.byref(p), _u8(mask), _dp(wall_u), _dp(rho0), int(nsteps), C.byref(spec), int(perturb),
                           _dp(v), float(h), C.byref(L), C.byref(dL), int(threads))
    assert rc == 0, rc
    return L.value, dL.value


def adjoint(params: Params, rho0, nsteps: int, kind: int, window: int = 2, u_target=None, mask=None,
            wall_u=None, max_tape: int = 60_000_000):
    """The oracle's own discrete adjoint of the loss (reverse sweep of a recorded tape).
    Returns (L, dL/drho0 [ny, nx], dL/dG, dL/d|F|).  Small lattices only: the tape holds
    about 1,000 entries per node and step."""
    shp = (params.ny, params.nx)
    rho0 = _f64(rho0, shp)
    mask = _mask(mask, shp)
    wall_u = _f64(wall_u, (2,) + shp)
    ut = _f64(u_target, shp)
    spec = _Loss()
    spec.kind = kind
    spec.window = window
    spec.u_target = _dp(ut)
    L, dG, dF = C.c_double(0.0), C.c_double(0.0), C.c_double(0.0)
    g = np.zeros(shp)
    p = params.to_c()
    rc = lib().oracle_adjoint(C.byref(p), _u8(mask), _dp(wall_u), _dp(rho0), int(nsteps), C.byref(spec),
                              int(max_tape), C.byref(L), _dp(g), C.byref(dG), C.byref(dF))
    assert rc == 0, rc
    return L.value, g, dG.value, dF.value
