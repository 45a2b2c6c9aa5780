"""Shared test plumbing: conversion of a workload into oracle parameters."""
from __future__ import annotations

from oracle import oracle as O


def oracle_params(w, **over) -> O.Params:
    """Oracle parameters of a workload (paper_2604_13407_amd.workloads.Workload)."""
    kw = dict(nx=w.nx, ny=w.ny, periodic_x=w.periodic_x, periodic_y=w.periodic_y, eos_kind=w.eos_kind,
              a=w.a, b=w.b, R=w.R, T=w.T, k_eos=w.k_eos, G=w.G, s=tuple(w.s), scheme=w.scheme,
              eps=w.eps, k1=w.k1, k2=w.k2, force_mode=w.force_mode, fx=w.fx, fy=w.fy,
              rho_g=w.rho_g, rho_l=w.rho_l, rho_s=w.rho_s)
    kw.update(over)
    return O.Params(**kw)


def oracle_for(w, threads: int = 0, **over) -> O.Oracle:
    """An oracle lattice initialised with the workload's seeded inputs."""
    o = O.Oracle(oracle_params(w, **over), mask=w.mask(), wall_u=w.wall_velocity(), threads=threads)
    return o.init(w.rho0())


def fp64_bar(steps: int) -> float:
    """The FP64 comparison bar of a run of `steps` steps: 1e-12, or 5e-15 per
    step (about 20 ulp) for long runs.  Two FP64 implementations that round
    differently (fused multiply-adds, summation order) drift apart by a few
    ulp per step: near a steady state the same rounding repeats every step,
    so the difference grows linearly (measured GPU against the oracle: 5e-17
    per step on a converged cylindrical Couette flow, 5e-16 on the aligned
    channel over 20,000 steps, 2.4e-15 on the oblique channel over 50,000)."""
    return max(1e-12, 5e-15 * steps)
