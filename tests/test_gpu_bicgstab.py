"""GPU BiCGStab bottom solver (opts bottom_solver = 1) against the oracle's
``bicgstab_bottom``: whole multigrid solves with per-cycle residual
histories and solutions, a single-level problem solved by the bottom solver
alone, and FP32 V-cycles inside FP64 refinement."""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_util import gpu_solver, lib, oracle_level, rel_l2, to_global
from test_gpu_solve import _check_history, _run_pair

BICG = dict(bottom_solver=1)
OBICG = dict(bottom_solver="bicgstab")


@pytest.mark.gpu
def test_bicgstab_bottom_c0_periodic_singular():
    print("[bicgstab] C0 32^3 periodic Poisson", flush=True)
    cfg = W.config_c0()
    g, gphi, o, ophi = _run_pair(cfg, opts=BICG, oracle_opts=OBICG)
    assert g["converged"] and g["nlevels"] == 3
    _check_history(g, o)
    assert rel_l2(gphi, ophi) <= 1e-9
    assert abs(gphi.mean()) <= 1e-14


@pytest.mark.gpu
@pytest.mark.parametrize("aggregate", [0, 1])
def test_bicgstab_bottom_lognormal(aggregate):
    print(f"[bicgstab] lognormal 64^3, 8 boxes, aggregate {aggregate}", flush=True)
    cfg = W.config_lognormal(64, 32)
    g, gphi, o, ophi = _run_pair(cfg, opts=BICG, oracle_opts=OBICG, aggregate=aggregate)
    assert g["converged"]
    _check_history(g, o)
    assert rel_l2(gphi, ophi) <= 1e-9


@pytest.mark.gpu
def test_bicgstab_single_level():
    """Boxes too small to coarsen: the solve is the bottom solver on level 0,
    in correction form each cycle."""
    print("[bicgstab] 12^3 in 8 boxes of 6^3 (one level)", flush=True)
    cfg = W.config_lognormal(12, 6)
    g, gphi, o, ophi = _run_pair(cfg, opts=BICG, oracle_opts=OBICG)
    assert g["nlevels"] == 1 and o["nlevels"] == 1
    assert g["converged"]
    _check_history(g, o, rtol=1e-5)
    assert rel_l2(gphi, ophi) <= 1e-9


@pytest.mark.gpu
def test_bicgstab_loose_bottom_converges_like_oracle():
    """At the default bottom tolerance (1e-4) the bottom solve stops early each
    cycle; roundoff may move its stopping point by an iteration, so the cycle
    counts agree within one and the solutions to the solve's accuracy."""
    print("[bicgstab] lognormal 32^3, bottom tol 1e-4", flush=True)
    P = lib()
    cfg = W.config_lognormal(32, 16)
    boxes = cfg["boxes"]
    s = gpu_solver(cfg, opts=dict(bottom_solver=1, bottom_rel_tol=1e-4))
    f = W.scatter_cells(cfg["rhs"], boxes)
    phi = s.cell_mf(1, fill=0.0)
    g = s.solve(phi, P.MultiFab.from_numpy(boxes, f, 0), 1e-10, history=True)
    torch.cuda.synchronize()
    gphi = to_global(phi, boxes, 32)
    s.close()
    lev = oracle_level(cfg)
    ophi = O.new_cell_data(lev)
    o = O.solve(lev, ophi, f, 1e-10, opts=O.Opts(bottom_solver="bicgstab", bottom_tol=1e-4))
    assert g["converged"] and o["converged"]
    assert abs(g["iters"] - o["iters"]) <= 1
    assert rel_l2(gphi, W.gather_cells(ophi, boxes, 32, ng=1)) <= 1e-8


@pytest.mark.gpu
def test_bicgstab_bottom_fp32_refinement():
    print("[bicgstab] FP32 V-cycles + FP64 refinement, lognormal 64^3", flush=True)
    P = lib()
    cfg = W.config_lognormal(64, 32)
    boxes = cfg["boxes"]
    s = gpu_solver(cfg, opts=dict(precision=1, bottom_solver=1, bottom_rel_tol=1e-6))
    f = W.scatter_cells(cfg["rhs"], boxes)
    phi = s.cell_mf(1, fill=0.0)
    g = s.solve(phi, P.MultiFab.from_numpy(boxes, f, 0), 1e-10)
    torch.cuda.synchronize()
    gphi = to_global(phi, boxes, 64)
    s.close()
    lev = oracle_level(cfg)
    ophi = O.new_cell_data(lev)
    o = O.solve(lev, ophi, f, 1e-10, opts=O.Opts(bottom_tol=1e-12))
    assert g["converged"] and o["converged"]
    assert rel_l2(gphi, W.gather_cells(ophi, boxes, 64, ng=1)) <= 1e-8
