"""GPU multigrid-preconditioned CG (opts.krylov = 1) against the oracle's
pcg_solve: same iteration count, residual histories to roundoff, solutions
to rel-L2 1e-9; and the same solution as the V-cycle solve."""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_util import gpu_solver, lib, oracle_level, rel_l2, to_global

TIGHT = 1e-12

CASES = [
    ("c0_periodic_singular", W.config_c0, 4, 0),
    ("lognormal64_32boxes", lambda: W.config_lognormal(64, 32), 4, 0),
    ("lognormal64_aggregated", lambda: W.config_lognormal(64, 16), 4, 1),
    ("lognormal48_uneven_periodic_x",
     lambda: dict(W.config_lognormal(48, 24,
                                      boxes=[((0, 0, 0), (23, 47, 47)), ((24, 0, 0), (47, 23, 47)),
                                             ((24, 24, 0), (47, 47, 47))]),
                  periodic=(True, False, False)), 4, 0),
]


@pytest.mark.gpu
@pytest.mark.parametrize("name,make,min_edge,agg", CASES, ids=[c[0] for c in CASES])
def test_pcg_matches_oracle(name, make, min_edge, agg):
    print(f"[pcg] {name}", flush=True)
    P = lib()
    cfg = make()
    if cfg["faces"] is not None and cfg["periodic"] != (False, False, False):
        cfg["faces"] = W.harmonic_faces(cfg["bcell"], cfg["periodic"])
    n, boxes = cfg["n"], cfg["boxes"]
    f = cfg["rhs"] - (cfg["rhs"].mean() if all(cfg["periodic"]) else 0.0)
    f_boxes = W.scatter_cells(f, boxes)
    s = gpu_solver(cfg, opts=dict(krylov=1, bottom_rel_tol=TIGHT, min_bottom_edge=min_edge,
                                  aggregate=agg))
    rhs = P.MultiFab.from_numpy(boxes, f_boxes, 0)
    phi = s.cell_mf(1, fill=0.0)
    g = s.solve(phi, rhs, 1e-10, history=True)
    torch.cuda.synchronize()
    gphi = to_global(phi, boxes, n)
    s.close()
    lev = oracle_level(cfg)
    ophi = O.new_cell_data(lev)
    o = O.pcg_solve(lev, ophi, f_boxes, 1e-10,
                    opts=O.Opts(bottom_tol=TIGHT, min_bottom_edge=min_edge, aggregate=bool(agg)))
    print(f"  GPU {g['iters']} iterations, oracle {o['iters']}")
    assert g["converged"] and o["converged"]
    assert g["iters"] == o["iters"], (g["history"], o["history"])
    nf = float(o["normf"])
    for k, (a, b) in enumerate(zip(g["history"], o["history"])):
        assert abs(a - b) <= 1e-6 * b + 1e-12 * nf, (k, a, b)
    err = rel_l2(gphi, W.gather_cells(ophi, boxes, n, ng=1))
    print(f"  rel-L2 vs oracle {err:.2e}")
    assert err <= 1e-9


@pytest.mark.gpu
def test_pcg_and_vcycles_reach_the_same_solution():
    print("[pcg] PCG vs V-cycles, lognormal 64^3", flush=True)
    P = lib()
    cfg = W.config_lognormal(64, 32)
    boxes = cfg["boxes"]
    rhs = P.MultiFab.from_numpy(boxes, W.scatter_cells(cfg["rhs"], boxes), 0)
    out = {}
    for k in (0, 1):
        s = gpu_solver(cfg, opts=dict(krylov=k))
        phi = s.cell_mf(1, fill=0.0)
        info = s.solve(phi, rhs, 1e-12)
        torch.cuda.synchronize()
        out[k] = (info, to_global(phi, boxes, 64))
        s.close()
    print(f"  V-cycles {out[0][0]['iters']}, PCG iterations {out[1][0]['iters']}")
    assert out[1][0]["iters"] < out[0][0]["iters"]
    assert rel_l2(out[1][1], out[0][1]) <= 1e-9


@pytest.mark.gpu
@pytest.mark.parametrize("name,make", [("lognormal64_32boxes", lambda: W.config_lognormal(64, 32)),
                                       ("c0_periodic_singular", W.config_c0)])
def test_pcg_float32_preconditioner_vs_oracle(name, make):
    """FP32 V-cycle as the preconditioner, FP64 CG: iteration count and
    solution against the oracle's pcg_solve with a float32 inner V-cycle."""
    print(f"[pcg] FP32 preconditioner {name}", flush=True)
    P = lib()
    cfg = make()
    n, boxes = cfg["n"], cfg["boxes"]
    f = cfg["rhs"] - (cfg["rhs"].mean() if all(cfg["periodic"]) else 0.0)
    f_boxes = W.scatter_cells(f, boxes)
    s = gpu_solver(cfg, opts=dict(krylov=1, precision=1, bottom_rel_tol=TIGHT))
    phi = s.cell_mf(1, fill=0.0)
    g = s.solve(phi, P.MultiFab.from_numpy(boxes, f_boxes, 0), 1e-10, history=True)
    torch.cuda.synchronize()
    gphi = to_global(phi, boxes, n)
    s.close()
    lev = oracle_level(cfg)
    ophi = O.new_cell_data(lev)
    o = O.pcg_solve(lev, ophi, f_boxes, 1e-10, opts=O.Opts(bottom_tol=TIGHT),
                    inner_dtype=np.float32)
    print(f"  GPU {g['iters']} iterations, oracle {o['iters']}")
    assert g["converged"] and o["converged"]
    assert abs(g["iters"] - o["iters"]) <= 1
    err = rel_l2(gphi, W.gather_cells(ophi, boxes, n, ng=1))
    print(f"  rel-L2 vs FP64-CG oracle with FP32 V-cycle {err:.2e}")
    assert err <= 1e-8


@pytest.mark.gpu
def test_pcg_option_errors():
    P = lib()
    cfg = W.config_lognormal(16, 8)
    with pytest.raises(P.MGError) as e:
        gpu_solver(cfg, opts=dict(krylov=2))
    assert e.value.code == P._lib.MG_ERR_ARG
