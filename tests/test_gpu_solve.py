"""GPU multigrid solve against the CPU oracle.

Small cases (seconds for the oracle, several tiles and boxes per level):
per-cycle residual histories, one-cycle iterates element by element and
converged solutions.  Full 256^3 size (the benchmark's launch
configuration): the residual of the GPU solution recomputed by the oracle's
operator on every cell, and the GPU operator checked against the oracle's.
"""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_util import gpu_solver, lib, oracle_level, rel_l2, to_global

TIGHT = 1e-12  # bottom CG tolerance for parity: roundoff cannot move its stopping point


def _run_pair(cfg, opts=None, rel_tol=1e-10, max_iter=100, a_cells=None, min_edge=4,
              aggregate=0, oracle_opts=None):
    P = lib()
    n, boxes = cfg["n"], cfg["boxes"]
    gopts = dict(bottom_rel_tol=TIGHT, max_iter=max_iter, min_bottom_edge=min_edge,
                 aggregate=aggregate)
    gopts.update(opts or {})
    s = gpu_solver(cfg, opts=gopts, a_cells=a_cells)
    f_boxes = W.scatter_cells(cfg["rhs"], boxes)
    rhs = P.MultiFab.from_numpy(boxes, f_boxes, 0)
    phi = s.cell_mf(1, fill=0.0)
    ginfo = s.solve(phi, rhs, rel_tol, history=True, raise_on_fail=False)
    torch.cuda.synchronize()
    gphi = to_global(phi, boxes, n)
    lev = oracle_level(cfg, a_cells=a_cells)
    ophi = O.new_cell_data(lev)
    oinfo = O.solve(lev, ophi, f_boxes, rel_tol,
                    opts=O.Opts(bottom_tol=TIGHT, max_iter=max_iter, min_bottom_edge=min_edge,
                                aggregate=bool(aggregate), **(oracle_opts or {})))
    s.close()
    return ginfo, gphi, oinfo, W.gather_cells(ophi, boxes, n, ng=1)


def _check_history(g, o, rtol=1e-6):
    """Same cycle count; each max-norm residual equal to rtol, with an absolute
    allowance of 1e-12 max|f| for entries already at the roundoff floor of
    f - A phi (the two sides sum the stencil in different orders)."""
    assert g["iters"] == o["iters"], (g["history"], o["history"])
    nf = float(o["normf"])
    worst_rel = max(abs(a - b) / b for a, b in zip(g["history"], o["history"]))
    worst_abs = max(abs(a - b) for a, b in zip(g["history"], o["history"])) / nf
    print(f"history: {g['iters']} cycles, worst |gpu - oracle| {worst_rel:.2e} relative, "
          f"{worst_abs:.2e} max|f|")
    for k, (a, b) in enumerate(zip(g["history"], o["history"])):
        assert abs(a - b) <= rtol * b + 1e-12 * nf, (k, a, b)


@pytest.mark.gpu
def test_c0_periodic_poisson():
    print("[solve] C0 32^3 periodic Poisson", flush=True)
    cfg = W.config_c0()
    g, gphi, o, ophi = _run_pair(cfg)
    assert g["converged"] and g["nlevels"] == 3
    _check_history(g, o)
    assert rel_l2(gphi, ophi) <= 1e-9
    h = 1.0 / 32
    lam = 12 * np.sin(np.pi * h) ** 2 / h ** 2
    assert rel_l2(gphi, cfg["rhs"] / lam) <= 1e-9
    assert abs(gphi.mean()) <= 1e-14


@pytest.mark.gpu
def test_lognormal_dirichlet_64():
    print("[solve] lognormal 64^3, 8 boxes of 32^3", flush=True)
    cfg = W.config_lognormal(64, 32)
    g, gphi, o, ophi = _run_pair(cfg)
    assert g["converged"] and g["nlevels"] == 4
    _check_history(g, o)
    assert rel_l2(gphi, ophi) <= 1e-9


@pytest.mark.gpu
@pytest.mark.parametrize("which", ["c0", "lognormal64", "uneven96"])
def test_aggregated_hierarchy(which):
    """Boxes merged once they stop coarsening (one box down to 4^3)."""
    print(f"[solve] aggregated hierarchy {which}", flush=True)
    if which == "c0":
        cfg = W.config_c0()
    elif which == "lognormal64":
        cfg = W.config_lognormal(64, 16)
    else:
        cfg = W.config_lognormal(96, None, boxes=_uneven_boxes_96())
    g, gphi, o, ophi = _run_pair(cfg, aggregate=1)
    assert g["converged"] and g["nlevels"] == o["nlevels"]
    _check_history(g, o)
    assert rel_l2(gphi, ophi) <= 1e-9


@pytest.mark.gpu
def test_mixed_bc_with_cell_coefficient():
    print("[solve] 32^3 periodic-x, a != 1, alpha 0.5", flush=True)
    cfg = W.config_lognormal(32, 16)
    cfg["periodic"] = (True, False, False)
    cfg["faces"] = W.harmonic_faces(W.lognormal_cells(32, 1.0, 1), cfg["periodic"])
    cfg["alpha"] = 0.5
    a = W.lognormal_cells(32, 0.3, 9)
    g, gphi, o, ophi = _run_pair(cfg, a_cells=a)
    assert g["converged"]
    _check_history(g, o)
    assert rel_l2(gphi, ophi) <= 1e-9


@pytest.mark.gpu
def test_one_cycle_elementwise():
    """After exactly one V-cycle the iterates agree cell by cell."""
    print("[solve] one V-cycle, 48^3 in 8 boxes of 24^3", flush=True)
    cfg = W.config_lognormal(48, 24)
    g, gphi, o, ophi = _run_pair(cfg, max_iter=1, min_edge=3)
    assert g["iters"] == 1 and not g["converged"]
    scale = np.max(np.abs(ophi))
    assert np.max(np.abs(gphi - ophi)) <= 1e-12 * scale


@pytest.mark.gpu
def test_single_level_bottom_only():
    """Boxes too small to coarsen: the solve is CG on level 0."""
    print("[solve] 12^3 in 8 boxes of 6^3 (one level)", flush=True)
    cfg = W.config_lognormal(12, 6)
    g, gphi, o, ophi = _run_pair(cfg)
    assert g["nlevels"] == 1 and o["nlevels"] == 1
    assert g["converged"]
    _check_history(g, o, rtol=1e-5)
    assert rel_l2(gphi, ophi) <= 1e-9


def _uneven_boxes_96():
    """96^3 cut at x=32, y=48, z=64: boxes of edges (32|64) x 48 x (64|32); the
    48-edge boxes stop coarsening at 6, the others keep going."""
    out = []
    for zl, zh in ((0, 63), (64, 95)):
        for yl, yh in ((0, 47), (48, 95)):
            for xl, xh in ((0, 31), (32, 95)):
                out.append(((xl, yl, zl), (xh, yh, zh)))
    return out


@pytest.mark.gpu
def test_uneven_boxes():
    print("[solve] 96^3 uneven boxes", flush=True)
    boxes = _uneven_boxes_96()
    cfg = W.config_lognormal(96, None, boxes=boxes)
    g, gphi, o, ophi = _run_pair(cfg)
    assert g["converged"] and g["nlevels"] == 4
    _check_history(g, o)
    assert rel_l2(gphi, ophi) <= 1e-9


@pytest.mark.gpu
def test_guillotine256_full_residual():
    """256^3 guillotine boxes (the 512^3 generator's structure at 256): the
    oracle's operator recomputes the residual of the GPU solution everywhere."""
    print("[solve] guillotine 256^3", flush=True)
    P = lib()
    boxes = W.guillotine_boxes(256)
    cfg = W.config_lognormal(256, None, boxes=boxes)
    s = gpu_solver(cfg)
    f_boxes = W.scatter_cells(cfg["rhs"], boxes)
    rhs = P.MultiFab.from_numpy(boxes, f_boxes, 0)
    phi = s.cell_mf(1, fill=0.0)
    info = s.solve(phi, rhs, 1e-10)
    print(f"guillotine256: {len(boxes)} boxes, {info['nlevels']} levels, {info['iters']} cycles, "
          f"{info['solve_ms']:.1f} ms")
    lev = oracle_level(cfg)
    oA = O.apply_op(lev, phi.to_numpy())
    r = max(float(np.max(np.abs(fb - a))) for fb, a in zip(f_boxes, oA))
    normf = max(float(np.max(np.abs(x))) for x in f_boxes)
    assert r <= 1e-10 * normf * (1 + 1e-3)
    s.close()


@pytest.mark.gpu
def test_float32_refinement_vs_fp64_oracle():
    print("[solve] FP32 V-cycle + FP64 refinement, 64^3", flush=True)
    P = lib()
    cfg = W.config_lognormal(64, 32)
    boxes = cfg["boxes"]
    s = gpu_solver(cfg, opts=dict(precision=1))
    f_boxes = W.scatter_cells(cfg["rhs"], boxes)
    rhs = P.MultiFab.from_numpy(boxes, f_boxes, 0)
    phi = s.cell_mf(1, fill=0.0)
    info = s.solve(phi, rhs, 1e-10, history=True)
    assert info["converged"] and info["rel_resid"] <= 1e-10
    lev = oracle_level(cfg)
    ophi = O.new_cell_data(lev)
    O.solve(lev, ophi, f_boxes, 1e-12, opts=O.Opts(bottom_tol=TIGHT))
    err = rel_l2(to_global(phi, boxes, 64), W.gather_cells(ophi, boxes, 64, ng=1))
    print(f"FP32+refine rel-L2 vs FP64 oracle: {err:.3e} ({info['iters']} refinement steps)")
    assert err <= 1e-8
    s.close()


@pytest.mark.gpu
def test_tile_shapes_and_graph_bitwise_identical():
    """Red/black updates within a colour are independent: any tiling, with or
    without graph replay, must give the same bits (a race or overlap would not)."""
    print("[solve] tile-shape invariance 64^3", flush=True)
    P = lib()
    cfg = W.config_lognormal(64, 32)
    boxes = cfg["boxes"]
    rhs = P.MultiFab.from_numpy(boxes, W.scatter_cells(cfg["rhs"], boxes), 0)
    outs = []
    # kernels 0-2 on half-sweep levels (fused sweeps off), kernel 3 = fused sweep,
    # kernel 4 = the residual pass restricting into level 1
    shapes = [None, (0, 16, 4, 4, 1), (0, 32, 8, 32, 2), (0, 64, 4, 64, 4), (0, 32, 2, 2, 2),
              (0, 32, 8, 1, 1), (2, 32, 4, 4, 2), (2, 16, 4, 8, 1), (1, 32, 2, 8, 1),
              (1, 128, 2, 64, 4), (1, 64, 4, 4, 2), (3, 64, 8, 16, 1), (3, 32, 8, 4, 1),
              (3, 64, 4, 32, 1), (3, 32, 16, 8, 1), (4, 32, 2, 2, 2), (4, 64, 2, 8, 2),
              (4, 128, 2, 4, 2), (4, 32, 8, 2, 2)]
    for graph in (1, 0):
        for sh in shapes:
            fused = 32 if sh is not None and sh[0] == 3 else 0
            s = gpu_solver(cfg, opts=dict(max_iter=2, use_graph=graph, tune=0,
                                          fused_min_edge=fused))
            if sh is not None:
                s.set_tile_shape(*sh)
            phi = s.cell_mf(1, fill=0.0)
            s.solve(phi, rhs, 1e-10, raise_on_fail=False)
            torch.cuda.synchronize()
            # valid cells only: which ghosts hold current values depends on the
            # path (write-through fills face ghosts, the fused path exchanges)
            outs.append(to_global(phi, boxes, 64))
            s.close()
    ref = outs[0]
    assert np.all(np.isfinite(ref))
    for o in outs[1:]:
        assert np.array_equal(o, ref)


@pytest.mark.gpu
@pytest.mark.parametrize("precision", [0, 1])
def test_tuned_shapes_bitwise_identical(precision, tmp_path, monkeypatch):
    """The tuner picks level-0 and level-1 tile shapes (search, then the cached
    entries): the solution keeps the bits of the default tiling."""
    print(f"[solve] tuned shapes 64^3 precision={precision}", flush=True)
    P = lib()
    cfg = W.config_lognormal(64, 32)
    boxes = cfg["boxes"]
    rhs = P.MultiFab.from_numpy(boxes, W.scatter_cells(cfg["rhs"], boxes), 0)
    cache = tmp_path / "tiles.txt"
    monkeypatch.setenv("AMRMG_TUNE_CACHE", str(cache))
    outs = []
    for tune in (0, 2, 1):
        s = gpu_solver(cfg, opts=dict(max_iter=3, tune=tune, precision=precision))
        phi = s.cell_mf(1, fill=0.0)
        s.solve(phi, rhs, 1e-10, raise_on_fail=False)
        torch.cuda.synchronize()
        outs.append(to_global(phi, boxes, 64))
        s.close()
    lines = cache.read_text().split("\n")
    tag = "f32" if precision else "f64"
    # level 0 boxes and level 1 boxes (half their edges) each have entries
    keys = [ln.split()[0] for ln in lines if ln.strip()]
    for kern in ("gsrb", "resid"):
        dims = sorted({k.split("|")[-2] for k in keys if f"|{kern}|{tag}|" in k})
        assert len(dims) == 2, keys
    assert np.all(np.isfinite(outs[0]))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.gpu
@pytest.mark.parametrize("precision", [0, 1])
def test_class_tile_shapes_bitwise_identical(precision, tmp_path, monkeypatch):
    """Level-0 smoother tiles chosen per box class (x extent) inside one launch
    -- forced shapes, including one-plane tiles and tiles wider than their
    boxes, and the tuner's own per-class choice -- give the bits of the
    uniform default tiling on uneven boxes (192^3: x extents 32, 48, 64, 96)."""
    print(f"[solve] class tile shapes 192^3 guillotine precision={precision}", flush=True)
    P = lib()
    cfg = W.config_lognormal(192, None, boxes=W.guillotine_boxes(192))
    boxes = cfg["boxes"]
    rhs = P.MultiFab.from_numpy(boxes, W.scatter_cells(cfg["rhs"], boxes), 0)
    monkeypatch.setenv("AMRMG_TUNE_CACHE", str(tmp_path / "tiles.txt"))
    forced = [{96: (16, 16, 4), 48: (64, 4, 2), 64: (32, 8, 8), 32: (16, 16, 16)},
              {96: (32, 8, 2), 48: (16, 16, 2)},
              {32: (64, 4, 4), 64: (16, 16, 2), 96: (64, 4, 16), 48: (32, 8, 4)}]
    outs = []
    for k in range(len(forced) + 2):
        tune = 2 if k == len(forced) + 1 else 0
        s = gpu_solver(cfg, opts=dict(max_iter=3, tune=tune, precision=precision))
        if 1 <= k <= len(forced):
            for x, (lx, ly, tz) in forced[k - 1].items():
                s.set_class_tile_shape(x, lx, ly, tz)
            assert s.class_tile_shapes() == forced[k - 1]
        phi = s.cell_mf(1, fill=0.0)
        s.solve(phi, rhs, 1e-10, raise_on_fail=False)
        torch.cuda.synchronize()
        outs.append(to_global(phi, boxes, 192))
        s.close()
    assert np.all(np.isfinite(outs[0]))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    # a shape that is not a candidate of the launch is refused
    s = gpu_solver(cfg, opts=dict(tune=0, precision=precision))
    with pytest.raises(P.MGError):
        s.set_class_tile_shape(96, 16, 4, 4)
    with pytest.raises(P.MGError):
        s.set_class_tile_shape(80, 32, 8, 4)
    s.close()


FUSED_CASES = [
    # (name, cfg, boxes or None, fused_min_edge, precision)
    ("lognormal64_32boxes_f64", lambda: W.config_lognormal(64, 32), None, 32, 0),
    ("lognormal64_32boxes_f32", lambda: W.config_lognormal(64, 32), None, 32, 1),
    ("lognormal64_16boxes_all_levels", lambda: W.config_lognormal(64, 16), None, 4, 0),
    ("poisson32_periodic", W.config_c0, None, 8, 0),
    ("uneven_periodic_y", lambda: dict(W.config_c0(), periodic=(False, True, False)),
     [((0, 0, 0), (15, 31, 31)), ((16, 0, 0), (31, 15, 31)), ((16, 16, 0), (31, 31, 15)),
      ((16, 16, 16), (31, 31, 31))], 8, 0),
]


@pytest.mark.gpu
@pytest.mark.parametrize("name,make,boxes,edge,prec", FUSED_CASES, ids=[c[0] for c in FUSED_CASES])
def test_fused_sweeps_bitwise_equal_half_sweeps(name, make, boxes, edge, prec):
    """A fused sweep (one pass into a second buffer, rim pass after an
    exchange) performs the same arithmetic on the same values as a red and a
    black half-sweep: solutions after a few cycles must agree bit for bit."""
    print(f"[solve] fused vs half-sweeps {name}", flush=True)
    P = lib()
    cfg = make()
    boxes = boxes or cfg["boxes"]
    f = cfg["rhs"] - (cfg["rhs"].mean() if all(cfg["periodic"]) else 0.0)
    rhs = P.MultiFab.from_numpy(boxes, W.scatter_cells(f, boxes), 0)
    outs, iters = [], []
    for fme in (edge, 0):
        s = gpu_solver(cfg, boxes=boxes, opts=dict(max_iter=3, tune=0, fused_min_edge=fme,
                                                   precision=prec))
        phi = s.cell_mf(1, fill=0.0)
        info = s.solve(phi, rhs, 1e-10, raise_on_fail=False, history=True)
        torch.cuda.synchronize()
        outs.append(to_global(phi, boxes, cfg["n"]))
        iters.append(list(info["history"]))
        s.close()
    assert np.all(np.isfinite(outs[0]))
    assert np.array_equal(outs[0], outs[1])
    assert iters[0] == iters[1]


WT_CASES = [
    # (name, cfg maker, boxes or None, opts)
    ("lognormal64_32boxes_f64", lambda: W.config_lognormal(64, 32), None, {}),
    ("lognormal64_32boxes_f32", lambda: W.config_lognormal(64, 32), None, dict(precision=1)),
    ("lognormal64_16boxes_pcg", lambda: W.config_lognormal(64, 16), None, dict(krylov=1)),
    ("poisson32_periodic_self_images", W.config_c0, None, {}),
    ("one_box_periodic", W.config_c0, [W.domain_box(32)], {}),
    ("uneven_periodic_y", lambda: dict(W.config_c0(), periodic=(False, True, False)),
     [((0, 0, 0), (15, 31, 31)), ((16, 0, 0), (31, 15, 31)), ((16, 16, 0), (31, 31, 15)),
      ((16, 16, 16), (31, 31, 31))], {}),
    ("uneven96", lambda: W.config_lognormal(96, None, boxes=_uneven_boxes_96()), None, {}),
    # 192^3: a half-sweep's arrays (340 MB) exceed the last-level cache, so the
    # write-through path loads through buffer descriptors
    ("lognormal192_27boxes_buffer_loads", lambda: W.config_lognormal(192, 64), None, {}),
    # 256^3 FP32: the FP32 arrays stream too, and the folded half-sweep then
    # also loads the coarse correction through a buffer descriptor
    ("lognormal256_64boxes_f32_buffer_loads", lambda: W.config_lognormal(256, 64), None,
     dict(precision=1)),
]


@pytest.mark.gpu
@pytest.mark.parametrize("name,make,boxes,extra", WT_CASES, ids=[c[0] for c in WT_CASES])
def test_ghost_write_through_bitwise_equal_exchanges(name, make, boxes, extra):
    """Half-sweeps that store boundary updates straight into the neighbours'
    face ghosts (no exchange between half-sweeps), with and without the
    interpolation folded into the first post-smoothing half-sweep and the
    restriction folded into a coarse level's first pre-smoothing half-sweep,
    give the same bits as separate interpolation and restriction passes and
    an exchange before every half-sweep."""
    print(f"[solve] ghost write-through vs exchanges {name}", flush=True)
    P = lib()
    cfg = make()
    boxes = boxes or cfg["boxes"]
    f = cfg["rhs"] - (cfg["rhs"].mean() if all(cfg["periodic"]) else 0.0)
    rhs = P.MultiFab.from_numpy(boxes, W.scatter_cells(f, boxes), 0)
    outs, hist, interp = [], [], []
    for gw, fold, rfold in ((1, 1, 2), (1, 1, 1), (1, 0, 2), (0, 1, 2), (1, 1, 0), (0, 0, 0)):
        s = gpu_solver(cfg, boxes=boxes, opts=dict(max_iter=3, tune=0, ghost_write=gw,
                                                   interp_fold=fold, restrict_fold=rfold,
                                                   **extra))
        phi = s.cell_mf(1, fill=0.0)
        s.profile(True)
        info = s.solve(phi, rhs, 1e-10, raise_on_fail=False, history=True)
        torch.cuda.synchronize()
        interp.append(s.kernel_stats(P._lib.FAM_PROLONG)[1])
        s.profile(False)
        outs.append(to_global(phi, boxes, cfg["n"]))
        hist.append(list(info["history"]))
        s.close()
    assert np.all(np.isfinite(outs[0]))
    for o, h in zip(outs[1:], hist[1:]):
        assert np.array_equal(outs[0], o)
        assert hist[0] == h
    # one level-0 interpolation per V-cycle either way (folded or a pass)
    assert interp[0] > 0 and all(x == interp[0] for x in interp)


STOP_FOLD_CASES = [
    # (name, cfg maker, boxes or None, opts, rel_tol)
    ("lognormal64_32boxes_converged", lambda: W.config_lognormal(64, 32), None, {}, 1e-10),
    ("lognormal64_32boxes_max_iter", lambda: W.config_lognormal(64, 32), None,
     dict(max_iter=3), 1e-10),
    ("lognormal64_16boxes_no_graph_no_write_through", lambda: W.config_lognormal(64, 16), None,
     dict(use_graph=0, ghost_write=0), 1e-10),
    ("lognormal64_16boxes_nu1_nu2_1", lambda: W.config_lognormal(64, 16), None,
     dict(nu1=1, nu2=1), 1e-9),
    ("lognormal64_16boxes_nu2_0", lambda: W.config_lognormal(64, 16), None,
     dict(nu1=3, nu2=0), 1e-8),
    ("poisson32_periodic_singular", W.config_c0, None, {}, 1e-10),
    ("uneven_periodic_y", lambda: dict(W.config_c0(), periodic=(False, True, False)),
     [((0, 0, 0), (15, 31, 31)), ((16, 0, 0), (31, 15, 31)), ((16, 16, 0), (31, 31, 15)),
      ((16, 16, 16), (31, 31, 31))], {}, 1e-10),
    ("lognormal192_27boxes_buffer_loads", lambda: W.config_lognormal(192, 64), None, {}, 1e-10),
]


@pytest.mark.gpu
@pytest.mark.parametrize("name,make,boxes,extra,tol", STOP_FOLD_CASES,
                         ids=[c[0] for c in STOP_FOLD_CASES])
def test_stop_fold_bitwise_equal_plain_loop(name, make, boxes, extra, tol):
    """The stop test's residual pass that also performs the next cycle's red
    half-sweep into the second level-0 array (iterates alternating between
    the two, norms read one pass behind) gives the same norms, cycle count,
    status and solution bits as a norm-only residual pass before each cycle."""
    print(f"[solve] folded stop test vs plain loop {name}", flush=True)
    P = lib()
    cfg = make()
    boxes = boxes or cfg["boxes"]
    f = cfg["rhs"] - (cfg["rhs"].mean() if all(cfg["periodic"]) else 0.0)
    rhs = P.MultiFab.from_numpy(boxes, W.scatter_cells(f, boxes), 0)
    outs, infos = [], []
    for sf in (1, 0):
        s = gpu_solver(cfg, boxes=boxes, opts=dict(tune=0, bottom_rel_tol=TIGHT, stop_fold=sf,
                                                   **extra))
        phi = s.cell_mf(1, fill=0.0)
        info = s.solve(phi, rhs, tol, raise_on_fail=False, history=True)
        torch.cuda.synchronize()
        outs.append(to_global(phi, boxes, cfg["n"]))
        infos.append(info)
        s.close()
    assert np.all(np.isfinite(outs[0]))
    assert np.array_equal(outs[0], outs[1])
    assert infos[0]["iters"] == infos[1]["iters"]
    assert infos[0]["converged"] == infos[1]["converged"]
    assert list(infos[0]["history"]) == list(infos[1]["history"])
    if "max_iter" in extra:
        assert not infos[0]["converged"] and infos[0]["iters"] == extra["max_iter"]
    else:
        assert infos[0]["converged"]


@pytest.mark.gpu
def test_quad_smoother_bitwise_fp32_256():
    """The FP32 smoother with one x-quad per lane (two cells of the colour,
    16-byte loads; level-0 FP32 arrays that stream through buffer loads, so
    256^3) gives the bits of the x-pair mapping: the same FP32+refine
    history and solution for every quad shape, with one and two planes in
    flight, including the zero-guess and folded-interpolation half-sweeps."""
    print("[solve] quad smoother mapping FP32 256^3", flush=True)
    P = lib()
    cfg = W.config_c1()
    boxes = cfg["boxes"]
    rhs = P.MultiFab.from_numpy(boxes, W.scatter_cells(cfg["rhs"], boxes), 0)
    outs, hists = [], []
    for sh in (None, (5, 16, 16, 1, 1), (5, 16, 8, 2, 2), (5, 8, 16, 4, 1), (5, 32, 8, 1, 1)):
        s_ = gpu_solver(cfg, opts=dict(max_iter=3, tune=0, precision=1, aggregate=1))
        if sh is not None:
            s_.set_tile_shape(*sh)
            assert s_.tile_shape(0)[4] == 2
        phi = s_.cell_mf(1, fill=0.0)
        info = s_.solve(phi, rhs, 1e-10, raise_on_fail=False, history=True)
        torch.cuda.synchronize()
        outs.append(to_global(phi, boxes, cfg["n"]))
        hists.append(list(info["history"]))
        s_.close()
    assert np.all(np.isfinite(outs[0]))
    for o, h in zip(outs[1:], hists[1:]):
        assert h == hists[0]
        assert np.array_equal(o, outs[0])
    # not on an FP64 solver
    s_ = gpu_solver(cfg, opts=dict(max_iter=1, tune=0, aggregate=1))
    with pytest.raises(Exception):
        s_.set_tile_shape(5, 16, 16, 1, 1)
    s_.close()


@pytest.mark.gpu
def test_quad_smoother_bitwise_fp32_uneven_boxes():
    """The same on 256^3 cut into 62 guillotine boxes with x extents 32, 48,
    64, 96 and 128: quad tiles of 32, 64 and 128 cells per row leave ragged
    last tiles (a quad partly or wholly past its box, a row's last quad with
    one cell of the colour) and boxes whose x faces meet several
    neighbours."""
    print("[solve] quad smoother mapping FP32 256^3 guillotine boxes", flush=True)
    P = lib()
    cfg = W.config_c2(256)
    boxes = cfg["boxes"]
    assert sorted({h[0] - l[0] + 1 for l, h in boxes}) == [32, 48, 64, 96, 128]
    rhs = P.MultiFab.from_numpy(boxes, W.scatter_cells(cfg["rhs"], boxes), 0)
    outs, hists = [], []
    for sh in (None, (5, 8, 16, 1, 1), (5, 16, 8, 2, 2), (5, 32, 8, 1, 1)):
        s_ = gpu_solver(cfg, opts=dict(max_iter=3, tune=0, precision=1, aggregate=1))
        if sh is not None:
            s_.set_tile_shape(*sh)
            assert s_.tile_shape(0)[4] == 2
        phi = s_.cell_mf(1, fill=0.0)
        info = s_.solve(phi, rhs, 1e-10, raise_on_fail=False, history=True)
        torch.cuda.synchronize()
        outs.append(to_global(phi, boxes, cfg["n"]))
        hists.append(list(info["history"]))
        s_.close()
    assert np.all(np.isfinite(outs[0]))
    assert hists[0][-1] < hists[0][0]
    for o, h in zip(outs[1:], hists[1:]):
        assert h == hists[0]
        assert np.array_equal(o, outs[0])
    # x extents 126 and 130 (2 mod 4): a row's last quad would reach past
    # the end of the last row's arrays, so the mapping is refused
    c1 = W.config_c1()
    odd = [((x0, y0, z0), (x1, y0 + 63, z0 + 63)) for x0, x1 in ((0, 125), (126, 255))
           for y0 in range(0, 256, 64) for z0 in range(0, 256, 64)]
    s_ = gpu_solver(c1, boxes=odd, opts=dict(max_iter=1, tune=0, precision=1, aggregate=1))
    with pytest.raises(Exception):
        s_.set_tile_shape(5, 16, 16, 1, 1)
    assert s_.tile_shape(0)[4] != 2
    s_.close()


TAIL_CASES = [
    # (name, cfg maker, boxes or None, opts (coarse_tail: the threshold), rel_tol, a != 1,
    #  first tail level)
    ("lognormal64_8boxes_aggregated_default", lambda: W.config_lognormal(64, 32), None,
     dict(aggregate=1), 1e-10, False, 3),
    ("lognormal64_8boxes_two_levels", lambda: W.config_lognormal(64, 32), None,
     dict(coarse_tail=4096), 1e-10, False, 2),
    ("lognormal64_8boxes_aggregated_three_levels", lambda: W.config_lognormal(64, 32), None,
     dict(aggregate=1, coarse_tail=4096), 1e-10, False, 2),
    ("lognormal64_tail_from_level1", lambda: W.config_lognormal(64, 32), None,
     dict(coarse_tail=32768), 1e-10, False, 1),
    ("poisson32_periodic_singular_from_level1", W.config_c0, None, dict(coarse_tail=4096),
     1e-10, False, 1),
    ("poisson32_periodic_singular_aggregated_default", W.config_c0, None, dict(aggregate=1),
     1e-10, False, 2),
    ("uneven_periodic_y", lambda: dict(W.config_c0(), periodic=(False, True, False)),
     [((0, 0, 0), (15, 31, 31)), ((16, 0, 0), (31, 15, 31)), ((16, 16, 0), (31, 31, 15)),
      ((16, 16, 16), (31, 31, 31))], dict(coarse_tail=4096), 1e-10, False, 1),
    ("lognormal64_f32_refine", lambda: W.config_lognormal(64, 32), None,
     dict(precision=1, aggregate=1, coarse_tail=4096), 1e-10, False, 2),
    ("lognormal64_mgpcg", lambda: W.config_lognormal(64, 32), None,
     dict(krylov=1, aggregate=1), 1e-10, False, 3),
    ("lognormal64_mgpcg_f32", lambda: W.config_lognormal(64, 32), None,
     dict(krylov=1, precision=1, coarse_tail=4096), 1e-10, False, 2),
    ("lognormal64_nu1_nu2_1", lambda: W.config_lognormal(64, 32), None,
     dict(nu1=1, nu2=1, coarse_tail=4096), 1e-9, False, 2),
    ("lognormal64_nu2_0", lambda: W.config_lognormal(64, 32), None,
     dict(nu1=3, nu2=0, coarse_tail=4096), 1e-8, False, 2),
    ("lognormal64_no_graph_max_iter_3", lambda: W.config_lognormal(64, 32), None,
     dict(use_graph=0, max_iter=3, coarse_tail=4096), 1e-10, False, 2),
    ("lognormal32_periodic_x_cell_coefficient",
     lambda: dict(W.config_lognormal(32, 16), periodic=(True, False, False), alpha=0.5), None,
     dict(coarse_tail=4096), 1e-10, True, 1),
]


@pytest.mark.gpu
@pytest.mark.parametrize("name,make,boxes,extra,tol,with_a,level", TAIL_CASES,
                         ids=[c[0] for c in TAIL_CASES])
def test_coarse_tail_bitwise_equal_launches(name, make, boxes, extra, tol, with_a, level):
    """The coarsest levels run as one single-work-group launch per cycle
    (default) give the same norms, cycle count and solution bits as a launch
    per pass (coarse_tail = 0)."""
    print(f"[solve] coarse tail vs a launch per pass {name}", flush=True)
    P = lib()
    cfg = make()
    boxes = boxes or cfg["boxes"]
    f = cfg["rhs"] - (cfg["rhs"].mean() if all(cfg["periodic"]) else 0.0)
    rhs = P.MultiFab.from_numpy(boxes, W.scatter_cells(f, boxes), 0)
    a_cells = None
    if with_a:
        a_cells = np.random.default_rng(5).uniform(0.5, 2.0, size=(cfg["n"],) * 3)
    outs, infos = [], []
    for tail in (extra.get("coarse_tail", 1024), 0):
        opts = dict(extra, tune=0, bottom_rel_tol=TIGHT, coarse_tail=tail)
        s = gpu_solver(cfg, boxes=boxes, opts=opts, a_cells=a_cells)
        phi = s.cell_mf(1, fill=0.0)
        info = s.solve(phi, rhs, tol, raise_on_fail=False, history=True)
        torch.cuda.synchronize()
        outs.append(to_global(phi, boxes, cfg["n"]))
        infos.append(info)
        s.close()
    assert infos[0]["tail_level"] == level and infos[1]["tail_level"] == 0
    assert np.all(np.isfinite(outs[0]))
    assert np.array_equal(outs[0], outs[1])
    assert infos[0]["iters"] == infos[1]["iters"]
    assert infos[0]["bottom_iters"] == infos[1]["bottom_iters"]
    assert infos[0]["converged"] == infos[1]["converged"]
    assert list(infos[0]["history"]) == list(infos[1]["history"])
    if "max_iter" in extra:
        assert infos[0]["iters"] == extra["max_iter"]
    else:
        assert infos[0]["converged"]


@pytest.mark.gpu
@pytest.mark.parametrize("variant", ["f64", "f32_refine", "f64_mgpcg"])
def test_c1_bench_configuration(variant, monkeypatch):
    """256^3 in the benchmark's launch configuration (aggregated hierarchy,
    tiles searched at set-up, coarse levels replayed from the graph, folded
    restriction chosen by the tuner): the oracle's operator recomputes
    f - A phi on every cell.  V-cycle solves keep the bits of the default
    tiling; MG-PCG sums p.q per residual tile, so there the residual's tile
    shape moves the last bits and both solutions are checked instead."""
    print(f"[solve] C1 256^3 bench configuration {variant}", flush=True)
    monkeypatch.delenv("AMRMG_TUNE_CACHE", raising=False)
    P = lib()
    cfg = W.config_c1()
    n, boxes = cfg["n"], cfg["boxes"]
    f_boxes = W.scatter_cells(cfg["rhs"], boxes)
    rhs = P.MultiFab.from_numpy(boxes, f_boxes, 0)
    opts = dict(aggregate=1, precision=1 if variant == "f32_refine" else 0,
                krylov=1 if variant.endswith("mgpcg") else 0)
    sols, infos = [], []
    for tune in (2, 0):
        s = gpu_solver(cfg, opts=dict(opts, tune=tune))
        phi = s.cell_mf(1, fill=0.0)
        info = s.solve(phi, rhs, 1e-10)
        torch.cuda.synchronize()
        assert info["converged"] and info["nlevels"] == 7
        infos.append(info)
        sols.append(phi.to_numpy())
        s.close()
        del phi
    print(f"C1 {variant}: {infos[0]['iters']} iterations, {infos[0]['solve_ms']:.1f} ms")
    assert infos[0]["iters"] == infos[1]["iters"]
    pcg = variant.endswith("mgpcg")
    if not pcg:
        assert all(np.array_equal(a[1:-1, 1:-1, 1:-1], b[1:-1, 1:-1, 1:-1])
                   for a, b in zip(sols[0], sols[1]))
    lev = oracle_level(cfg)
    normf = max(float(np.max(np.abs(x))) for x in f_boxes)
    for sol in sols[:2 if pcg else 1]:
        oA = O.apply_op(lev, sol)
        r = max(float(np.max(np.abs(fb - a))) for fb, a in zip(f_boxes, oA))
        assert r <= 1e-10 * normf * (1 + 1e-3)
    torch.cuda.empty_cache()


@pytest.mark.gpu
def test_error_paths():
    print("[solve] error paths", flush=True)
    P = lib()
    cfg = W.config_lognormal(16, 8)
    boxes = cfg["boxes"]
    s = gpu_solver(cfg, opts=dict(max_iter=1))
    f = W.scatter_cells(cfg["rhs"], boxes)
    rhs = P.MultiFab.from_numpy(boxes, f, 0)
    phi = s.cell_mf(1, fill=0.0)
    info = s.solve(phi, rhs, 1e-10, raise_on_fail=False)
    assert info["status"] == P._lib.MG_ERR_NOT_CONVERGED and info["iters"] == 1
    assert np.all(np.isfinite(to_global(phi, boxes, 16)))
    bad = [x.copy() for x in f]
    bad[3][1, 2, 3] = np.nan
    with pytest.raises(P.MGError) as e:
        s.solve(s.cell_mf(1, fill=0.0), P.MultiFab.from_numpy(boxes, bad, 0), 1e-10)
    assert e.value.code == P._lib.MG_ERR_NAN
    zero = P.MultiFab.from_numpy(boxes, [np.zeros_like(x) for x in f], 0)
    phi = s.cell_mf(1, fill=5.0)
    info = s.solve(phi, zero, 1e-10)
    assert info["converged"] and not np.any(to_global(phi, boxes, 16))
    other = P.MultiFab(W.uniform_boxes(16, 16), 1, fill=0.0)
    with pytest.raises(P.MGError) as e:
        s.solve(other, rhs, 1e-10)
    assert e.value.code == P._lib.MG_ERR_MISMATCH
    s.close()


@pytest.mark.gpu
def test_c1_full_size_residual_and_operator():
    """256^3, 64 boxes of 64^3, lognormal b: the launch configuration of the
    benchmark.  The oracle's operator recomputes f - A phi on every cell."""
    print("[solve] C1 256^3 full size", flush=True)
    P = lib()
    cfg = W.config_c1()
    n, boxes = cfg["n"], cfg["boxes"]
    s = gpu_solver(cfg)
    f_boxes = W.scatter_cells(cfg["rhs"], boxes)
    rhs = P.MultiFab.from_numpy(boxes, f_boxes, 0)
    phi = s.cell_mf(1, fill=0.0)
    info = s.solve(phi, rhs, 1e-10, history=True)
    print(f"C1: {info['iters']} cycles, {info['solve_ms']:.1f} ms, rel {info['rel_resid']:.2e}")
    assert info["converged"] and info["nlevels"] == 5
    out = s.cell_mf(0)
    s.apply(phi, out)
    torch.cuda.synchronize()
    lev = oracle_level(cfg)
    ophi = phi.to_numpy()
    oA = O.apply_op(lev, ophi)
    gA = out.valid_numpy()
    scale = max(float(np.max(np.abs(x))) for x in oA)
    err = max(float(np.max(np.abs(a - b))) for a, b in zip(gA, oA))
    assert err <= 1e-12 * scale * 10
    r = max(float(np.max(np.abs(fb - a))) for fb, a in zip(f_boxes, oA))
    normf = max(float(np.max(np.abs(x))) for x in f_boxes)
    assert abs(r - info["abs_resid"]) <= 1e-6 * r + 1e-13 * scale
    assert r <= 1e-10 * normf * (1 + 1e-3)
    s.close()
