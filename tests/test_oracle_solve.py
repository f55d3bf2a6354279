"""Pins of the oracle's whole solve (no GPU).

* closed form: sin(2 pi x) sin(2 pi y) sin(2 pi z) is an eigenvector of the
  periodic 7-point Laplacian with eigenvalue 12 sin^2(pi h) / h^2, so the
  discrete solution of the periodic Poisson problem is f / lambda_h;
* second-order convergence to a manufactured smooth solution with a variable
  coefficient and Dirichlet walls;
* dense direct solves of independently assembled matrices on 8^3 grids;
* V-cycle contraction factors and the equivalence of the direct and the
  correction (refinement) forms.
"""

import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from dense_ref import assemble


def _level_from(cfg, boxes=None, min_a=None):
    boxes = boxes or cfg["boxes"]
    b = None
    if cfg["faces"] is not None:
        b = [W.scatter_faces(cfg["faces"][d], boxes, d) for d in range(3)]
    return O.make_level(boxes, W.domain_box(cfg["n"]), cfg["periodic"], cfg["alpha"], cfg["beta"],
                        None, b)


def _periodic_poisson(n, m):
    boxes = W.uniform_boxes(n, m)
    lev = O.make_level(boxes, W.domain_box(n), (True,) * 3, 0.0, 1.0)
    f = W.sin_rhs(n)
    return lev, f


def test_c0_closed_form():
    cfg = W.config_c0()
    lev = _level_from(cfg)
    phi = O.new_cell_data(lev)
    info = O.solve(lev, phi, W.scatter_cells(cfg["rhs"], lev.boxes), 1e-10)
    assert info["converged"] and info["nlevels"] == 3
    h = 1.0 / 32
    lam_h = 12 * math.sin(math.pi * h) ** 2 / h ** 2
    assert abs(lam_h - 118.0552372026) < 1e-9
    G = W.gather_cells(phi, lev.boxes, 32, ng=1)
    ex = cfg["rhs"] / lam_h
    assert np.linalg.norm(G - ex) / np.linalg.norm(ex) <= 1e-9
    assert abs(G.mean()) <= 1e-15
    # contraction per V-cycle
    hist = info["history"]
    rho = [hist[i + 1] / hist[i] for i in range(len(hist) - 1)]
    assert max(rho) <= 0.25


def test_periodic_second_order_in_h():
    errs = []
    for n in (16, 32, 64):
        lev, f = _periodic_poisson(n, n // 2)
        phi = O.new_cell_data(lev)
        info = O.solve(lev, phi, W.scatter_cells(f, lev.boxes), 1e-11)
        assert info["converged"]
        G = W.gather_cells(phi, lev.boxes, n, ng=1)
        ex = f / (12 * math.pi ** 2)
        errs.append(np.linalg.norm(G - ex) / np.linalg.norm(ex))
        h = 1.0 / n
        lam_h = 12 * math.sin(math.pi * h) ** 2 / h ** 2
        assert abs(errs[-1] - (12 * math.pi ** 2 - lam_h) / lam_h) <= 1e-8
    assert abs(errs[0] / errs[1] - 4) < 0.05 and abs(errs[1] / errs[2] - 4) < 0.02


def test_cycle_factor_grid_independent():
    rhos = []
    for n in (32, 64):
        lev, f = _periodic_poisson(n, n // 2)
        phi = O.new_cell_data(lev)
        info = O.solve(lev, phi, W.scatter_cells(f, lev.boxes), 1e-10)
        h = info["history"]
        rhos.append((h[-1] / h[0]) ** (1.0 / (len(h) - 1)))
    assert max(rhos) <= 0.25
    assert abs(rhos[0] - rhos[1]) <= 0.05


def _manufactured(n):
    x = (np.arange(n) + 0.5) / n
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    pi = math.pi
    phi_e = np.sin(pi * X) * np.sin(pi * Y) * np.sin(pi * Z)
    b = 1 + 0.5 * np.sin(2 * pi * X) * np.sin(2 * pi * Y) * np.sin(2 * pi * Z)
    gb = [pi * np.cos(2 * pi * X) * np.sin(2 * pi * Y) * np.sin(2 * pi * Z),
          pi * np.sin(2 * pi * X) * np.cos(2 * pi * Y) * np.sin(2 * pi * Z),
          pi * np.sin(2 * pi * X) * np.sin(2 * pi * Y) * np.cos(2 * pi * Z)]
    gp = [pi * np.cos(pi * X) * np.sin(pi * Y) * np.sin(pi * Z),
          pi * np.sin(pi * X) * np.cos(pi * Y) * np.sin(pi * Z),
          pi * np.sin(pi * X) * np.sin(pi * Y) * np.cos(pi * Z)]
    f = phi_e + 3 * pi ** 2 * b * phi_e - sum(g1 * g2 for g1, g2 in zip(gb, gp))
    faces = []
    xf = np.arange(n + 1) / n
    for d in range(3):
        c = [x, x, x]
        c[d] = xf
        A, B, C = np.meshgrid(*c, indexing="ij")
        faces.append(1 + 0.5 * np.sin(2 * pi * A) * np.sin(2 * pi * B) * np.sin(2 * pi * C))
    return phi_e, f, faces


def test_manufactured_dirichlet_second_order():
    e2, einf = [], []
    for n in (16, 32, 64):
        phi_e, f, faces = _manufactured(n)
        boxes = W.uniform_boxes(n, n // 2)
        lev = O.make_level(boxes, W.domain_box(n), (False,) * 3, 1.0, 1.0, None,
                           [W.scatter_faces(faces[d], boxes, d) for d in range(3)])
        phi = O.new_cell_data(lev)
        info = O.solve(lev, phi, W.scatter_cells(f, boxes), 1e-11)
        assert info["converged"]
        G = W.gather_cells(phi, boxes, n, ng=1)
        e2.append(np.linalg.norm(G - phi_e) / np.linalg.norm(phi_e))
        einf.append(np.max(np.abs(G - phi_e)))
    for e in (e2, einf):
        assert 3.5 < e[0] / e[1] < 4.5 and 3.5 < e[1] / e[2] < 4.5


@pytest.mark.parametrize("m", [8, 4])
@pytest.mark.parametrize("periodic", [(False, False, False), (True, False, False)])
def test_dense_direct_8cubed(m, periodic):
    n = 8
    bc = W.lognormal_cells(n, 1.0, 11)
    faces = W.harmonic_faces(bc, periodic)
    f = W.uniform_rhs(n, 12)
    boxes = W.uniform_boxes(n, m)
    lev = O.make_level(boxes, W.domain_box(n), periodic, 1.0, 1.0, None,
                       [W.scatter_faces(faces[d], boxes, d) for d in range(3)])
    opts = O.Opts(min_bottom_edge=2, bottom_tol=1e-12)
    phi = O.new_cell_data(lev)
    info = O.solve(lev, phi, W.scatter_cells(f, boxes), 1e-12, opts=opts)
    assert info["converged"] and info["nlevels"] >= 2
    A = assemble(n, faces, 1.0, 1.0, periodic)
    x = np.linalg.solve(A, f.ravel()).reshape(n, n, n)
    G = W.gather_cells(phi, boxes, n, ng=1)
    assert np.linalg.norm(G - x) / np.linalg.norm(x) <= 1e-10


def test_dense_direct_singular_periodic():
    n = 8
    bc = W.lognormal_cells(n, 0.5, 13)
    per = (True, True, True)
    faces = W.harmonic_faces(bc, per)
    f = W.uniform_rhs(n, 14)
    f -= f.mean()
    boxes = W.uniform_boxes(n, 4)
    lev = O.make_level(boxes, W.domain_box(n), per, 0.0, 1.0, None,
                       [W.scatter_faces(faces[d], boxes, d) for d in range(3)])
    phi = O.new_cell_data(lev)
    info = O.solve(lev, phi, W.scatter_cells(f, boxes), 1e-12,
                   opts=O.Opts(min_bottom_edge=2, bottom_tol=1e-12))
    assert info["converged"]
    N = n ** 3
    A = assemble(n, faces, 0.0, 1.0, per) + np.ones((N, N)) / N
    x = np.linalg.solve(A, f.ravel()).reshape(n, n, n)
    G = W.gather_cells(phi, boxes, n, ng=1)
    assert np.linalg.norm(G - x) / np.linalg.norm(x) <= 1e-10


def test_cg_bottom_equals_direct():
    n = 8
    per = (False, True, False)
    bc = W.lognormal_cells(n, 1.0, 15)
    faces = W.harmonic_faces(bc, per)
    boxes = W.uniform_boxes(n, 4)
    lev = O.make_level(boxes, W.domain_box(n), per, 1.0, 1.0, None,
                       [W.scatter_faces(faces[d], boxes, d) for d in range(3)])
    f = W.uniform_rhs(n, 16)
    x, its = O.cg_bottom(lev, W.scatter_cells(f, boxes), tol=1e-13)
    assert its <= n ** 3
    ref = np.linalg.solve(assemble(n, faces, 1.0, 1.0, per), f.ravel()).reshape(n, n, n)
    G = W.gather_cells(x, boxes, n, ng=1)
    assert np.linalg.norm(G - ref) / np.linalg.norm(ref) <= 1e-12


def _small_lognormal(n=32, m=16, sigma=1.0):
    cfg = W.config_lognormal(n, m, sigma)
    return cfg, _level_from(cfg)


def test_refinement_form_equals_direct_form():
    cfg, lev = _small_lognormal()
    f = W.scatter_cells(cfg["rhs"], lev.boxes)
    opts = O.Opts(bottom_tol=1e-12)
    p1 = O.new_cell_data(lev)
    i1 = O.solve(lev, p1, f, 1e-10, opts=opts)
    p2 = O.new_cell_data(lev)
    i2 = O.solve_refine(lev, p2, f, 1e-10, opts=opts, inner_dtype=np.float64)
    assert i1["iters"] == i2["iters"]
    nf = i1["normf"]
    for a, b in zip(i1["history"], i2["history"]):
        assert abs(a - b) <= 1e-6 * a + 1e-13 * nf
    for a, b in zip(i1["history"][:4], i2["history"][:4]):
        assert abs(a - b) <= 1e-10 * a
    G1 = W.gather_cells(p1, lev.boxes, 32, ng=1)
    G2 = W.gather_cells(p2, lev.boxes, 32, ng=1)
    assert np.linalg.norm(G1 - G2) / np.linalg.norm(G1) <= 1e-10


def test_float32_refinement_reaches_fp64_accuracy():
    cfg, lev = _small_lognormal()
    f = W.scatter_cells(cfg["rhs"], lev.boxes)
    p1 = O.new_cell_data(lev)
    O.solve(lev, p1, f, 1e-12, opts=O.Opts(bottom_tol=1e-12))
    p2 = O.new_cell_data(lev)
    info = O.solve_refine(lev, p2, f, 1e-10, inner_dtype=np.float32)
    assert info["converged"]
    G1 = W.gather_cells(p1, lev.boxes, 32, ng=1)
    G2 = W.gather_cells(p2, lev.boxes, 32, ng=1)
    assert np.linalg.norm(G1 - G2) / np.linalg.norm(G1) <= 1e-8


def test_not_converged_and_zero_rhs():
    cfg, lev = _small_lognormal(16, 8)
    f = W.scatter_cells(cfg["rhs"], lev.boxes)
    phi = O.new_cell_data(lev)
    info = O.solve(lev, phi, f, 1e-10, opts=O.Opts(max_iter=1))
    assert not info["converged"] and info["iters"] == 1 and len(info["history"]) == 2
    z = [np.zeros_like(x) for x in f]
    phi = O.new_cell_data(lev)
    for v in phi:
        v[...] = 3.0
    info = O.solve(lev, phi, z, 1e-10)
    assert info["converged"] and all(not np.any(v) for v in phi)
    bad = [x.copy() for x in f]
    bad[0][1, 1, 1] = np.nan
    info = O.solve(lev, O.new_cell_data(lev), bad, 1e-10)
    assert not info["converged"]


def test_aggregated_solve_matches_dense_and_plain():
    n = 8
    bc = W.lognormal_cells(n, 1.0, 17)
    faces = W.harmonic_faces(bc)
    f = W.uniform_rhs(n, 18)
    boxes = W.uniform_boxes(n, 4)
    lev = O.make_level(boxes, W.domain_box(n), (False,) * 3, 1.0, 1.0, None,
                       [W.scatter_faces(faces[d], boxes, d) for d in range(3)])
    opts = O.Opts(min_bottom_edge=2, bottom_tol=1e-12, aggregate=True)
    phi = O.new_cell_data(lev)
    info = O.solve(lev, phi, W.scatter_cells(f, boxes), 1e-12, opts=opts)
    assert info["converged"] and info["nlevels"] == 3
    x = np.linalg.solve(assemble(n, faces, 1.0, 1.0, (False,) * 3), f.ravel()).reshape(n, n, n)
    assert np.linalg.norm(W.gather_cells(phi, boxes, n, ng=1) - x) / np.linalg.norm(x) <= 1e-10


def test_aggregation_speeds_convergence_not_answer():
    cfg, lev = _small_lognormal(64, 32)
    f = W.scatter_cells(cfg["rhs"], lev.boxes)
    p1 = O.new_cell_data(lev)
    i1 = O.solve(lev, p1, f, 1e-10)
    p2 = O.new_cell_data(lev)
    i2 = O.solve(lev, p2, f, 1e-10, opts=O.Opts(aggregate=True))
    assert i2["nlevels"] > i1["nlevels"] and i1["converged"] and i2["converged"]
    G1 = W.gather_cells(p1, lev.boxes, 64, ng=1)
    G2 = W.gather_cells(p2, lev.boxes, 64, ng=1)
    assert np.linalg.norm(G1 - G2) / np.linalg.norm(G1) <= 1e-9
    assert i2["iters"] <= i1["iters"] + 1
