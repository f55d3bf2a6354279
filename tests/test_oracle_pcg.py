"""Pins of the oracle's multigrid-preconditioned conjugate gradients (no GPU).

* the symmetric V-cycle (post-smoothing black then red) is a symmetric,
  positive operator, while the plain V-cycle is not (so a missed reversal
  fails the pin);
* with the identity as preconditioner the iterates are those of SciPy's CG on
  the independently assembled matrix;
* the solve reaches the dense direct solution (Dirichlet and mixed periodic)
  and the closed form f / lambda_h of the periodic Poisson problem;
* on the rough lognormal problem it needs fewer iterations than V-cycles.
"""

import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
import workloads as W
from dense_ref import assemble


def _level(n, m, periodic=(False, False, False), sigma=1.0, seed=41):
    bc = W.lognormal_cells(n, sigma, seed)
    faces = W.harmonic_faces(bc, periodic)
    boxes = W.uniform_boxes(n, m)
    lev = O.make_level(boxes, W.domain_box(n), periodic, 1.0, 1.0, None,
                       [W.scatter_faces(faces[d], boxes, d) for d in range(3)])
    return lev, faces


EXACT_BOTTOM = dict(min_bottom_edge=2, bottom_tol=1e-15)


@pytest.mark.parametrize("symmetric", [True, False])
def test_symmetric_vcycle_is_symmetric_positive(symmetric):
    n = 16
    lev, _ = _level(n, 8)
    opts = O.Opts(symmetric=symmetric, **EXACT_BOTTOM)
    levels = O.build_levels(lev, opts.min_bottom_edge)
    rng = np.random.default_rng(3)
    u = [rng.standard_normal(O.box_shape(b)) for b in lev.boxes]
    v = [rng.standard_normal(O.box_shape(b)) for b in lev.boxes]
    Mu = O.vcycle_precond(levels, u, opts)
    Mv = O.vcycle_precond(levels, v, opts)
    vMu = sum(float(np.sum(a * O.valid(b))) for a, b in zip(v, Mu))
    uMv = sum(float(np.sum(a * O.valid(b))) for a, b in zip(u, Mv))
    uMu = sum(float(np.sum(a * O.valid(b))) for a, b in zip(u, Mu))
    asym = abs(vMu - uMv) / abs(vMu)
    if symmetric:
        assert asym <= 1e-10 and uMu > 0
    else:
        assert asym > 1e-6


def test_identity_preconditioner_is_scipy_cg():
    n = 8
    lev, faces = _level(n, 4)
    A = assemble(n, faces, 1.0, 1.0, lev.periodic)
    f = W.uniform_rhs(n, 16)
    fb = W.scatter_cells(f, lev.boxes)

    def ident(r):
        z = O.new_cell_data(lev)
        for zb, rb in zip(z, r):
            O.valid(zb)[...] = rb
        return z

    for k in (1, 3, 6):
        phi = O.new_cell_data(lev)
        O.pcg_solve(lev, phi, fb, rel_tol=0.0, opts=O.Opts(max_iter=k), precond=ident)
        ref, _ = spla.cg(A, f.ravel(), x0=np.zeros(n ** 3), rtol=0.0, atol=0.0, maxiter=k)
        got = W.gather_cells(phi, lev.boxes, n, ng=1).ravel()
        assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("periodic,inner", [((False, False, False), np.float64),
                                            ((True, False, True), np.float64),
                                            ((False, False, False), np.float32)])
def test_pcg_matches_dense_direct(periodic, inner):
    """Also with a float32 V-cycle as the preconditioner: the float64 CG loop
    still reaches the float64 solution."""
    n = 16
    lev, faces = _level(n, 8, periodic)
    A = assemble(n, faces, 1.0, 1.0, periodic)
    f = W.uniform_rhs(n, 16)
    phi = O.new_cell_data(lev)
    info = O.pcg_solve(lev, phi, W.scatter_cells(f, lev.boxes), 1e-13,
                       opts=O.Opts(min_bottom_edge=2, bottom_tol=1e-12), inner_dtype=inner)
    assert info["converged"]
    ref = np.linalg.solve(A, f.ravel()).reshape(n, n, n)
    got = W.gather_cells(phi, lev.boxes, n, ng=1)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-10


def test_pcg_periodic_poisson_closed_form():
    cfg = W.config_c0()
    boxes = cfg["boxes"]
    lev = O.make_level(boxes, W.domain_box(32), (True,) * 3, 0.0, 1.0)
    phi = O.new_cell_data(lev)
    info = O.pcg_solve(lev, phi, W.scatter_cells(cfg["rhs"], boxes), 1e-12)
    assert info["converged"]
    h = 1.0 / 32
    lam_h = 12 * math.sin(math.pi * h) ** 2 / h ** 2
    G = W.gather_cells(phi, boxes, 32, ng=1)
    ex = cfg["rhs"] / lam_h
    assert np.linalg.norm(G - ex) / np.linalg.norm(ex) <= 1e-10
    assert abs(G.mean()) <= 1e-15


def test_pcg_needs_fewer_iterations_than_vcycles():
    cfg = W.config_lognormal(32, 16)
    boxes = cfg["boxes"]
    lev = O.make_level(boxes, W.domain_box(32), cfg["periodic"], 1.0, 1.0, None,
                       [W.scatter_faces(cfg["faces"][d], boxes, d) for d in range(3)])
    f = W.scatter_cells(cfg["rhs"], boxes)
    a, b = O.new_cell_data(lev), O.new_cell_data(lev)
    mg = O.solve(lev, a, f, 1e-10)
    pcg = O.pcg_solve(lev, b, f, 1e-10)
    assert mg["converged"] and pcg["converged"]
    assert pcg["iters"] <= mg["iters"] - 2
    A_ = W.gather_cells(a, boxes, 32, ng=1)
    B_ = W.gather_cells(b, boxes, 32, ng=1)
    assert np.linalg.norm(A_ - B_) / np.linalg.norm(A_) <= 1e-9
