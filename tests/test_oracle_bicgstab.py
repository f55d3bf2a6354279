"""Pins of the oracle's BiCGStab bottom solver (no GPU).

* its k-th iterate equals SciPy's ``bicgstab`` (an independent
  implementation of the same stabilised bi-conjugate gradient recurrences)
  after k steps on the independently assembled matrix;
* run to a tight tolerance it reaches the dense direct solution;
* on a singular all-periodic problem it returns the mean-free solution of the
  projected system;
* a multigrid solve with it as the bottom solver reaches the closed-form
  periodic Poisson solution f / lambda_h and the CG-bottom solution.
"""

import math

import numpy as np
import pytest
from scipy.sparse.linalg import bicgstab

import oracle as O
import workloads as W
from dense_ref import assemble


def _level(n, per, alpha, sigma, seed, m=4):
    bc = W.lognormal_cells(n, sigma, seed)
    faces = W.harmonic_faces(bc, per)
    boxes = W.uniform_boxes(n, m)
    lev = O.make_level(boxes, W.domain_box(n), per, alpha, 1.0, None,
                       [W.scatter_faces(faces[d], boxes, d) for d in range(3)])
    return lev, boxes, faces


@pytest.mark.parametrize("k", [1, 2, 5])
def test_iterates_equal_scipy_bicgstab(k):
    n, per = 8, (False, True, False)
    lev, boxes, faces = _level(n, per, 1.0, 1.0, 21)
    f = W.uniform_rhs(n, 22)
    x, its = O.bicgstab_bottom(lev, W.scatter_cells(f, boxes), tol=0.0, max_iter=k)
    assert its == k
    A = assemble(n, faces, 1.0, 1.0, per)
    ref, info = bicgstab(A, f.ravel(), x0=np.zeros(n ** 3), rtol=0.0, atol=0.0, maxiter=k)
    assert info == k
    G = W.gather_cells(x, boxes, n, ng=1).ravel()
    assert np.linalg.norm(G - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("per", [(False, False, False), (True, False, True)])
def test_tight_tolerance_equals_direct(per):
    n = 8
    lev, boxes, faces = _level(n, per, 1.0, 1.0, 23)
    f = W.uniform_rhs(n, 24)
    x, its = O.bicgstab_bottom(lev, W.scatter_cells(f, boxes), tol=1e-13)
    assert 0 < its < n ** 3
    ref = np.linalg.solve(assemble(n, faces, 1.0, 1.0, per), f.ravel()).reshape(n, n, n)
    G = W.gather_cells(x, boxes, n, ng=1)
    assert np.linalg.norm(G - ref) <= 1e-11 * np.linalg.norm(ref)


def test_singular_periodic_projected():
    n, per = 8, (True, True, True)
    lev, boxes, faces = _level(n, per, 0.0, 0.5, 25)
    f = W.uniform_rhs(n, 26)
    x, its = O.bicgstab_bottom(lev, W.scatter_cells(f, boxes), tol=1e-13)
    G = W.gather_cells(x, boxes, n, ng=1)
    assert abs(G.mean()) <= 1e-13 * np.abs(G).max()
    N = n ** 3
    A = assemble(n, faces, 0.0, 1.0, per)
    resid = A @ G.ravel() - (f.ravel() - f.mean())
    assert np.linalg.norm(resid) <= 1e-10 * np.linalg.norm(f)


def test_zero_rhs_takes_no_iteration():
    lev, boxes, _ = _level(8, (False,) * 3, 1.0, 1.0, 27)
    x, its = O.bicgstab_bottom(lev, [np.zeros((4, 4, 4)) for _ in boxes], tol=1e-4)
    assert its == 0
    assert all(not np.any(v) for v in x)


def test_multigrid_with_bicgstab_bottom_closed_form():
    cfg = W.config_c0()
    n = cfg["n"]
    lev = O.make_level(cfg["boxes"], W.domain_box(n), cfg["periodic"], cfg["alpha"], cfg["beta"])
    phi = O.new_cell_data(lev)
    f = cfg["rhs"]
    info = O.solve(lev, phi, W.scatter_cells(f, cfg["boxes"]), 1e-11,
                   opts=O.Opts(bottom_solver="bicgstab", bottom_tol=1e-10))
    assert info["converged"]
    lam = 12.0 * math.sin(math.pi / n) ** 2 * n * n
    G = W.gather_cells(phi, cfg["boxes"], n, ng=1)
    assert np.abs(G - f / lam).max() <= 1e-9 * np.abs(f / lam).max()


def test_multigrid_bottom_solvers_reach_one_solution():
    cfg = W.config_lognormal(32, 16)
    lev = O.make_level(cfg["boxes"], W.domain_box(32), cfg["periodic"], 1.0, 1.0, None,
                       [W.scatter_faces(cfg["faces"][d], cfg["boxes"], d) for d in range(3)])
    f = W.scatter_cells(cfg["rhs"], cfg["boxes"])
    out = []
    for name in ("cg", "bicgstab"):
        phi = O.new_cell_data(lev)
        info = O.solve(lev, phi, f, 1e-11, opts=O.Opts(bottom_solver=name, bottom_tol=1e-6))
        assert info["converged"]
        out.append(W.gather_cells(phi, cfg["boxes"], 32, ng=1))
    assert np.linalg.norm(out[0] - out[1]) <= 1e-9 * np.linalg.norm(out[0])
