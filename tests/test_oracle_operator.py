"""Pins of the oracle's operator, smoother and transfers (no GPU).

The operator is pinned to an independent global flux-form formulation with
explicit ghost values (tests/dense_ref.py), to exact symmetry and definiteness,
and to box-decomposition invariance.  The smoother is pinned to a sequential
pure-Python Gauss-Seidel in red-then-black order.
"""

import numpy as np
import pytest

import oracle as O
import workloads as W
from dense_ref import apply_global, assemble

BCS = [(False, False, False), (True, True, True), (True, False, True)]


def _level(n, m, periodic, alpha=1.0, beta=1.0, sigma=1.0, seed=1, with_a=False):
    boxes = W.uniform_boxes(n, m)
    bc = W.lognormal_cells(n, sigma, seed)
    faces = W.harmonic_faces(bc, periodic)
    acell = None
    a = None
    if with_a:
        acell = W.lognormal_cells(n, 0.3, seed + 10)
        a = W.scatter_cells(acell, boxes)
    lev = O.make_level(boxes, W.domain_box(n), periodic, alpha, beta, a,
                       [W.scatter_faces(faces[d], boxes, d) for d in range(3)])
    return lev, faces, acell


@pytest.mark.parametrize("periodic", BCS)
@pytest.mark.parametrize("with_a", [False, True])
def test_apply_matches_flux_form(periodic, with_a):
    n = 16
    lev, faces, acell = _level(n, 8, periodic, alpha=0.7, beta=1.3, with_a=with_a)
    u = np.random.default_rng(3).standard_normal((n, n, n))
    phi = W.scatter_cells(u, lev.boxes, ng=1, fill=np.nan)
    got = W.gather_cells(O.apply_op(lev, phi), lev.boxes, n)
    ref = apply_global(u, faces, 0.7, 1.3, lev.h, periodic, acell)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_apply_is_box_decomposition_invariant():
    n = 16
    for periodic in BCS:
        lev8, faces, _ = _level(n, 8, periodic)
        lev1 = O.make_level([W.domain_box(n)], W.domain_box(n), periodic, 1.0, 1.0, None,
                            [W.scatter_faces(faces[d], [W.domain_box(n)], d) for d in range(3)])
        u = np.random.default_rng(4).standard_normal((n, n, n))
        a8 = W.gather_cells(O.apply_op(lev8, W.scatter_cells(u, lev8.boxes, 1)), lev8.boxes, n)
        a1 = W.gather_cells(O.apply_op(lev1, W.scatter_cells(u, lev1.boxes, 1)), lev1.boxes, n)
        assert np.array_equal(a8, a1)


def _oracle_matrix(lev, n):
    N = n ** 3
    A = np.zeros((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        phi = W.scatter_cells(e.reshape(n, n, n), lev.boxes, ng=1)
        A[:, k] = W.gather_cells(O.apply_op(lev, phi), lev.boxes, n).ravel()
    return A


@pytest.mark.parametrize("periodic", BCS)
def test_operator_symmetric_and_definite(periodic):
    n = 8
    lev, faces, _ = _level(n, 4, periodic, alpha=0.0 if all(periodic) else 1.0)
    A = _oracle_matrix(lev, n)
    assert np.array_equal(A, A.T)
    Aref = assemble(n, faces, lev.alpha, 1.0, periodic)
    assert np.max(np.abs(A - Aref)) <= 1e-12 * np.max(np.abs(Aref))
    w = np.linalg.eigvalsh(A)
    if all(periodic):
        # semidefinite, null space = constants
        assert abs(w[0]) <= 1e-9 * w[-1] and w[1] > 1e-6 * w[-1]
        ones = np.ones(n ** 3)
        assert np.max(np.abs(A @ ones)) <= 1e-10 * w[-1]
    else:
        assert w[0] > 0


def test_inner_product_symmetry_multibox():
    n = 32
    lev, _, _ = _level(n, 16, (False, True, False), with_a=True)
    rng = np.random.default_rng(5)
    u = rng.standard_normal((n, n, n))
    v = rng.standard_normal((n, n, n))
    Au = W.gather_cells(O.apply_op(lev, W.scatter_cells(u, lev.boxes, 1)), lev.boxes, n)
    Av = W.gather_cells(O.apply_op(lev, W.scatter_cells(v, lev.boxes, 1)), lev.boxes, n)
    a, b = np.sum(u * Av), np.sum(Au * v)
    assert abs(a - b) <= 1e-14 * np.sum(np.abs(u * Av)) * 10


def _sequential_gs(u, f, faces, alpha, beta, h, periodic):
    """Red sweep then black sweep, one cell at a time, reading current values."""
    n = u.shape[0]
    u = u.copy()
    for colour in (0, 1):
        for i in range(n):
            for j in range(n):
                for k in range(n):
                    if (i + j + k) % 2 != colour:
                        continue
                    diag = alpha
                    off = 0.0
                    for d in range(3):
                        idx = [i, j, k]
                        for side in (0, 1):
                            fidx = list(idx)
                            fidx[d] = idx[d] + side
                            c = beta * faces[d][tuple(fidx)] / (h[d] * h[d])
                            nb = list(idx)
                            nb[d] = idx[d] + (1 if side else -1)
                            if 0 <= nb[d] < n:
                                diag += c
                                off += c * u[tuple(nb)]
                            elif periodic[d]:
                                nb[d] %= n
                                diag += c
                                off += c * u[tuple(nb)]
                            else:
                                # ghost value -u_i: c (ghost - u) = -2 c u
                                diag += 2 * c
                    u[i, j, k] = (f[i, j, k] + off) / diag
    return u


@pytest.mark.parametrize("periodic", [(False, False, False), (True, False, True)])
def test_gsrb_matches_sequential_gauss_seidel(periodic):
    n = 8
    lev, faces, _ = _level(n, 4, periodic, alpha=0.5)
    rng = np.random.default_rng(6)
    u = rng.standard_normal((n, n, n))
    f = rng.standard_normal((n, n, n))
    phi = W.scatter_cells(u, lev.boxes, ng=1)
    fb = W.scatter_cells(f, lev.boxes)
    O.gsrb_halfsweep(lev, phi, fb, 0)
    O.gsrb_halfsweep(lev, phi, fb, 1)
    got = W.gather_cells(phi, lev.boxes, n, ng=1)
    ref = _sequential_gs(u, f, faces, 0.5, 1.0, lev.h, periodic)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_gsrb_is_box_decomposition_invariant():
    n = 16
    for periodic in BCS:
        lev8, faces, _ = _level(n, 8, periodic)
        lev2 = O.make_level(W.uniform_boxes(n, 16), W.domain_box(n), periodic, 1.0, 1.0, None,
                            [W.scatter_faces(faces[d], W.uniform_boxes(n, 16), d) for d in range(3)])
        rng = np.random.default_rng(7)
        u = rng.standard_normal((n, n, n))
        f = rng.standard_normal((n, n, n))
        outs = []
        for lev in (lev8, lev2):
            phi = W.scatter_cells(u, lev.boxes, 1)
            fb = W.scatter_cells(f, lev.boxes)
            for c in (0, 1, 0, 1):
                O.gsrb_halfsweep(lev, phi, fb, c)
            outs.append(W.gather_cells(phi, lev.boxes, n, ng=1))
        assert np.array_equal(outs[0], outs[1])


def test_transfers():
    n = 16
    lev, _, _ = _level(n, 8, (False, False, False))
    levc = O.coarsen_level(lev)
    rng = np.random.default_rng(8)
    ones = [np.ones(O.box_shape(b)) for b in lev.boxes]
    assert all(np.array_equal(x, np.ones_like(x)) for x in O.restrict(lev, ones))
    # R P = I exactly; P^T = 8 R in the inner product; cell sums scaled by volume
    ec = rng.standard_normal((n // 2,) * 3)
    phi = W.scatter_cells(np.zeros((n, n, n)), lev.boxes, 1)
    O.prolong_add(phi, W.scatter_cells(ec, levc.boxes, 1))
    Pe = W.gather_cells(phi, lev.boxes, n, ng=1)
    RPe = W.gather_cells(O.restrict(lev, W.scatter_cells(Pe, lev.boxes)), levc.boxes, n // 2)
    assert np.array_equal(RPe, ec)
    r = rng.standard_normal((n, n, n))
    Rr = W.gather_cells(O.restrict(lev, W.scatter_cells(r, lev.boxes)), levc.boxes, n // 2)
    assert abs(np.sum(Pe * r) - 8 * np.sum(ec * Rr)) <= 1e-12 * np.sum(np.abs(Pe * r))
    assert abs(np.sum(r) * lev.h[0] ** 3 - np.sum(Rr) * levc.h[0] ** 3) <= 1e-13
    # averaged unit coefficients stay exactly one; h doubles
    lev1 = O.make_level(lev.boxes, lev.domain, lev.periodic, 1.0, 1.0)
    c1 = O.coarsen_level(lev1)
    assert all(np.array_equal(x, np.ones_like(x)) for d in range(3) for x in c1.b[d])
    assert c1.h == (2.0 / n,) * 3


def test_coefficient_coarsening_values():
    n = 8
    lev, faces, _ = _level(n, 4, (False, False, False), with_a=True)
    c = O.coarsen_level(lev)
    A = W.gather_cells(lev.a, lev.boxes, n)
    Ac = W.gather_cells(c.a, c.boxes, n // 2)
    assert np.allclose(Ac[1, 2, 3], A[2:4, 4:6, 6:8].mean(), rtol=1e-15)
    # coarse x-face 2 (between coarse cells 1 and 2) at (j, k) = (1, 3)
    got = [x for bx, x in zip(c.boxes, c.b[0]) if bx[0] == (0, 0, 2)][0][2, 1, 1]
    assert np.isclose(got, faces[0][4, 2:4, 6:8].mean(), rtol=1e-15)


def test_merged_level_transfers_and_coefficients():
    """Coarsening onto a merged single box equals coarsening the same data held
    as one box; R P = I and P^T = 8 R hold across the merge."""
    n = 16
    lev8, faces, _ = _level(n, 8, (False, False, False), with_a=True)
    one = [W.domain_box(n)]
    lev1 = O.make_level(one, W.domain_box(n), (False,) * 3, 1.0, 1.0,
                        [W.gather_cells(lev8.a, lev8.boxes, n)],
                        [W.scatter_faces(faces[d], one, d) for d in range(3)])
    cm = O.coarsen_level(lev8, merged=True)
    c1 = O.coarsen_level(lev1)
    assert cm.boxes == c1.boxes and cm.merged
    assert np.array_equal(cm.a[0], c1.a[0])
    for d in range(3):
        assert np.array_equal(cm.b[d][0], c1.b[d][0])
    rng = np.random.default_rng(9)
    ec = rng.standard_normal((n // 2,) * 3)
    phi = W.scatter_cells(np.zeros((n, n, n)), lev8.boxes, 1)
    O.prolong_add(phi, W.scatter_cells(ec, cm.boxes, 1), lev8, cm)
    Pe = W.gather_cells(phi, lev8.boxes, n, ng=1)
    assert np.array_equal(Pe, np.repeat(np.repeat(np.repeat(ec, 2, 0), 2, 1), 2, 2))
    RPe = O.restrict(lev8, W.scatter_cells(Pe, lev8.boxes), cm)[0]
    assert np.array_equal(RPe, ec)
    r = rng.standard_normal((n, n, n))
    Rr = O.restrict(lev8, W.scatter_cells(r, lev8.boxes), cm)[0]
    assert abs(np.sum(Pe * r) - 8 * np.sum(ec * Rr)) <= 1e-12 * np.sum(np.abs(Pe * r))


def test_aggregated_hierarchy_depths():
    def depth(boxes, n, m=4):
        return [O.box_shape(b[1])[0] for b in O.mg_hierarchy(boxes, W.domain_box(n), m, True)]
    assert depth(W.uniform_boxes(256, 64), 256) == [256, 128, 64, 32, 16, 8, 4]
    assert depth(W.uniform_boxes(32, 16), 32) == [32, 16, 8, 4]
    assert depth(W.uniform_boxes(128, 64), 128) == [128, 64, 32, 16, 8, 4]
    assert depth(W.guillotine_boxes(512), 512) == [512, 256, 128, 64, 32, 16, 8, 4]
    h = O.mg_hierarchy(W.uniform_boxes(256, 64), W.domain_box(256), 4, True)
    assert [m for _, _, m in h] == [False] * 5 + [True, False]
