"""Pins of the oracle's adjoint gradient (no GPU).

The reference is torch autograd through a dense solve of the operator assembled
in flux form from exp(log b) face tensors (tests/dense_ref.py), so the adjoint
algebra, the Dirichlet-wall factor and the periodic wrap face are all checked
against differentiation that knows nothing of them.
"""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from dense_ref import apply_global


def _dense_grad(n, logb, f, phi_t, periodic, beta=1.0, alpha=1.0):
    lb = [torch.tensor(x, dtype=torch.float64, requires_grad=True) for x in logb]
    faces = [torch.exp(x) for x in lb]
    N = n ** 3
    E = torch.eye(N, dtype=torch.float64).reshape(N, n, n, n)
    cols = apply_global(E, faces, alpha, beta, (1.0 / n,) * 3, periodic, xp=torch)
    A = cols.reshape(N, N).T
    ft = torch.tensor(f.ravel(), dtype=torch.float64, requires_grad=True)
    phi = torch.linalg.solve(A, ft)
    L = 0.5 * torch.sum((phi - torch.tensor(phi_t.ravel())) ** 2)
    L.backward()
    return ([x.grad.numpy() for x in lb], ft.grad.numpy().reshape(n, n, n),
            phi.detach().numpy().reshape(n, n, n))


def _oracle_grad(n, m, logb, f, phi_t, periodic):
    boxes = W.uniform_boxes(n, m)
    faces = [np.exp(x) for x in logb]
    lev = O.make_level(boxes, W.domain_box(n), periodic, 1.0, 1.0, None,
                       [W.scatter_faces(faces[d], boxes, d) for d in range(3)])
    opts = O.Opts(min_bottom_edge=2, bottom_tol=1e-13)
    phi = O.new_cell_data(lev)
    O.solve(lev, phi, W.scatter_cells(f, boxes), 1e-13, opts=opts)
    P = W.gather_cells(phi, boxes, n, ng=1)
    lam = O.new_cell_data(lev)
    O.solve(lev, lam, W.scatter_cells(P - phi_t, boxes), 1e-13, opts=opts)
    return O.grad_logb(lev, phi, lam), W.gather_cells(lam, boxes, n, ng=1), P


@pytest.mark.parametrize("periodic", [(False, False, False), (True, False, False)])
def test_adjoint_matches_dense_autograd(periodic):
    n = 8
    rng = np.random.default_rng(21)
    bc = W.lognormal_cells(n, 0.5, 22)
    logb = [np.log(x) for x in W.harmonic_faces(bc, periodic)]
    f = W.uniform_rhs(n, 23)
    phi_t = rng.standard_normal((n, n, n)) * 1e-2
    g_ref, gf_ref, P_ref = _dense_grad(n, logb, f, phi_t, periodic)
    g, gf, P = _oracle_grad(n, 4, logb, f, phi_t, periodic)
    assert np.linalg.norm(P - P_ref) <= 1e-10 * np.linalg.norm(P_ref)
    assert np.linalg.norm(gf - gf_ref) <= 1e-9 * np.linalg.norm(gf_ref)
    for d in range(3):
        ref = g_ref[d].copy()
        got = g[d].copy()
        if periodic[d]:
            # faces 0 and n are one parameter; torch sees it as face 0 and n separately
            # only through the wrapped ghost (face n), so compare their sum
            n_ = ref.shape[d]
            s0 = [slice(None)] * 3
            s1 = [slice(None)] * 3
            s0[d] = 0
            s1[d] = n_ - 1
            ref_w = ref[tuple(s0)] + ref[tuple(s1)]
            assert np.allclose(got[tuple(s0)], ref_w, rtol=1e-8, atol=1e-12 * np.abs(ref).max())
            assert np.array_equal(got[tuple(s0)], got[tuple(s1)])
            ref[tuple(s0)] = 0
            ref[tuple(s1)] = 0
            got[tuple(s0)] = 0
            got[tuple(s1)] = 0
        assert np.linalg.norm(got - ref) <= 1e-8 * np.linalg.norm(ref)


def test_adjoint_dirichlet_faces_nonzero():
    n = 8
    bc = W.lognormal_cells(n, 0.5, 24)
    logb = [np.log(x) for x in W.harmonic_faces(bc)]
    f = W.uniform_rhs(n, 25)
    g, _, _ = _oracle_grad(n, 8, logb, f, np.zeros((n, n, n)), (False,) * 3)
    # with phi_t = 0 the loss grows with |phi|; every face gradient has the sign of -phi.lam
    assert np.all(np.abs(g[0][0]) > 0) and np.all(np.abs(g[0][-1]) > 0)


def test_finite_difference_small():
    """Central differences of L in log b on a few faces, from solution differences."""
    n = 16
    per = (False, False, False)
    bc = W.lognormal_cells(n, 0.5, 26)
    logb = [np.log(x) for x in W.harmonic_faces(bc, per)]
    f = W.uniform_rhs(n, 27)
    phi_t = 0.01 * W.uniform_rhs(n, 28)
    g, _, P0 = _oracle_grad(n, 8, logb, f, phi_t, per)
    boxes = W.uniform_boxes(n, 8)
    rng = np.random.default_rng(W.SEED_FD)
    eps = 1e-6
    gmax = max(np.abs(x).max() for x in g)
    for _ in range(6):
        d = int(rng.integers(3))
        idx = tuple(int(rng.integers(s)) for s in logb[d].shape)
        sols = []
        for sgn in (1, -1):
            lb = [x.copy() for x in logb]
            lb[d][idx] += sgn * eps
            lev = O.make_level(boxes, W.domain_box(n), per, 1.0, 1.0, None,
                               [W.scatter_faces(np.exp(lb[a]), boxes, a) for a in range(3)])
            phi = W.scatter_cells(P0, boxes, ng=1)
            O.solve(lev, phi, W.scatter_cells(f, boxes), 0.0, 1e-14 * np.abs(f).max(),
                    opts=O.Opts(bottom_tol=1e-12))
            sols.append(W.gather_cells(phi, boxes, n, ng=1))
        dL = 0.5 * np.sum((sols[0] - sols[1]) * (sols[0] + sols[1] - 2 * phi_t))
        fd = dL / (2 * eps)
        # solve roundoff puts an absolute floor under dL, hence the gmax term
        assert abs(fd - g[d][idx]) <= 1e-4 * abs(g[d][idx]) + 1e-6 * gmax
