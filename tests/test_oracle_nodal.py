"""Pins of the nodal oracle (oracle/nodal.py) against things other than itself:
an independent finite-element assembly (Gauss quadrature of the trilinear
shape functions, tests/nodal_ref.py), the interpolation matrix built from the
coarse hat functions at the fine nodes' coordinates, the closed-form symbol of
the constant-coefficient stencil, dense direct solves, a manufactured solution
and sequential loops."""

import itertools
import math

import numpy as np
import pytest
import scipy.sparse.linalg as sla

import oracle.nodal as N
from nodal_ref import assemble, element_stiffness, from_vec, interp_matrix, to_vec

CASES = [
    ((8, 8, 8), (False, False, False)),
    ((8, 6, 4), (True, False, True)),
    ((6, 6, 6), (True, True, True)),
    ((4, 8, 6), (False, True, False)),
]


def _sigma(n, seed=0):
    return np.exp(np.random.default_rng(seed).standard_normal(n))


def test_element_matrix_equals_quadrature():
    """Moment-integral element stiffness = Gauss quadrature of the shape
    functions' gradients, also for a non-cubic cell; rows sum to zero."""
    for h in [(0.25, 0.25, 0.25), (0.1, 0.2, 0.05)]:
        K = N.element_matrix(h)
        corners, Kq = element_stiffness(h)
        perm = [corners.index(c) for c in N.CORNERS]
        assert np.allclose(K, Kq[np.ix_(perm, perm)], rtol=1e-14, atol=1e-15)
        assert np.abs(K.sum(axis=1)).max() < 1e-14 * np.abs(K).max()
    # cubic cell: diagonal 1/3 h, edge neighbours 0, face and body diagonals -h/12
    K = N.element_matrix((1.0, 1.0, 1.0))
    for ia, a in enumerate(N.CORNERS):
        for ib, b in enumerate(N.CORNERS):
            k = sum(a[d] != b[d] for d in range(3))
            assert abs(K[ia, ib] - {0: 1 / 3, 1: 0.0, 2: -1 / 12, 3: -1 / 12}[k]) < 1e-15


@pytest.mark.parametrize("n,per", CASES)
def test_operator_equals_independent_assembly(n, per):
    sig = _sigma(n)
    lev = N.make_nodal_level(sig, per)
    A, m = assemble(sig, per)
    assert m == list(lev.m)
    x = np.random.default_rng(1).standard_normal(lev.m)
    got = N.apply_nodal(lev, x)
    ref = from_vec(A @ to_vec(x), lev.m)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_constant_coefficient_symbol():
    """Constant sigma, periodic: a product of cosines is an eigenvector with
    lambda = sum_d (2 - 2 cos t_d) / h_d^2 prod_{e != d} (2 + cos t_e) / 3."""
    n = (8, 12, 16)
    lev = N.make_nodal_level(np.full(n, 2.5), (True, True, True))
    k = (1, 2, 3)
    t = [2 * math.pi * k[d] / n[d] for d in range(3)]
    h = [1.0 / n[d] for d in range(3)]
    I, J, K = np.meshgrid(*[np.arange(n[d]) for d in range(3)], indexing="ij")
    u = np.cos(t[0] * I) * np.cos(t[1] * J) * np.cos(t[2] * K)
    lam = 0.0
    for d in range(3):
        term = (2 - 2 * math.cos(t[d])) / h[d] ** 2
        for e in range(3):
            if e != d:
                term *= (2 + math.cos(t[e])) / 3
        lam += term
    lam *= 2.5
    assert np.abs(N.apply_nodal(lev, u) - lam * u).max() <= 1e-12 * lam


def test_symmetry_definiteness_and_null_space():
    sig = _sigma((8, 8, 8), 2)
    Ad, _ = assemble(sig, (False,) * 3)
    for per in [(False,) * 3, (True, True, True)]:
        lev = N.make_nodal_level(sig, per)
        m = lev.m
        M = np.zeros((int(np.prod(m)),) * 2)
        for c in range(M.shape[0]):
            e = np.zeros(M.shape[0])
            e[c] = 1
            M[:, c] = to_vec(N.apply_nodal(lev, from_vec(e, m)))
        assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
        ev = np.linalg.eigvalsh(0.5 * (M + M.T))
        if all(per):
            assert abs(ev[0]) < 1e-9 * ev[-1] and ev[1] > 1e-6 * ev[-1]
            assert np.abs(N.apply_nodal(lev, np.ones(m))).max() < 1e-9
        else:
            assert ev[0] > 0
    del Ad


@pytest.mark.parametrize("n,per", [((8, 8, 8), (False,) * 3), ((8, 8, 4), (True, False, True)),
                                   ((8, 4, 8), (True, True, True))])
def test_galerkin_equals_dense_triple_product(n, per):
    """The coarse operator equals P^T A P / 8 with A from the independent
    assembly and P from the coarse hat functions at the fine nodes; it is
    exactly symmetric."""
    sig = _sigma(n, 3)
    lev = N.make_nodal_level(sig, per)
    lc = N.galerkin(lev)
    A, _ = assemble(sig, per)
    P = interp_matrix(lc.n, per)
    Ac = (P.T @ A @ P) / 8.0
    x = np.random.default_rng(4).standard_normal(lc.m)
    got = N.apply_nodal(lc, x)
    ref = from_vec(Ac @ to_vec(x), lc.m)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    m = lc.m
    M = np.zeros((int(np.prod(m)),) * 2)
    for c in range(M.shape[0]):
        e = np.zeros(M.shape[0])
        e[c] = 1
        M[:, c] = to_vec(N.apply_nodal(lc, from_vec(e, m)))
    assert np.array_equal(M, M.T)


def test_galerkin_of_block_constant_sigma_is_the_coarse_discretisation():
    """Nested trilinear spaces: with sigma constant on every 2x2x2 block the
    Galerkin coarse operator is the finite-element operator of the coarse grid
    with the block values."""
    for per in [(False,) * 3, (True, False, True)]:
        sc = _sigma((4, 4, 4), 5)
        sf = np.repeat(np.repeat(np.repeat(sc, 2, 0), 2, 1), 2, 2)
        lc = N.galerkin(N.make_nodal_level(sf, per))
        direct = N.make_nodal_level(sc, per)
        scale = np.abs(direct.w[(0, 0, 0)]).max()
        ones = np.ones(lc.m)
        for o in N.OFFSETS:
            # couplings to wall nodes multiply 0 and are not compared
            inner = N.shift(ones, o, per) > 0
            assert np.abs(lc.w[o] - direct.w[o])[inner].max() <= 1e-13 * scale
        x = np.random.default_rng(14).standard_normal(lc.m)
        assert np.abs(N.apply_nodal(lc, x) - N.apply_nodal(direct, x)).max() <= 1e-12 * scale


@pytest.mark.parametrize("per", [(False,) * 3, (True, False, True), (True, True, True)])
def test_transfers(per):
    """Interpolation = the hat-function matrix; restriction = its transpose / 8;
    constants restrict and interpolate to constants where no wall is near."""
    n = (8, 8, 8)
    lev = N.make_nodal_level(_sigma(n), per)
    lc = N.NodalLevel(N.coarsen_n(n), per, tuple(2 * x for x in lev.h))
    P = interp_matrix(lc.n, per)
    rng = np.random.default_rng(6)
    e = rng.standard_normal(lc.m)
    got = N.interp_add(lev, lc, np.zeros(lev.m), e)
    assert np.abs(got - from_vec(P @ to_vec(e), lev.m)).max() <= 1e-15
    r = rng.standard_normal(lev.m)
    got = N.restrict_nodal(lev, lc, r)
    assert np.abs(got - from_vec(P.T @ to_vec(r), lc.m) / 8).max() <= 1e-15
    if all(per):
        assert np.array_equal(N.restrict_nodal(lev, lc, np.ones(lev.m)), np.ones(lc.m))
        assert np.array_equal(N.interp_add(lev, lc, np.zeros(lev.m), np.ones(lc.m)),
                              np.ones(lev.m))


def test_jacobi_equals_loop():
    """One sweep = a plain loop over the nodes reading only old values."""
    n, per = (4, 6, 4), (True, False, False)
    lev = N.make_nodal_level(_sigma(n, 7), per)
    rng = np.random.default_rng(8)
    phi = rng.standard_normal(lev.m)
    f = rng.standard_normal(lev.m)
    got = N.jacobi(lev, phi, f, 0.7)
    m = lev.m
    ref = np.empty(m)
    for i, j, k in itertools.product(*[range(x) for x in m]):
        s = 0.0
        for o in N.OFFSETS:
            q = [i + o[0], j + o[1], k + o[2]]
            val = 0.0
            ok = True
            for d in range(3):
                if per[d]:
                    q[d] %= m[d]
                elif q[d] < 0 or q[d] >= m[d]:
                    ok = False
            if ok:
                val = phi[q[0], q[1], q[2]]
            s += lev.w[o][i, j, k] * val
        ref[i, j, k] = phi[i, j, k] + 0.7 * (f[i, j, k] - s) / lev.w[(0, 0, 0)][i, j, k]
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_bottom_cg_equals_direct():
    n, per = (8, 8, 8), (False, True, False)
    sig = _sigma(n, 9)
    lev = N.make_nodal_level(sig, per)
    A, m = assemble(sig, per)
    b = np.random.default_rng(10).standard_normal(lev.m)
    x, it = N.nodal_cg_bottom(lev, b, tol=1e-13)
    ref = from_vec(sla.spsolve(A.tocsc(), to_vec(b)), m)
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)
    assert 0 < it <= b.size


@pytest.mark.parametrize("n,per", [((16, 16, 16), (False,) * 3), ((16, 16, 16), (True, False, True)),
                                   ((8, 8, 8), (False, True, False))])
def test_solve_equals_direct(n, per):
    sig = _sigma(n, 11)
    A, m = assemble(sig, per)
    f = np.random.default_rng(12).uniform(-1, 1, m)
    phi, info = N.nodal_solve(sig, per, f, 1e-12,
                              opts=N.NodalOpts(bottom_tol=1e-13, min_bottom_cells=4))
    ref = from_vec(sla.spsolve(A.tocsc(), to_vec(f)), m)
    assert info["converged"] and info["nlevels"] >= 2
    assert np.linalg.norm(phi - ref) <= 1e-10 * np.linalg.norm(ref)


def test_periodic_closed_form_solution():
    """Constant sigma, all periodic: f = a zero-mean cosine mode, phi = f / lambda."""
    n = (16, 16, 16)
    per = (True, True, True)
    I, J, K = np.meshgrid(*[np.arange(16)] * 3, indexing="ij")
    t = 2 * math.pi / 16
    f = np.cos(t * I) * np.cos(2 * t * J) * np.cos(t * K)
    h2 = (1 / 16) ** 2
    lam = ((2 - 2 * math.cos(t)) * (2 + math.cos(2 * t)) * (2 + math.cos(t)) / 9
           + (2 - 2 * math.cos(2 * t)) * (2 + math.cos(t)) ** 2 / 9
           + (2 - 2 * math.cos(t)) * (2 + math.cos(t)) * (2 + math.cos(2 * t)) / 9) / h2
    phi, info = N.nodal_solve(np.ones(n), per, f, 1e-12,
                              opts=N.NodalOpts(bottom_tol=1e-13, min_bottom_cells=4))
    assert info["converged"]
    assert np.linalg.norm(phi - f / lam) <= 1e-10 * np.linalg.norm(f / lam)


def _manufactured(nn):
    h = 1.0 / nn
    xc = (np.arange(nn) + 0.5) * h
    X, Y, Z = np.meshgrid(xc, xc, xc, indexing="ij")
    s, c, pi = np.sin, np.cos, np.pi
    sig = 1 + 0.5 * s(2 * pi * X) * s(2 * pi * Y) * s(2 * pi * Z)
    xn = np.arange(1, nn) * h
    X, Y, Z = np.meshgrid(xn, xn, xn, indexing="ij")
    phi = s(pi * X) * s(pi * Y) * s(pi * Z)
    sg = 1 + 0.5 * s(2 * pi * X) * s(2 * pi * Y) * s(2 * pi * Z)
    g = [pi * c(pi * X) * s(pi * Y) * s(pi * Z), pi * s(pi * X) * c(pi * Y) * s(pi * Z),
         pi * s(pi * X) * s(pi * Y) * c(pi * Z)]
    sd = [pi * c(2 * pi * X) * s(2 * pi * Y) * s(2 * pi * Z),
          pi * s(2 * pi * X) * c(2 * pi * Y) * s(2 * pi * Z),
          pi * s(2 * pi * X) * s(2 * pi * Y) * c(2 * pi * Z)]
    f = -(sg * (-3 * pi * pi * phi) + sd[0] * g[0] + sd[1] * g[1] + sd[2] * g[2])
    return sig, f, phi


def test_manufactured_second_order():
    """-div(sigma grad phi) = f with phi = sin(pi x) sin(pi y) sin(pi z) (zero on
    the walls), sigma = 1 + sin(2 pi x) sin(2 pi y) sin(2 pi z) / 2 at cell
    centres: nodal errors fall by ~4 per halving of h (L2 and max)."""
    errs = []
    for nn in (8, 16, 32):
        sig, f, phi = _manufactured(nn)
        u, info = N.nodal_solve(sig, (False,) * 3, f, 1e-12,
                                opts=N.NodalOpts(bottom_tol=1e-13, min_bottom_cells=4))
        assert info["converged"]
        e = u - phi
        errs.append((np.sqrt(np.mean(e ** 2)) / np.sqrt(np.mean(phi ** 2)),
                     np.abs(e).max() / np.abs(phi).max()))
    for a, b in zip(errs, errs[1:]):
        for q in range(2):
            assert 3.6 < a[q] / b[q] < 4.4, errs


def test_vcycle_contraction_grid_independent():
    """Constant sigma: the V(2,2) contraction stays below 0.35 and changes
    little from 16^3 to 32^3 cells."""
    rho = []
    for nn in (16, 32):
        n = (nn,) * 3
        f = np.random.default_rng(13).uniform(-1, 1, N.unknown_shape(n, (False,) * 3))
        _, info = N.nodal_solve(np.ones(n), (False,) * 3, f, 1e-10,
                                opts=N.NodalOpts(bottom_tol=1e-12, min_bottom_cells=4))
        h = info["history"]
        rho.append((h[-1] / h[0]) ** (1.0 / info["iters"]))
    assert max(rho) < 0.35 and abs(rho[0] - rho[1]) < 0.05, rho


def _matrix(fn, m):
    M = np.zeros((int(np.prod(m)),) * 2)
    for c in range(M.shape[0]):
        e = np.zeros(M.shape[0])
        e[c] = 1
        M[:, c] = to_vec(fn(from_vec(e, m)))
    return M


@pytest.mark.parametrize("nu", [(2, 2), (2, 1)])
def test_vcycle_preconditioner_symmetric_positive(nu):
    """nu1 = nu2: M is symmetric positive definite; nu1 != nu2 breaks the
    symmetry (so the pin fails if pre and post smoothing differ)."""
    n, per = (8, 8, 8), (False, True, False)
    sig = _sigma(n, 15)
    opts = N.NodalOpts(nu1=nu[0], nu2=nu[1], bottom_tol=1e-15, min_bottom_cells=2)
    levs = N.build_nodal_levels(sig, per, opts)
    M = _matrix(lambda r: N.nodal_precond(levs, r, opts), levs[0].m)
    asym = np.abs(M - M.T).max() / np.abs(M).max()
    if nu[0] == nu[1]:
        assert asym < 1e-10
        assert np.linalg.eigvalsh(0.5 * (M + M.T))[0] > 0
    else:
        assert asym > 1e-6


def test_pcg_identity_equals_scipy_cg_iterates():
    """With the identity as preconditioner the k-th iterate is SciPy's CG
    iterate on the independently assembled matrix."""
    n, per = (8, 8, 8), (False, False, False)
    sig = _sigma(n, 16)
    A, m = assemble(sig, per)
    f = np.random.default_rng(17).uniform(-1, 1, m)
    for k in (1, 3, 6):
        phi, info = N.nodal_pcg_solve(sig, per, f, 0.0, opts=N.NodalOpts(max_iter=k),
                                      precond=lambda r: r.copy())
        assert info["iters"] == k
        ref, _ = sla.cg(A, to_vec(f), x0=np.zeros(A.shape[0]), maxiter=k, rtol=0.0, atol=0.0)
        assert np.linalg.norm(to_vec(phi) - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("n,per", [((16, 16, 16), (False,) * 3), ((16, 16, 16), (True, False, True)),
                                   ((8, 8, 8), (True, True, True))])
def test_pcg_solve_equals_direct(n, per):
    sig = _sigma(n, 18)
    A, m = assemble(sig, per)
    f = np.random.default_rng(19).uniform(-1, 1, m)
    if all(per):
        f = f - f.mean()
    phi, info = N.nodal_pcg_solve(sig, per, f, 1e-12,
                                  opts=N.NodalOpts(bottom_tol=1e-13, min_bottom_cells=2))
    assert info["converged"]
    if all(per):
        # singular: the solution with zero mean of A x = f
        Ad = A.toarray() + np.ones((A.shape[0],) * 2) / A.shape[0]
        ref = from_vec(np.linalg.solve(Ad, to_vec(f)), m)
        ref = ref - ref.mean()
    else:
        ref = from_vec(sla.spsolve(A.tocsc(), to_vec(f)), m)
    assert np.linalg.norm(phi - ref) <= 1e-10 * np.linalg.norm(ref)


def test_pcg_needs_fewer_iterations_than_vcycles():
    n, per = (32, 32, 32), (False,) * 3
    sig = _sigma(n, 20)
    f = np.random.default_rng(21).uniform(-1, 1, N.unknown_shape(n, per))
    o = N.NodalOpts(min_bottom_cells=4)
    levs = N.build_nodal_levels(sig, per, o)
    _, iv = N.nodal_solve(sig, per, f, 1e-10, opts=o, levs=levs)
    phi, ip = N.nodal_pcg_solve(sig, per, f, 1e-10, opts=o, levs=levs)
    assert ip["converged"] and ip["iters"] < 0.7 * iv["iters"], (ip["iters"], iv["iters"])
    phv, _ = N.nodal_solve(sig, per, f, 1e-12, opts=o, levs=levs)
    assert np.linalg.norm(phi - phv) <= 1e-8 * np.linalg.norm(phv)
