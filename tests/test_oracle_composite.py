"""Pins of the oracle's two-level composite operator and solve (no GPU).

* the operator equals an independent sparse assembly from the definition
  (tests/composite_ref.py) on random fields;
* the composite solve reaches the direct solution of that sparse system;
* a fine level covering the whole domain reduces to a single-level fine solve;
* linear fields are reproduced by the coarse/fine interpolation (zero
  operator away from walls when alpha = 0 and b = 1);
* conservation: the volume-weighted sum of A phi over composite cells equals
  the alpha term plus the wall fluxes.
"""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
import workloads as W
from composite_ref import CompositeRef
from oracle import composite as OC
from workloads import amr


def _setup(nc, cbox, fine_boxes, sigma=1.0, alpha=1.0, b_const=False):
    bc = np.ones((nc,) * 3) if b_const else W.lognormal_cells(nc, sigma, 31)
    cf = W.harmonic_faces(bc)
    cboxes = W.uniform_boxes(nc, cbox)
    lc = O.make_level(cboxes, W.domain_box(nc), (False,) * 3, alpha, 1.0, None,
                      [W.scatter_faces(cf[d], cboxes, d) for d in range(3)])
    fb = [amr.fine_faces(bc, cf, fine_boxes, d) for d in range(3)]
    comp = OC.make_composite(lc, fine_boxes, fb)
    # global fine faces for the reference (injection over the whole fine grid)
    gf = [amr.fine_faces(bc, cf, [((0, 0, 0), (2 * nc - 1,) * 3)], d)[0] for d in range(3)]
    ref = CompositeRef(nc, fine_boxes, bc, cf, gf, alpha=alpha)
    return comp, ref, bc, cf


def _patch_boxes():
    # one 8^3 fine patch over coarse cells 6..9, cut at the coarse box boundary (fine 16)
    return amr.chop([((12, 12, 12), (19, 19, 19))], 8, 2, 16)


def _fields(comp, ref, rng):
    Ff = rng.standard_normal((ref.nf,) * 3)
    Fc = rng.standard_normal((ref.nc,) * 3)
    phi_f = W.scatter_cells(Ff, comp.lf.boxes, ng=1, fill=np.nan)
    phi_c = W.scatter_cells(Fc, comp.lc.boxes, ng=1, fill=np.nan)
    return Ff, Fc, phi_f, phi_c


@pytest.mark.parametrize("alpha", [1.0, 0.0])
def test_operator_matches_independent_assembly(alpha):
    comp, ref, _, _ = _setup(16, 8, _patch_boxes(), alpha=alpha)
    assert ref.n == 16 ** 3 - 64 + 512
    A = ref.matrix()
    rng = np.random.default_rng(2)
    for _ in range(3):
        Ff, Fc, phi_f, phi_c = _fields(comp, ref, rng)
        Af, Ac = OC.composite_apply(comp, phi_f, phi_c)
        got = ref.pack(W.gather_cells(Af, comp.lf.boxes, (32,) * 3),
                       W.gather_cells(Ac, comp.lc.boxes, 16))
        want = A @ ref.pack(Ff, Fc)
        assert np.max(np.abs(got - want)) <= 1e-11 * np.max(np.abs(want))


def test_generated_boxes_operator_matches_assembly():
    nc = 16
    fc = amr.blob_rhs(nc, amr.blob_centres())
    fboxes = amr.fine_boxes(fc, block=1, coarse_box=8)
    assert len(fboxes) > 4
    comp, ref, _, _ = _setup(nc, 8, fboxes)
    A = ref.matrix()
    rng = np.random.default_rng(3)
    Ff, Fc, phi_f, phi_c = _fields(comp, ref, rng)
    Af, Ac = OC.composite_apply(comp, phi_f, phi_c)
    got = ref.pack(W.gather_cells(Af, comp.lf.boxes, (32,) * 3), W.gather_cells(Ac, comp.lc.boxes, nc))
    want = A @ ref.pack(Ff, Fc)
    assert np.max(np.abs(got - want)) <= 1e-11 * np.max(np.abs(want))


def test_composite_solve_matches_direct():
    comp, ref, _, _ = _setup(16, 8, _patch_boxes())
    rng = np.random.default_rng(4)
    Gf = rng.uniform(-1, 1, (32,) * 3)
    Gc = rng.uniform(-1, 1, (16,) * 3)
    f_f = W.scatter_cells(Gf, comp.lf.boxes)
    f_c = W.scatter_cells(Gc, comp.lc.boxes)
    phi_f = O.new_cell_data(comp.lf)
    phi_c = O.new_cell_data(comp.lc)
    info = OC.composite_solve(comp, phi_f, phi_c, f_f, f_c, 1e-12,
                              opts=O.Opts(min_bottom_edge=2, bottom_tol=1e-12))
    assert info["converged"]
    x = spla.spsolve(ref.matrix().tocsc(), ref.pack(Gf, Gc))
    got = ref.pack(W.gather_cells(phi_f, comp.lf.boxes, (32,) * 3, ng=1),
                   W.gather_cells(phi_c, comp.lc.boxes, 16, ng=1))
    assert np.linalg.norm(got - x) / np.linalg.norm(x) <= 1e-10
    h = info["history"]
    assert (h[-1] / h[0]) ** (1.0 / (len(h) - 1)) <= 0.5


def test_full_cover_reduces_to_fine_single_level():
    nc = 8
    fboxes = W.uniform_boxes(16, 8)
    comp, _, bc, cf = _setup(nc, 4, fboxes)
    rng = np.random.default_rng(5)
    Gf = rng.uniform(-1, 1, (16,) * 3)
    f_f = W.scatter_cells(Gf, fboxes)
    f_c = O.new_cell_data(comp.lc)
    f_c = [O.valid(x) for x in f_c]
    phi_f = O.new_cell_data(comp.lf)
    phi_c = O.new_cell_data(comp.lc)
    info = OC.composite_solve(comp, phi_f, phi_c, f_f, f_c, 1e-12,
                              opts=O.Opts(min_bottom_edge=2, bottom_tol=1e-12))
    assert info["converged"]
    lf = O.make_level(fboxes, W.domain_box(16), (False,) * 3, 1.0, 1.0, None,
                      [amr.fine_faces(bc, cf, fboxes, d) for d in range(3)])
    p = O.new_cell_data(lf)
    O.solve(lf, p, f_f, 1e-12, opts=O.Opts(min_bottom_edge=2, bottom_tol=1e-12))
    a = W.gather_cells(phi_f, fboxes, 16, ng=1)
    b = W.gather_cells(p, fboxes, 16, ng=1)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) <= 1e-10


def test_linear_field_reproduced():
    """alpha = 0, b = 1: a linear field has zero operator at every composite cell
    whose stencil (incl. interpolation) stays off the walls."""
    comp, ref, _, _ = _setup(16, 8, _patch_boxes(), alpha=0.0, b_const=True)
    c = np.array([0.3, -0.7, 0.45])
    xf = (np.arange(32) + 0.5) / 32
    xc = (np.arange(16) + 0.5) / 16
    Lf = (c[0] * xf[:, None, None] + c[1] * xf[None, :, None] + c[2] * xf[None, None, :])
    Lc = (c[0] * xc[:, None, None] + c[1] * xc[None, :, None] + c[2] * xc[None, None, :])
    phi_f = W.scatter_cells(Lf, comp.lf.boxes, ng=1)
    phi_c = W.scatter_cells(Lc, comp.lc.boxes, ng=1)
    Af, Ac = OC.composite_apply(comp, phi_f, phi_c)
    assert max(float(np.max(np.abs(a))) for a in Af) <= 1e-9
    Gc = W.gather_cells(Ac, comp.lc.boxes, 16)
    assert np.max(np.abs(Gc[2:-2, 2:-2, 2:-2])) <= 1e-9


def test_conservation():
    """sum over composite cells of (A phi) * volume = sum alpha a phi * volume
    minus the net outward flux through the domain walls."""
    comp, ref, bc, cf = _setup(16, 8, _patch_boxes())
    rng = np.random.default_rng(6)
    Ff, Fc, phi_f, phi_c = _fields(comp, ref, rng)
    Af, Ac = OC.composite_apply(comp, phi_f, phi_c)
    vf, vc = (1 / 32) ** 3, (1 / 16) ** 3
    lhs = sum(float(np.sum(a)) for a in Af) * vf + sum(float(np.sum(a)) for a in Ac) * vc
    # alpha term
    Fc_unc = Fc * (~ref.covered)
    rhs = np.sum(Ff * ref.fine) * vf + np.sum(Fc_unc) * vc
    # wall fluxes (the patch is interior, so walls are all coarse): folded ghost -phi
    h = 1 / 16
    wall = 0.0
    for d in range(3):
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[d] = 0
        sl_hi[d] = -1
        bl = cf[d][tuple(sl_lo)]
        bh = cf[d][tuple(sl_hi)]
        wall += np.sum(bl * 2 * Fc[tuple(sl_lo)] / h) * h * h
        wall += np.sum(bh * 2 * Fc[tuple(sl_hi)] / h) * h * h
    rhs += wall
    assert abs(lhs - rhs) <= 1e-10 * (abs(lhs) + abs(rhs) + wall)


def _unpack(ref, comp, x):
    """Packed composite unknowns -> fine / coarse per-box arrays (ghost-free)."""
    Gf = np.zeros((ref.nf,) * 3)
    Gc = np.zeros((ref.nc,) * 3)
    for p, r in ref.fid.items():
        Gf[p] = x[r]
    for p, r in ref.cid.items():
        Gc[p] = x[r]
    return W.scatter_cells(Gf, comp.lf.boxes), W.scatter_cells(Gc, comp.lc.boxes)


@pytest.mark.parametrize("k", [1, 3, 5])
def test_fgmres_identity_minimises_over_krylov_space(k):
    """With the identity as preconditioner, k iterations from phi = 0 give the
    minimiser of ||f - A x||_2 over the Krylov space span{f, A f, ..}, found
    here by a least-squares solve on an orthonormal basis of that space built
    from the independent sparse assembly."""
    comp, ref, _, _ = _setup(16, 8, _patch_boxes())
    A = ref.matrix().tocsr()
    rng = np.random.default_rng(7)
    Gf = rng.uniform(-1, 1, (32,) * 3)
    Gc = rng.uniform(-1, 1, (16,) * 3)
    b = ref.pack(Gf, Gc)
    f_f = W.scatter_cells(Gf, comp.lf.boxes)
    f_c = W.scatter_cells(Gc, comp.lc.boxes)

    def ident(Rf, Rc):
        return [np.pad(x, 1) for x in Rf], [np.pad(x, 1) for x in Rc]

    phi_f = O.new_cell_data(comp.lf)
    phi_c = O.new_cell_data(comp.lc)
    info = OC.composite_fgmres(comp, phi_f, phi_c, f_f, f_c, rel_tol=0.0, restart=k,
                               opts=O.Opts(max_iter=k), precond=ident)
    assert info["iters"] == k and info["cycles"] == 1
    K = [b]
    for _ in range(k - 1):
        K.append(A @ K[-1])
    Q, _ = np.linalg.qr(np.stack(K, axis=1))
    c, *_ = np.linalg.lstsq(A @ Q, b, rcond=None)
    want = Q @ c
    got = ref.pack(W.gather_cells(phi_f, comp.lf.boxes, (32,) * 3, ng=1),
                   W.gather_cells(phi_c, comp.lc.boxes, 16, ng=1))
    assert np.linalg.norm(got - want) <= 1e-9 * np.linalg.norm(want)


def test_fgmres_matches_direct():
    comp, ref, _, _ = _setup(16, 8, _patch_boxes())
    rng = np.random.default_rng(4)
    Gf = rng.uniform(-1, 1, (32,) * 3)
    Gc = rng.uniform(-1, 1, (16,) * 3)
    phi_f = O.new_cell_data(comp.lf)
    phi_c = O.new_cell_data(comp.lc)
    info = OC.composite_fgmres(comp, phi_f, phi_c, W.scatter_cells(Gf, comp.lf.boxes),
                               W.scatter_cells(Gc, comp.lc.boxes), 1e-12,
                               opts=O.Opts(min_bottom_edge=2, bottom_tol=1e-12))
    assert info["converged"]
    x = spla.spsolve(ref.matrix().tocsc(), ref.pack(Gf, Gc))
    got = ref.pack(W.gather_cells(phi_f, comp.lf.boxes, (32,) * 3, ng=1),
                   W.gather_cells(phi_c, comp.lc.boxes, 16, ng=1))
    assert np.linalg.norm(got - x) / np.linalg.norm(x) <= 1e-10


def test_fgmres_needs_fewer_corrections_than_the_stationary_solve():
    nc = 32
    fcg = amr.blob_rhs(nc, amr.blob_centres())
    fboxes = amr.fine_boxes(fcg, block=2, coarse_box=16)
    comp, _, _, _ = _setup(nc, 16, fboxes)
    f_f = amr.fine_rhs(fboxes, amr.blob_centres(), 2 * nc)
    f_c = W.scatter_cells(fcg, comp.lc.boxes)
    a_f, a_c = O.new_cell_data(comp.lf), O.new_cell_data(comp.lc)
    st = OC.composite_solve(comp, a_f, a_c, f_f, f_c, 1e-10)
    b_f, b_c = O.new_cell_data(comp.lf), O.new_cell_data(comp.lc)
    gm = OC.composite_fgmres(comp, b_f, b_c, f_f, f_c, 1e-10)
    assert st["converged"] and gm["converged"]
    assert gm["iters"] <= st["iters"] - 4
    A_ = np.concatenate([O.valid(x).ravel() for x in a_f])
    B_ = np.concatenate([O.valid(x).ravel() for x in b_f])
    assert np.linalg.norm(A_ - B_) / np.linalg.norm(A_) <= 1e-8
