"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case patches one oracle function with a plausible error (a wrong wall
weight, a dropped face term, a swapped colour order, a wrong transfer scale,
a flipped sign in CG, a wrong interpolation sign) and checks that the
independent reference that pins that function now disagrees.
"""

import numpy as np
import pytest

import oracle as O
import oracle.mlmg as M
import workloads as W
from dense_ref import apply_global


def _lev(n=8, m=4, periodic=(False, False, False)):
    bc = W.lognormal_cells(n, 1.0, 41)
    faces = W.harmonic_faces(bc, periodic)
    boxes = W.uniform_boxes(n, m)
    lev = O.make_level(boxes, W.domain_box(n), periodic, 1.0, 1.0, None,
                       [W.scatter_faces(faces[d], boxes, d) for d in range(3)])
    return lev, faces


def _operator_error(lev, faces, n=8):
    u = np.random.default_rng(1).standard_normal((n, n, n))
    got = W.gather_cells(O.apply_op(lev, W.scatter_cells(u, lev.boxes, 1)), lev.boxes, n)
    ref = apply_global(u, faces, 1.0, 1.0, lev.h, lev.periodic)
    return np.max(np.abs(got - ref)) / np.max(np.abs(ref))


def test_reference_agrees_unpatched():
    lev, faces = _lev()
    assert _operator_error(lev, faces) <= 1e-12


def _patched_stencil(mutation):
    orig = M.stencil

    def st(lev):
        lev._stencil = None
        out = orig(lev)
        lev._stencil = None
        res = []
        for diag, faces in out:
            faces = list(faces)
            if mutation == "wall_weight_1":
                diag = diag - sum(np.where(m, c, 0.0) for c, m in faces)
            elif mutation == "drop_zhi":
                c, m = faces[5]
                diag = diag - np.where(m, 2 * c, c)
                faces[5] = (np.zeros_like(c), m)
            elif mutation == "swap_xy_faces":
                faces[0], faces[2] = faces[2], faces[0]
            res.append((diag, faces))
        return res
    return st


@pytest.mark.parametrize("mutation", ["wall_weight_1", "drop_zhi", "swap_xy_faces"])
def test_operator_mutations_caught(monkeypatch, mutation):
    lev, faces = _lev()
    monkeypatch.setattr(M, "stencil", _patched_stencil(mutation))
    assert _operator_error(lev, faces) > 1e-6


def test_colour_order_mutation_caught(monkeypatch):
    from test_oracle_operator import _sequential_gs
    lev, faces = _lev(8, 4)
    orig = M.gsrb_halfsweep
    monkeypatch.setattr(M, "gsrb_halfsweep", lambda l, p, f, c: orig(l, p, f, 1 - c))
    rng = np.random.default_rng(6)
    u = rng.standard_normal((8, 8, 8))
    f = rng.standard_normal((8, 8, 8))
    phi = W.scatter_cells(u, lev.boxes, 1)
    fb = W.scatter_cells(f, lev.boxes)
    M.gsrb_halfsweep(lev, phi, fb, 0)
    M.gsrb_halfsweep(lev, phi, fb, 1)
    got = W.gather_cells(phi, lev.boxes, 8, ng=1)
    ref = _sequential_gs(u, f, faces, 1.0, 1.0, lev.h, lev.periodic)
    assert np.max(np.abs(got - ref)) > 1e-6 * np.max(np.abs(ref))


def test_restriction_scale_mutation_caught(monkeypatch):
    orig = M._avg8
    monkeypatch.setattr(M, "_avg8", lambda r: orig(r) * 2)
    lev, _ = _lev(16, 8)
    ones = [np.ones(O.box_shape(b)) for b in lev.boxes]
    assert not all(np.array_equal(x, np.ones_like(x)) for x in M.restrict(lev, ones))


def test_cg_sign_mutation_caught(monkeypatch):
    """CG run on -A (a sign dropped in the operator it applies) lands on -A^{-1} b."""
    from dense_ref import assemble
    n = 8
    lev, faces = _lev(n, 4)
    orig = M.apply_op
    monkeypatch.setattr(M, "apply_op", lambda l, p: [-x for x in orig(l, p)])
    f = W.uniform_rhs(n, 16)
    x, _ = M.cg_bottom(lev, W.scatter_cells(f, lev.boxes), tol=1e-13)
    ref = np.linalg.solve(assemble(n, faces, 1.0, 1.0, lev.periodic), f.ravel()).reshape(n, n, n)
    G = W.gather_cells(x, lev.boxes, n, ng=1)
    assert np.linalg.norm(G - ref) / np.linalg.norm(ref) > 1e-3


def test_interpolation_sign_mutation_caught(monkeypatch):
    """Flip the coarse/fine slope sign: the independent composite assembly disagrees."""
    from oracle import composite as OC
    from test_oracle_composite import _fields, _patch_boxes, _setup
    comp, ref, _, _ = _setup(16, 8, _patch_boxes())
    A = ref.matrix()
    orig = OC.fill_fine_ghosts

    def flipped(c, pf, pc):
        saved = [g[1] for g in c.ghosts]
        c.ghosts = [(loc, tuple(glob[a] + (1 - 2 * (glob[a] % 2)) if a == 0 else glob[a]
                                for a in range(3))) for loc, glob in c.ghosts]
        try:
            orig(c, pf, pc)
        finally:
            c.ghosts = [(g[0], s) for g, s in zip(c.ghosts, saved)]
    monkeypatch.setattr(OC, "fill_fine_ghosts", flipped)
    rng = np.random.default_rng(2)
    Ff, Fc, phi_f, phi_c = _fields(comp, ref, rng)
    Af, Ac = OC.composite_apply(comp, phi_f, phi_c)
    got = ref.pack(W.gather_cells(Af, comp.lf.boxes, (32,) * 3), W.gather_cells(Ac, comp.lc.boxes, 16))
    want = A @ ref.pack(Ff, Fc)
    assert np.max(np.abs(got - want)) > 1e-6 * np.max(np.abs(want))
