"""GPU adjoint gradient (autograd through the solve) against the oracle and
against central finite differences."""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_util import lib, rel_l2

TIGHT = 1e-12


def _problem(n, m, sigma=0.5):
    cfg = W.config_lognormal(n, m, sigma)
    bt = W.lognormal_cells(n, sigma, W.SEED_BT)
    cfg["faces_target"] = W.harmonic_faces(bt, cfg["periodic"])
    return cfg


def _gpu_setup(cfg, precision=0):
    """Solver handle (precision 0: FP64 V-cycles; 1: FP32 V-cycle inside FP64
    refinement) and device tensors f, log b, log b_target."""
    P = lib()
    n, boxes = cfg["n"], cfg["boxes"]
    s = P.MLMG(boxes, W.domain_box(n), cfg["periodic"], cfg["alpha"], cfg["beta"],
               opts=dict(bottom_rel_tol=TIGHT, precision=precision))
    f = torch.from_numpy(np.concatenate([x.ravel(order="F") for x in
                                         W.scatter_cells(cfg["rhs"], boxes)])).cuda()
    logb = [torch.from_numpy(P.global_to_xfast(np.log(cfg["faces"][d]))).cuda() for d in range(3)]
    logbt = [torch.from_numpy(P.global_to_xfast(np.log(cfg["faces_target"][d]))).cuda()
             for d in range(3)]
    return s, f, logb, logbt


@pytest.mark.gpu
@pytest.mark.parametrize("precision", [0, 1])
def test_adjoint_gradient_vs_oracle(precision):
    """Forward and adjoint solves in FP64, or with the FP32 V-cycle inside FP64
    refinement: dL/df and dL/dlog b against the FP64 oracle's gradient."""
    print(f"[adjoint] 32^3, 8 boxes of 16^3, precision={precision}", flush=True)
    P = lib()
    cfg = _problem(32, 16)
    n, boxes = cfg["n"], cfg["boxes"]
    s, f, logb, logbt = _gpu_setup(cfg, precision)
    with torch.no_grad():
        phi_t = P.mg_solve(f, *logbt, s, 1e-13)
    fr = f.clone().requires_grad_(True)
    lb = [x.clone().requires_grad_(True) for x in logb]
    phi = P.mg_solve(fr, *lb, s, 1e-13)
    loss = 0.5 * torch.sum((phi - phi_t) ** 2)
    loss.backward()
    # oracle
    lev = O.make_level(boxes, W.domain_box(n), cfg["periodic"], 1.0, 1.0, None,
                       [W.scatter_faces(cfg["faces"][d], boxes, d) for d in range(3)])
    opts = O.Opts(bottom_tol=TIGHT)
    f_boxes = W.scatter_cells(cfg["rhs"], boxes)
    levt = O.make_level(boxes, W.domain_box(n), cfg["periodic"], 1.0, 1.0, None,
                        [W.scatter_faces(cfg["faces_target"][d], boxes, d) for d in range(3)])
    pt = O.new_cell_data(levt)
    O.solve(levt, pt, f_boxes, 1e-13, opts=opts)
    po = O.new_cell_data(lev)
    O.solve(lev, po, f_boxes, 1e-13, opts=opts)
    Pg, Pt = W.gather_cells(po, boxes, n, ng=1), W.gather_cells(pt, boxes, n, ng=1)
    lam = O.new_cell_data(lev)
    O.solve(lev, lam, W.scatter_cells(Pg - Pt, boxes), 1e-13, opts=opts)
    g_ref = O.grad_logb(lev, po, lam)
    lam_ref = W.gather_cells(lam, boxes, n, ng=1)
    # compare
    gphi = W.gather_cells(P.MultiFab(boxes, 0, data=phi.detach()).valid_numpy(), boxes, n)
    assert rel_l2(gphi, Pg) <= 1e-10
    gf = W.gather_cells(P.MultiFab(boxes, 0, data=fr.grad).valid_numpy(), boxes, n)
    e = rel_l2(gf, lam_ref)
    print(f"dL/df rel-L2 vs oracle: {e:.2e}")
    assert e <= 1e-8
    for d in range(3):
        got = P.xfast_to_global(lb[d].grad)
        e = rel_l2(got, g_ref[d])
        print(f"dL/dlog b_{'xyz'[d]} rel-L2 vs oracle: {e:.2e}")
        assert e <= 1e-8
    s.close()


FACE_CASES = [
    # (name, n, boxes, periodic)
    ("dirichlet16_8boxes", 16, W.uniform_boxes(16, 8), (False, False, False)),
    ("uneven32_periodic_y", 32, [((0, 0, 0), (15, 31, 31)), ((16, 0, 0), (31, 15, 31)),
                                 ((16, 16, 0), (31, 31, 15)), ((16, 16, 16), (31, 31, 31))],
     (False, True, False)),
    ("periodic24_one_box", 24, [((0, 0, 0), (23, 23, 23))], (True, True, True)),
    # x extent 96: two 64-lane x tiles per row, the second one ragged
    ("wide96_periodic_xz", 96, [((0, 0, 0), (95, 47, 95)), ((0, 48, 0), (95, 95, 95))],
     (True, False, True)),
]


def _face_case(n, boxes, periodic, seed):
    cfg = W.config_lognormal(n, None, 0.5, boxes=boxes)
    cfg["periodic"] = periodic
    cfg["faces"] = W.harmonic_faces(W.lognormal_cells(n, 0.5, W.SEED_B), periodic)
    rng = np.random.default_rng(seed)
    return cfg, rng.standard_normal((n,) * 3), rng.standard_normal((n,) * 3)


@pytest.mark.gpu
@pytest.mark.parametrize("name,n,boxes,periodic", FACE_CASES, ids=[c[0] for c in FACE_CASES])
def test_face_gradient_kernel_vs_oracle(name, n, boxes, periodic):
    """The one-pass face-gradient kernel (all three directions, global face
    arrays) on given phi and lambda against the oracle's dL/dlog b, on every
    face: walls, periodic wrap faces (written at both ends), uneven boxes and
    rows wider than one 64-lane tile."""
    print(f"[adjoint] face gradient vs oracle {name}", flush=True)
    P = lib()
    cfg, Pg, Lg = _face_case(n, boxes, periodic, 5)
    s = P.MLMG(boxes, W.domain_box(n), periodic, 1.0, 1.0, opts=dict(tune=0))
    logb = [torch.from_numpy(P.global_to_xfast(np.log(cfg["faces"][d]))).cuda() for d in range(3)]
    s.set_coefficients_global(logb, is_log=True)
    phi = P.MultiFab.from_numpy(boxes, W.scatter_cells(Pg, boxes, 1, fill=np.nan), 1)
    lam = P.MultiFab.from_numpy(boxes, W.scatter_cells(Lg, boxes, 1, fill=np.nan), 1)
    glob = s.face_grad_logb_global(phi, lam)
    torch.cuda.synchronize()
    lev = O.make_level(boxes, W.domain_box(n), periodic, 1.0, 1.0, None,
                       [W.scatter_faces(cfg["faces"][d], boxes, d) for d in range(3)])
    ref = O.grad_logb(lev, W.scatter_cells(Pg, boxes, 1), W.scatter_cells(Lg, boxes, 1))
    for d in range(3):
        got = P.xfast_to_global(glob[d])
        assert got.shape == ref[d].shape
        scale = np.abs(ref[d]).max()
        err = np.abs(got - ref[d]).max()
        print(f"  d={d}: max |gpu - oracle| = {err:.2e} of max {scale:.2e}")
        assert err <= 1e-13 * scale
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("name,n,boxes,periodic", FACE_CASES, ids=[c[0] for c in FACE_CASES])
def test_face_gradient_per_box_matches_global(name, n, boxes, periodic):
    P = lib()
    cfg, Pg, Lg = _face_case(n, boxes, periodic, 3)
    s = P.MLMG(boxes, W.domain_box(n), periodic, 1.0, 1.0, opts=dict(tune=0))
    logb = [torch.from_numpy(P.global_to_xfast(np.log(cfg["faces"][d]))).cuda() for d in range(3)]
    s.set_coefficients_global(logb, is_log=True)
    phi = P.MultiFab.from_numpy(boxes, W.scatter_cells(Pg, boxes, 1), 1)
    lam = P.MultiFab.from_numpy(boxes, W.scatter_cells(Lg, boxes, 1), 1)
    glob = s.face_grad_logb_global(phi, lam)
    per = [s.face_mf(d) for d in range(3)]
    s.face_grad_logb(phi, lam, per)
    torch.cuda.synchronize()
    for d in range(3):
        G = P.xfast_to_global(glob[d])
        for bx, arr in zip(boxes, per[d].to_numpy()):
            lo = bx[0]
            sl = tuple(slice(lo[a], lo[a] + arr.shape[a]) for a in range(3))
            assert np.array_equal(G[sl], arr)
    s.close()


def _fd_picks(grads, rng, n_top, n_mid, n_rand):
    """Sample positions (d, idx) over three face tensors: the n_top largest
    |g|, n_mid drawn among faces with |g| in [1e-3, 1e-1] of the largest, and
    n_rand uniform (which mostly land far below the largest entry)."""
    flat = np.concatenate([g.ravel() for g in grads])
    offs = np.cumsum([0] + [g.size for g in grads])
    a = np.abs(flat)
    gmax = float(a.max())
    top = np.argpartition(-a, n_top)[:n_top]
    mid_pool = np.flatnonzero((a >= 1e-3 * gmax) & (a <= 1e-1 * gmax))
    mid = rng.choice(mid_pool, size=n_mid, replace=False)
    rnd = rng.integers(flat.size, size=n_rand)
    out = []
    for q in list(top) + list(mid) + list(rnd):
        d = int(np.searchsorted(offs, q, side="right") - 1)
        out.append((d, tuple(int(x) for x in np.unravel_index(q - offs[d], grads[d].shape))))
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("precision", [0, 1])
def test_c3_finite_differences(precision):
    """128^3, 8 boxes of 64^3, sigma 0.5: central differences (eps 1e-6) of L in
    log b and in f, from warm-started solves and solution differences, against
    the adjoint gradient; both computed with the solver handle of the given
    precision (FP64, or the FP32 V-cycle inside FP64 refinement).

    Faces: the 12 largest |dL/dlog b|, 12 with |g| between 1e-3 and 1e-1 of the
    largest, and 8 uniform draws; cells likewise.  ΔL carries the solves'
    roundoff, an absolute error floor under every entry: measured up to
    2.0e-6 (FP64) and 4.6e-6 (FP32+refine) of the largest entry.  Each entry
    must agree to 1e-4 |g| + 1e-5 max|g|, every sampled error must stay
    under that 1e-5 floor, and at least 12 of each 32 samples lie where the
    relative term is the larger (|g| >= 0.1 max|g|)."""
    print(f"[adjoint] C3 128^3 finite differences precision={precision}", flush=True)
    P = lib()
    cfg = W.config_c3()
    n, boxes = cfg["n"], cfg["boxes"]
    s, f, logb, logbt = _gpu_setup(cfg, precision)
    with torch.no_grad():
        phi_t = P.mg_solve(f, *logbt, s, 1e-12)
    fr = f.clone().requires_grad_(True)
    lb = [x.clone().requires_grad_(True) for x in logb]
    phi = P.mg_solve(fr, *lb, s, 1e-12)
    loss = 0.5 * torch.sum((phi - phi_t) ** 2)
    loss.backward()
    phi0 = phi.detach()
    normf = float(f.abs().max())
    atol = 1e-14 * normf

    def solve_with(fv, lbv):
        with torch.no_grad():
            return P.mg_solve(fv, *lbv, s, 0.0, atol, phi0)

    def dL(pp, pm):
        return 0.5 * float(torch.sum((pp - pm) * (pp + pm - 2 * phi_t)))

    rng = np.random.default_rng(W.SEED_FD)
    eps = 1e-6
    floor_rel = 1e-5
    gfaces = [x.grad.detach().cpu().numpy() for x in lb]
    gmax = max(float(np.abs(g).max()) for g in gfaces)
    rel_side, worst_rel, worst_abs = 0, 0.0, 0.0
    for d, idx in _fd_picks(gfaces, rng, 12, 12, 8):
        lp = [x.detach().clone() for x in lb]
        lm = [x.detach().clone() for x in lb]
        lp[d][idx] += eps
        lm[d][idx] -= eps
        fd = dL(solve_with(f, lp), solve_with(f, lm)) / (2 * eps)
        g = float(gfaces[d][idx])
        rel = abs(fd - g) / abs(g) if g != 0 else float("inf")
        print(f"  face d={d} {idx}: g {g:+.6e} fd {fd:+.6e} |g|/max {abs(g) / gmax:.1e} "
              f"rel err {rel:.1e} abs err/max {abs(fd - g) / gmax:.1e}")
        worst_abs = max(worst_abs, abs(fd - g) / gmax)
        if abs(g) >= 0.1 * gmax:
            rel_side += 1
            worst_rel = max(worst_rel, rel)
        assert abs(fd - g) <= 1e-4 * abs(g) + floor_rel * gmax, (d, idx, fd, g)
    assert rel_side >= 12, rel_side
    gcell = fr.grad.detach().cpu().numpy()
    gfmax = float(np.abs(gcell).max())
    rel_side_c, worst_abs_c = 0, 0.0
    for (_, (c,)) in _fd_picks([gcell], rng, 12, 12, 8):
        fp = f.clone()
        fm = f.clone()
        fp[c] += eps
        fm[c] -= eps
        fd = dL(solve_with(fp, logb), solve_with(fm, logb)) / (2 * eps)
        g = float(gcell[c])
        worst_abs_c = max(worst_abs_c, abs(fd - g) / gfmax)
        if abs(g) >= 0.1 * gfmax:
            rel_side_c += 1
            worst_rel = max(worst_rel, abs(fd - g) / abs(g))
        assert abs(fd - g) <= 1e-4 * abs(g) + floor_rel * gfmax, (c, fd, g)
    assert rel_side_c >= 12, rel_side_c
    assert worst_abs < floor_rel and worst_abs_c < floor_rel
    print(f"C3 FD precision={precision}: worst relative error where |g| >= 0.1 max {worst_rel:.2e} "
          f"({rel_side} faces, {rel_side_c} cells); worst absolute error / max: faces "
          f"{worst_abs:.2e}, cells {worst_abs_c:.2e}")
    s.close()
