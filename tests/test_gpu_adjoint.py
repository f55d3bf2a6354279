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


def _gpu_setup(cfg):
    P = lib()
    n, boxes = cfg["n"], cfg["boxes"]
    s = P.MLMG(boxes, W.domain_box(n), cfg["periodic"], cfg["alpha"], cfg["beta"],
               opts=dict(bottom_rel_tol=TIGHT))
    f = torch.from_numpy(np.concatenate([x.ravel(order="F") for x in
                                         W.scatter_cells(cfg["rhs"], boxes)])).cuda()
    logb = [torch.from_numpy(P.global_to_xfast(np.log(cfg["faces"][d]))).cuda() for d in range(3)]
    logbt = [torch.from_numpy(P.global_to_xfast(np.log(cfg["faces_target"][d]))).cuda()
             for d in range(3)]
    return s, f, logb, logbt


@pytest.mark.gpu
def test_adjoint_gradient_vs_oracle():
    print("[adjoint] 32^3, 8 boxes of 16^3", flush=True)
    P = lib()
    cfg = _problem(32, 16)
    n, boxes = cfg["n"], cfg["boxes"]
    s, f, logb, logbt = _gpu_setup(cfg)
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
    assert rel_l2(gf, lam_ref) <= 1e-8
    for d in range(3):
        got = P.xfast_to_global(lb[d].grad)
        e = rel_l2(got, g_ref[d])
        print(f"dL/dlog b_{'xyz'[d]} rel-L2 vs oracle: {e:.2e}")
        assert e <= 1e-8
    s.close()


@pytest.mark.gpu
def test_face_gradient_per_box_matches_global():
    P = lib()
    cfg = _problem(16, 8)
    n, boxes = cfg["n"], cfg["boxes"]
    s, f, logb, _ = _gpu_setup(cfg)
    s.set_coefficients_global(logb, is_log=True)
    rng = np.random.default_rng(3)
    phi = P.MultiFab.from_numpy(boxes, W.scatter_cells(rng.standard_normal((n,) * 3), boxes, 1), 1)
    lam = P.MultiFab.from_numpy(boxes, W.scatter_cells(rng.standard_normal((n,) * 3), boxes, 1), 1)
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


@pytest.mark.gpu
def test_c3_finite_differences():
    """128^3, 8 boxes of 64^3, sigma 0.5: central differences (eps 1e-6) of L in
    log b on 32 seeded faces and in f on 32 seeded cells, from warm-started
    solves and solution differences."""
    print("[adjoint] C3 128^3 finite differences", flush=True)
    P = lib()
    cfg = W.config_c3()
    n, boxes = cfg["n"], cfg["boxes"]
    s, f, logb, logbt = _gpu_setup(cfg)
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
    gmax = max(float(x.grad.abs().max()) for x in lb)
    worst = 0.0
    for _ in range(32):
        d = int(rng.integers(3))
        shp = s.global_face_shape(d)
        idx = tuple(int(rng.integers(x)) for x in shp)
        lp = [x.detach().clone() for x in lb]
        lm = [x.detach().clone() for x in lb]
        lp[d][idx] += eps
        lm[d][idx] -= eps
        fd = dL(solve_with(f, lp), solve_with(f, lm)) / (2 * eps)
        g = float(lb[d].grad[idx])
        worst = max(worst, abs(fd - g) / (abs(g) + 1e-5 * gmax))
        # solve roundoff gives dL an absolute floor: 1e-5 of the largest entry
        assert abs(fd - g) <= 1e-4 * abs(g) + 1e-5 * gmax, (d, idx, fd, g)
    gfmax = float(fr.grad.abs().max())
    for _ in range(32):
        c = int(rng.integers(f.numel()))
        fp = f.clone()
        fm = f.clone()
        fp[c] += eps
        fm[c] -= eps
        fd = dL(solve_with(fp, logb), solve_with(fm, logb)) / (2 * eps)
        g = float(fr.grad[c])
        assert abs(fd - g) <= 1e-4 * abs(g) + 1e-5 * gfmax, (c, fd, g)
    print(f"C3 FD: worst relative face error {worst:.2e}")
    s.close()
