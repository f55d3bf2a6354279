"""Two-level composite solve (coarse level + one finer level at ratio 2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper names multi-level geometric multigrid ("Linear Solvers"),
coarse-to-fine interpolation that fills fine ghost cells only where no fine
data exists, restriction by averaging, and refluxing of coarse fluxes at
coarse/fine faces with fine ones ("Operations between levels").  It gives none
of the formulas; the readings taken here:

* unknowns: every fine valid cell and every coarse cell not covered by the
  refinement of a fine box; a covered coarse cell holds the mean of its 8
  fine children ("average down") and is not an unknown;
* a fine ghost cell that no fine box supplies is interpolated from the coarse
  level: phi_g = phi_C + (1/4) sum_d sigma_d s_d with C the coarse parent,
  sigma_d = +1 / -1 for the high / low half of C along d and the unlimited
  central slope s_d = (phi_{C+e_d} - phi_{C-e_d}) / 2; past a Dirichlet wall
  the missing neighbour is the folded ghost -phi_C;
* fine cells use the 7-point operator with those ghosts; an uncovered coarse
  cell uses the coarse operator except that across a coarse/fine face the
  coarse flux is replaced by the mean of the 4 fine fluxes through it;
* fine face coefficients come from the coarse ones by injection (generated
  with the inputs); walls are Dirichlet (periodic composites are not built);
* the solve is an outer iteration on the exact composite residual, each step
  a two-level correction: 2 nu1 fine Gauss-Seidel sweeps with ghosts from a
  zero coarse correction, the composite residual of that fine correction,
  its fine part averaged onto covered coarse cells, one coarse V-cycle on the
  whole coarse level, the coarse correction added to the fine cells under it,
  2 nu2 fine sweeps with ghosts from the coarse correction, then the update and
  an average down.  The converged answer does not depend on these choices.
"""

from dataclasses import dataclass

import numpy as np

from .boxes import box_shape, coarsen_box, intersect, refine_box
from .mlmg import (NG, Opts, apply_op, build_levels, gsrb_halfsweep, max_norm, new_cell_data,
                   valid, vcycle)


@dataclass
class Composite:
    lc: object          # coarse Level (covers its domain)
    lf: object          # fine Level (boxes in fine index space; does not cover)
    parent: list        # fine box -> coarse box that contains it
    covered: np.ndarray  # global coarse bool array
    nc: tuple           # coarse domain extent
    ghosts: list        # per fine box: (local index arrays, global fine index arrays)
    cf_faces: list      # (coarse box, coarse local idx, d, side, fine box, fine valid local
                        #  idx list (4), fine ghost local idx list (4), fine face local idx list)
    levels_c: list = None


def make_composite(lc, fine_boxes, fine_b, fine_a=None):
    """Build the composite from the coarse Level and the fine boxes/coefficients."""
    from .mlmg import make_level
    dom_f = refine_box(lc.domain)
    lf = make_level(fine_boxes, dom_f, lc.periodic, lc.alpha, lc.beta, fine_a, fine_b,
                    prob_len=tuple(lc.h[d] * box_shape(lc.domain)[d] for d in range(3)))
    assert not any(lc.periodic), "composite solves are built for Dirichlet walls only"
    nc = box_shape(lc.domain)
    covered = np.zeros(nc, dtype=bool)
    parent = []
    for fb in fine_boxes:
        cb = coarsen_box(fb)
        assert refine_box(cb) == fb, "fine boxes must be unions of whole coarse cells"
        covered[cb[0][0]:cb[1][0] + 1, cb[0][1]:cb[1][1] + 1, cb[0][2]:cb[1][2] + 1] = True
        p = [i for i, b in enumerate(lc.boxes) if intersect(b, cb) == cb]
        assert p, "a fine box must lie inside one coarse box"
        parent.append(p[0])
    # fine ghost cells needing interpolation: face neighbours of valid fine cells
    # that lie inside the domain and in no fine box
    fine_owner = {}
    ghosts = []
    for ib, (lo, hi) in enumerate(fine_boxes):
        shp = box_shape((lo, hi))
        locs, globs = [], []
        for d in range(3):
            for side in (-1, 1):
                idx = [np.arange(shp[a]) for a in range(3)]
                idx[d] = np.array([0 if side < 0 else shp[d] + 1])
                for a in range(3):
                    if a != d:
                        idx[a] = idx[a] + 1
                L = np.meshgrid(*idx, indexing="ij")
                G = [L[a] - 1 + lo[a] for a in range(3)]
                inside = np.ones(L[0].shape, bool)
                for a in range(3):
                    inside &= (G[a] >= dom_f[0][a]) & (G[a] <= dom_f[1][a])
                cov = np.zeros_like(inside)
                for jb, (lo2, hi2) in enumerate(fine_boxes):
                    m = np.ones_like(inside)
                    for a in range(3):
                        m &= (G[a] >= lo2[a]) & (G[a] <= hi2[a])
                    cov |= m
                sel = inside & ~cov
                locs.append(tuple(L[a][sel] for a in range(3)))
                globs.append(tuple(G[a][sel] for a in range(3)))
        ghosts.append((tuple(np.concatenate([x[a] for x in locs]) for a in range(3)),
                       tuple(np.concatenate([x[a] for x in globs]) for a in range(3))))
    del fine_owner
    # coarse/fine faces: uncovered coarse cell I next to covered cell J
    cf = []
    for ib, (lo, hi) in enumerate(fine_boxes):
        cb = coarsen_box((lo, hi))
        for d in range(3):
            for side in (-1, 1):
                # coarse cells just outside this fine box's coarsened face
                rng_ = [np.arange(cb[0][a], cb[1][a] + 1) for a in range(3)]
                rng_[d] = np.array([cb[0][d] - 1 if side < 0 else cb[1][d] + 1])
                I = np.meshgrid(*rng_, indexing="ij")
                for t in zip(*(x.ravel() for x in I)):
                    if not (0 <= t[d] < nc[d]):
                        continue
                    if covered[t]:
                        continue
                    J = list(t)
                    J[d] -= side       # covered neighbour, inside this fine box's coarsening
                    # the 4 fine cells of J next to the face and their ghosts in I
                    fv, fg, ff = [], [], []
                    tr = [a for a in range(3) if a != d]
                    for o1 in (0, 1):
                        for o2 in (0, 1):
                            fc = [0, 0, 0]
                            fc[tr[0]] = 2 * J[tr[0]] + o1
                            fc[tr[1]] = 2 * J[tr[1]] + o2
                            fc[d] = 2 * J[d] + (0 if side < 0 else 1)
                            gc = list(fc)
                            gc[d] += side
                            fv.append(tuple(fc[a] - lo[a] + NG for a in range(3)))
                            fg.append(tuple(gc[a] - lo[a] + NG for a in range(3)))
                            face = list(fc)
                            if side > 0:
                                face[d] += 1
                            ff.append(tuple(face[a] - lo[a] for a in range(3)))
                    cbox = [k for k, b in enumerate(lc.boxes) if intersect(b, (t, t)) is not None][0]
                    cl = tuple(t[a] - lc.boxes[cbox][0][a] + NG for a in range(3))
                    jl = tuple(J[a] - lc.boxes[cbox][0][a] + NG for a in range(3))
                    cf.append((cbox, cl, d, side, ib, fv, fg, ff, t, tuple(J)))
    comp = Composite(lc, lf, parent, covered, nc, ghosts, cf)
    return comp


def _avg8(r):
    z0 = ((r[0::2, 0::2, 0::2] + r[1::2, 0::2, 0::2]) + (r[0::2, 1::2, 0::2] + r[1::2, 1::2, 0::2]))
    z1 = ((r[0::2, 0::2, 1::2] + r[1::2, 0::2, 1::2]) + (r[0::2, 1::2, 1::2] + r[1::2, 1::2, 1::2]))
    return (z0 + z1) * 0.125


def average_down(comp, phi_f, phi_c, ng_f=NG, ng_c=NG):
    """Covered coarse cells take the mean of their 8 fine children."""
    for ib, fb in enumerate(comp.lf.boxes):
        v = phi_f[ib][ng_f:-ng_f, ng_f:-ng_f, ng_f:-ng_f] if ng_f else phi_f[ib]
        cb = coarsen_box(fb)
        p = comp.parent[ib]
        plo = comp.lc.boxes[p][0]
        sl = tuple(slice(cb[0][a] - plo[a] + ng_c, cb[1][a] - plo[a] + ng_c + 1) for a in range(3))
        phi_c[p][sl] = _avg8(v)


def _coarse_global(comp, phi_c):
    G = np.zeros(comp.nc)
    for (lo, hi), a in zip(comp.lc.boxes, phi_c):
        G[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1] = valid(a)
    return G


def fill_fine_ghosts(comp, phi_f, phi_c):
    """Fine ghosts from other fine boxes, then the rest by coarse interpolation.
    phi_c must hold the average-down values in covered cells."""
    from .boxes import fill_boundary
    lf = comp.lf
    fill_boundary(phi_f, lf.boxes, lf.domain, lf.periodic, NG)
    G = _coarse_global(comp, phi_c)
    nc = comp.nc
    for ib, (loc, glob) in enumerate(comp.ghosts):
        if len(loc[0]) == 0:
            continue
        C = [g // 2 for g in glob]
        val = G[C[0], C[1], C[2]]
        acc = np.zeros_like(val)
        for d in range(3):
            hi_ = [c.copy() for c in C]
            lo_ = [c.copy() for c in C]
            hi_[d] = C[d] + 1
            lo_[d] = C[d] - 1
            in_hi = hi_[d] < nc[d]
            in_lo = lo_[d] >= 0
            vhi = np.where(in_hi, G[np.minimum(hi_[0], nc[0] - 1), np.minimum(hi_[1], nc[1] - 1),
                                    np.minimum(hi_[2], nc[2] - 1)], -val)
            vlo = np.where(in_lo, G[np.maximum(lo_[0], 0), np.maximum(lo_[1], 0),
                                    np.maximum(lo_[2], 0)], -val)
            s = 0.5 * (vhi - vlo)
            sign = np.where(glob[d] % 2 == 1, 1.0, -1.0)
            acc = acc + sign * s
        phi_f[ib][loc] = val + 0.25 * acc


def composite_apply(comp, phi_f, phi_c):
    """A phi on fine valid cells and on uncovered coarse cells (covered entries 0).
    Overwrites the covered cells of phi_c (average down) and the fine ghosts."""
    average_down(comp, phi_f, phi_c)
    fill_fine_ghosts(comp, phi_f, phi_c)
    Af = apply_op(comp.lf, phi_f)
    Ac = apply_op(comp.lc, phi_c)
    hc = comp.lc.h
    hf = comp.lf.h
    beta = comp.lc.beta
    for (cbox, cl, d, side, ib, fv, fg, ff, t, J) in comp.cf_faces:
        # coarse term of this face in (A phi)_I: c (phi_I - phi_J); I = J + side e_d,
        # so the shared face is I's low face for side > 0 and its high face otherwise
        cb = comp.lc.b[d][cbox]
        fidx = [cl[a] - NG for a in range(3)]
        if side < 0:
            fidx[d] += 1
        c = (beta * cb[tuple(fidx)]) / (hc[d] * hc[d])
        pI = phi_c[cbox][cl]
        jl = list(cl)
        jl[d] -= side
        term_c = c * (pI - phi_c[cbox][tuple(jl)]) if _in_box(comp.lc.boxes[cbox], J) else \
            c * (pI - _coarse_value(comp, phi_c, J))
        # fine replacement: (1/h_c) * mean of beta b_f (phi_g - phi_in) / h_f
        fl = []
        for v_, g_, f_ in zip(fv, fg, ff):
            bf = comp.lf.b[d][ib][f_]
            fl.append(beta * bf * (phi_f[ib][g_] - phi_f[ib][v_]) / hf[d])
        term_f = (((fl[0] + fl[1]) + (fl[2] + fl[3])) * 0.25) / hc[d]
        Ac[cbox][tuple(cl[a] - NG for a in range(3))] += term_f - term_c
    for ib, (lo, hi) in enumerate(comp.lc.boxes):
        m = comp.covered[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1]
        Ac[ib][m] = 0.0
    return Af, Ac


def _in_box(b, p):
    return all(b[0][a] <= p[a] <= b[1][a] for a in range(3))


def _coarse_value(comp, phi_c, p):
    for k, b in enumerate(comp.lc.boxes):
        if _in_box(b, p):
            return phi_c[k][tuple(p[a] - b[0][a] + NG for a in range(3))]
    raise ValueError(p)


def composite_residual(comp, phi_f, phi_c, f_f, f_c):
    Af, Ac = composite_apply(comp, phi_f, phi_c)
    Rf = [f - a for f, a in zip(f_f, Af)]
    Rc = []
    for ib, (lo, hi) in enumerate(comp.lc.boxes):
        r = f_c[ib] - Ac[ib]
        m = comp.covered[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1]
        r[m] = 0.0
        Rc.append(r)
    return Rf, Rc


def composite_norm(comp, Rf, Rc):
    return max(max_norm(Rf) if Rf else 0.0, max_norm(Rc))


def _fine_sweep(comp, e_f, e_c, rhs_f, colour):
    average_down(comp, e_f, e_c)
    fill_fine_ghosts(comp, e_f, e_c)
    gsrb_halfsweep(comp.lf, e_f, rhs_f, colour)


def composite_precond(comp, Rf, Rc, opts, nf1, nf2):
    """One two-level correction (e_f, e_c) of the composite residual (Rf, Rc)
    from a zero guess: nf1 fine Gauss-Seidel sweeps with ghosts from a zero
    coarse correction, the composite residual of that fine correction, its
    fine part averaged onto covered coarse cells, one coarse V-cycle on the
    whole coarse level, the coarse correction added to the fine cells under
    it, nf2 fine sweeps with ghosts from the coarse correction.  Returns
    per-box arrays with one ghost layer."""
    e_f = new_cell_data(comp.lf)
    e_c = new_cell_data(comp.lc)
    for _ in range(nf1):
        _fine_sweep(comp, e_f, e_c, Rf, 0)
        _fine_sweep(comp, e_f, e_c, Rf, 1)
    Af, Ac = composite_apply(comp, e_f, e_c)
    rf = [r - a for r, a in zip(Rf, Af)]
    rc = [r - a for r, a in zip(Rc, Ac)]
    rcg = [np.pad(x, NG) for x in rc]
    average_down(comp, rf, rcg, ng_f=0)
    rc = [valid(x) for x in rcg]
    ec = new_cell_data(comp.lc)
    vcycle(comp.levels_c, 0, ec, rc, opts)
    for ib, fb in enumerate(comp.lf.boxes):
        cb = coarsen_box(fb)
        p = comp.parent[ib]
        plo = comp.lc.boxes[p][0]
        E = ec[p][tuple(slice(cb[0][a] - plo[a] + NG, cb[1][a] - plo[a] + NG + 1)
                         for a in range(3))]
        valid(e_f[ib])[...] += np.repeat(np.repeat(np.repeat(E, 2, 0), 2, 1), 2, 2)
    for _ in range(nf2):
        _fine_sweep(comp, e_f, ec, Rf, 0)
        _fine_sweep(comp, e_f, ec, Rf, 1)
    return e_f, ec


def _add_correction(comp, phi_f, phi_c, e_f, e_c, scale=1.0):
    """phi_f += scale e_f; uncovered phi_c += scale e_c (covered cells are
    set by the caller's average down)."""
    for ib in range(len(phi_f)):
        valid(phi_f[ib])[...] += scale * valid(e_f[ib])
    for ib, (lo, hi) in enumerate(comp.lc.boxes):
        m = ~comp.covered[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1]
        valid(phi_c[ib])[m] += scale * valid(e_c[ib])[m]


def _sweeps(opts, fine_sweeps):
    nf1 = 2 * opts.nu1 if fine_sweeps is None else fine_sweeps
    nf2 = 2 * opts.nu2 if fine_sweeps is None else fine_sweeps
    return nf1, nf2


def _normf(comp, f_f, f_c):
    fz = []
    for ib, (lo, hi) in enumerate(comp.lc.boxes):
        x = f_c[ib].copy()
        x[comp.covered[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1]] = 0.0
        fz.append(x)
    return max(max_norm(f_f) if f_f else 0.0, max_norm(fz))


def composite_solve(comp, phi_f, phi_c, f_f, f_c, rel_tol=1e-10, abs_tol=0.0, opts=None,
                    fine_sweeps=None):
    """Outer iteration on the composite residual with two-level corrections.
    phi_f / phi_c: per-box arrays with one ghost layer (initial guess, updated).
    Stop when max |R| over composite cells <= max(rel_tol * max|f|, abs_tol),
    max|f| taken over the same cells.  fine_sweeps: red/black sweeps on the
    fine level before and after the coarse correction (default: 2 nu1 and
    2 nu2; the fine level is a small part of the cells and two sweeps per side
    leave its error decaying at about 0.5 per step, four at about 0.35)."""
    opts = opts or Opts()
    nf1, nf2 = _sweeps(opts, fine_sweeps)
    if comp.levels_c is None:
        comp.levels_c = build_levels(comp.lc, opts.min_bottom_edge, opts.aggregate)
    normf = _normf(comp, f_f, f_c)
    tol = max(rel_tol * normf, abs_tol)
    info = {"history": [], "iters": 0, "converged": False, "normf": normf}
    it = 0
    while True:
        Rf, Rc = composite_residual(comp, phi_f, phi_c, f_f, f_c)
        rn = composite_norm(comp, Rf, Rc)
        info["history"].append(rn)
        if not np.isfinite(rn):
            break
        if rn <= tol:
            info["converged"] = True
            break
        if it == opts.max_iter:
            break
        e_f, ec = composite_precond(comp, Rf, Rc, opts, nf1, nf2)
        _add_correction(comp, phi_f, phi_c, e_f, ec)
        average_down(comp, phi_f, phi_c)
        it += 1
    info["iters"] = it
    return info


def _cdot(uf, uc, vf, vc):
    """Dot product over fine cells and coarse cells of residual-shaped
    (ghost-free) composite vectors (covered coarse entries are zero)."""
    return float(sum(np.sum(a * b) for a, b in zip(uf, vf)) +
                 sum(np.sum(a * b) for a, b in zip(uc, vc)))


def composite_fgmres(comp, phi_f, phi_c, f_f, f_c, rel_tol=1e-10, abs_tol=0.0, opts=None,
                     fine_sweeps=None, restart=20, precond=None):
    """Flexible GMRES on the composite system, right-preconditioned by the
    two-level correction (the paper's Krylov solvers with its multigrid as the
    preconditioner; the composite operator is not symmetric, and the
    correction's bottom CG makes the preconditioner vary a little, hence the
    flexible form that keeps each z_j = M v_j).

    Each cycle: R = f - A phi (true composite residual; its max norm is the
    history entry and the stop test, as in composite_solve); beta = ||R||_2,
    v_1 = R / beta; for j = 1.. restart: z_j = M v_j, w = A z_j, classical
    Gram-Schmidt against v_1..v_j (coefficients from w before any
    subtraction), h_{j+1,j} = ||w||_2, v_{j+1} = w / h_{j+1,j}, Givens
    rotations on H and g = beta e_1; the cycle ends when |g_{j+1}| (the 2-norm
    of the residual) <= tol * beta / max|R| (the residual's 2-norm to
    max-norm ratio at the start of the cycle carried over to the target), at
    restart, or when the iteration budget (opts.max_iter) is used up.  Then
    y = H^{-1} g (triangular), phi += sum y_j z_j, average down.  Dot products
    run over fine cells and uncovered coarse cells.  precond(Rf, Rc) ->
    (e_f, e_c) (ghost layer 1) replaces the two-level correction.
    Returns a dict: history (max |R| at the start of each cycle), iters
    (preconditioner applications), cycles, converged."""
    opts = opts or Opts()
    nf1, nf2 = _sweeps(opts, fine_sweeps)
    if comp.levels_c is None:
        comp.levels_c = build_levels(comp.lc, opts.min_bottom_edge, opts.aggregate)
    if precond is None:
        def precond(Rf, Rc):
            return composite_precond(comp, Rf, Rc, opts, nf1, nf2)
    normf = _normf(comp, f_f, f_c)
    tol = max(rel_tol * normf, abs_tol)
    info = {"history": [], "iters": 0, "cycles": 0, "converged": False, "normf": normf}
    total = 0
    while True:
        Rf, Rc = composite_residual(comp, phi_f, phi_c, f_f, f_c)
        rn = composite_norm(comp, Rf, Rc)
        info["history"].append(rn)
        if not np.isfinite(rn):
            break
        if rn <= tol:
            info["converged"] = True
            break
        if total >= opts.max_iter:
            break
        beta = np.sqrt(_cdot(Rf, Rc, Rf, Rc))
        target = tol * beta / rn
        Vf, Vc = [[x / beta for x in Rf]], [[x / beta for x in Rc]]
        Z = []
        m = restart
        H = np.zeros((m + 1, m))
        g = np.zeros(m + 1)
        g[0] = beta
        cs, sn = np.zeros(m), np.zeros(m)
        k = 0
        for j in range(m):
            zf, zc = precond(Vf[j], Vc[j])
            Z.append((zf, zc))
            wf, wc = composite_apply(comp, zf, zc)
            h = [_cdot(wf, wc, Vf[i], Vc[i]) for i in range(j + 1)]
            for i in range(j + 1):
                wf = [a - h[i] * b for a, b in zip(wf, Vf[i])]
                wc = [a - h[i] * b for a, b in zip(wc, Vc[i])]
            hn = np.sqrt(_cdot(wf, wc, wf, wc))
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            r = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / r, H[j + 1, j] / r
            H[j, j], H[j + 1, j] = r, 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            k = j + 1
            if hn == 0.0 or abs(g[j + 1]) <= target or total >= opts.max_iter:
                break
            Vf.append([x / hn for x in wf])
            Vc.append([x / hn for x in wc])
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
        for i in range(k):
            _add_correction(comp, phi_f, phi_c, Z[i][0], Z[i][1], y[i])
        average_down(comp, phi_f, phi_c)
        info["cycles"] += 1
    info["iters"] = total
    return info
