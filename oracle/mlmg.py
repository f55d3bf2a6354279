"""Cell-centred variable-coefficient operator and its geometric multigrid solve.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The operator is the one of the paper's "Linear Solvers" section,
``alpha*a*phi - beta*div(b grad phi) = f`` (the paper's scalars and
coefficients renamed: alpha, beta scalars; ``a`` per cell; ``b`` per face).
Its standard 7-point cell-centred discretisation on a level with mesh size h:

    (A phi)_i = alpha a_i phi_i
                - beta sum_d [ b_{d,i+e_d} (phi_{i+e_d} - phi_i)
                              - b_{d,i}     (phi_i - phi_{i-e_d}) ] / h_d^2

Face array ``b[d][box]`` holds, at index i, the face on the low side of cell i
along d (indices lo_d .. hi_d+1).  Readings taken where the paper is silent:

* domain = unit cube, h_d = 1 / n_d;
* periodic directions go through ghost cells filled by the exchange;
* a homogeneous Dirichlet wall (phi = 0 on the face) uses the linear ghost
  value phi_ghost = -phi_i folded into the stencil: that face adds 2 c_f to the
  diagonal and has no neighbour term (symmetric, so CG and the adjoint work);
* smoother = red/black Gauss-Seidel, colour = (i+j+k) mod 2 in global level
  indices, red (0) first, ghost exchange before every half-sweep;
* restriction = average of the 8 children, interpolation = piecewise constant
  (the averaging and interpolation of "Operations between levels");
* coefficients coarsened by averaging (a: 8 cells, b: the 4 fine faces on a
  coarse face) and the operator re-discretised at h_c = 2h;
* bottom = unpreconditioned CG from a zero guess, stopped on the 2-norm
  (or BiCGStab, the paper's other native Krylov solver, with the same stop);
* outer stop test on the max norm relative to max|f|.
"""

import math
from dataclasses import dataclass, field

import numpy as np

from .boxes import box_shape, coarsen_box, fill_boundary

NG = 1  # ghost width of cell data used by the solver


@dataclass
class Level:
    boxes: list
    domain: tuple
    periodic: tuple
    h: tuple
    alpha: float
    beta: float
    a: list            # per box, valid shape; None means a == 1
    b: list            # b[d][box], face arrays (valid shape + e_d)
    dtype: type = np.float64
    merged: bool = False   # one box covering several boxes of the level above
    _stencil: list = field(default=None, repr=False)


def make_level(boxes, domain, periodic, alpha, beta, a=None, b=None, prob_len=(1.0, 1.0, 1.0),
               dtype=np.float64):
    """Build level-0 of a solve.  ``a`` and ``b`` are per-box lists (None = 1)."""
    n = box_shape(domain)
    h = tuple(prob_len[d] / n[d] for d in range(3))
    if b is None:
        b = []
        for d in range(3):
            e = [0, 0, 0]
            e[d] = 1
            b.append([np.ones(tuple(box_shape(bx)[a_] + e[a_] for a_ in range(3)), dtype=dtype)
                      for bx in boxes])
    if a is not None:
        a = [np.asarray(x, dtype=dtype) for x in a]
    b = [[np.asarray(x, dtype=dtype) for x in b[d]] for d in range(3)]
    return Level(list(boxes), domain, tuple(bool(p) for p in periodic), h, float(alpha),
                 float(beta), a, b, dtype)


def new_cell_data(level, ng=NG, dtype=None):
    dt = level.dtype if dtype is None else dtype
    return [np.zeros(tuple(e + 2 * ng for e in box_shape(bx)), dtype=dt) for bx in level.boxes]


def valid(arr, ng=NG):
    return arr[ng:-ng, ng:-ng, ng:-ng] if ng > 0 else arr


def _parent(lev_c, ib):
    """Box of the coarse level holding the coarsened fine box ib."""
    return 0 if lev_c.merged else ib


def _place(out, ib_parent, lev_c, sub, fine_box, extra=(0, 0, 0), ng=0):
    """Write ``sub`` (an array over coarsen(fine_box), grown by ``extra`` at the
    high end) into the coarse box's array at the matching position."""
    clo = coarsen_box(fine_box)[0]
    plo = lev_c.boxes[ib_parent][0]
    sl = tuple(slice(clo[a] - plo[a] + ng, clo[a] - plo[a] + ng + sub.shape[a]) for a in range(3))
    out[ib_parent][sl] = sub


def coarsen_level(lev, merged=False):
    """Next multigrid level: boxes coarsened by 2, coefficients averaged.

    a_c = mean of the 8 child cells; b_c on a coarse d-face = mean of the 4 fine
    d-faces that make it up.  Coarsening is done in float64.  With ``merged``
    the next level is the single box coarsen(domain) and each fine box's
    averages land in their place inside it.
    """
    cdom = coarsen_box(lev.domain)
    boxes = [cdom] if merged else [coarsen_box(bx) for bx in lev.boxes]
    h = tuple(2.0 * x for x in lev.h)
    out = Level(boxes, cdom, lev.periodic, h, lev.alpha, lev.beta, None, None, np.float64,
                merged)
    a = None
    if lev.a is not None:
        a = [np.zeros(box_shape(b)) for b in boxes]
        for ib, af in enumerate(lev.a):
            af = af.astype(np.float64)
            z0 = ((af[0::2, 0::2, 0::2] + af[1::2, 0::2, 0::2])
                  + (af[0::2, 1::2, 0::2] + af[1::2, 1::2, 0::2]))
            z1 = ((af[0::2, 0::2, 1::2] + af[1::2, 0::2, 1::2])
                  + (af[0::2, 1::2, 1::2] + af[1::2, 1::2, 1::2]))
            _place(a, _parent(out, ib), out, (z0 + z1) * 0.125, lev.boxes[ib])
    b = []
    for d in range(3):
        t1, t2 = [x for x in range(3) if x != d]
        e = [0, 0, 0]
        e[d] = 1
        bl = [np.zeros(tuple(box_shape(bx)[q] + e[q] for q in range(3))) for bx in boxes]
        for ib, bf in enumerate(lev.b[d]):
            bf = bf.astype(np.float64)
            sl = [slice(None)] * 3
            sl[d] = slice(0, None, 2)       # fine faces 0, 2, ..., n_d lie on coarse faces
            sub = bf[tuple(sl)]
            parts = []
            for o1 in (0, 1):
                for o2 in (0, 1):
                    s2 = [slice(None)] * 3
                    s2[t1] = slice(o1, None, 2)
                    s2[t2] = slice(o2, None, 2)
                    parts.append(sub[tuple(s2)])
            _place(bl, _parent(out, ib), out, ((parts[0] + parts[1]) + (parts[2] + parts[3])) * 0.25,
                   lev.boxes[ib])
        b.append(bl)
    out.a = a
    out.b = b
    return out


def cast_level(lev, dtype):
    """Same level with its coefficients rounded to ``dtype``."""
    a = None if lev.a is None else [x.astype(dtype) for x in lev.a]
    b = [[x.astype(dtype) for x in lev.b[d]] for d in range(3)]
    return Level(lev.boxes, lev.domain, lev.periodic, lev.h, lev.alpha, lev.beta, a, b, dtype,
                 lev.merged)


def stencil(lev):
    """Per box: (diag, [(c, dirichlet_mask) for faces xlo, xhi, ylo, yhi, zlo, zhi]).

    c_f = beta * b_f / h_d^2.  A face on a Dirichlet wall has weight 2 in the
    diagonal and no neighbour term; every other face has weight 1.  The diagonal
    is summed in the fixed face order xlo, xhi, ylo, yhi, zlo, zhi.
    """
    if lev._stencil is not None:
        return lev._stencil
    dt = lev.dtype
    out = []
    for ib, bx in enumerate(lev.boxes):
        shp = box_shape(bx)
        lo, hi = bx
        if lev.a is None:
            diag = np.full(shp, lev.alpha, dtype=dt)
        else:
            diag = (dt(lev.alpha) * lev.a[ib]).astype(dt)
        faces = []
        for d in range(3):
            inv_h2 = dt(1.0 / (lev.h[d] * lev.h[d]))
            bf = lev.b[d][ib]
            sl_lo = [slice(None)] * 3
            sl_hi = [slice(None)] * 3
            sl_lo[d] = slice(0, shp[d])
            sl_hi[d] = slice(1, shp[d] + 1)
            for side, sl in (("lo", sl_lo), ("hi", sl_hi)):
                c = (dt(lev.beta) * bf[tuple(sl)]) * inv_h2
                mask = np.zeros(shp, dtype=bool)
                if not lev.periodic[d]:
                    edge = [slice(None)] * 3
                    if side == "lo" and lo[d] == lev.domain[0][d]:
                        edge[d] = slice(0, 1)
                        mask[tuple(edge)] = True
                    if side == "hi" and hi[d] == lev.domain[1][d]:
                        edge[d] = slice(shp[d] - 1, shp[d])
                        mask[tuple(edge)] = True
                faces.append((c.astype(dt), mask))
        for (c, m) in faces:
            diag = diag + np.where(m, dt(2) * c, c)
        out.append((diag.astype(dt), faces))
    lev._stencil = out
    return out


def _neighbours(P, ng=NG):
    """Views of the six neighbours of every valid cell: xlo, xhi, ylo, yhi, zlo, zhi."""
    n0, n1, n2 = (P.shape[0] - 2 * ng, P.shape[1] - 2 * ng, P.shape[2] - 2 * ng)
    g = ng
    return [
        P[g - 1:g - 1 + n0, g:g + n1, g:g + n2], P[g + 1:g + 1 + n0, g:g + n1, g:g + n2],
        P[g:g + n0, g - 1:g - 1 + n1, g:g + n2], P[g:g + n0, g + 1:g + 1 + n1, g:g + n2],
        P[g:g + n0, g:g + n1, g - 1:g - 1 + n2], P[g:g + n0, g:g + n1, g + 1:g + 1 + n2],
    ]


def _offsum(faces, P):
    dt = P.dtype
    s = None
    for (c, m), nb in zip(faces, _neighbours(P)):
        t = np.where(m, dt.type(0), c * nb)
        s = t if s is None else s + t
    return s


def exchange(lev, data):
    fill_boundary(data, lev.boxes, lev.domain, lev.periodic, NG)


def apply_op(lev, phi):
    """A phi on every valid cell (ghosts of phi are filled first)."""
    exchange(lev, phi)
    out = []
    for ib, (diag, faces) in enumerate(stencil(lev)):
        P = phi[ib]
        out.append(diag * valid(P) - _offsum(faces, P))
    return out


def residual(lev, phi, f):
    """r = f - A phi (valid cells only)."""
    Aphi = apply_op(lev, phi)
    return [f[ib] - Aphi[ib] for ib in range(len(lev.boxes))]


def colour_mask(bx, colour):
    lo, hi = bx
    I = np.arange(lo[0], hi[0] + 1)[:, None, None]
    J = np.arange(lo[1], hi[1] + 1)[None, :, None]
    K = np.arange(lo[2], hi[2] + 1)[None, None, :]
    return ((I + J + K) % 2) == colour


def gsrb_halfsweep(lev, phi, f, colour):
    """One Gauss-Seidel half-sweep over the cells of one colour.

    phi_i <- (f_i + sum_{non-wall faces} c_f phi_nbr) / diag_i.  Cells of one
    colour only neighbour cells of the other colour, so updating all of them
    from the same old values is exact Gauss-Seidel for that colour.
    """
    exchange(lev, phi)
    for ib, (diag, faces) in enumerate(stencil(lev)):
        P = phi[ib]
        new = (f[ib] + _offsum(faces, P)) / diag
        V = valid(P)
        m = colour_mask(lev.boxes[ib], colour)
        V[m] = new[m]


def restrict(lev_f, r_f, lev_c=None):
    """Coarse value = mean of the 8 children.  Box b of the coarse level is
    coarsen(box b), or, for a merged coarse level, each fine box's averages go
    to their place in its single box."""
    if lev_c is None or not lev_c.merged:
        out = []
        for r in r_f:
            out.append(_avg8(r))
        return out
    out = [np.zeros(box_shape(b), dtype=r_f[0].dtype) for b in lev_c.boxes]
    for ib, r in enumerate(r_f):
        _place(out, 0, lev_c, _avg8(r), lev_f.boxes[ib])
    return out


def _avg8(r):
    # pairwise: ((x pairs) + (y pairs)) per z layer, then the two z layers, so
    # that eight equal values average back to exactly that value
    z0 = ((r[0::2, 0::2, 0::2] + r[1::2, 0::2, 0::2]) + (r[0::2, 1::2, 0::2] + r[1::2, 1::2, 0::2]))
    z1 = ((r[0::2, 0::2, 1::2] + r[1::2, 0::2, 1::2]) + (r[0::2, 1::2, 1::2] + r[1::2, 1::2, 1::2]))
    return ((z0 + z1) * r.dtype.type(0.125)).astype(r.dtype)


def prolong_add(phi_f, e_c, lev_f=None, lev_c=None):
    """Fine valid cell += coarse value of its parent (piecewise-constant interpolation)."""
    for ib in range(len(phi_f)):
        V = valid(phi_f[ib])
        if lev_c is not None and lev_c.merged:
            cb = coarsen_box(lev_f.boxes[ib])
            plo = lev_c.boxes[0][0]
            E = e_c[0][tuple(slice(cb[0][a] - plo[a] + NG, cb[1][a] - plo[a] + NG + 1)
                             for a in range(3))]
        else:
            E = valid(e_c[ib])
        V += np.repeat(np.repeat(np.repeat(E, 2, axis=0), 2, axis=1), 2, axis=2)


def _dot(u, v):
    """Sum of products over all valid cells, accumulated in float64."""
    return float(sum(np.sum(x.astype(np.float64) * y.astype(np.float64)) for x, y in zip(u, v)))


def _mean(u):
    n = sum(x.size for x in u)
    return float(sum(np.sum(x.astype(np.float64)) for x in u)) / n


def is_singular(lev):
    if not all(lev.periodic):
        return False
    if lev.alpha == 0.0:
        return True
    return lev.a is not None and all(not np.any(x) for x in lev.a)


def cg_bottom(lev, rhs, tol=1e-4, max_iter=None, singular=None):
    """Unpreconditioned CG on ``A x = rhs`` from x = 0 (the paper's CG "bottom solve").

    Stops when ||r||_2 <= tol * ||rhs||_2 (2-norm over all cells) or after
    ``max_iter`` iterations (default: number of cells).  For a singular
    all-periodic problem the mean of rhs is removed first and the mean of x at
    the end (CG's r and p recurrences do not involve x, so removing it at the
    end equals removing it from every iterate).  Dot products are accumulated
    in float64.  Returns (x with ghosts, iterations).
    """
    dt = lev.dtype
    if singular is None:
        singular = is_singular(lev)
    ncell = sum(int(np.prod(box_shape(b))) for b in lev.boxes)
    if max_iter is None:
        max_iter = ncell
    x = new_cell_data(lev)
    r = [np.array(v, dtype=dt, copy=True) for v in rhs]
    if singular:
        m = dt(_mean(r))
        r = [(v - m).astype(dt) for v in r]
    rho = _dot(r, r)
    bnorm = math.sqrt(rho)
    if bnorm == 0.0:
        return x, 0
    p = new_cell_data(lev)
    for ib in range(len(p)):
        valid(p[ib])[...] = r[ib]
    it = 0
    while it < max_iter:
        q = apply_op(lev, p)
        pq = _dot([valid(v) for v in p], q)
        al = rho / pq
        for ib in range(len(x)):
            valid(x[ib])[...] += dt(al) * valid(p[ib])
            r[ib] -= dt(al) * q[ib]
        it += 1
        rho_new = _dot(r, r)
        if math.sqrt(rho_new) <= tol * bnorm:
            break
        bt = rho_new / rho
        for ib in range(len(p)):
            valid(p[ib])[...] = r[ib] + dt(bt) * valid(p[ib])
        rho = rho_new
    if singular:
        m = dt(_mean([valid(v) for v in x]))
        for v in x:
            valid(v)[...] -= m
    return x, it


def bicgstab_bottom(lev, rhs, tol=1e-4, max_iter=None, singular=None):
    """Unpreconditioned BiCGStab on ``A x = rhs`` from x = 0: the bi-conjugate
    gradient member of the paper's native Krylov solvers ("CG and BiCG",
    "Linear Solvers"), used as the bottom solve.

    Stabilised BiCG with the shadow residual fixed at r^ = r_0.  Iteration i
    (rho_0 = alpha = omega = 1, p = v = 0 before the first):

        rho_i = (r^, r);   p = r + (rho_i / rho_{i-1}) (alpha / omega) (p - omega v)
        v = A p;           alpha = rho_i / (r^, v);   s = r - alpha v
        t = A s;           omega = (t, s) / (t, t)
        x = x + alpha p + omega s;   r = s - omega t

    Stops when ||r||_2 <= tol * ||rhs||_2, or earlier in an iteration when
    ||s||_2 is already there (x += alpha p), or after ``max_iter`` iterations
    (default: number of cells).  A zero rho_i or (r^, v) ends the solve with x
    as it stands; a zero (t, t) takes x += alpha p, r = s and ends it.  For a
    singular all-periodic problem the mean of rhs is removed first and the
    mean of x at the end (A maps onto mean-free fields there, so r, s, v and t
    stay mean-free).  Dot products accumulate in float64; vectors and the
    scalars applied to them are in the level's precision.  Returns (x with
    ghosts, iterations).
    """
    dt = lev.dtype
    if singular is None:
        singular = is_singular(lev)
    ncell = sum(int(np.prod(box_shape(b))) for b in lev.boxes)
    if max_iter is None:
        max_iter = ncell
    x = new_cell_data(lev)
    r = [np.array(v, dtype=dt, copy=True) for v in rhs]
    if singular:
        m = dt(_mean(r))
        r = [(v - m).astype(dt) for v in r]
    bnorm = math.sqrt(_dot(r, r))
    if bnorm == 0.0:
        return x, 0
    rh = [v.copy() for v in r]
    p = new_cell_data(lev)
    s = new_cell_data(lev)
    v = [np.zeros_like(w) for w in r]
    rho_prev, alpha, omega = 1.0, 1.0, 1.0
    it = 0
    while it < max_iter:
        rho = _dot(rh, r)
        if rho == 0.0:
            break
        beta = (rho / rho_prev) * (alpha / omega)
        for ib in range(len(p)):
            P = valid(p[ib])
            P[...] = r[ib] + dt(beta) * (P - dt(omega) * v[ib])
        v = apply_op(lev, p)
        rv = _dot(rh, v)
        if rv == 0.0:
            break
        alpha = rho / rv
        for ib in range(len(s)):
            valid(s[ib])[...] = r[ib] - dt(alpha) * v[ib]
        it += 1
        if not math.sqrt(_dot([valid(w) for w in s], [valid(w) for w in s])) > tol * bnorm:
            for ib in range(len(x)):
                valid(x[ib])[...] += dt(alpha) * valid(p[ib])
            break
        t = apply_op(lev, s)
        tt = _dot(t, t)
        if tt == 0.0:
            for ib in range(len(x)):
                valid(x[ib])[...] += dt(alpha) * valid(p[ib])
            break
        omega = _dot(t, [valid(w) for w in s]) / tt
        for ib in range(len(x)):
            X = valid(x[ib])
            X[...] = (X + dt(alpha) * valid(p[ib])) + dt(omega) * valid(s[ib])
            r[ib] = valid(s[ib]) - dt(omega) * t[ib]
        if not math.sqrt(_dot(r, r)) > tol * bnorm:
            break
        if omega == 0.0:
            break
        rho_prev = rho
    if singular:
        m = dt(_mean([valid(w) for w in x]))
        for w in x:
            valid(w)[...] -= m
    return x, it


BOTTOM_SOLVERS = {"cg": cg_bottom, "bicgstab": bicgstab_bottom}


@dataclass
class Opts:
    nu1: int = 2
    nu2: int = 2
    max_iter: int = 100
    bottom_tol: float = 1e-4
    bottom_max_iter: int = None
    # "cg" or "bicgstab"
    bottom_solver: str = "cg"
    min_bottom_edge: int = 4
    aggregate: bool = False
    # post-smoothing in black-then-red order on every level, which makes the
    # V-cycle (from a zero guess, exact bottom solve, nu1 = nu2) a symmetric
    # operator: the preconditioner of pcg_solve
    symmetric: bool = False


def vcycle(levels, l, phi, f, opts, stats=None):
    """V(l, phi, f): nu1 pre-smoothing sweeps, residual, restrict, recurse on a zero
    coarse guess, add the interpolated correction, nu2 post-smoothing sweeps; the
    bottom level is solved by CG (or BiCGStab) on its residual equation."""
    lev = levels[l]
    if l == len(levels) - 1:
        r = residual(lev, phi, f)
        e, its = BOTTOM_SOLVERS[opts.bottom_solver](lev, r, opts.bottom_tol, opts.bottom_max_iter)
        for ib in range(len(phi)):
            valid(phi[ib])[...] += valid(e[ib])
        if stats is not None:
            stats.setdefault("bottom_iters", []).append(its)
        return
    for _ in range(opts.nu1):
        gsrb_halfsweep(lev, phi, f, 0)
        gsrb_halfsweep(lev, phi, f, 1)
    r = residual(lev, phi, f)
    fc = restrict(lev, r, levels[l + 1])
    ec = new_cell_data(levels[l + 1])
    vcycle(levels, l + 1, ec, fc, opts, stats)
    prolong_add(phi, ec, lev, levels[l + 1])
    first, second = (1, 0) if opts.symmetric else (0, 1)
    for _ in range(opts.nu2):
        gsrb_halfsweep(lev, phi, f, first)
        gsrb_halfsweep(lev, phi, f, second)


def max_norm(u):
    return float(max(np.max(np.abs(x)) for x in u))


def build_levels(lev0, min_bottom_edge=4, aggregate=False):
    """Level 0 plus its coarsened copies, following ``boxes.mg_hierarchy``'s rule."""
    from .boxes import mg_hierarchy
    hier = mg_hierarchy(lev0.boxes, lev0.domain, min_bottom_edge, aggregate)
    levels = [lev0]
    for (_, _, merged) in hier[1:]:
        levels.append(coarsen_level(levels[-1], merged))
    return levels


def solve(lev0, phi, f, rel_tol=1e-10, abs_tol=0.0, opts=None, levels=None):
    """Iterate V-cycles on level 0 until max|f - A phi| <= max(rel_tol*max|f|, abs_tol).

    ``phi`` (per-box arrays with one ghost layer) is the initial guess and is
    updated in place.  Returns a dict with the per-cycle max-norm residual
    history (entry k is the residual after k cycles), the cycle count and
    whether the tolerance was met.  For a singular all-periodic problem the
    returned phi has its mean removed.
    """
    opts = opts or Opts()
    if levels is None:
        levels = build_levels(lev0, opts.min_bottom_edge, opts.aggregate)
    normf = max_norm(f)
    info = {"history": [], "iters": 0, "converged": False, "bottom_iters": [],
            "nlevels": len(levels)}
    if normf == 0.0:
        for v in phi:
            v[...] = 0.0
        info["converged"] = True
        return info
    tol = max(rel_tol * normf, abs_tol)
    it = 0
    while True:
        rn = max_norm(residual(lev0, phi, f))
        info["history"].append(rn)
        if not np.isfinite(rn):
            break
        if rn <= tol:
            info["converged"] = True
            break
        if it == opts.max_iter:
            break
        vcycle(levels, 0, phi, f, opts, info)
        it += 1
    info["iters"] = it
    info["normf"] = normf
    if is_singular(lev0):
        m = _mean([valid(v) for v in phi])
        for v in phi:
            valid(v)[...] -= m
    return info


def solve_refine(lev0, phi, f, rel_tol=1e-10, abs_tol=0.0, opts=None, inner_dtype=np.float64,
                 levels=None):
    """Iterative refinement: float64 residual, one V-cycle in ``inner_dtype`` on the
    residual equation from a zero guess, float64 update.

    With ``inner_dtype`` float64 the iterates equal those of ``solve`` in exact
    arithmetic (Gauss-Seidel commutes with the shift phi = phi_k + e).  The
    coefficient hierarchy is coarsened in float64 and then rounded.
    """
    opts = opts or Opts()
    if levels is None:
        levels = build_levels(lev0, opts.min_bottom_edge, opts.aggregate)
    inner = [cast_level(L, inner_dtype) for L in levels]
    normf = max_norm(f)
    info = {"history": [], "iters": 0, "converged": False, "bottom_iters": [],
            "nlevels": len(levels)}
    if normf == 0.0:
        for v in phi:
            v[...] = 0.0
        info["converged"] = True
        return info
    tol = max(rel_tol * normf, abs_tol)
    it = 0
    while True:
        r = residual(lev0, phi, f)
        rn = max_norm(r)
        info["history"].append(rn)
        if not np.isfinite(rn):
            break
        if rn <= tol:
            info["converged"] = True
            break
        if it == opts.max_iter:
            break
        r_in = [x.astype(inner_dtype) for x in r]
        e = new_cell_data(inner[0], dtype=inner_dtype)
        vcycle(inner, 0, e, r_in, opts, info)
        for ib in range(len(phi)):
            valid(phi[ib])[...] += valid(e[ib]).astype(np.float64)
        it += 1
    info["iters"] = it
    info["normf"] = normf
    if is_singular(lev0):
        m = _mean([valid(v) for v in phi])
        for v in phi:
            valid(v)[...] -= m
    return info


def vcycle_precond(levels, r, opts):
    """z = M r: one V-cycle on A z = r from z = 0, in the precision of
    ``levels`` (r rounded to it, z returned in float64); mean removed for a
    singular all-periodic problem."""
    dt = levels[0].dtype
    z = new_cell_data(levels[0], dtype=dt)
    vcycle(levels, 0, z, [x.astype(dt) for x in r], opts)
    z = [x.astype(np.float64) for x in z]
    if is_singular(levels[0]):
        m = _mean([valid(v) for v in z])
        for v in z:
            valid(v)[...] -= m
    return z


def pcg_solve(lev0, phi, f, rel_tol=1e-10, abs_tol=0.0, opts=None, levels=None, precond=None,
              inner_dtype=np.float64):
    """Preconditioned conjugate gradients on A phi = f (the paper's Krylov CG
    with its multigrid as preconditioner; "Linear Solvers").

    Default preconditioner: one symmetric V-cycle from a zero guess
    (``opts.symmetric`` is forced on), run in ``inner_dtype`` on a copy of the
    hierarchy coarsened in float64 and then rounded (float32: the mixed
    precision of ``solve_refine`` with CG as the outer loop).
    ``precond(r) -> z`` replaces it (identity gives plain CG).  From r = f - A phi, z = M r, p = z, rho = r.z,
    each iteration: q = A p, alpha = rho / p.q, phi += alpha p, r -= alpha q;
    stop when max|r| <= tol (tol as in ``solve``), confirmed on the true
    residual f - A phi (if that is still above tol, r is replaced by it and the
    recurrence restarts with p = M r); else z = M r, rho' = r.z,
    p = z + (rho'/rho) p.  Dots accumulate in float64.  For a singular
    all-periodic problem the mean is taken out of r at the start and of phi at
    the end.  Returns a dict like ``solve``: history[k] = max|r| after k
    iterations, iters, converged.
    """
    opts = opts or Opts()
    opts = Opts(**{**opts.__dict__, "symmetric": True})
    if levels is None:
        levels = build_levels(lev0, opts.min_bottom_edge, opts.aggregate)
    if precond is None:
        inner = levels if inner_dtype == np.float64 else [cast_level(L, inner_dtype) for L in levels]

        def precond(r):
            return vcycle_precond(inner, r, opts)
    singular = is_singular(lev0)
    normf = max_norm(f)
    info = {"history": [], "iters": 0, "converged": False, "nlevels": len(levels),
            "restarts": 0}
    if normf == 0.0:
        for v in phi:
            v[...] = 0.0
        info["converged"] = True
        return info
    tol = max(rel_tol * normf, abs_tol)

    def true_residual():
        r = residual(lev0, phi, f)
        if singular:
            m = _mean(r)
            r = [x - m for x in r]
        return r

    r = true_residual()
    it = 0
    p = rho = None
    while True:
        rn = max_norm(r)
        info["history"].append(rn)
        if not np.isfinite(rn):
            break
        if rn <= tol:
            rt = true_residual()
            if max_norm(rt) <= tol:
                info["converged"] = True
                break
            r = rt
            p = None
            info["restarts"] += 1
        if it == opts.max_iter:
            break
        z = precond(r)
        rho_new = _dot(r, [valid(v) for v in z])
        if p is None:
            p = [np.array(v, copy=True) for v in z]
        else:
            bt = rho_new / rho
            for ib in range(len(p)):
                valid(p[ib])[...] = valid(z[ib]) + bt * valid(p[ib])
        rho = rho_new
        q = apply_op(lev0, p)
        pq = _dot([valid(v) for v in p], q)
        al = rho / pq
        for ib in range(len(phi)):
            valid(phi[ib])[...] += al * valid(p[ib])
            r[ib] = r[ib] - al * q[ib]
        it += 1
    info["iters"] = it
    info["normf"] = normf
    if singular:
        m = _mean([valid(v) for v in phi])
        for v in phi:
            valid(v)[...] -= m
    return info
