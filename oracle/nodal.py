"""Node-centred variable-coefficient Poisson operator from finite elements, and
its multigrid solve.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's "Linear Solvers" section says that the nodal solver is built on a
finite-element approach, that its stencil comes from pre-computed moment
integrals over the cells, and that its coarse operators come from an
algebraic coarsening.  Written out:

* Unknowns phi at the nodes of the cell grid of the unit cube (n_d cells along
  d, h_d = 1 / n_d, node i at x_d = i h_d); sigma is one positive value per cell.
* phi is the continuous piecewise-trilinear function with these nodal values.
  The equation is the Galerkin form of -div(sigma grad phi) = f tested with
  every nodal hat function N_p, with the right-hand side lumped to the node
  (f_p times the cell volume V = h_x h_y h_z) and the whole row divided by V:

      (A phi)_p = (1/V) sum_{cells c at p} sigma_c sum_{corners q of c} K_pq phi_q.

  K is the stiffness of one trilinear cell, assembled from the moment
  integrals of the 1D linear functions l_0 = 1 - t, l_1 = t over a cell of
  width h: int l_a l_b = h/3 (a = b) or h/6; int l_a' l_b' = 1/h (a = b) or
  -1/h.  For corners a, b in {0, 1}^3:

      K_ab = sum_d k_d(a_d, b_d) prod_{e != d} m_e(a_e, b_e).

* Walls are homogeneous Dirichlet: the nodes on a wall face hold 0 and are not
  unknowns.  A periodic direction wraps (node n_d is node 0).

Readings taken where the paper gives no detail:

* levels: halve the cell count along every direction while all of them stay
  even and half of each is >= min_bottom_cells;
* interpolation P: trilinear (a coarse node's value at its fine node, the mean
  of the two coarse neighbours at a fine node between them, per direction);
  restriction R = P^T V_f / V_c = P^T / 8 (full weighting);
* coarse operator A_c = R A P (the Galerkin product: the algebraic coarsening),
  kept as 27 coefficients per node.  The coefficient of the coupling from node
  I to node I + o is computed for the 14 offsets o >= 0 in (z, y, x)
  lexicographic order and mirrored for the other 13 (A_c[I, -o] =
  A_c[I - o, o]), so every coarse operator is exactly symmetric;
* smoother: Jacobi, phi <- phi + omega (f - A phi) / diag (the 27-point
  couplings admit no red/black colouring), nu1 = nu2 = 2 sweeps, omega = 1:
  for the trilinear stencil the high-frequency eigenvalues of diag^-1 A lie
  in [1/2, 3/2] (1/2 at the (pi, pi, pi) mode, 3/2 at (pi, 0, 0)), so
  omega = 2 / (1/2 + 3/2) = 1 is the damping that smooths best (factor 1/2);
* bottom: unpreconditioned CG from zero, stopped on the 2-norm relative to the
  bottom right-hand side (the mean projected out when every direction is
  periodic, as for the cell-centred solver);
* stop test: max norm of f - A phi over the unknowns relative to max |f|.

Arrays hold the unknowns only, indexed [i, j, k] (x first): shape n_d - 1
along a Dirichlet direction (global nodes 1 .. n_d - 1) and n_d along a
periodic one (global nodes 0 .. n_d - 1).
"""

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

# the 27 offsets in (z, y, x) lexicographic order, and the 14 that are >= 0
OFFSETS = [(ox, oy, oz) for oz in (-1, 0, 1) for oy in (-1, 0, 1) for ox in (-1, 0, 1)]
UPPER = [o for o in OFFSETS if (o[2], o[1], o[0]) >= (0, 0, 0)]
CORNERS = [(ax, ay, az) for az in (0, 1) for ay in (0, 1) for ax in (0, 1)]


@dataclass
class NodalLevel:
    n: tuple                 # cells per direction
    periodic: tuple
    h: tuple
    sigma: np.ndarray = None  # cell coefficient (finest level only)
    w: dict = field(default=None, repr=False)  # offset -> coefficient array over the unknowns

    @property
    def m(self):
        return unknown_shape(self.n, self.periodic)


def unknown_shape(n, periodic):
    return tuple(n[d] if periodic[d] else n[d] - 1 for d in range(3))


def element_matrix(h):
    """K_ab of one trilinear cell (8 x 8, corners in CORNERS order) from the
    1D moment integrals."""
    def m1(hd, a, b):
        return hd / 3.0 if a == b else hd / 6.0

    def k1(hd, a, b):
        return 1.0 / hd if a == b else -1.0 / hd

    K = np.zeros((8, 8))
    for ia, a in enumerate(CORNERS):
        for ib, b in enumerate(CORNERS):
            s = 0.0
            for d in range(3):
                t = k1(h[d], a[d], b[d])
                for e in range(3):
                    if e != d:
                        t *= m1(h[e], a[e], b[e])
                s += t
            K[ia, ib] = s
    return K


def shift(U, o, periodic):
    """V[u] = U[u + o] for every unknown u: wrapped along a periodic direction,
    0 past a wall (the wall node's value)."""
    V = U
    for d in range(3):
        if o[d] == 0:
            continue
        if periodic[d]:
            V = np.roll(V, -o[d], axis=d)
        else:
            W = np.zeros_like(V)
            sl_dst = [slice(None)] * 3
            sl_src = [slice(None)] * 3
            if o[d] > 0:
                sl_dst[d] = slice(0, V.shape[d] - o[d])
                sl_src[d] = slice(o[d], None)
            else:
                sl_dst[d] = slice(-o[d], None)
                sl_src[d] = slice(0, V.shape[d] + o[d])
            W[tuple(sl_dst)] = V[tuple(sl_src)]
            V = W
    return V


def _cells_at(sigma, s, periodic, m):
    """sigma of the cell at corner offset s in {0, 1}^3 of every unknown node:
    the cell whose low corner is node (global) g - 1 + s."""
    out = sigma
    for d in range(3):
        if periodic[d]:
            # unknown u = global node u; cell u - 1 + s_d, wrapped
            out = np.roll(out, 1 - s[d], axis=d)
            sl = [slice(None)] * 3
            sl[d] = slice(0, m[d])
            out = out[tuple(sl)]
        else:
            # unknown u = global node u + 1; cell u + s_d
            sl = [slice(None)] * 3
            sl[d] = slice(s[d], s[d] + m[d])
            out = out[tuple(sl)]
    return out


def make_nodal_level(sigma, periodic, h=None):
    """Finest level from the cell coefficient (n_x, n_y, n_z); cell widths h
    (default: the unit cube, h_d = 1 / n_d)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    n = sigma.shape
    h = tuple(1.0 / n[d] for d in range(3)) if h is None else tuple(float(x) for x in h)
    lev = NodalLevel(tuple(n), tuple(bool(p) for p in periodic), h, sigma)
    lev.w = fine_weights(lev)
    return lev


def fine_weights(lev):
    """The 27 coefficients of the finest level at every unknown node: for each
    of the 8 cells at the node (corner offset s, the node being corner 1 - s of
    the cell) and each corner b of that cell, sigma_c K_{1-s, b} / V goes to the
    coupling with offset b - (1 - s)."""
    K = element_matrix(lev.h)
    V = lev.h[0] * lev.h[1] * lev.h[2]
    m = lev.m
    w = {o: np.zeros(m) for o in OFFSETS}
    for s in CORNERS:
        sig = _cells_at(lev.sigma, s, lev.periodic, m)
        a = tuple(1 - s[d] for d in range(3))
        ia = CORNERS.index(a)
        for ib, b in enumerate(CORNERS):
            o = tuple(b[d] - a[d] for d in range(3))
            w[o] = w[o] + sig * (K[ia, ib] / V)
    return w


def apply_nodal(lev, phi):
    """A phi at every unknown: sum over the 27 offsets (OFFSETS order)."""
    out = np.zeros(lev.m)
    for o in OFFSETS:
        out = out + lev.w[o] * shift(phi, o, lev.periodic)
    return out


def nodal_residual(lev, phi, f):
    return f - apply_nodal(lev, phi)


def jacobi(lev, phi, f, omega, zero_guess=False):
    """One damped Jacobi sweep: phi + omega (f - A phi) / diag (from phi = 0:
    omega f / diag)."""
    d = lev.w[(0, 0, 0)]
    if zero_guess:
        return omega * f / d
    return phi + omega * (f - apply_nodal(lev, phi)) / d


def coarsen_n(n):
    return tuple(x // 2 for x in n)


def nodal_levels_n(n, periodic, min_bottom_cells=8):
    """Cell counts of the levels: halve while every count is even and half of
    it is >= min_bottom_cells."""
    out = [tuple(n)]
    while all(x % 2 == 0 and x // 2 >= min_bottom_cells for x in out[-1]):
        out.append(coarsen_n(out[-1]))
    return out


def _fine_index(lev_f, lev_c, d, u):
    """Fine unknown index along d of fine node 2 G + u (G the global coarse
    node of each coarse unknown), wrapped along a periodic direction."""
    mc, mf = lev_c.m[d], lev_f.m[d]
    off = 0 if lev_f.periodic[d] else 1
    idx = 2 * np.arange(mc) + off + u
    return idx % mf


def _fine_at(W, lev_f, lev_c, u):
    ix = [_fine_index(lev_f, lev_c, d, u[d]) for d in range(3)]
    return W[np.ix_(ix[0], ix[1], ix[2])]


def _pw(t):
    """1D interpolation weight of a coarse node at fine distance t."""
    return 1.0 if t == 0 else (0.5 if abs(t) == 1 else 0.0)


def galerkin(lev_f):
    """Next coarser level: A_c = R A_f P with R = P^T / 8, for the 14 upper
    offsets; the lower 13 mirrored.

    A_c[I, o] = 1/8 sum_u r(u) sum_v A_f[2I+u, 2I+u+v] P[2I+u+v, I+o], where
    u, v run over {-1, 0, 1}^3, r(u) = P[2I+u, I] = prod_d w(u_d) and
    P[2I+u+v, I+o] = prod_d w(u_d + v_d - 2 o_d) with w(0) = 1, w(+-1) = 1/2.
    """
    nc = coarsen_n(lev_f.n)
    lev_c = NodalLevel(nc, lev_f.periodic, tuple(2.0 * x for x in lev_f.h))
    w = {}
    for o in UPPER:
        acc = np.zeros(lev_c.m)
        for u in OFFSETS:
            ru = _pw(u[0]) * _pw(u[1]) * _pw(u[2])
            for v in OFFSETS:
                p = _pw(u[0] + v[0] - 2 * o[0]) * _pw(u[1] + v[1] - 2 * o[1]) * \
                    _pw(u[2] + v[2] - 2 * o[2])
                if p == 0.0:
                    continue
                acc = acc + (ru * p) * _fine_at(lev_f.w[v], lev_f, lev_c, u)
        w[o] = acc * 0.125
    for o in UPPER:
        if o == (0, 0, 0):
            continue
        mo = (-o[0], -o[1], -o[2])
        w[mo] = shift(w[o], mo, lev_c.periodic)
    lev_c.w = w
    return lev_c


def restrict_nodal(lev_f, lev_c, r_f):
    """r_c(I) = 1/8 sum_u r(u) r_f(2I + u): full weighting, R = P^T / 8."""
    out = np.zeros(lev_c.m)
    for u in OFFSETS:
        ru = _pw(u[0]) * _pw(u[1]) * _pw(u[2])
        out = out + ru * _fine_at(r_f, lev_f, lev_c, u)
    return out * 0.125


def _global_nodes(U, periodic):
    """All nodes 0 .. n_d of a level from its unknowns (0 on walls, node n_d =
    node 0 along a periodic direction)."""
    G = U
    for d in range(3):
        if periodic[d]:
            first = [slice(None)] * 3
            first[d] = slice(0, 1)
            G = np.concatenate([G, G[tuple(first)]], axis=d)
        else:
            shp = list(G.shape)
            shp[d] = 1
            z = np.zeros(shp)
            G = np.concatenate([z, G, z], axis=d)
    return G


def _unknowns(G, periodic):
    sl = []
    for d in range(3):
        n = G.shape[d] - 1
        sl.append(slice(0, n) if periodic[d] else slice(1, n))
    return G[tuple(sl)]


def interp_add(lev_f, lev_c, phi_f, e_c):
    """phi_f + P e_c, P trilinear: along each direction in turn, even fine node
    2G takes coarse node G and odd node 2G + 1 the mean of G and G + 1."""
    E = _global_nodes(e_c, lev_c.periodic)
    for d in range(3):
        nc = E.shape[d] - 1
        shp = list(E.shape)
        shp[d] = 2 * nc + 1
        F = np.zeros(shp)
        ev = [slice(None)] * 3
        ev[d] = slice(0, 2 * nc + 1, 2)
        F[tuple(ev)] = E
        od = [slice(None)] * 3
        od[d] = slice(1, 2 * nc, 2)
        lo = [slice(None)] * 3
        lo[d] = slice(0, nc)
        hi = [slice(None)] * 3
        hi[d] = slice(1, nc + 1)
        F[tuple(od)] = 0.5 * (E[tuple(lo)] + E[tuple(hi)])
        E = F
    return phi_f + _unknowns(E, lev_f.periodic)


def is_singular_nodal(lev):
    return all(lev.periodic)


def nodal_cg_bottom(lev, rhs, tol=1e-4, max_iter=None):
    """Unpreconditioned CG on A x = rhs from x = 0, stopped at ||r||_2 <= tol
    ||rhs||_2 or after max_iter (default: number of unknowns) iterations.  All
    periodic (singular): the mean is removed from rhs first and from x at the
    end.  Returns (x, iterations)."""
    b = rhs.astype(np.float64)
    if is_singular_nodal(lev):
        b = b - b.mean()
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = float(np.sum(r * r))
    nb = math.sqrt(float(np.sum(b * b)))
    limit = max_iter if max_iter is not None else b.size
    it = 0
    if nb == 0.0:
        return x, 0
    while it < limit and math.sqrt(rr) > tol * nb:
        q = apply_nodal(lev, p)
        alpha = rr / float(np.sum(p * q))
        x = x + alpha * p
        r = r - alpha * q
        rr_new = float(np.sum(r * r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    if is_singular_nodal(lev):
        x = x - x.mean()
    return x, it


@dataclass
class NodalOpts:
    nu1: int = 2
    nu2: int = 2
    omega: float = 1.0
    max_iter: int = 100
    bottom_tol: float = 1e-4
    bottom_max_iter: int = None
    min_bottom_cells: int = 8


def build_nodal_levels(sigma, periodic, opts=None):
    opts = opts or NodalOpts()
    levs = [make_nodal_level(sigma, periodic)]
    for _ in nodal_levels_n(levs[0].n, periodic, opts.min_bottom_cells)[1:]:
        levs.append(galerkin(levs[-1]))
    return levs


def nodal_vcycle(levs, l, phi, f, opts, zero_guess=False):
    """One V-cycle on level l (direct form; coarse levels solve for the
    correction from zero).  Returns the new phi."""
    lev = levs[l]
    if l + 1 == len(levs):
        x, _ = nodal_cg_bottom(lev, f, opts.bottom_tol, opts.bottom_max_iter)
        return x
    for k in range(opts.nu1):
        phi = jacobi(lev, phi, f, opts.omega, zero_guess and k == 0)
    if opts.nu1 == 0 and zero_guess:
        phi = np.zeros(lev.m)
    r = nodal_residual(lev, phi, f)
    rc = restrict_nodal(lev, levs[l + 1], r)
    ec = nodal_vcycle(levs, l + 1, None, rc, opts, zero_guess=True)
    phi = interp_add(lev, levs[l + 1], phi, ec)
    for _ in range(opts.nu2):
        phi = jacobi(lev, phi, f, opts.omega)
    return phi


def nodal_solve(sigma, periodic, f, rel_tol=1e-10, abs_tol=0.0, opts=None, phi0=None,
                levs=None):
    """V-cycles from phi0 (default 0) until max|f - A phi| <= max(rel_tol max|f|,
    abs_tol).  All periodic: phi's mean is removed at the end.  Returns (phi,
    info) with the max-norm history."""
    opts = opts or NodalOpts()
    levs = levs or build_nodal_levels(sigma, periodic, opts)
    lev = levs[0]
    f = np.asarray(f, dtype=np.float64)
    phi = np.zeros(lev.m) if phi0 is None else np.array(phi0, dtype=np.float64)
    normf = float(np.max(np.abs(f)))
    info = {"iters": 0, "history": [], "converged": False, "normf": normf,
            "nlevels": len(levs)}
    if normf == 0.0:
        info["converged"] = True
        return np.zeros(lev.m), info
    tol = max(rel_tol * normf, abs_tol)
    it = 0
    while True:
        rn = float(np.max(np.abs(nodal_residual(lev, phi, f))))
        info["history"].append(rn)
        if rn <= tol:
            info["converged"] = True
            break
        if it == opts.max_iter:
            break
        phi = nodal_vcycle(levs, 0, phi, f, opts)
        it += 1
    if is_singular_nodal(lev):
        phi = phi - phi.mean()
    info["iters"] = it
    return phi, info


def nodal_precond(levs, r, opts):
    """One V-cycle from a zero guess on the finest level: z = M r.  With
    nu1 = nu2 the cycle is a symmetric operator (a Jacobi sweep is
    self-adjoint in the energy inner product, the coarse correction
    P (R A P)^-1 R with R = P^T / 8 is symmetric)."""
    return nodal_vcycle(levs, 0, None, r, opts, zero_guess=True)


def nodal_pcg_solve(sigma, periodic, f, rel_tol=1e-10, abs_tol=0.0, opts=None, phi0=None,
                    levs=None, precond=None):
    """Conjugate gradients on A phi = f preconditioned by one V-cycle per
    iteration (the paper's Krylov CG with its multigrid as preconditioner).

    From r = f - A phi: z = M r, rho = r.z, p = z (then p = z + (rho/rho_old)
    p), q = A p, alpha = rho / p.q, phi += alpha p, r -= alpha q.  Stop when
    max|r| <= max(rel_tol max|f|, abs_tol), confirmed on the true residual f -
    A phi; if that is above the tolerance, r is replaced by it and the
    recurrence restarts from p = M r.  Dots are float64 sums.  All periodic:
    the mean is taken out of r at the start and after a restart, out of every
    z, and out of phi at the end.  ``precond(r) -> z`` replaces the V-cycle
    (the identity gives plain CG).  Returns (phi, info) with info["history"][k]
    = max|r| after k iterations."""
    opts = opts or NodalOpts()
    levs = levs or build_nodal_levels(sigma, periodic, opts)
    lev = levs[0]
    singular = is_singular_nodal(lev)
    if precond is None:
        def precond(r):
            return nodal_precond(levs, r, opts)
    f = np.asarray(f, dtype=np.float64)
    phi = np.zeros(lev.m) if phi0 is None else np.array(phi0, dtype=np.float64)
    normf = float(np.max(np.abs(f)))
    info = {"iters": 0, "history": [], "converged": False, "normf": normf,
            "nlevels": len(levs), "restarts": 0}
    if normf == 0.0:
        info["converged"] = True
        return np.zeros(lev.m), info
    tol = max(rel_tol * normf, abs_tol)

    def true_residual():
        r = nodal_residual(lev, phi, f)
        return r - r.mean() if singular else r

    r = true_residual()
    p = None
    rho = None
    it = 0
    while True:
        rn = float(np.max(np.abs(r)))
        info["history"].append(rn)
        if not np.isfinite(rn):
            break
        if rn <= tol:
            rt = true_residual()
            if float(np.max(np.abs(rt))) <= tol:
                info["converged"] = True
                break
            r = rt
            p = None
            info["restarts"] += 1
        if it == opts.max_iter:
            break
        z = precond(r)
        if singular:
            z = z - z.mean()
        rho_new = float(np.sum(r * z))
        p = z.copy() if p is None else z + (rho_new / rho) * p
        rho = rho_new
        q = apply_nodal(lev, p)
        alpha = rho / float(np.sum(p * q))
        phi = phi + alpha * p
        r = r - alpha * q
        it += 1
    if singular:
        phi = phi - phi.mean()
    info["iters"] = it
    return phi, info
