"""Independent global-array formulations used to pin the oracle.

Nothing here uses boxes, ghost exchange or the oracle's folded stencil: the
operator is written in flux form on one global array padded with explicit ghost
values (wrapped copies for periodic directions, phi_ghost = -phi_inside for a
homogeneous Dirichlet wall, the linear-extrapolation reading of phi = 0 on the
wall).
"""

import numpy as np


def pad_ghosts(u, periodic, xp=np):
    """One ghost layer around a global (n0, n1, n2) array (batched over leading dims)."""
    nd = u.ndim
    for d in range(3):
        ax = nd - 3 + d
        n = u.shape[ax]
        lo_idx = [slice(None)] * nd
        hi_idx = [slice(None)] * nd
        if periodic[d]:
            lo_idx[ax] = slice(n - 1, n)
            hi_idx[ax] = slice(0, 1)
            lo = u[tuple(lo_idx)]
            hi = u[tuple(hi_idx)]
        else:
            lo_idx[ax] = slice(0, 1)
            hi_idx[ax] = slice(n - 1, n)
            lo = -u[tuple(lo_idx)]
            hi = -u[tuple(hi_idx)]
        u = xp.concatenate([lo, u, hi], axis=ax)
    return u


def apply_global(u, faces, alpha, beta, h, periodic, acell=None, xp=np):
    """(A u) = alpha a u - beta sum_d [b_hi (u_hi - u) - b_lo (u - u_lo)] / h_d^2."""
    P = pad_ghosts(u, periodic, xp)
    nd = u.ndim
    core = tuple([slice(None)] * (nd - 3) + [slice(1, -1)] * 3)
    out = alpha * (u if acell is None else acell * u)
    for d in range(3):
        ax = nd - 3 + d
        n = u.shape[ax]
        s_lo = [slice(None)] * (nd - 3) + [slice(1, -1)] * 3
        s_hi = list(s_lo)
        s_lo[ax] = slice(0, n)
        s_hi[ax] = slice(2, n + 2)
        f_lo = [slice(None)] * 3
        f_hi = [slice(None)] * 3
        f_lo[d] = slice(0, n)
        f_hi[d] = slice(1, n + 1)
        blo = faces[d][tuple(f_lo)]
        bhi = faces[d][tuple(f_hi)]
        flux = bhi * (P[tuple(s_hi)] - P[core]) - blo * (P[core] - P[tuple(s_lo)])
        out = out - beta * flux / (h[d] * h[d])
    return out


def assemble(n, faces, alpha, beta, periodic, acell=None):
    """Dense matrix of the operator on an n^3 grid (unknown index = C order of [i, j, k])."""
    N = n ** 3
    h = (1.0 / n,) * 3
    E = np.eye(N).reshape(N, n, n, n)
    cols = apply_global(E, faces, alpha, beta, h, periodic, acell)
    return cols.reshape(N, N).T.copy()
