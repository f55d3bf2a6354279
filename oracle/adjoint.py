"""Adjoint gradient of a quadratic loss through the solve.

TEST INFRASTRUCTURE ONLY (see the package docstring).

With A(b) phi = f for the operator of the paper's "Linear Solvers" section and
L = 1/2 sum_cells (phi - phi_t)^2, the adjoint state is lambda = A^{-T}
(phi - phi_t) = A^{-1} (phi - phi_t) (A is symmetric with the folded Dirichlet
wall), dL/df = lambda and dL/db_f = -lambda^T (dA/db_f) phi.  A face coefficient
enters A only through c_f = beta b_f / h_d^2:

* interior or periodic face between cells i and j adds c_f (e_i - e_j)(e_i - e_j)^T,
  so dL/db_f = -beta (phi_j - phi_i)(lambda_j - lambda_i) / h_d^2;
* a Dirichlet wall face next to cell i adds 2 c_f e_i e_i^T,
  so dL/db_f = -2 beta phi_i lambda_i / h_d^2.

dL/dlog b_f = b_f dL/db_f.  The parameters are one value per physical face:
global face arrays of shape (n_x+1, n_y, n_z), (n_x, n_y+1, n_z),
(n_x, n_y, n_z+1); in a periodic direction faces 0 and n are the same face and
both entries carry its gradient.
"""

import numpy as np

from .boxes import box_shape


def gather_cells(lev, data, ng=1):
    """Valid cells of per-box arrays into one global array."""
    n = box_shape(lev.domain)
    dlo = lev.domain[0]
    G = np.zeros(n, dtype=np.float64)
    for bx, arr in zip(lev.boxes, data):
        lo, hi = bx
        v = arr[ng:-ng, ng:-ng, ng:-ng] if ng > 0 else arr
        G[lo[0] - dlo[0]:hi[0] - dlo[0] + 1, lo[1] - dlo[1]:hi[1] - dlo[1] + 1,
          lo[2] - dlo[2]:hi[2] - dlo[2] + 1] = v
    return G


def gather_faces(lev, d):
    """Per-box face arrays of direction d into one global face array."""
    n = list(box_shape(lev.domain))
    dlo = lev.domain[0]
    n[d] += 1
    G = np.zeros(n, dtype=np.float64)
    for bx, arr in zip(lev.boxes, lev.b[d]):
        lo = bx[0]
        sl = tuple(slice(lo[a] - dlo[a], lo[a] - dlo[a] + arr.shape[a]) for a in range(3))
        G[sl] = arr
    return G


def loss(phi_cells, phi_t_cells):
    """L = 1/2 sum (phi - phi_t)^2 over all cells (plain sum, no cell volume)."""
    d = phi_cells - phi_t_cells
    return 0.5 * float(np.sum(d * d))


def grad_logb(lev, phi, lam, ng=1):
    """dL/dlog b on every physical face, from the solution and adjoint state.

    ``phi`` and ``lam`` are per-box arrays with ``ng`` ghost layers.  Returns a
    list of three global face arrays.
    """
    P = gather_cells(lev, phi, ng)
    Lm = gather_cells(lev, lam, ng)
    out = []
    for d in range(3):
        B = gather_faces(lev, d)
        inv_h2 = 1.0 / (lev.h[d] * lev.h[d])
        n = P.shape[d]
        g = np.zeros_like(B)
        sl = lambda a, b_: tuple(slice(a, b_) if x == d else slice(None) for x in range(3))  # noqa: E731
        # interior faces 1..n-1 lie between cells k-1 and k
        dP = P[sl(1, n)] - P[sl(0, n - 1)]
        dL = Lm[sl(1, n)] - Lm[sl(0, n - 1)]
        g[sl(1, n)] = -lev.beta * dP * dL * inv_h2
        if lev.periodic[d]:
            dPw = P[sl(0, 1)] - P[sl(n - 1, n)]
            dLw = Lm[sl(0, 1)] - Lm[sl(n - 1, n)]
            gw = -lev.beta * dPw * dLw * inv_h2
            g[sl(0, 1)] = gw
            g[sl(n, n + 1)] = gw
        else:
            g[sl(0, 1)] = -2.0 * lev.beta * P[sl(0, 1)] * Lm[sl(0, 1)] * inv_h2
            g[sl(n, n + 1)] = -2.0 * lev.beta * P[sl(n - 1, n)] * Lm[sl(n - 1, n)] * inv_h2
        out.append(g * B)
    return out
