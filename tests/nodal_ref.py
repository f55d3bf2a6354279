"""Independent sparse assembly of the nodal finite-element operator, for the
oracle's pins (test code; shares nothing with oracle/nodal.py).

Each cell's stiffness is integrated with the 2-point Gauss rule per direction
(exact for the products of trilinear gradients) from the trilinear shape
functions themselves; the row of a node is divided by the cell volume (the
lumped mass).  The interpolation matrix evaluates the coarse trilinear hat
functions at the fine nodes' coordinates.
"""

import itertools

import numpy as np
import scipy.sparse as sp


def _node_ids(n, periodic):
    """Global node (i, j, k), 0 <= i <= n_d, -> unknown id or -1 (wall node)."""
    m = [n[d] if periodic[d] else n[d] - 1 for d in range(3)]

    def uid(g):
        u = []
        for d in range(3):
            x = g[d]
            if periodic[d]:
                x %= n[d]
            else:
                if x == 0 or x == n[d]:
                    return -1
                x -= 1
            u.append(x)
        return u[0] + m[0] * (u[1] + m[1] * u[2])
    return m, uid


def _shape_grad(a, xi):
    """Gradient (in reference coordinates on [0,1]^3) of the trilinear shape
    function of corner a at point xi."""
    def l(ad, t):
        return t if ad == 1 else 1.0 - t

    def dl(ad):
        return 1.0 if ad == 1 else -1.0
    g = np.empty(3)
    for d in range(3):
        v = dl(a[d])
        for e in range(3):
            if e != d:
                v *= l(a[e], xi[e])
        g[d] = v
    return g


def element_stiffness(h):
    corners = list(itertools.product((0, 1), repeat=3))
    gp = [0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)]
    K = np.zeros((8, 8))
    J = np.array(h, dtype=float)
    vol = float(np.prod(J))
    for q in itertools.product(gp, repeat=3):
        grads = [_shape_grad(a, q) / J for a in corners]
        for i in range(8):
            for j in range(8):
                K[i, j] += float(np.dot(grads[i], grads[j])) * vol / 8.0
    return corners, K


def assemble(sigma, periodic):
    """Sparse A over the unknowns (x fastest): sum over cells of sigma_c K_c / V."""
    n = sigma.shape
    h = [1.0 / n[d] for d in range(3)]
    vol = h[0] * h[1] * h[2]
    corners, K = element_stiffness(h)
    m, uid = _node_ids(n, periodic)
    N = m[0] * m[1] * m[2]
    rows, cols, vals = [], [], []
    for c in itertools.product(range(n[0]), range(n[1]), range(n[2])):
        ids = [uid((c[0] + a[0], c[1] + a[1], c[2] + a[2])) for a in corners]
        s = sigma[c]
        for i in range(8):
            if ids[i] < 0:
                continue
            for j in range(8):
                if ids[j] < 0:
                    continue
                rows.append(ids[i])
                cols.append(ids[j])
                vals.append(s * K[i, j] / vol)
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N)), m


def interp_matrix(nc, periodic):
    """P: coarse unknowns -> fine unknowns, the coarse trilinear hat functions
    evaluated at the fine nodes' coordinates."""
    nf = tuple(2 * x for x in nc)
    mf, uidf = _node_ids(nf, periodic)
    mc, uidc = _node_ids(nc, periodic)
    Nf, Nc = mf[0] * mf[1] * mf[2], mc[0] * mc[1] * mc[2]
    rows, cols, vals = [], [], []
    hc = [1.0 / nc[d] for d in range(3)]
    for g in itertools.product(*[range(nf[d] + 1) for d in range(3)]):
        i = uidf(g)
        if i < 0:
            continue
        x = [g[d] / nf[d] for d in range(3)]
        if any(periodic[d] and g[d] == nf[d] for d in range(3)):
            continue  # the same node as index 0
        # the coarse cell holding x and the hat functions of its corners
        base = [min(int(np.floor(x[d] / hc[d])), nc[d] - 1) for d in range(3)]
        for a in itertools.product((0, 1), repeat=3):
            G = tuple(base[d] + a[d] for d in range(3))
            w = 1.0
            for d in range(3):
                t = x[d] / hc[d] - base[d]
                w *= t if a[d] == 1 else 1.0 - t
            if w == 0.0:
                continue
            j = uidc(G)
            if j < 0:
                continue
            rows.append(i)
            cols.append(j)
            vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(Nf, Nc))


def to_vec(U):
    """Unknown array [i, j, k] -> vector, x fastest."""
    return np.asarray(U).ravel(order="F")


def from_vec(v, m):
    return np.asarray(v).reshape(m, order="F")
