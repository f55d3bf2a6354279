"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module generates data only: box lists, coefficient fields and right-hand
sides drawn from fixed seeds, plus plain scatter/gather between a global array
and per-box arrays.  It holds none of the solver's arithmetic, so both the GPU
path and the CPU oracle may take their inputs from it.

Conventions: the domain is the unit cube with n cells per side; a global cell
array has shape (n, n, n) indexed [i, j, k] (i along x); a global face array of
direction d has n+1 entries along d, entry i being the face on the low side of
cell i.  Seeds: cell b = 1, rhs = 2, target b = 3, boxes = 4, blobs = 5,
finite-difference picks = 6.
"""

import numpy as np

SEED_B = 1
SEED_RHS = 2
SEED_BT = 3
SEED_BOXES = 4
SEED_BLOBS = 5
SEED_FD = 6

EDGES = (32, 48, 64, 96, 128)


def domain_box(n):
    return ((0, 0, 0), (n - 1, n - 1, n - 1))


def uniform_boxes(n, max_grid_size):
    """Chop the n^3 domain into boxes of edge max_grid_size (x varies fastest)."""
    m = max_grid_size
    assert n % m == 0
    out = []
    for k in range(0, n, m):
        for j in range(0, n, m):
            for i in range(0, n, m):
                out.append(((i, j, k), (i + m - 1, j + m - 1, k + m - 1)))
    return out


def guillotine_boxes(n, seed=SEED_BOXES):
    """Seeded recursive guillotine chop with edges from {32, 48, 64, 96, 128}.

    A box with an edge outside that set is split along its longest such axis
    (ties: lowest axis).  Otherwise it is kept if its longest edge is <= 64, and
    else split along its longest axis (ties: lowest) with probability 1/2.  A
    split cuts off a low part whose edge is drawn uniformly from the set members
    that leave a remainder >= 32 that is a multiple of 16.  Recursion is
    depth-first, low part first; the random draws happen in that order.
    """
    rng = np.random.default_rng(seed)
    out = []

    def rec(lo, hi):
        e = [hi[d] - lo[d] + 1 for d in range(3)]
        bad = [d for d in range(3) if e[d] not in EDGES]
        if bad:
            ax = max(bad, key=lambda d: (e[d], -d))
        else:
            if max(e) <= 64:
                out.append((tuple(lo), tuple(hi)))
                return
            if rng.random() >= 0.5:
                out.append((tuple(lo), tuple(hi)))
                return
            ax = max(range(3), key=lambda d: (e[d], -d))
        choices = [c for c in EDGES if e[ax] - c >= 32 and (e[ax] - c) % 16 == 0]
        cut = choices[int(rng.integers(len(choices)))]
        hi1 = list(hi)
        hi1[ax] = lo[ax] + cut - 1
        lo2 = list(lo)
        lo2[ax] = lo[ax] + cut
        rec(list(lo), hi1)
        rec(lo2, list(hi))

    rec([0, 0, 0], [n - 1, n - 1, n - 1])
    return out


def lognormal_cells(n, sigma=1.0, seed=SEED_B):
    """b = exp(sigma * Z), Z standard normal drawn as one (n, n, n) array."""
    rng = np.random.default_rng(seed)
    return np.exp(sigma * rng.standard_normal((n, n, n)))


def uniform_rhs(n, seed=SEED_RHS):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, (n, n, n))


def sin_rhs(n):
    """sin(2 pi x) sin(2 pi y) sin(2 pi z) at cell centres, minus its mean."""
    x = (np.arange(n) + 0.5) / n
    s = np.sin(2.0 * np.pi * x)
    f = s[:, None, None] * s[None, :, None] * s[None, None, :]
    return f - f.mean()


def harmonic_faces(bcell, periodic=(False, False, False)):
    """Face coefficients from cell values: harmonic mean of the two neighbours.

    On a non-periodic domain face the single interior cell's value is used; on a
    periodic one the harmonic mean with the wrapped cell (faces 0 and n equal).
    Returns [bx, by, bz] global face arrays.
    """
    out = []
    for d in range(3):
        n = bcell.shape[d]
        shp = list(bcell.shape)
        shp[d] += 1
        F = np.empty(shp)

        def sl(a, b_):
            return tuple(slice(a, b_) if x == d else slice(None) for x in range(3))

        L = bcell[sl(0, n - 1)]
        R = bcell[sl(1, n)]
        F[sl(1, n)] = 2.0 * L * R / (L + R)
        if periodic[d]:
            L = bcell[sl(n - 1, n)]
            R = bcell[sl(0, 1)]
            w = 2.0 * L * R / (L + R)
            F[sl(0, 1)] = w
            F[sl(n, n + 1)] = w
        else:
            F[sl(0, 1)] = bcell[sl(0, 1)]
            F[sl(n, n + 1)] = bcell[sl(n - 1, n)]
        out.append(F)
    return out


def scatter_cells(G, boxes, ng=0, fill=0.0, dlo=(0, 0, 0)):
    """Per-box arrays (with ng ghost layers set to ``fill``) from a global cell array."""
    out = []
    for lo, hi in boxes:
        shp = tuple(hi[d] - lo[d] + 1 + 2 * ng for d in range(3))
        a = np.full(shp, fill, dtype=G.dtype)
        v = G[lo[0] - dlo[0]:hi[0] - dlo[0] + 1, lo[1] - dlo[1]:hi[1] - dlo[1] + 1,
              lo[2] - dlo[2]:hi[2] - dlo[2] + 1]
        if ng > 0:
            a[ng:-ng, ng:-ng, ng:-ng] = v
        else:
            a[...] = v
        out.append(a)
    return out


def scatter_faces(F, boxes, d, dlo=(0, 0, 0)):
    """Per-box face arrays of direction d (valid shape + e_d) from a global face array."""
    out = []
    for lo, hi in boxes:
        e = [0, 0, 0]
        e[d] = 1
        sl = tuple(slice(lo[a] - dlo[a], hi[a] - dlo[a] + 1 + e[a]) for a in range(3))
        out.append(np.array(F[sl]))
    return out


def gather_cells(per_box, boxes, n, ng=0, dlo=(0, 0, 0)):
    G = np.zeros((n, n, n) if np.isscalar(n) else tuple(n), dtype=per_box[0].dtype)
    for (lo, hi), a in zip(boxes, per_box):
        v = a[ng:-ng, ng:-ng, ng:-ng] if ng > 0 else a
        G[lo[0] - dlo[0]:hi[0] - dlo[0] + 1, lo[1] - dlo[1]:hi[1] - dlo[1] + 1,
          lo[2] - dlo[2]:hi[2] - dlo[2] + 1] = v
    return G


# ---------------------------------------------------------------------------
# The five benchmark workloads (all on the unit cube).

def config_c0():
    """32^3 periodic Poisson: 8 boxes of 16^3, alpha = 0, beta = 1, b = 1,
    rhs = sin(2 pi x) sin(2 pi y) sin(2 pi z) minus its mean."""
    n = 32
    return dict(name="poisson32_periodic", n=n, boxes=uniform_boxes(n, 16),
                periodic=(True, True, True), alpha=0.0, beta=1.0, bcell=None, faces=None,
                rhs=sin_rhs(n))


def config_lognormal(n, max_grid_size, sigma=1.0, boxes=None, seed_b=SEED_B, seed_rhs=SEED_RHS):
    """Dirichlet-0 variable-coefficient problem: alpha = beta = 1, a = 1, cell
    b = exp(sigma Z) (seed 1), face b harmonic, rhs ~ U[-1, 1] (seed 2)."""
    bc = lognormal_cells(n, sigma, seed_b)
    per = (False, False, False)
    return dict(name=f"lognormal{n}", n=n,
                boxes=boxes if boxes is not None else uniform_boxes(n, max_grid_size),
                periodic=per, alpha=1.0, beta=1.0, bcell=bc, faces=harmonic_faces(bc, per),
                rhs=uniform_rhs(n, seed_rhs))


def config_c1():
    """256^3, 64 boxes of 64^3, Dirichlet 0, lognormal b (sigma 1)."""
    c = config_lognormal(256, 64)
    c["name"] = "abec256_lognormal_64boxes"
    return c


def config_c2(n=512):
    """512^3 guillotine-chopped boxes (seed 4), lognormal b (sigma 1)."""
    c = config_lognormal(n, None, boxes=guillotine_boxes(n))
    c["name"] = f"abec{n}_guillotine"
    return c


def config_c3():
    """128^3, 8 boxes of 64^3, Dirichlet 0, b = exp(0.5 Z) (seed 1), target b seed 3."""
    c = config_lognormal(128, 64, sigma=0.5)
    bt = lognormal_cells(128, 0.5, SEED_BT)
    c["faces_target"] = harmonic_faces(bt, c["periodic"])
    c["name"] = "adjoint128"
    return c


# ---------------------------------------------------------------------------
# Nodal workload: node-centred unknowns on the same cell grid.

def nodal_unknown_shape(n, periodic):
    """Unknown nodes per direction: interior nodes along a wall direction,
    nodes 0 .. n-1 along a periodic one."""
    n = (n,) * 3 if np.isscalar(n) else tuple(n)
    return tuple(n[d] if periodic[d] else n[d] - 1 for d in range(3))


def nodes_from_unknowns(U, n, periodic):
    """All nodes 0 .. n_d (shape n + 1) from the unknowns: 0 on wall nodes,
    node n_d = node 0 along a periodic direction."""
    n = (n,) * 3 if np.isscalar(n) else tuple(n)
    G = np.zeros(tuple(x + 1 for x in n), dtype=U.dtype)
    sl = tuple(slice(0, n[d]) if periodic[d] else slice(1, n[d]) for d in range(3))
    G[sl] = U
    for d in range(3):
        if periodic[d]:
            a = [slice(None)] * 3
            b = [slice(None)] * 3
            a[d] = slice(n[d], n[d] + 1)
            b[d] = slice(0, 1)
            G[tuple(a)] = G[tuple(b)]
    return G


def unknowns_from_nodes(G, periodic):
    n = tuple(x - 1 for x in G.shape)
    sl = tuple(slice(0, n[d]) if periodic[d] else slice(1, n[d]) for d in range(3))
    return np.array(G[sl])


def scatter_nodes(G, boxes, ng=0, fill=0.0, dlo=(0, 0, 0)):
    """Per-box nodal arrays (nodes lo .. hi+1, ghost nodes set to ``fill``)
    from an array of all nodes (shape n + 1)."""
    out = []
    for lo, hi in boxes:
        shp = tuple(hi[d] - lo[d] + 2 + 2 * ng for d in range(3))
        a = np.full(shp, fill, dtype=G.dtype)
        v = G[lo[0] - dlo[0]:hi[0] - dlo[0] + 2, lo[1] - dlo[1]:hi[1] - dlo[1] + 2,
              lo[2] - dlo[2]:hi[2] - dlo[2] + 2]
        if ng > 0:
            a[ng:-ng, ng:-ng, ng:-ng] = v
        else:
            a[...] = v
        out.append(a)
    return out


def config_nodal(n, max_grid_size, sigma=1.0, periodic=(False, False, False), seed_b=SEED_B,
                 seed_rhs=SEED_RHS):
    """Nodal -div(sigma grad phi) = f: cell sigma = exp(sigma Z) (seed 1), f ~
    U[-1, 1] on the unknown nodes (seed 2, one draw of the unknown shape)."""
    per = tuple(bool(p) for p in periodic)
    rng = np.random.default_rng(seed_rhs)
    f = rng.uniform(-1.0, 1.0, nodal_unknown_shape(n, per))
    return dict(name=f"nodal{n}", n=n, boxes=uniform_boxes(n, max_grid_size), periodic=per,
                sigma_cells=lognormal_cells(n, sigma, seed_b), rhs_unknowns=f)
