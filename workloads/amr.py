"""Inputs of the two-level composite problem: blob right-hand side, error
tagging, Berger-Rigoutsos clustering and box chopping ("Regridding and load
balancing" in the paper: tag cells above a tolerance, group the tags into
rectangles with the Berger-Rigoutsos algorithm, keep edges divisible by the
blocking factor and no longer than max_grid_size).

These functions produce the fine box array and the coefficient and rhs data
that both the oracle and the GPU path take as input; they hold none of the
solver's arithmetic.  Fine index space = coarse index space refined by 2.
"""

import numpy as np

from . import SEED_BLOBS


def blob_centres(seed=SEED_BLOBS, count=4):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.2, 0.8, (count, 3))


def blob_rhs(n, centres, sigma=0.05):
    """sum_m exp(-|x - c_m|^2 / (2 sigma^2)) at the centres of an n^3 grid on [0,1]^3."""
    x = (np.arange(n) + 0.5) / n
    f = np.zeros((n, n, n))
    for c in centres:
        gx = np.exp(-(x - c[0]) ** 2 / (2 * sigma ** 2))
        gy = np.exp(-(x - c[1]) ** 2 / (2 * sigma ** 2))
        gz = np.exp(-(x - c[2]) ** 2 / (2 * sigma ** 2))
        f += gx[:, None, None] * gy[None, :, None] * gz[None, None, :]
    return f


def tag_cells(f, frac=0.5):
    """Cells where |f| exceeds frac * max|f|."""
    a = np.abs(f)
    return a > frac * a.max()


def _split_index(sig):
    """Berger-Rigoutsos cut of one signature (sum of tags over the other two
    axes): a zero (hole) nearest the middle, else the largest jump of the
    discrete second derivative, else None.  Returns the length of the low part."""
    n = len(sig)
    if n < 2:
        return None
    mid = (n - 1) / 2.0
    holes = [i for i in range(1, n - 1) if sig[i] == 0]
    if holes:
        i = min(holes, key=lambda i: (abs(i - mid), i))
        return i  # low part = [0, i), cell i (a hole) starts the high part
    if n < 4:
        return None
    lap = [sig[i + 1] - 2 * sig[i] + sig[i - 1] for i in range(1, n - 1)]
    best, where = 0, None
    for k in range(1, len(lap)):
        if (lap[k - 1] < 0) != (lap[k] < 0):
            jump = abs(lap[k] - lap[k - 1])
            cut = k + 1  # between cells k and k+1
            if jump > best or (jump == best and where is not None
                               and abs(cut - mid) < abs(where - mid)):
                best, where = jump, cut
    return where


def berger_rigoutsos(tags, efficiency=0.7):
    """Cluster a boolean array of tags into boxes (inclusive index corners).

    Each box is the bounding box of its tags; it is accepted when the tagged
    fraction reaches ``efficiency``, otherwise cut at a hole or inflection of
    the tag signatures (longest usable axis first) and both halves are
    clustered again; with no usable cut it is halved along its longest axis.
    """
    out = []

    def rec(lo, hi):
        sub = tags[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1]
        if not sub.any():
            return
        idx = [np.nonzero(sub.any(axis=tuple(a for a in range(3) if a != d)))[0] for d in range(3)]
        lo = [lo[d] + int(idx[d][0]) for d in range(3)]
        hi = [lo0 + int(idx[d][-1]) - int(idx[d][0]) for d, lo0 in enumerate(lo)]
        sub = tags[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1]
        if sub.mean() >= efficiency:
            out.append((tuple(lo), tuple(hi)))
            return
        axes = sorted(range(3), key=lambda d: (-(hi[d] - lo[d]), d))
        cut = None
        for d in axes:
            sig = sub.sum(axis=tuple(a for a in range(3) if a != d))
            c = _split_index(list(sig))
            if c is not None and 0 < c < len(sig):
                cut = (d, c)
                break
        if cut is None:
            d = axes[0]
            if hi[d] == lo[d]:
                out.append((tuple(lo), tuple(hi)))
                return
            cut = (d, (hi[d] - lo[d] + 1) // 2)
        d, c = cut
        hi1 = list(hi)
        hi1[d] = lo[d] + c - 1
        lo2 = list(lo)
        lo2[d] = lo[d] + c
        rec(lo, hi1)
        rec(lo2, hi)

    rec([0, 0, 0], [s - 1 for s in tags.shape])
    return out


def chop(boxes, max_edge, align, cut_every):
    """Split boxes so that no edge exceeds max_edge; cuts fall on multiples of
    ``align`` and on every multiple of ``cut_every`` (the coarse box grid)."""
    out = []
    for lo, hi in boxes:
        ranges = []
        for d in range(3):
            cuts = [lo[d]]
            x = lo[d]
            while x <= hi[d]:
                nxt = min(hi[d] + 1, x + max_edge, (x // cut_every + 1) * cut_every)
                cuts.append(nxt)
                x = nxt
            ranges.append([(cuts[i], cuts[i + 1] - 1) for i in range(len(cuts) - 1)])
        for zr in ranges[2]:
            for yr in ranges[1]:
                for xr in ranges[0]:
                    out.append(((xr[0], yr[0], zr[0]), (xr[1], yr[1], zr[1])))
    for lo, hi in out:
        for d in range(3):
            assert lo[d] % align == 0 and (hi[d] + 1) % align == 0
    return out


def fine_boxes(f_coarse, block=4, efficiency=0.7, max_edge=32, coarse_box=64, frac=0.5):
    """Fine box array (fine index space) over the tagged coarse cells.

    Tags are coarsened to blocks of ``block`` coarse cells (blocking factor
    2*block fine cells), clustered, refined to fine cells and chopped to edges
    <= max_edge fine cells, never crossing a coarse box boundary."""
    tags = tag_cells(f_coarse, frac)
    n = tags.shape[0]
    nb = n // block
    bt = tags.reshape(nb, block, nb, block, nb, block).any(axis=(1, 3, 5))
    bboxes = berger_rigoutsos(bt, efficiency)
    fb = [(tuple(2 * block * x for x in lo), tuple(2 * block * x + 2 * block - 1 for x in hi))
          for lo, hi in bboxes]
    return chop(fb, max_edge, 2 * block, 2 * coarse_box)


def fine_faces(bcell, cfaces, boxes, d):
    """Fine face coefficients by injection: a fine face lying on a coarse face
    takes that face's value, a fine face inside a coarse cell takes the cell's
    value (the harmonic mean of the two injected fine cells).  Per fine box."""
    out = []
    for lo, hi in boxes:
        e = [0, 0, 0]
        e[d] = 1
        idx = [np.arange(lo[a], hi[a] + 1 + e[a]) for a in range(3)]
        I, J, K = np.meshgrid(*idx, indexing="ij")
        F = (I, J, K)[d]
        on_coarse = (F % 2) == 0
        c = [I // 2, J // 2, K // 2]
        cf = list(c)
        cf[d] = F // 2
        ncell = bcell.shape[d]
        val_cell = bcell[c[0].clip(0, bcell.shape[0] - 1), c[1].clip(0, bcell.shape[1] - 1),
                         c[2].clip(0, bcell.shape[2] - 1)]
        val_face = cfaces[d][cf[0], cf[1], cf[2]]
        del ncell
        out.append(np.where(on_coarse, val_face, val_cell))
    return out


def config_c4(n=256, coarse_box=64, sigma_b=1.0):
    """Two-level problem: coarse n^3 in boxes of coarse_box^3, Dirichlet walls,
    alpha = beta = 1, lognormal b (seed 1), rhs = 4 Gaussian blobs (seed 5);
    fine level (ratio 2) over cells with |rhs| > 0.5 max|rhs|."""
    from . import harmonic_faces, lognormal_cells, uniform_boxes
    bc = lognormal_cells(n, sigma_b)
    cf = harmonic_faces(bc)
    cen = blob_centres()
    fc = blob_rhs(n, cen)
    fboxes = fine_boxes(fc, coarse_box=coarse_box)
    ff = blob_rhs(2 * n, cen) if n <= 64 else None
    return dict(name=f"composite{n}", n=n, boxes=uniform_boxes(n, coarse_box), fine_boxes=fboxes,
                periodic=(False, False, False), alpha=1.0, beta=1.0, bcell=bc, faces=cf,
                rhs=fc, rhs_fine_global=ff, centres=cen)


def fine_rhs(boxes, centres, n_fine, sigma=0.05):
    """Blob rhs at fine cell centres, per fine box (no global fine array)."""
    out = []
    for lo, hi in boxes:
        xs = [(np.arange(lo[d], hi[d] + 1) + 0.5) / n_fine for d in range(3)]
        f = np.zeros(tuple(len(x) for x in xs))
        for c in centres:
            g = [np.exp(-(xs[d] - c[d]) ** 2 / (2 * sigma ** 2)) for d in range(3)]
            f += g[0][:, None, None] * g[1][None, :, None] * g[2][None, None, :]
        out.append(f)
    return out
