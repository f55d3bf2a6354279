"""Boxes, box arrays, the multigrid box hierarchy and the ghost-cell exchange.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A box is a pair ``(lo, hi)`` of 3-tuples of inclusive cell indices, as in the
paper's description of ``Box`` (section "Basic data structures"): a logically
rectangular region given by its lower and upper corner.  All boxes here are
cell-centred.  Per-box data are NumPy arrays indexed ``[i, j, k]`` over the box
grown by ``ngrow`` ghost cells on each side ("Containers for mesh data").
"""

import itertools

import numpy as np

Box = tuple


def box_shape(b):
    lo, hi = b
    return tuple(hi[d] - lo[d] + 1 for d in range(3))


def box_ok(b):
    lo, hi = b
    return all(hi[d] >= lo[d] for d in range(3))


def grow(b, g):
    lo, hi = b
    return (tuple(x - g for x in lo), tuple(x + g for x in hi))


def shift_box(b, s):
    lo, hi = b
    return (tuple(lo[d] + s[d] for d in range(3)), tuple(hi[d] + s[d] for d in range(3)))


def intersect(a, b):
    """Intersection of two boxes, or None when empty."""
    lo = tuple(max(a[0][d], b[0][d]) for d in range(3))
    hi = tuple(min(a[1][d], b[1][d]) for d in range(3))
    r = (lo, hi)
    return r if box_ok(r) else None


def coarsen_box(b, r=2):
    """Coarsen by ratio r with floor division (a fine cell i has parent i // r)."""
    lo, hi = b
    return (tuple(x // r for x in lo), tuple(x // r for x in hi))


def refine_box(b, r=2):
    lo, hi = b
    return (tuple(x * r for x in lo), tuple(x * r + r - 1 for x in hi))


def validate_boxarray(boxes, domain, require_cover=True):
    """Check the conditions the paper puts on a BoxArray ("Basic data structures").

    Boxes must be non-empty, pairwise non-intersecting and inside the domain.
    For a single-level solve they must also cover the domain exactly (this is
    the solver's requirement, checked by counting cells).  Raises ValueError.
    """
    if len(boxes) == 0:
        raise ValueError("empty box array")
    for b in boxes:
        if not box_ok(b):
            raise ValueError(f"empty box {b}")
        if intersect(b, domain) != b:
            raise ValueError(f"box {b} outside domain {domain}")
    for i in range(len(boxes)):
        for j in range(i + 1, len(boxes)):
            if intersect(boxes[i], boxes[j]) is not None:
                raise ValueError(f"boxes {i} and {j} intersect")
    if require_cover:
        ncell = sum(int(np.prod(box_shape(b))) for b in boxes)
        if ncell != int(np.prod(box_shape(domain))):
            raise ValueError("box array does not cover the domain")


def _coarsenable(bs, dom, min_bottom_edge):
    for b in bs:
        for d, e in enumerate(box_shape(b)):
            if e % 2 != 0 or e // 2 < min_bottom_edge or b[0][d] % 2 != 0:
                return False
    for d, e in enumerate(box_shape(dom)):
        if e % 2 != 0 or dom[0][d] % 2 != 0:
            return False
    return True


def mg_hierarchy(boxes, domain, min_bottom_edge=4, aggregate=False):
    """Box arrays of the multigrid levels.

    Reading taken (the paper names coarsening and "blocking_factor" improving
    multigrid efficiency, section "Regridding and load balancing", but gives no
    rule): level l+1 is every box of level l coarsened by 2, which is done only
    while every edge of every box at level l is even and half of it is at least
    ``min_bottom_edge`` and every box (and the domain) starts at an even index,
    so that each coarse cell has its 8 children in one box.

    Aggregation (the paper's "Linear Solvers" section: merging boxes at a level
    of the hierarchy to allow further coarsening): when that rule stops and
    ``aggregate`` is set, a level whose boxes cover its domain in whole 2x2x2
    blocks gets a next level made of the single box coarsen(domain) (if the
    domain passes the rule), and coarsening continues from there.

    Returns a list of ``(boxes, domain, merged)``; ``merged`` marks a level
    that is one box covering several boxes of the level above.
    """
    levels = [(list(boxes), domain, False)]
    while True:
        bs, dom, _ = levels[-1]
        if _coarsenable(bs, dom, min_bottom_edge):
            levels.append(([coarsen_box(b) for b in bs], coarsen_box(dom), False))
            continue
        if not aggregate or len(bs) == 1:
            break
        ncell = sum(int(np.prod(box_shape(b))) for b in bs)
        even = all(b[0][d] % 2 == 0 and box_shape(b)[d] % 2 == 0 for b in bs for d in range(3))
        if not even or ncell != int(np.prod(box_shape(dom))):
            break
        if not _coarsenable([dom], dom, min_bottom_edge):
            break
        cd = coarsen_box(dom)
        levels.append(([cd], cd, True))
    return levels


def copy_tags(boxes, domain, periodic, ngrow):
    """Brute-force ghost-exchange metadata ("Operations on a level", "Communication").

    For every destination box B, every source box S and every periodic image
    shift s (a multiple of the domain length in each periodic direction, zero
    otherwise), the region grow(B, ngrow) intersected with S shifted by s is
    copied from S: destination cell p takes the value of source cell p - s.
    The pair (S = B, s = 0) is skipped (it is B's own valid region).  Ghost
    cells outside the domain in a non-periodic direction are never written.

    The paper builds this list with a hash over the boxes; this oracle checks
    every pair, which is slower but has no hashing logic to get wrong.  Tags
    are returned in the canonical order (dst, src, shift, region lo).
    Each tag is ``(dst, src, (lo, hi), shift)``.
    """
    L = box_shape(domain)
    shifts_1d = [[-L[d], 0, L[d]] if periodic[d] else [0] for d in range(3)]
    tags = []
    for bi, B in enumerate(boxes):
        gb = grow(B, ngrow)
        for si, S in enumerate(boxes):
            for s in itertools.product(*shifts_1d):
                if si == bi and s == (0, 0, 0):
                    continue
                R = intersect(gb, shift_box(S, s))
                if R is None:
                    continue
                tags.append((bi, si, R, tuple(s)))
    tags.sort(key=lambda t: (t[0], t[1], t[3], t[2][0]))
    return tags


def fill_boundary(data, boxes, domain, periodic, ngrow):
    """Apply the copy tags in place: ``dst[p] = src[p - shift]``.

    ``data[b]`` is box b's array over grow(boxes[b], ngrow).  Only valid cells
    are ever read, so the order in which tags are applied does not matter.
    """
    for (d, s, R, sh) in copy_tags(boxes, domain, periodic, ngrow):
        dlo = boxes[d][0]
        slo = boxes[s][0]
        lo, hi = R
        dsl = tuple(slice(lo[a] - dlo[a] + ngrow, hi[a] - dlo[a] + ngrow + 1) for a in range(3))
        ssl = tuple(slice(lo[a] - sh[a] - slo[a] + ngrow, hi[a] - sh[a] - slo[a] + ngrow + 1)
                    for a in range(3))
        data[d][dsl] = data[s][ssl]
