"""Pins of the oracle's box metadata and ghost exchange (no GPU).

The ghost exchange is checked against its plain definition: after it, every
ghost cell whose (periodically wrapped) index lies in the domain holds the
global array's value there, and no other ghost cell is touched.  This uses no
intersection logic at all.
"""

import numpy as np
import pytest

import oracle as O
import workloads as W


def _global_spec_check(boxes, n, periodic, ngrow, seed=0):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n, n))
    data = W.scatter_cells(G, boxes, ng=ngrow, fill=np.nan)
    O.fill_boundary(data, boxes, W.domain_box(n), periodic, ngrow)
    for (lo, hi), a in zip(boxes, data):
        idx = [np.arange(lo[d] - ngrow, hi[d] + ngrow + 1) for d in range(3)]
        I, J, K = np.meshgrid(*idx, indexing="ij")
        inside = np.ones(I.shape, bool)
        wrapped = []
        for d, X in enumerate((I, J, K)):
            if periodic[d]:
                wrapped.append(X % n)
            else:
                inside &= (X >= 0) & (X < n)
                wrapped.append(np.clip(X, 0, n - 1))
        expect = G[wrapped[0], wrapped[1], wrapped[2]]
        assert np.array_equal(a[inside], expect[inside])
        assert np.all(np.isnan(a[~inside]))


@pytest.mark.parametrize("periodic", [(True, True, True), (False, False, False), (True, False, True)])
def test_fill_boundary_matches_global_array(periodic):
    _global_spec_check(W.uniform_boxes(16, 8), 16, periodic, 1)


def test_fill_boundary_two_ghosts_and_uneven_boxes():
    boxes = [((0, 0, 0), (5, 11, 11)), ((6, 0, 0), (11, 5, 11)), ((6, 6, 0), (11, 11, 11))]
    _global_spec_check(boxes, 12, (True, False, True), 2)
    _global_spec_check(boxes, 12, (False, True, False), 1)


def test_fill_boundary_guillotine_boxes():
    boxes = W.guillotine_boxes(256)
    O.validate_boxarray(boxes, W.domain_box(256))
    _global_spec_check(boxes, 256, (False, False, False), 1)


def test_tags_cover_each_ghost_once_and_are_canonical():
    n = 16
    boxes = W.uniform_boxes(n, 8)
    for periodic in [(True, True, True), (False, False, False)]:
        tags = O.copy_tags(boxes, W.domain_box(n), periodic, 1)
        keys = [(t[0], t[1], t[3], t[2][0]) for t in tags]
        assert keys == sorted(keys)
        count = [np.zeros((10, 10, 10), int) for _ in boxes]
        for (d, s, (lo, hi), sh) in tags:
            blo = boxes[d][0]
            count[d][lo[0] - blo[0] + 1:hi[0] - blo[0] + 2, lo[1] - blo[1] + 1:hi[1] - blo[1] + 2,
                     lo[2] - blo[2] + 1:hi[2] - blo[2] + 2] += 1
        for c in count:
            assert c[1:-1, 1:-1, 1:-1].max() == 0       # valid cells never written
            assert c.max() == 1                           # nothing written twice
        if periodic[0]:
            assert all(c.sum() == 10 ** 3 - 8 ** 3 for c in count)
    # 8 boxes of 8^3, all periodic: each box touches 26 neighbour images
    tags = O.copy_tags(boxes, W.domain_box(n), (True, True, True), 1)
    assert len(tags) == 8 * 26


def test_validate_boxarray_errors():
    dom = W.domain_box(8)
    with pytest.raises(ValueError):
        O.validate_boxarray([((0, 0, 0), (7, 7, 7)), ((0, 0, 0), (1, 1, 1))], dom)
    with pytest.raises(ValueError):
        O.validate_boxarray([((0, 0, 0), (8, 7, 7))], dom)
    with pytest.raises(ValueError):
        O.validate_boxarray([((0, 0, 0), (3, 7, 7))], dom)
    O.validate_boxarray([((0, 0, 0), (3, 7, 7))], dom, require_cover=False)
    O.validate_boxarray(W.uniform_boxes(8, 4), dom)


def test_hierarchy_depths():
    def depth(boxes, n, m=4):
        return [O.box_shape(b[1]) for b in O.mg_hierarchy(boxes, W.domain_box(n), m)]
    assert [h[0] for h in depth(W.uniform_boxes(32, 16), 32)] == [32, 16, 8]
    assert [h[0] for h in depth(W.uniform_boxes(256, 64), 256)] == [256, 128, 64, 32, 16]
    assert [h[0] for h in depth(W.uniform_boxes(128, 64), 128)] == [128, 64, 32, 16, 8]
    g = W.guillotine_boxes(512)
    O.validate_boxarray(g, W.domain_box(512))
    assert all(e in W.EDGES for b in g for e in O.box_shape(b))
    assert [h[0] for h in depth(g, 512)] == [512, 256, 128, 64]
    assert [h[0] for h in depth(g, 512, 2)] == [512, 256, 128, 64, 32]


def test_guillotine_is_seeded():
    assert W.guillotine_boxes(512) == W.guillotine_boxes(512)
    assert W.guillotine_boxes(512, seed=7) != W.guillotine_boxes(512)
