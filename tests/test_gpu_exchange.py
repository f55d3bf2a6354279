"""GPU ghost exchange (fused copy kernel) against the oracle, bit for bit.

Ghost cells are NaN-poisoned before the exchange, so a ghost that should be
filled and is not shows up as a NaN mismatch; ghosts outside a wall stay NaN.
"""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_util import lib

CASES = [
    ("c0_periodic", W.uniform_boxes(32, 16), 32, (True, True, True), 1),
    ("c1_boxes_dirichlet", W.uniform_boxes(256, 64), 256, (False, False, False), 1),
    ("mixed_bc_two_ghosts", W.uniform_boxes(32, 8), 32, (True, False, True), 2),
    ("guillotine256", W.guillotine_boxes(256), 256, (False, False, False), 1),
    ("uneven_periodic", [((0, 0, 0), (5, 11, 11)), ((6, 0, 0), (11, 5, 11)),
                         ((6, 6, 0), (11, 11, 11))], 12, (True, True, False), 1),
]


@pytest.mark.gpu
@pytest.mark.parametrize("name,boxes,n,periodic,ng", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_fill_boundary_bitexact(name, boxes, n, periodic, ng, dtype):
    P = lib()
    print(f"[exchange] {name} n={n} ng={ng} {dtype}", flush=True)
    rng = np.random.default_rng(11)
    G = rng.standard_normal((n, n, n))
    if dtype == torch.float32:
        G = G.astype(np.float32)
    arrays = W.scatter_cells(G, boxes, ng=ng, fill=np.nan)
    mf = P.MultiFab.from_numpy(boxes, arrays, ng, dtype=dtype)
    P.fill_boundary(mf, W.domain_box(n), periodic)
    torch.cuda.synchronize()
    got = mf.to_numpy()
    O.fill_boundary(arrays, boxes, W.domain_box(n), periodic, ng)
    for b, (x, y) in enumerate(zip(got, arrays)):
        assert np.array_equal(x, y, equal_nan=True), f"box {b}"


@pytest.mark.gpu
def test_fill_boundary_plan_cache_and_second_layout():
    P = lib()
    boxes = W.uniform_boxes(16, 8)
    for ng in (1, 1, 2):
        arrays = W.scatter_cells(np.arange(16 ** 3, dtype=np.float64).reshape(16, 16, 16), boxes,
                                 ng=ng, fill=-1.0)
        mf = P.MultiFab.from_numpy(boxes, arrays, ng)
        P.fill_boundary(mf, W.domain_box(16), (True, True, True))
        torch.cuda.synchronize()
        O.fill_boundary(arrays, boxes, W.domain_box(16), (True, True, True), ng)
        assert all(np.array_equal(x, y) for x, y in zip(mf.to_numpy(), arrays))
    P.release_caches()
