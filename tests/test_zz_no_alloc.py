"""The allocation-free ghost exchange (mg_fill_boundary_noalloc) against
fill_boundary, bit for bit, on consecutive calls that share the library's
static device scratch: a larger layout first, then smaller ones, so a stale
plan left in the scratch by the previous call would show as a mismatch.
Ghosts are NaN-poisoned before each exchange.
"""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_util import lib

CALLS = [
    # name, boxes, n, periodic, ngrow, dtype
    ("128_periodic_64boxes", W.uniform_boxes(128, 32), 128, (True, True, True), 1, torch.float64),
    ("12_uneven_periodic_f32", [((0, 0, 0), (5, 11, 11)), ((6, 0, 0), (11, 5, 11)),
                                ((6, 6, 0), (11, 11, 11))], 12, (True, True, False), 1,
     torch.float32),
    ("32_mixed_two_ghosts", W.uniform_boxes(32, 8), 32, (True, False, True), 2, torch.float64),
]


def _poisoned(P, boxes, n, ng, dtype, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n, n))
    if dtype == torch.float32:
        G = G.astype(np.float32)
    arrays = W.scatter_cells(G, boxes, ng=ng, fill=np.nan)
    return arrays, P.MultiFab.from_numpy(boxes, arrays, ng, dtype=dtype)


@pytest.mark.gpu
def test_noalloc_exchange_equals_fill_boundary_on_consecutive_calls():
    P = lib()
    for i, (name, boxes, n, per, ng, dtype) in enumerate(CALLS):
        print(f"[noalloc] call {i}: {name} n={n} ng={ng} {dtype}", flush=True)
        arrays, mf_a = _poisoned(P, boxes, n, ng, dtype, 20 + i)
        _, mf_b = _poisoned(P, boxes, n, ng, dtype, 20 + i)
        P.fill_boundary_noalloc(mf_a, W.domain_box(n), per)
        P.fill_boundary(mf_b, W.domain_box(n), per)
        torch.cuda.synchronize()
        got, ref = mf_a.to_numpy(), mf_b.to_numpy()
        O.fill_boundary(arrays, boxes, W.domain_box(n), per, ng)
        for b in range(len(boxes)):
            assert np.array_equal(got[b], ref[b], equal_nan=True), f"{name}: box {b} vs fill_boundary"
            assert np.array_equal(got[b], arrays[b], equal_nan=True), f"{name}: box {b} vs oracle"


@pytest.mark.gpu
def test_noalloc_exchange_repeated_on_one_layout_after_another():
    P = lib()
    # the same small layout twice around a different one: each call re-stages its plan
    seq = [CALLS[2], CALLS[1], CALLS[2]]
    for i, (name, boxes, n, per, ng, dtype) in enumerate(seq):
        print(f"[noalloc] repeat {i}: {name}", flush=True)
        arrays, mf = _poisoned(P, boxes, n, ng, dtype, 40 + i)
        P.fill_boundary_noalloc(mf, W.domain_box(n), per)
        torch.cuda.synchronize()
        O.fill_boundary(arrays, boxes, W.domain_box(n), per, ng)
        assert all(np.array_equal(x, y, equal_nan=True) for x, y in zip(mf.to_numpy(), arrays))


@pytest.mark.gpu
def test_noalloc_exchange_rejects_a_plan_beyond_the_scratch():
    P = lib()
    # 4096 boxes of 4^3 in a periodic 64^3 domain: ~106k copy tags, a plan of
    # several MiB, more than the static scratch holds
    boxes = W.uniform_boxes(64, 4)
    mf = P.MultiFab(boxes, 1, torch.float64, fill=3.0)
    print(f"[noalloc] oversize plan: {len(boxes)} boxes", flush=True)
    with pytest.raises(P.MGError) as ei:
        P.fill_boundary_noalloc(mf, W.domain_box(64), (True, True, True))
    assert ei.value.code == P._lib.MG_ERR_WORKSPACE
    assert "static scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((mf.data == 3.0).all())
