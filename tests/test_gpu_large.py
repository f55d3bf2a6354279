"""The 512^3 uneven-box problem at full size (the configuration bench.py
--workload c2 times): residual of the GPU solution recomputed by the oracle's
operator on sampled boxes (ghosts taken from the gathered global solution):
one box of each of the 104 distinct box shapes, then seeded draws up to 160
of the 670."""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_util import lib


@pytest.mark.gpu
@pytest.mark.parametrize("precision", [0, 1])
def test_c2_full_size_sampled_residual(precision):
    print(f"[large] 512^3 guillotine precision={precision}", flush=True)
    P = lib()
    cfg = W.config_c2()
    n, boxes = cfg["n"], cfg["boxes"]
    b = []
    for d in range(3):
        e = [0, 0, 0]
        e[d] = 1
        b.append(P.MultiFab.from_numpy(boxes, W.scatter_faces(cfg["faces"][d], boxes, d), 0,
                                       ixtype=tuple(e)))
    f_boxes = W.scatter_cells(cfg["rhs"], boxes)
    rhs = P.MultiFab.from_numpy(boxes, f_boxes, 0)
    s = P.MLMG(boxes, W.domain_box(n), cfg["periodic"], 1.0, 1.0, b=b,
               opts=dict(precision=precision, aggregate=1, tune=0))
    phi = s.cell_mf(1, fill=0.0)
    info = s.solve(phi, rhs, 1e-10)
    print(f"c2: {len(boxes)} boxes, {info['nlevels']} levels, {info['iters']} cycles, "
          f"{info['solve_ms']:.1f} ms", flush=True)
    assert info["converged"]
    G = W.gather_cells(phi.valid_numpy(), boxes, n)
    del phi
    rng = np.random.default_rng(7)
    first = {}
    for i, (lo, hi) in enumerate(boxes):
        first.setdefault(tuple(h - l + 1 for l, h in zip(lo, hi)), i)
    rest = [i for i in range(len(boxes)) if i not in set(first.values())]
    extra = rng.choice(rest, size=max(0, 160 - len(first)), replace=False).tolist()
    pick = sorted(set(first.values()) | set(extra))
    pboxes = [boxes[i] for i in pick]
    lev = O.make_level(pboxes, W.domain_box(n), cfg["periodic"], 1.0, 1.0, None,
                       [W.scatter_faces(cfg["faces"][d], pboxes, d) for d in range(3)])
    pad = np.pad(G, 1)   # wall ghosts are never read by the folded stencil
    ph = [pad[lo[0]:hi[0] + 3, lo[1]:hi[1] + 3, lo[2]:hi[2] + 3].copy() for lo, hi in pboxes]
    Aphi = O.apply_op(lev, ph)
    normf = max(float(np.max(np.abs(x))) for x in f_boxes)
    r = max(float(np.max(np.abs(f_boxes[i] - a))) for i, a in zip(pick, Aphi))
    print(f"c2: {len(pick)} boxes ({len(first)} shapes) checked, max residual {r / normf:.2e} "
          f"of max|f|", flush=True)
    assert r <= 1e-10 * normf * (1 + 1e-3) and r <= info["abs_resid"] + 1e-12 * normf
    s.close()
    torch.cuda.empty_cache()
