"""Helpers shared by the GPU tests: build solver inputs from the workload
generators and compare GPU MultiFabs with the oracle's per-box arrays."""

import numpy as np
import torch

import oracle as O
import workloads as W


def lib():
    import paper_2009_12009_amd as P
    return P


def oracle_level(cfg, boxes=None, a_cells=None):
    boxes = boxes or cfg["boxes"]
    b = None
    if cfg.get("faces") is not None:
        b = [W.scatter_faces(cfg["faces"][d], boxes, d) for d in range(3)]
    a = W.scatter_cells(a_cells, boxes) if a_cells is not None else None
    return O.make_level(boxes, W.domain_box(cfg["n"]), cfg["periodic"], cfg["alpha"],
                        cfg["beta"], a, b)


def gpu_solver(cfg, boxes=None, opts=None, a_cells=None):
    P = lib()
    boxes = boxes or cfg["boxes"]
    b = None
    if cfg.get("faces") is not None:
        b = []
        for d in range(3):
            e = [0, 0, 0]
            e[d] = 1
            b.append(P.MultiFab.from_numpy(boxes, W.scatter_faces(cfg["faces"][d], boxes, d), 0,
                                           ixtype=tuple(e)))
    a = None
    if a_cells is not None:
        a = P.MultiFab.from_numpy(boxes, W.scatter_cells(a_cells, boxes), 0)
    return P.MLMG(boxes, W.domain_box(cfg["n"]), cfg["periodic"], cfg["alpha"], cfg["beta"],
                  a=a, b=b, opts=opts)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_global(mf, boxes, n):
    return W.gather_cells(mf.valid_numpy(), boxes, n)


def sync():
    torch.cuda.synchronize()
