"""Nodal solver binding: -div(sigma grad phi) = f on the nodes of the cell grid
(trilinear finite elements, Galerkin coarse operators), through the C ABI
(mg_nodal_*, include/amrmg.h).  Argument marshalling only."""

import ctypes as C

import torch

from . import _lib as L
from .multifab import MultiFab
from .solver import _stream_handle

NODE = (1, 1, 1)


def nodal_workspace_bytes(boxes, domain, periodic, opts):
    bx = L.boxes_array(boxes)
    g = L.geom_struct(domain, periodic)
    n = C.c_size_t()
    L.check(L.lib.mg_nodal_query_workspace(bx, len(boxes), C.byref(g), C.byref(opts), C.byref(n)),
            "mg_nodal_query_workspace")
    return n.value


class NodalMLMG:
    """boxes: (lo, hi) cell boxes covering ``domain``; periodic: 3 bools (other
    directions have phi = 0 on their wall nodes); sigma: cell MultiFab (ngrow 0)
    or None (sigma = 1); opts: keyword overrides of mg_opts_t."""

    def __init__(self, boxes, domain, periodic, sigma=None, opts=None, stream=None):
        self.boxes = [(tuple(lo), tuple(hi)) for lo, hi in boxes]
        self.domain = domain
        self.periodic = tuple(bool(p) for p in periodic)
        self.n = tuple(domain[1][d] - domain[0][d] + 1 for d in range(3))
        self.opts = L.default_opts(**(opts or {}))
        self._bx = L.boxes_array(self.boxes)
        self._geom = L.geom_struct(domain, periodic)
        bc = (C.c_int32 * 3)(*[L.MG_BC_PERIODIC if p else L.MG_BC_DIRICHLET0 for p in periodic])
        nbytes = nodal_workspace_bytes(self.boxes, domain, periodic, self.opts)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        self._ws_ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        sm = sigma.c_struct() if sigma is not None else None
        h = C.c_void_p()
        L.check(L.lib.mg_nodal_create(self._bx, len(self.boxes), C.byref(self._geom), bc, bc,
                                      C.byref(sm) if sm is not None else None,
                                      C.byref(self.opts), C.c_void_p(self._ws_ptr), nbytes,
                                      _stream_handle(stream), C.byref(h)), "mg_nodal_create")
        self.handle = h
        self._stream = stream

    def close(self):
        if getattr(self, "handle", None):
            L.lib.mg_nodal_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def node_mf(self, ngrow=0, fill=None):
        return MultiFab(self.boxes, ngrow, ixtype=NODE, fill=fill)

    def num_levels(self):
        n = C.c_int32()
        L.check(L.lib.mg_nodal_num_levels(self.handle, C.byref(n)), "mg_nodal_num_levels")
        return n.value

    def solve(self, phi, rhs, rel_tol=1e-10, abs_tol=0.0, history=False, raise_on_fail=True):
        pm, rm = phi.c_struct(), rhs.c_struct()
        info = L.MgInfo()
        hist = (C.c_double * (self.opts.max_iter + 1))() if history else None
        code = L.lib.mg_nodal_solve(self.handle, C.byref(pm), C.byref(rm), float(rel_tol),
                                    float(abs_tol), C.byref(info), hist)
        if raise_on_fail and code != L.MG_OK:
            L.check(code, "mg_nodal_solve")
        out = {"status": code, "iters": info.iters, "nlevels": info.nlevels,
               "bottom_iters": info.bottom_iters, "converged": bool(info.converged),
               "rel_resid": info.rel_resid, "abs_resid": info.abs_resid,
               "setup_ms": info.setup_ms, "solve_ms": info.solve_ms}
        if history:
            out["history"] = list(hist[:info.iters + 1])
        return out

    def time_smoother(self, reps=20):
        """Mean ms of one finest-level Jacobi sweep (HIP events, solver stream)."""
        ms = C.c_double()
        L.check(L.lib.mg_nodal_time_smoother(self.handle, int(reps), C.byref(ms)),
                "mg_nodal_time_smoother")
        return ms.value

    def apply(self, phi, out):
        pm, om = phi.c_struct(), out.c_struct()
        L.check(L.lib.mg_nodal_apply(self.handle, C.byref(pm), C.byref(om)), "mg_nodal_apply")
