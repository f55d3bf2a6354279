"""Python face of the C ABI: MLMG solver handle, fill_boundary, copy tags.

Only marshalling: every numerical step runs in libamrmg.so.  Device memory
(MultiFab data and the solver's workspace) comes from PyTorch's allocator.
"""

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from .multifab import MultiFab


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def copy_tags(boxes, domain, periodic, ngrow):
    """Ghost-exchange copy tags from the library's hash intersection (host only).

    Returns tuples (dst, src, (lo, hi), shift) in canonical order."""
    bx = L.boxes_array(boxes)
    g = L.geom_struct(domain, periodic)
    n = C.c_int32(0)
    L.check(L.lib.mg_copy_tags(bx, len(boxes), C.byref(g), ngrow, None, 0, C.byref(n)),
            "mg_copy_tags")
    arr = (L.MgCopyTag * max(1, n.value))()
    L.check(L.lib.mg_copy_tags(bx, len(boxes), C.byref(g), ngrow, arr, n.value, C.byref(n)),
            "mg_copy_tags")
    out = []
    for t in arr[:n.value]:
        out.append((t.dst, t.src, (tuple(t.dst_region.lo), tuple(t.dst_region.hi)), tuple(t.shift)))
    return out


def workspace_bytes(boxes, domain, periodic, opts=None, has_acoef=False):
    bx = L.boxes_array(boxes)
    g = L.geom_struct(domain, periodic)
    o = opts if opts is not None else L.default_opts()
    n = C.c_size_t(0)
    L.check(L.lib.mg_query_workspace(bx, len(boxes), C.byref(g), C.byref(o), int(has_acoef),
                                     C.byref(n)), "mg_query_workspace")
    return n.value


def num_levels(boxes, domain, periodic, opts=None):
    bx = L.boxes_array(boxes)
    g = L.geom_struct(domain, periodic)
    o = opts if opts is not None else L.default_opts()
    n = C.c_int32(0)
    L.check(L.lib.mg_num_levels(bx, len(boxes), C.byref(g), C.byref(o), C.byref(n)),
            "mg_num_levels")
    return n.value


def fill_boundary(mf, domain, periodic, stream=None):
    """Fill mf's ghost cells from neighbouring boxes and periodic images."""
    g = L.geom_struct(domain, periodic)
    m = mf.c_struct()
    L.check(L.lib.fill_boundary(C.byref(m), C.byref(g), _stream_handle(stream)), "fill_boundary")


def fill_boundary_noalloc(mf, domain, periodic, stream=None):
    """fill_boundary without device allocation (plan staged in the library's
    static device scratch; overlapping calls on one device race)."""
    g = L.geom_struct(domain, periodic)
    m = mf.c_struct()
    L.check(L.lib.mg_fill_boundary_noalloc(C.byref(m), C.byref(g), _stream_handle(stream)),
            "mg_fill_boundary_noalloc")


def stream_copy(dst, src, stream=None):
    """dst.copy_(src) with the library's streaming kernel (contiguous device
    tensors of equal byte size, 16-byte aligned)."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes and src.is_contiguous() and dst.is_contiguous()
    L.check(L.lib.mg_stream_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nbytes,
                                 _stream_handle(stream)), "mg_stream_copy")


class MLMG:
    """Multigrid solver of alpha*a*phi - beta*div(b grad phi) = f on one level.

    boxes: list of (lo, hi) cell boxes covering ``domain``; periodic: 3 bools
    (other directions are homogeneous Dirichlet walls); a: cell MultiFab or
    None (a = 1); b: three face MultiFabs or None (b = 1); opts: keyword
    overrides of mg_opts_t (see include/amrmg.h)."""

    def __init__(self, boxes, domain, periodic, alpha, beta, a=None, b=None, opts=None,
                 prob_lo=(0.0, 0.0, 0.0), prob_hi=(1.0, 1.0, 1.0), stream=None):
        self.boxes = [(tuple(lo), tuple(hi)) for lo, hi in boxes]
        self.domain = domain
        self.periodic = tuple(bool(p) for p in periodic)
        self.n = tuple(domain[1][d] - domain[0][d] + 1 for d in range(3))
        self.opts = L.default_opts(**(opts or {}))
        self._bx = L.boxes_array(self.boxes)
        self._geom = L.geom_struct(domain, periodic, prob_lo, prob_hi)
        bc = (C.c_int32 * 3)(*[L.MG_BC_PERIODIC if p else L.MG_BC_DIRICHLET0 for p in periodic])
        nbytes = workspace_bytes(self.boxes, domain, periodic, self.opts, a is not None)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        ptr = self.workspace.data_ptr()
        self._ws_ptr = (ptr + 255) // 256 * 256
        self._stream = stream
        am = a.c_struct() if a is not None else None
        if b is not None:
            bms = [x.c_struct() for x in b]
            barr = (C.POINTER(L.MgMultiFab) * 3)(*[C.pointer(x) for x in bms])
            bptr = C.cast(barr, C.POINTER(C.POINTER(L.MgMultiFab)))
        else:
            bptr = None
        h = C.c_void_p()
        L.check(L.lib.mg_create(self._bx, len(self.boxes), C.byref(self._geom), bc, bc,
                                float(alpha), float(beta), C.byref(am) if am is not None else None,
                                bptr, C.byref(self.opts), C.c_void_p(self._ws_ptr), nbytes,
                                _stream_handle(stream), C.byref(h)), "mg_create")
        self.handle = h
        self.has_a = a is not None
        self.coef_version = 0

    def close(self):
        if getattr(self, "handle", None):
            L.lib.mg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- MultiFab factories over the solver's boxes ----------------------------
    def cell_mf(self, ngrow=0, fill=None):
        return MultiFab(self.boxes, ngrow, fill=fill)

    def face_mf(self, d, fill=None):
        e = [0, 0, 0]
        e[d] = 1
        return MultiFab(self.boxes, 0, ixtype=tuple(e), fill=fill)

    # -- calls ------------------------------------------------------------------
    def solve(self, phi, rhs, rel_tol=1e-10, abs_tol=0.0, history=False, raise_on_fail=True):
        pm, rm = phi.c_struct(), rhs.c_struct()
        info = L.MgInfo()
        hist = (C.c_double * (self.opts.max_iter + 1))() if history else None
        code = L.lib.mg_solve(self.handle, C.byref(pm), C.byref(rm), float(rel_tol),
                              float(abs_tol), C.byref(info), hist)
        if raise_on_fail and code != L.MG_OK:
            L.check(code, "mg_solve")
        out = {"status": code, "iters": info.iters, "nlevels": info.nlevels,
               "bottom_iters": info.bottom_iters, "converged": bool(info.converged),
               "rel_resid": info.rel_resid, "abs_resid": info.abs_resid,
               "setup_ms": info.setup_ms, "solve_ms": info.solve_ms,
               "tail_level": info.tail_level}
        if history:
            out["history"] = list(hist[:info.iters + 1])
        return out

    def apply(self, phi, out):
        pm, om = phi.c_struct(), out.c_struct()
        L.check(L.lib.mg_apply(self.handle, C.byref(pm), C.byref(om)), "mg_apply")

    def copy_valid(self, src, dst):
        sm, dm = src.c_struct(), dst.c_struct()
        L.check(L.lib.mg_copy_valid(self.handle, C.byref(sm), C.byref(dm)), "mg_copy_valid")

    def face_grad_logb(self, phi, lam, grads):
        pm, lm = phi.c_struct(), lam.c_struct()
        gms = [g.c_struct() for g in grads]
        arr = (C.POINTER(L.MgMultiFab) * 3)(*[C.pointer(x) for x in gms])
        L.check(L.lib.mg_face_grad_logb(self.handle, C.byref(pm), C.byref(lm),
                                        C.cast(arr, C.POINTER(C.POINTER(L.MgMultiFab)))),
                "mg_face_grad_logb")

    def global_face_shape(self, d):
        """Shape (nz, ny, nx) + e_d of an x-fastest global face tensor."""
        n = list(self.n)
        n[d] += 1
        return (n[2], n[1], n[0])

    def face_grad_logb_global(self, phi, lam):
        outs = [torch.empty(self.global_face_shape(d), dtype=torch.float64, device="cuda")
                for d in range(3)]
        pm, lm = phi.c_struct(), lam.c_struct()
        ptrs = (C.c_void_p * 3)(*[t.data_ptr() for t in outs])
        L.check(L.lib.mg_face_grad_logb_global(self.handle, C.byref(pm), C.byref(lm), ptrs),
                "mg_face_grad_logb_global")
        return outs

    def set_coefficients_global(self, bfaces, is_log=True, a_global=None):
        """bfaces: three contiguous float64 device tensors of x-fastest global faces."""
        for d, t in enumerate(bfaces):
            assert t.is_contiguous() and t.dtype == torch.float64
            assert tuple(t.shape) == self.global_face_shape(d)
        ptrs = (C.c_void_p * 3)(*[t.data_ptr() for t in bfaces])
        ap = C.c_void_p(a_global.data_ptr()) if a_global is not None else None
        L.check(L.lib.mg_set_coefficients_global(self.handle, ap, ptrs, int(bool(is_log))),
                "mg_set_coefficients_global")
        self.coef_version += 1

    def set_coefficients(self, a=None, b=None):
        am = a.c_struct() if a is not None else None
        if b is not None:
            bms = [x.c_struct() for x in b]
            barr = (C.POINTER(L.MgMultiFab) * 3)(*[C.pointer(x) for x in bms])
            bptr = C.cast(barr, C.POINTER(C.POINTER(L.MgMultiFab)))
        else:
            bptr = None
        L.check(L.lib.mg_set_coefficients(self.handle, C.byref(am) if am is not None else None,
                                          bptr), "mg_set_coefficients")
        self.coef_version += 1

    def profile(self, enable=True):
        L.check(L.lib.mg_profile(self.handle, int(enable)), "mg_profile")

    def kernel_stats(self, family):
        t = C.c_double(0)
        n = C.c_int64(0)
        L.check(L.lib.mg_kernel_stats(self.handle, family, C.byref(t), C.byref(n)),
                "mg_kernel_stats")
        return t.value, n.value

    def tile_shape(self, kernel):
        """Level-0 tile shape in use: kernel 0 smoother (lx, ly, tz, unroll, whole_pairs),
        1 cell kernels (lx, ly, tz, unroll, 0), 3 fused sweep (lx, ly, tz, in_use, 0),
        4 residual pass restricting into level 1 (lx, ly, tz, in_use, 0)."""
        out = (C.c_int32 * 5)()
        L.check(L.lib.mg_get_tile_shape(self.handle, kernel, out), "mg_get_tile_shape")
        return tuple(out)

    def set_tile_shape(self, kernel, lx, ly, tz, unroll=1):
        L.check(L.lib.mg_set_tile_shape(self.handle, kernel, lx, ly, tz, unroll),
                "mg_set_tile_shape")

    def set_class_tile_shape(self, x_extent, lx, ly, tz):
        L.check(L.lib.mg_set_class_tile_shape(self.handle, x_extent, lx, ly, tz),
                "mg_set_class_tile_shape")

    def class_tile_shapes(self):
        """{x extent: (lx, ly, tz)} of the level-0 smoother's per-class tiles ({} = uniform)."""
        n = C.c_int32()
        L.check(L.lib.mg_get_class_tile_shapes(self.handle, None, 0, C.byref(n)),
                "mg_get_class_tile_shapes")
        buf = (C.c_int32 * max(1, 4 * n.value))()
        L.check(L.lib.mg_get_class_tile_shapes(self.handle, buf, n.value, C.byref(n)),
                "mg_get_class_tile_shapes")
        return {buf[4 * i]: (buf[4 * i + 1], buf[4 * i + 2], buf[4 * i + 3]) for i in range(n.value)}

    def time_smoother(self, phi, rhs, reps=20):
        pm, rm = phi.c_struct(), rhs.c_struct()
        ms = C.c_double(0)
        L.check(L.lib.mg_time_smoother(self.handle, C.byref(pm), C.byref(rm), reps, C.byref(ms)),
                "mg_time_smoother")
        return ms.value


def release_caches():
    L.lib.mg_release_caches()


class CompositeMLMG:
    """Two-level composite solve: coarse boxes covering a Dirichlet-walled domain
    and fine boxes (coarse index space refined by 2) over part of it.

    b_c / b_f: three face MultiFabs on the coarse / fine boxes, or None for b = 1."""

    def __init__(self, coarse_boxes, fine_boxes, domain, alpha, beta, b_c=None, b_f=None,
                 opts=None, prob_lo=(0.0, 0.0, 0.0), prob_hi=(1.0, 1.0, 1.0), stream=None):
        self.boxes = [(tuple(lo), tuple(hi)) for lo, hi in coarse_boxes]
        self.fine_boxes = [(tuple(lo), tuple(hi)) for lo, hi in fine_boxes]
        self.domain = domain
        self.opts = L.default_opts(**(opts or {}))
        self._cb = L.boxes_array(self.boxes)
        self._fb = L.boxes_array(self.fine_boxes)
        self._geom = L.geom_struct(domain, (False, False, False), prob_lo, prob_hi)
        n = C.c_size_t(0)
        L.check(L.lib.mg_query_workspace_amr(self._cb, len(self.boxes), self._fb,
                                             len(self.fine_boxes), C.byref(self._geom),
                                             C.byref(self.opts), C.byref(n)),
                "mg_query_workspace_amr")
        nbytes = n.value
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        ws = (self.workspace.data_ptr() + 255) // 256 * 256

        def faces(mfs):
            if mfs is None:
                return None, None
            ms = [x.c_struct() for x in mfs]
            arr = (C.POINTER(L.MgMultiFab) * 3)(*[C.pointer(x) for x in ms])
            return C.cast(arr, C.POINTER(C.POINTER(L.MgMultiFab))), (ms, arr)

        bc, keep_c = faces(b_c)
        bf, keep_f = faces(b_f)
        h = C.c_void_p()
        L.check(L.lib.mg_create_amr(self._cb, len(self.boxes), self._fb, len(self.fine_boxes),
                                    C.byref(self._geom), float(alpha), float(beta), bc, bf,
                                    C.byref(self.opts), C.c_void_p(ws), nbytes,
                                    _stream_handle(stream), C.byref(h)), "mg_create_amr")
        del keep_c, keep_f
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            L.lib.mg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def coarse_mf(self, ngrow=0, fill=None):
        return MultiFab(self.boxes, ngrow, fill=fill)

    def fine_mf(self, ngrow=0, fill=None):
        return MultiFab(self.fine_boxes, ngrow, fill=fill)

    def solve(self, phi_c, phi_f, rhs_c, rhs_f, rel_tol=1e-10, abs_tol=0.0, history=False,
              raise_on_fail=True):
        pc, pf, rc, rf = phi_c.c_struct(), phi_f.c_struct(), rhs_c.c_struct(), rhs_f.c_struct()
        info = L.MgInfo()
        hist = (C.c_double * (self.opts.max_iter + 1))() if history else None
        code = L.lib.mg_solve_amr(self.handle, C.byref(pc), C.byref(pf), C.byref(rc), C.byref(rf),
                                  float(rel_tol), float(abs_tol), C.byref(info), hist)
        if raise_on_fail and code != L.MG_OK:
            L.check(code, "mg_solve_amr")
        out = {"status": code, "iters": info.iters, "nlevels": info.nlevels,
               "converged": bool(info.converged), "rel_resid": info.rel_resid,
               "abs_resid": info.abs_resid, "setup_ms": info.setup_ms, "solve_ms": info.solve_ms,
               "tail_level": info.tail_level}
        if history:
            out["history"] = list(hist[:info.iters + 1])
        return out
