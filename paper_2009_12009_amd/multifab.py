"""MultiFab: one level's data as a single flat device tensor plus box metadata.

Box b's array covers the box grown by ``ngrow`` cells (and one more cell along
d for face data, ixtype[d] = 1), is stored x-fastest, and starts at
``offsets[b]`` (canonical packing: boxes one after another).  This mirrors the
paper's FabArray/MultiFab of FArrayBoxes with nGrow ghost cells ("Containers
for mesh data").  Host-side helpers move per-box NumPy arrays indexed
[i, j, k] in and out; they only reorder memory.
"""

import ctypes as C

import numpy as np
import torch

from . import _lib as L


def box_shape(b, ngrow=0, ixtype=(0, 0, 0)):
    lo, hi = b
    return tuple(hi[d] - lo[d] + 1 + 2 * ngrow + ixtype[d] for d in range(3))


class MultiFab:
    def __init__(self, boxes, ngrow=0, dtype=torch.float64, ixtype=(0, 0, 0), device="cuda",
                 data=None, fill=None):
        self.boxes = [(tuple(int(x) for x in lo), tuple(int(x) for x in hi)) for lo, hi in boxes]
        self.ngrow = int(ngrow)
        self.ixtype = tuple(int(x) for x in ixtype)
        self.dtype = dtype
        self.shapes = [box_shape(b, self.ngrow, self.ixtype) for b in self.boxes]
        sizes = [int(np.prod(s)) for s in self.shapes]
        self.offsets = np.zeros(len(self.boxes), dtype=np.int64)
        if len(sizes) > 1:
            self.offsets[1:] = np.cumsum(sizes[:-1])
        self.size = int(sum(sizes))
        if data is None:
            data = torch.empty(self.size, dtype=dtype, device=device)
            if fill is not None:
                data.fill_(fill)
        else:
            assert data.numel() == self.size and data.dtype == dtype and data.is_contiguous()
        self.data = data
        self._boxes_c = L.boxes_array(self.boxes)
        self._offs_c = (C.c_int64 * len(self.boxes))(*[int(x) for x in self.offsets])

    # -- C view -----------------------------------------------------------
    def c_struct(self):
        m = L.MgMultiFab()
        m.nbox = len(self.boxes)
        m.boxes = C.cast(self._boxes_c, C.POINTER(L.MgBox))
        m.ngrow = self.ngrow
        m.ncomp = 1
        m.ixtype[:] = list(self.ixtype)
        m.dtype = L.MG_F64 if self.dtype == torch.float64 else L.MG_F32
        m.data = C.c_void_p(self.data.data_ptr())
        m.offsets = C.cast(self._offs_c, C.POINTER(C.c_int64))
        return m

    def like(self, ngrow=None, fill=None):
        return MultiFab(self.boxes, self.ngrow if ngrow is None else ngrow, self.dtype, self.ixtype,
                        self.data.device, fill=fill)

    # -- host transfer (layout only) ---------------------------------------
    def box_tensor(self, b):
        """View of box b's array indexed [k, j, i] (x fastest in memory)."""
        nx, ny, nz = self.shapes[b]
        o = int(self.offsets[b])
        return self.data[o:o + nx * ny * nz].view(nz, ny, nx)

    @classmethod
    def from_numpy(cls, boxes, arrays, ngrow=0, ixtype=(0, 0, 0), dtype=torch.float64,
                   device="cuda"):
        """From per-box NumPy arrays indexed [i, j, k] over the grown box."""
        mf = cls(boxes, ngrow, dtype, ixtype, device)
        flat = np.concatenate([np.asarray(a).ravel(order="F") for a in arrays])
        np_dt = np.float64 if dtype == torch.float64 else np.float32
        mf.data.copy_(torch.from_numpy(flat.astype(np_dt)))
        return mf

    def to_numpy(self):
        """Per-box NumPy arrays indexed [i, j, k] over the grown box."""
        flat = self.data.detach().cpu().numpy()
        out = []
        for s, o in zip(self.shapes, self.offsets):
            n = int(np.prod(s))
            out.append(flat[o:o + n].reshape(s, order="F"))
        return out

    def valid_numpy(self):
        g = self.ngrow
        return [a[g:a.shape[0] - g, g:a.shape[1] - g, g:a.shape[2] - g] if g else a
                for a in self.to_numpy()]


def global_to_xfast(a):
    """NumPy array indexed [i, j, k] -> torch-ready array of shape (nz, ny, nx) (x fastest)."""
    return np.ascontiguousarray(np.asarray(a).transpose(2, 1, 0))


def xfast_to_global(t):
    """Tensor/array of shape (nz, ny, nx) -> NumPy array indexed [i, j, k]."""
    if isinstance(t, torch.Tensor):
        t = t.detach().cpu().numpy()
    return np.asarray(t).transpose(2, 1, 0)
