"""Independent sparse assembly of the two-level composite operator.

Each row is built as a linear combination of unknowns from the definition:
flux form on both levels, fine ghost values written out as the coarse
interpolation formula, covered coarse values as the mean of their 8 fine
children, the folded Dirichlet ghost -phi at walls, and the coarse flux across
a coarse/fine face replaced by the mean of the 4 fine fluxes.  No boxes, no
ghost exchange and none of the oracle's code are used.
"""

import numpy as np
import scipy.sparse as sp


class CompositeRef:
    def __init__(self, nc, fine_boxes, bcell, cfaces, ffaces_global, alpha=1.0, beta=1.0):
        """nc: coarse cells per side; fine_boxes in fine index space; cfaces: global
        coarse face arrays; ffaces_global: global fine face arrays (2nc+1, 2nc, 2nc) etc."""
        self.nc = nc
        self.nf = 2 * nc
        self.hc = 1.0 / nc
        self.hf = 1.0 / self.nf
        self.alpha, self.beta = alpha, beta
        self.cfaces, self.ffaces = cfaces, ffaces_global
        self.fine = np.zeros((self.nf,) * 3, bool)
        for lo, hi in fine_boxes:
            self.fine[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1] = True
        self.covered = self.fine.reshape(nc, 2, nc, 2, nc, 2).all(axis=(1, 3, 5))
        self.fid = {}
        for p in zip(*np.nonzero(self.fine)):
            self.fid[tuple(int(x) for x in p)] = len(self.fid)
        self.cid = {}
        for p in zip(*np.nonzero(~self.covered)):
            self.cid[tuple(int(x) for x in p)] = len(self.fid) + len(self.cid)
        self.n = len(self.fid) + len(self.cid)

    # linear combinations are dicts {unknown: coefficient}
    @staticmethod
    def _add(a, b, s=1.0):
        out = dict(a)
        for k, v in b.items():
            out[k] = out.get(k, 0.0) + s * v
        return out

    @staticmethod
    def _scale(a, s):
        return {k: v * s for k, v in a.items()}

    def coarse_val(self, C):
        C = tuple(C)
        if self.covered[C]:
            out = {}
            for o in np.ndindex(2, 2, 2):
                out[self.fid[tuple(2 * C[a] + o[a] for a in range(3))]] = 0.125
            return out
        return {self.cid[C]: 1.0}

    def ghost_val(self, g):
        C = [x // 2 for x in g]
        vc = self.coarse_val(C)
        acc = dict(vc)
        for d in range(3):
            hi = list(C)
            lo = list(C)
            hi[d] += 1
            lo[d] -= 1
            vhi = self.coarse_val(hi) if hi[d] < self.nc else self._scale(vc, -1.0)
            vlo = self.coarse_val(lo) if lo[d] >= 0 else self._scale(vc, -1.0)
            sgn = 1.0 if g[d] % 2 == 1 else -1.0
            acc = self._add(acc, self._add(vhi, vlo, -1.0), 0.25 * 0.5 * sgn)
        return acc

    def fine_neighbour(self, p, q):
        """Value at fine position q next to fine valid cell p."""
        if any(x < 0 or x >= self.nf for x in q):
            return {self.fid[p]: -1.0}
        if self.fine[q]:
            return {self.fid[q]: 1.0}
        return self.ghost_val(q)

    def matrix(self, acell_f=None, acell_c=None):
        rows, cols, vals = [], [], []

        def put(r, comb):
            for k, v in comb.items():
                rows.append(r)
                cols.append(k)
                vals.append(v)

        for p, r in self.fid.items():
            me = {r: 1.0}
            a = 1.0 if acell_f is None else acell_f[p]
            comb = self._scale(me, self.alpha * a)
            for d in range(3):
                hi = list(p)
                lo = list(p)
                hi[d] += 1
                lo[d] -= 1
                bhi = self.ffaces[d][tuple(hi)]
                blo = self.ffaces[d][p]
                flux = self._add(self._scale(self._add(self.fine_neighbour(p, tuple(hi)), me, -1.0),
                                             bhi),
                                 self._scale(self._add(me, self.fine_neighbour(p, tuple(lo)), -1.0),
                                             -blo))
                comb = self._add(comb, flux, -self.beta / self.hf ** 2)
            put(r, comb)
        for I, r in self.cid.items():
            me = {r: 1.0}
            a = 1.0 if acell_c is None else acell_c[I]
            comb = self._scale(me, self.alpha * a)
            for d in range(3):
                for side in (1, -1):
                    J = list(I)
                    J[d] += side
                    J = tuple(J)
                    fidx = list(I)
                    if side > 0:
                        fidx[d] += 1
                    b = self.cfaces[d][tuple(fidx)]
                    if not (0 <= J[d] < self.nc):
                        nb = self._scale(me, -1.0)
                        F = self._scale(self._add(nb, me, -1.0) if side > 0 else
                                        self._add(me, nb, -1.0), self.beta * b / self.hc)
                    elif not self.covered[J]:
                        nb = {self.cid[J]: 1.0}
                        F = self._scale(self._add(nb, me, -1.0) if side > 0 else
                                        self._add(me, nb, -1.0), self.beta * b / self.hc)
                    else:
                        F = {}
                        tr = [x for x in range(3) if x != d]
                        for o1 in (0, 1):
                            for o2 in (0, 1):
                                fc = [0, 0, 0]
                                fc[tr[0]] = 2 * J[tr[0]] + o1
                                fc[tr[1]] = 2 * J[tr[1]] + o2
                                fc[d] = 2 * J[d] + (0 if side > 0 else 1)
                                g = list(fc)
                                g[d] -= side
                                face = list(fc) if side > 0 else list(g)
                                bf = self.ffaces[d][tuple(face)]
                                vin = {self.fid[tuple(fc)]: 1.0}
                                vg = self.ghost_val(tuple(g))
                                fl = self._add(vin, vg, -1.0) if side > 0 else self._add(vg, vin, -1.0)
                                F = self._add(F, fl, 0.25 * self.beta * bf / self.hf)
                    comb = self._add(comb, F, -side / self.hc)
            put(r, comb)
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.n, self.n))

    def pack(self, fine_global, coarse_global):
        x = np.zeros(self.n)
        for p, r in self.fid.items():
            x[r] = fine_global[p]
        for p, r in self.cid.items():
            x[r] = coarse_global[p]
        return x

    def unpack(self, x):
        F = np.zeros((self.nf,) * 3)
        C = np.zeros((self.nc,) * 3)
        for p, r in self.fid.items():
            F[p] = x[r]
        for p, r in self.cid.items():
            C[p] = x[r]
        return F, C
