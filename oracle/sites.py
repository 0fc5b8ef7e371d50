"""Unreduced lattice for the oracle: translations only (Sec. 4.1).

For every basis site b of the unit cell, list every lattice site whose bond
distance from (cell 0, b) is at most the truncation range L (Eq. 34).  The
bond distance is the minimal number of lattice bonds joining two sites,
found by breadth-first search over the bond graph of the unit cell.  No
point-group symmetry is used: the vertex is stored for each listed site
separately, so the oracle relies on no symmetry table.

TEST INFRASTRUCTURE ONLY (see the oracle package docstring).
"""

from __future__ import annotations

from collections import deque

import numpy as np


class UnreducedLattice:
    def __init__(self, model, L: int):
        cell = model.cell
        self.cell_def = cell
        self.L = int(L)
        nb = cell.n_basis
        self.nb = nb
        nbrs = [[] for _ in range(nb)]
        for (f, t, d0, d1, d2) in cell.bonds:
            nbrs[f].append(((d0, d1, d2), t))
            nbrs[t].append(((-d0, -d1, -d2), f))

        lists = []
        for b in range(nb):
            start = ((0, 0, 0), b)
            dist = {start: 0}
            order = [start]
            q = deque([start])
            while q:
                node = q.popleft()
                dn = dist[node]
                if dn == self.L:
                    continue
                (c, bb) = node
                for (d, b2) in nbrs[bb]:
                    nxt = ((c[0] + d[0], c[1] + d[1], c[2] + d[2]), b2)
                    if nxt not in dist:
                        dist[nxt] = dn + 1
                        order.append(nxt)
                        q.append(nxt)
            order.sort(key=lambda n: (dist[n], n[0], n[1]))
            lists.append((order, dist))

        self.nsites = np.array([len(o) for o, _ in lists], dtype=np.int32)
        ns = int(self.nsites.max())
        self.ns = ns
        self.cell = np.zeros((nb, ns, 3), dtype=np.int32)
        self.bas = np.zeros((nb, ns), dtype=np.int32)
        self.dist = np.full((nb, ns), -1, dtype=np.int32)
        for b, (order, dist) in enumerate(lists):
            for k, (c, bb) in enumerate(order):
                self.cell[b, k] = c
                self.bas[b, k] = bb
                self.dist[b, k] = dist[(c, bb)]
        rm = int(np.abs(self.cell).max()) if ns else 0
        self.rm = rm
        W = 2 * rm + 1
        self.lookup = np.full((nb, W, W, W, nb), -1, dtype=np.int32)
        for b in range(nb):
            for k in range(self.nsites[b]):
                c = self.cell[b, k]
                self.lookup[b, c[0] + rm, c[1] + rm, c[2] + rm, self.bas[b, k]] = k

        # positions, for chi(k) and for matching sites with other representations
        self.basis_pos = np.array(cell.basis, dtype=np.float64)
        self.site_pos = np.zeros((nb, ns, 3))
        for b in range(nb):
            for k in range(self.nsites[b]):
                self.site_pos[b, k] = cell.position(self.cell[b, k], self.bas[b, k])

        # couplings J_{(0,b),(c,b')}: each listed interaction and its reverse;
        # a Heisenberg model gives one number per site, an XYZ model (params
        # (Jx, Jy, Jz)) three: coupling[nb, ns, 3]; a general model (params
        # 3x3 matrices M, the term S_from . M . S_to of Sec. 5.3) a matrix per
        # site, coupling[nb, ns, 3, 3], the reverse direction getting M^T
        dims = {np.ndim(v) for v in model.params.values()}
        if 2 in dims:
            shape, zero = (nb, ns, 3, 3), np.zeros((3, 3))
        elif 1 in dims:
            shape, zero = (nb, ns, 3), np.zeros(3)
        else:
            shape, zero = (nb, ns), 0.0
        self.coupling = np.zeros(shape)
        for (pname, f, t, d0, d1, d2) in model.interactions:
            J = np.asarray(model.params.get(pname, zero), dtype=np.float64)
            if len(shape) == 4 and J.ndim < 2:       # a number or a diagonal in a general model
                J = np.diag(np.broadcast_to(J, (3,)).astype(np.float64))
            for (b1, d, b2, M) in ((f, (d0, d1, d2), t, J), (t, (-d0, -d1, -d2), f, J.T)):
                k = self.index(b1, d, b2)
                if k >= 0:
                    self.coupling[b1, k] += M

    def index(self, b1: int, d, b2: int) -> int:
        rm = self.rm
        if any(abs(int(x)) > rm for x in d):
            return -1
        return int(self.lookup[b1, d[0] + rm, d[1] + rm, d[2] + rm, b2])

    @property
    def n_total(self) -> int:
        """Sites within range of basis site 0 (N_s^total in Sec. 4.1)."""
        return int(self.nsites[0])
