"""Bisection refinement written out from its definition -- TEST INFRASTRUCTURE.

Only the test suite may import this module; the product package never does.

Sections 4.2 and 4.3 refine the mesh adaptively.  The definition used here
(Maubach's bisection of tagged simplices): a tetrahedron (x0, x1, x2, x3)
with tag d in {1, 2, 3} is cut at the midpoint z of its edge (x0, x_d) into
    (x0, ..., x_{d-1}, z, x_{d+1}, ..., x3)   and   (x1, ..., x_d, z, x_{d+1}, ..., x3),
both with tag d - 1 (3 after 1); the first child takes the parent's place in
the list, the second is appended.  The initial tetrahedra carry tag 3.
Marking follows Doerfler: sort by the squared indicator, largest first
(ties keep the list order), and take the shortest prefix whose sum reaches
theta times the total.  The marked tetrahedra are bisected in list order;
then, pass by pass, every tetrahedron (in list order) that has an edge
whose midpoint exists is bisected, until none has.  A vertex lies on the
boundary iff it belongs to a face of only one tetrahedron.  Plain Python
loops: small meshes only.
"""
from __future__ import annotations

import numpy as np


class Refiner:
    def __init__(self, xyz, tets):
        self.xyz = [tuple(map(float, p)) for p in np.asarray(xyz, dtype=np.float64)]
        self.tets = [list(map(int, t)) for t in np.asarray(tets)]
        self.tags = [3] * len(self.tets)
        self.mid = {}

    def _midpoint(self, a, b):
        k = (min(a, b), max(a, b))
        if k not in self.mid:
            pa, pb = self.xyz[a], self.xyz[b]
            self.xyz.append(tuple(0.5 * (pa[d] + pb[d]) for d in range(3)))
            self.mid[k] = len(self.xyz) - 1
        return self.mid[k]

    def _bisect(self, t):
        x = self.tets[t]
        d = self.tags[t]
        z = self._midpoint(x[0], x[d])
        c1 = x[:d] + [z] + x[d + 1:]
        c2 = x[1:d + 1] + [z] + x[d + 1:]
        nt = d - 1 if d > 1 else 3
        self.tets[t] = c1
        self.tags[t] = nt
        self.tets.append(c2)
        self.tags.append(nt)

    def _hanging(self, x):
        return any((min(x[a], x[b]), max(x[a], x[b])) in self.mid for a in range(4) for b in range(a + 1, 4))

    def refine(self, eta2, theta):
        eta2 = np.asarray(eta2, dtype=np.float64)
        order = sorted(range(len(eta2)), key=lambda e: -eta2[e])   # stable: ties keep list order
        total = float(eta2.sum())
        marked, acc = [], 0.0
        for e in order:
            if marked and acc >= theta * total:
                break
            marked.append(e)
            acc += eta2[e]
        for e in sorted(marked):
            self._bisect(e)
        while True:
            todo = [e for e in range(len(self.tets)) if self._hanging(self.tets[e])]
            if not todo:
                break
            for e in todo:
                self._bisect(e)
        return len(marked)

    def mesh(self):
        xyz = np.array(self.xyz, dtype=np.float64)
        tets = np.array(self.tets, dtype=np.int32)
        count = {}
        for t in self.tets:
            for a in range(4):
                f = tuple(sorted(t[:a] + t[a + 1:]))
                count[f] = count.get(f, 0) + 1
        dirichlet = np.zeros(len(xyz), dtype=np.uint8)
        for f, c in count.items():
            if c == 1:
                dirichlet[list(f)] = 1
        return xyz, tets, dirichlet
