"""Triangle and RWG geometry (oracle; test infrastructure only).

RWG basis (Sec. 3, ref. [14]): for edge k of length l_k shared by T+ and T-
with free vertices v+ and v-,
    S_k = +(l_k / 2A+) (r - v+) on T+,   S_k = -(l_k / 2A-) (r - v-) on T-,
    div S_k = +l_k/A+ on T+,  -l_k/A- on T-.
Each basis has two "halves" h = 0 (T+) and 1 (T-): triangle t[k,h], free
vertex f[k,h], sign s[k,h].  The basis centre is c_k = (centroid(T+) +
centroid(T-)) / 2.
"""
from __future__ import annotations

import numpy as np


class Surface:
    def __init__(self, xyz: np.ndarray, tri: np.ndarray, rwg: np.ndarray):
        self.xyz = np.asarray(xyz, dtype=np.float64)
        self.tri = np.asarray(tri, dtype=np.int64)
        self.rwg = np.asarray(rwg, dtype=np.int64)
        v = self.xyz[self.tri]                      # [nt,3,3]
        self.tv = v
        cr = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
        self.area = 0.5 * np.linalg.norm(cr, axis=1)
        self.normal = cr / (2.0 * self.area[:, None])
        self.centroid = (v[:, 0] + v[:, 1] + v[:, 2]) / 3.0
        ns = len(self.rwg)
        self.ns = ns
        tp, tm, e0, e1 = self.rwg.T
        self.length = np.linalg.norm(self.xyz[e1] - self.xyz[e0], axis=1)
        self.t = np.stack([tp, tm], axis=1)                      # [ns,2]
        self.s = np.tile(np.array([1.0, -1.0]), (ns, 1))          # [ns,2]
        loc = np.empty((ns, 2), dtype=np.int64)                  # local index of the free vertex
        for h in range(2):
            tt = self.tri[self.t[:, h]]
            isfree = (tt != e0[:, None]) & (tt != e1[:, None])
            if not np.all(isfree.sum(1) == 1):
                raise ValueError("RWG edge is not an edge of its triangle")
            loc[:, h] = np.argmax(isfree, axis=1)
        self.loc = loc
        self.free = self.tri[self.t, loc]                        # vertex ids [ns,2]
        self.c = (self.centroid[tp] + self.centroid[tm]) / 2.0

    def support_vertices(self) -> np.ndarray:
        """The four vertices of the support of each basis [ns,4,3]."""
        tp, tm, e0, e1 = self.rwg.T
        return np.stack([self.xyz[e0], self.xyz[e1], self.xyz[self.free[:, 0]],
                         self.xyz[self.free[:, 1]]], axis=1)
