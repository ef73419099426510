"""Structured box mesh, box decomposition and the orthonormal gluing matrix B.

Oracle (test infrastructure).

Numbering (fixed so that index maps can be compared bit for bit):
* global node (i, j, k) -> i + (Nx+1) * (j + (Ny+1) * k);
* subdomain (I, J, K) -> I + Sx * (J + Sy * K) when every box of the
  decomposition is present; boxes listed in the workload's ``absent`` are
  left out of the body (a hole through the decomposition) and the others
  keep that order;
* local nodes and local elements of a subdomain: lexicographic, x fastest;
* torn DOF of (subdomain p, local node a, component c): off_p + 3 a + c,
  subdomains stacked in order (Section 4.1: the torn vector stacks the
  subdomain vectors).

The constraint matrix B = [B_G; B_U] (Section 4.1) is built in orthonormal
form.  The paper only states that the redundant +1/-1 rows of each shared node
are orthonormalised and dependent rows removed; the reading used here, for
each (global node, component) whose copies live in subdomains p_1 < ... < p_k:

* Dirichlet-constrained (node, component): k rows of B_U, one per copy, each
  +1 at that copy, and no B_G rows (gluing rows there would make B rank
  deficient, violating the full-row-rank condition of Section 4.2);
* otherwise, if k > 1: Helmert rows j = 1..k-1 with +c_j at p_1..p_j and
  -j c_j at p_{j+1}, c_j = 1/sqrt(j (j+1)): classical Gram-Schmidt on the
  redundant rows e_{p_a} - e_{p_b} (a < b) in lexicographic order.

Row order: all B_G rows (node ascending, component, j), then all B_U rows
(node ascending, component, copy ascending).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import q1


@dataclass
class Subdomain:
    index: int
    IJK: tuple
    e0: tuple              # first global element index per axis
    n: tuple               # elements per axis (nx, ny, nz)
    n_nodes: int
    n_dofs: int
    off: int               # torn DOF offset
    l2g: np.ndarray        # local node -> global node
    elems: np.ndarray      # (n_el, 8) local node indices per element
    coords: np.ndarray     # (n_nodes, 3)


class Mesh:
    def __init__(self, w):
        self.w = w
        Sx, Sy, Sz = w.S
        self.S = (Sx, Sy, Sz)
        self.N = (sum(w.nx), sum(w.ny), sum(w.nz))
        self.h = tuple(w.extent[d] / self.N[d] for d in range(3))
        Nx, Ny, Nz = self.N
        self.n_gnodes = (Nx + 1) * (Ny + 1) * (Nz + 1)
        starts = [np.concatenate([[0], np.cumsum(a)[:-1]]).astype(int) for a in (w.nx, w.ny, w.nz)]
        self.subs: list[Subdomain] = []
        off = 0
        absent = set(tuple(b) for b in getattr(w, "absent", []) or [])
        p = -1
        for K in range(Sz):
            for J in range(Sy):
                for I in range(Sx):
                    if (I, J, K) in absent:
                        continue
                    p += 1
                    n = (w.nx[I], w.ny[J], w.nz[K])
                    e0 = (starts[0][I], starts[1][J], starts[2][K])
                    ni, nj, nk = n[0] + 1, n[1] + 1, n[2] + 1
                    kk, jj, ii = np.meshgrid(np.arange(nk), np.arange(nj), np.arange(ni), indexing="ij")
                    gi, gj, gk = ii.ravel() + e0[0], jj.ravel() + e0[1], kk.ravel() + e0[2]
                    l2g = gi + (Nx + 1) * (gj + (Ny + 1) * gk)
                    coords = np.stack([gi * self.h[0], gj * self.h[1], gk * self.h[2]], axis=1)
                    ek, ej, ei = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
                    ei, ej, ek = ei.ravel(), ej.ravel(), ek.ravel()
                    elems = np.stack([(ei + o[0]) + ni * ((ej + o[1]) + nj * (ek + o[2]))
                                      for o in q1.NODE_OFF], axis=1)
                    nn = ni * nj * nk
                    self.subs.append(Subdomain(p, (I, J, K), e0, n, nn, 3 * nn, off, l2g, elems, coords))
                    off += 3 * nn
        self.subs.sort(key=lambda s: s.index)
        # recompute offsets in subdomain order (loop order above is already p order)
        off = 0
        for s in self.subs:
            s.off = off
            off += s.n_dofs
        self.n_torn = off
        self.n_elems = sum(len(s.elems) for s in self.subs)
        # global nodes that belong to some subdomain (all, unless boxes are absent)
        self.used = np.zeros(self.n_gnodes, dtype=bool)
        for s in self.subs:
            self.used[s.l2g] = True
        self._build_dirichlet()
        self._build_B()

    # ------------------------------------------------------------------ boundary
    def node_ijk(self, g: np.ndarray):
        Nx, Ny, _ = self.N
        i = g % (Nx + 1)
        j = (g // (Nx + 1)) % (Ny + 1)
        k = g // ((Nx + 1) * (Ny + 1))
        return i, j, k

    def _build_dirichlet(self):
        """dir_mask[g, c] = True if component c of global node g is fixed."""
        Nx, Ny, Nz = self.N
        g = np.arange(self.n_gnodes)
        i, j, k = self.node_ijk(g)
        on_face = [i == 0, i == Nx, j == 0, j == Ny, k == 0, k == Nz]
        mask = np.zeros((self.n_gnodes, 3), dtype=bool)
        for f in range(6):
            for c in range(3):
                if self.w.dirichlet[f][c]:
                    mask[on_face[f], c] = True
        self.dir_mask = mask

    def _build_B(self):
        g_all = np.concatenate([s.l2g for s in self.subs])
        p_all = np.concatenate([np.full(s.n_nodes, s.index) for s in self.subs])
        a_all = np.concatenate([np.arange(s.n_nodes) for s in self.subs])
        order = np.lexsort((p_all, g_all))
        g_s, p_s, a_s = g_all[order], p_all[order], a_all[order]
        bounds = np.flatnonzero(np.diff(g_s)) + 1
        starts = np.concatenate([[0], bounds])
        ends = np.concatenate([bounds, [len(g_s)]])
        offs = np.array([s.off for s in self.subs])

        rows_G, rows_U = [], []      # each row: list of (torn dof, coef)
        for st, en in zip(starts, ends):
            g = g_s[st]
            copies = [(p_s[t], a_s[t]) for t in range(st, en)]
            k = len(copies)
            for c in range(3):
                dofs = [offs[p] + 3 * a + c for (p, a) in copies]
                if self.dir_mask[g, c]:
                    for d in dofs:
                        rows_U.append([(d, 1.0)])
                elif k > 1:
                    for j in range(1, k):
                        cj = 1.0 / np.sqrt(float(j * (j + 1)))
                        row = [(dofs[t], cj) for t in range(j)]
                        row.append((dofs[j], -float(j) * cj))
                        rows_G.append(row)
        rows = rows_G + rows_U
        self.m_G, self.m_U = len(rows_G), len(rows_U)
        self.m = len(rows)
        indptr = np.zeros(self.m + 1, dtype=np.int64)
        indptr[1:] = np.cumsum([len(r) for r in rows])
        idx = np.array([d for r in rows for (d, _) in r], dtype=np.int64)
        val = np.array([v for r in rows for (_, v) in r], dtype=np.float64)
        self.B = sp.csr_matrix((val, idx, indptr), shape=(self.m, self.n_torn))
        self.B_indptr, self.B_idx, self.B_val = indptr, idx, val

    # ------------------------------------------------------------------ loads
    def torn_load(self, load_factor: float = 1.0) -> np.ndarray:
        """Torn load vector f: each subdomain integrates the traction on its own
        part of the loaded faces (Section 4.1: f_p is the load on Omega^p and
        Gamma_N^p)."""
        f = np.zeros(self.n_torn)
        Nx, Ny, Nz = self.N
        hx, hy, hz = self.h
        for s in self.subs:
            ni, nj, nk = s.n[0] + 1, s.n[1] + 1, s.n[2] + 1
            for face in range(6):
                t = np.asarray(self.w.traction[face], dtype=np.float64) * load_factor
                if not np.any(t):
                    continue
                axis, side = face // 2, face % 2
                glob = (0, self.N[axis])[side]
                loc = (0, s.n[axis])[side]
                if s.e0[axis] + loc != glob:
                    continue
                # the two in-plane axes, in increasing order
                a1, a2 = [d for d in range(3) if d != axis]
                ha, hb = (hx, hy, hz)[a1], (hx, hy, hz)[a2]
                fl = q1.face_load((ha, hb), t)
                for ib in range(s.n[a2]):
                    for ia in range(s.n[a1]):
                        for q, (da, db) in enumerate(((0, 0), (1, 0), (1, 1), (0, 1))):
                            ijk = [0, 0, 0]
                            ijk[axis] = loc
                            ijk[a1] = ia + da
                            ijk[a2] = ib + db
                            a = ijk[0] + ni * (ijk[1] + nj * ijk[2])
                            f[s.off + 3 * a:s.off + 3 * a + 3] += fl[q]
        return f

    # ------------------------------------------------------------------ torn/untorn maps
    def untorn_index(self) -> np.ndarray:
        """For each global DOF 3g + c of a node that belongs to some subdomain
        (node ascending), the torn DOF of its lowest-p copy."""
        first = np.full(self.n_gnodes, -1, dtype=np.int64)
        for s in self.subs:
            sel = first[s.l2g] < 0
            first[s.l2g[sel]] = s.off + 3 * np.nonzero(sel)[0]
        idx = (first[self.used][:, None] + np.arange(3)[None, :]).ravel()
        return idx

    def used_dofs(self) -> np.ndarray:
        """Global DOF indices 3g + c of the nodes that belong to some subdomain,
        in the order of untorn_index."""
        g = np.nonzero(self.used)[0]
        return (3 * g[:, None] + np.arange(3)[None, :]).ravel()

    def tear(self, u_global: np.ndarray) -> np.ndarray:
        out = np.zeros(self.n_torn)
        for s in self.subs:
            out[s.off:s.off + s.n_dofs] = u_global.reshape(-1, 3)[s.l2g].ravel()
        return out

    def subdomain_slice(self, p: int) -> slice:
        s = self.subs[p]
        return slice(s.off, s.off + s.n_dofs)
