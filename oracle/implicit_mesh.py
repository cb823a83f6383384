"""Implicitly defined meshes in 2D (section 5, "Curved domain geometry"): a
level set cuts the cells of a background n x n Cartesian grid; every cell
holds one piece per phase it meets; pieces smaller than a quarter of a cell
are merged into a neighbour of the same phase; and the multigrid hierarchy
agglomerates, level by level, the elements of one phase whose host cells
share a parent (section 3, "Mesh hierarchy": agglomeration only between
elements of the same phase).

TEST INFRASTRUCTURE ONLY (part of the oracle).

Readings (the paper defers these details to its references):

* merging: a piece of area fraction < 1/4 joins the neighbouring piece of
  the same phase, across a cell face, with which it shares the longest
  stretch of that face, pieces of fraction >= 1/4 preferred; faces are
  tried in the order -x, +x, -y, +y and the first of equal candidates
  wins (lengths within a relative 1e-12 count as equal, so that the
  mirror-symmetric ties of a circle do not depend on rounding).  A merged element keeps the cell of its large piece as host cell;
* basis: Q_p on the host cell (the orthonormal Legendre basis of a full
  cell), orthonormalised over the element's actual domain by the Cholesky
  factor L of its mass matrix, psi = L^{-1} phi (L obtained from a QR
  factorisation of the weighted basis samples); an element that is one whole
  cell (or, on coarse levels, the 2^d whole children of one parent) keeps
  the cell's basis unchanged.  A change of basis within each element leaves
  the block Gauss-Seidel iterates and the coarse operators unchanged up to
  the same change of basis, so this fixes only the representation;
* coarse levels are not merged again.

Elements are numbered by (host cell index, phase), cells by i_0 + n i_1.
"""
from __future__ import annotations

import numpy as np

from .basis import ref_basis, tensor_gauss, gauss01
from .implicit_quad import cut_box_rules, segment_rules

FRAC_MIN = 0.25
TIE = 1e-12            # shared lengths within this relative margin count as equal
DIRS = ((0, -1), (0, 1), (1, -1), (1, 1))      # (axis, step): -x, +x, -y, +y


class Element:
    def __init__(self, host, phase, X, w, full):
        self.host = host            # (i0, i1) of the host cell
        self.phase = phase
        self.X = X                  # quadrature points (Q, 2)
        self.w = w                  # weights (Q,)
        self.full = full            # True: the basis needs no orthonormalisation
        self.Linv = None

    @property
    def area(self):
        return float(self.w.sum())


class Face:
    """One face: ``kind`` 0 intraphase, 1 interphase, 2 Dirichlet wall;
    ``minus`` / ``plus`` element ids (plus = -1 on walls); points X,
    weights w, unit normal per point (from minus to plus, outward on walls)."""

    def __init__(self, kind, minus, plus, X, w, normal):
        self.kind, self.minus, self.plus = kind, minus, plus
        self.X, self.w, self.normal = X, w, normal


class MeshLevel:
    """Elements of one level and their basis (host cell width h)."""

    def __init__(self, n, p, elements):
        self.n, self.p = n, p
        self.h = 1.0 / n
        self.nq = (p + 1) ** 2
        self.elements = elements
        self.NE = len(elements)
        for e in elements:
            if e.full:
                e.Linv = np.eye(self.nq)
            else:
                # the Cholesky factor L of the raw mass matrix R^T W R, taken
                # from a QR factorisation of W^{1/2} R (L = R_qr^T with a
                # positive diagonal) rather than from the mass matrix itself,
                # whose condition number is the square of the samples'
                R = self.raw_basis(e, e.X)
                Rq = np.linalg.qr(np.sqrt(e.w)[:, None] * R, mode="r")
                Rq = Rq * np.sign(np.diag(Rq))[:, None]
                e.Linv = np.linalg.inv(Rq.T)

    def raw_basis(self, e, X, deriv_axis=None):
        lo = np.asarray(e.host, dtype=float) * self.h
        B = ref_basis(self.p, (X - lo[None, :]) / self.h, deriv_axis=deriv_axis) / self.h
        return B / self.h if deriv_axis is not None else B

    def basis(self, eid, X, deriv_axis=None):
        """Values (or d/dx_axis) of element eid's orthonormal basis at X: (Q, nq)."""
        e = self.elements[eid]
        return self.raw_basis(e, X, deriv_axis) @ e.Linv.T

    def chi(self):
        return np.array([e.phase for e in self.elements])


class ImplicitMesh(MeshLevel):
    """The finest level: cut cells, merging, faces.  With ``void_outside``
    (a curved domain: section 5, "Curved domain geometry") phase 2 is not
    part of the domain: its pieces are dropped and the interface becomes a
    Dirichlet wall of the phase-1 elements, normal pointing out of the
    domain."""

    def __init__(self, n, p, ls, q_full, q_cut, void_outside=False):
        self.ls = ls
        self.void_outside = void_outside
        h = 1.0 / n
        self.n, self.h = n, h
        self.q_full, self.q_cut = q_full, q_cut
        tp, tw = tensor_gauss(q_full, 2)
        pieces = {}                         # (cell, chi) -> (X, w)
        self.cut_cells = []
        self.surf = {}
        for i1 in range(n):
            for i0 in range(n):
                c = i0 + n * i1
                lo = np.array([i0, i1], dtype=float) * h
                hi = lo + h
                mn, mx = ls.box_range(lo, hi)
                if mn < 0.0 < mx:
                    r = cut_box_rules(ls, lo, hi, q_cut)
                    for chi in ((1,) if void_outside else (1, 2)):
                        X, w = r["vol"][chi]
                        if w.size and w.sum() > 0.0:
                            pieces[(c, chi)] = (X, w)
                    self.cut_cells.append(c)
                    self.surf[c] = r["surf"]
                else:
                    chi = 1 if mx <= 0.0 else 2
                    if chi == 2 and void_outside:
                        continue
                    pieces[(c, chi)] = ((np.array([i0, i1])[None, :] + tp) * h, tw * h * h)
        self.pieces = pieces
        frac = {key: w.sum() / (h * h) for key, (X, w) in pieces.items()}
        self.frac = frac
        # merging
        target = {}
        for key in sorted(pieces):
            if frac[key] >= FRAC_MIN:
                continue
            c, chi = key
            i0, i1 = c % n, c // n
            best, best_rank = None, None
            for axis, step in DIRS:
                j = [i0, i1]
                j[axis] += step
                if not (0 <= j[0] < n and 0 <= j[1] < n):
                    continue
                c2 = j[0] + n * j[1]
                if (c2, chi) not in pieces:
                    continue
                L = self._shared_length(i0, i1, axis, step, chi)
                if L <= 0.0:
                    continue
                large = frac[(c2, chi)] >= FRAC_MIN
                if (best_rank is None or large > best_rank[0]
                        or (large == best_rank[0] and L > best_rank[1] * (1.0 + TIE))):
                    best, best_rank = (c2, chi), (large, L)
            if best is None:
                raise ValueError(f"piece {key} has no neighbour of its phase to merge with")
            target[key] = best
        root = {}
        for key in pieces:
            k, seen = key, set()
            while k in target:
                if k in seen:
                    raise ValueError("merging cycle")
                seen.add(k)
                k = target[k]
            root[key] = k
        roots = sorted({root[k] for k in pieces})
        self.elem_of = {}
        elements = []
        for eid, rk in enumerate(roots):
            members = sorted(k for k in pieces if root[k] == rk)
            X = np.concatenate([pieces[k][0] for k in members])
            w = np.concatenate([pieces[k][1] for k in members])
            c = rk[0]
            full = len(members) == 1 and c not in self.surf
            elements.append(Element((c % n, c // n), rk[1], X, w, full))
            for k in members:
                self.elem_of[k] = eid
        self.merged = target
        super().__init__(n, p, elements)
        self.faces = self._faces()

    def _edge_rules(self, axis, m, i_other):
        """Per-phase rules on the grid edge x_axis = m h, x_other in
        [i_other h, (i_other + 1) h]."""
        h, n = self.h, self.n
        a, b = i_other * h, (i_other + 1) * h
        lo = np.zeros(2)
        hi = np.zeros(2)
        lo[axis] = hi[axis] = m * h
        lo[1 - axis], hi[1 - axis] = a, b
        mn, mx = self.ls.box_range(lo, hi)
        if mn < 0.0 < mx:
            return segment_rules(self.ls, axis, m * h, a, b, self.q_cut)
        xg, wg = gauss01(self.q_full)
        X = np.zeros((xg.size, 2))
        X[:, axis] = m * h
        X[:, 1 - axis] = a + h * xg
        chi = 1 if mx <= 0.0 else 2
        empty = (np.zeros((0, 2)), np.zeros(0))
        return {chi: (X, wg * h), 3 - chi: empty}

    def _shared_length(self, i0, i1, axis, step, chi):
        ij = [i0, i1]
        m = ij[axis] + (1 if step > 0 else 0)
        r = self._edge_rules(axis, m, ij[1 - axis])
        return float(r[chi][1].sum())

    def _faces(self):
        n = self.n
        faces = []
        for axis in (0, 1):
            for m in range(n + 1):
                for io in range(n):
                    rules = self._edge_rules(axis, m, io)
                    for chi in ((1,) if self.void_outside else (1, 2)):
                        X, w = rules[chi]
                        if w.size == 0:
                            continue
                        lo_c = hi_c = None
                        if m > 0:
                            ij = [0, 0]
                            ij[axis], ij[1 - axis] = m - 1, io
                            lo_c = ij[0] + n * ij[1]
                        if m < n:
                            ij = [0, 0]
                            ij[axis], ij[1 - axis] = m, io
                            hi_c = ij[0] + n * ij[1]
                        nrm = np.zeros((w.size, 2))
                        if lo_c is None:
                            nrm[:, axis] = -1.0
                            faces.append(Face(2, self.elem_of[(hi_c, chi)], -1, X, w, nrm))
                        elif hi_c is None:
                            nrm[:, axis] = 1.0
                            faces.append(Face(2, self.elem_of[(lo_c, chi)], -1, X, w, nrm))
                        else:
                            e1, e2 = self.elem_of[(lo_c, chi)], self.elem_of[(hi_c, chi)]
                            if e1 != e2:
                                nrm[:, axis] = 1.0
                                faces.append(Face(0, e1, e2, X, w, nrm))
        for c in self.cut_cells:
            X, w, nrm = self.surf[c]
            if w.size == 0:
                continue
            if self.void_outside:
                faces.append(Face(2, self.elem_of[(c, 1)], -1, X, w, nrm))
            else:
                faces.append(Face(1, self.elem_of[(c, 1)], self.elem_of[(c, 2)], X, w, nrm))
        return faces


def coarsen_mesh(fine: MeshLevel):
    """The next level: fine elements grouped by (parent of host cell, phase);
    returns (coarse level, parent id of every fine element)."""
    nc = fine.n // 2
    groups = {}
    for fid, e in enumerate(fine.elements):
        pc = (e.host[0] // 2) + nc * (e.host[1] // 2)
        groups.setdefault((pc, e.phase), []).append(fid)
    keys = sorted(groups)
    parent = np.empty(fine.NE, dtype=int)
    elements = []
    for cid, key in enumerate(keys):
        kids = groups[key]
        X = np.concatenate([fine.elements[f].X for f in kids])
        w = np.concatenate([fine.elements[f].w for f in kids])
        full = len(kids) == 4 and all(fine.elements[f].full for f in kids)
        elements.append(Element((key[0] % nc, key[0] // nc), key[1], X, w, full))
        parent[kids] = cid
    return MeshLevel(nc, fine.p, elements), parent


def prolongation(fine: MeshLevel, coarse: MeshLevel, parent):
    """Scalar injection I (fine dofs x coarse dofs): the L2 projection of each
    coarse basis function onto the fine element's basis, by the fine
    element's quadrature (exact: the coarse polynomial restricted to a fine
    element lies in the fine element's space)."""
    import scipy.sparse as sp
    nq = fine.nq
    rows, cols, vals = [], [], []
    ar = np.arange(nq)
    for f, e in enumerate(fine.elements):
        c = parent[f]
        Bf = fine.basis(f, e.X)
        Bc = coarse.basis(c, e.X)
        blk = (Bf * e.w[:, None]).T @ Bc
        rows.append(np.repeat(f * nq + ar, nq))
        cols.append(np.tile(c * nq + ar, nq))
        vals.append(blk.ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(fine.NE * nq, coarse.NE * nq))
