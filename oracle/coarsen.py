"""Operator coarsening, Algorithms 2 and 3 of the paper (appendix B).

The interpolation operator is injection (section 3, "Interpolation operator"):
(I u)|_{E_f} = u|_{E_c}.  Its matrix is built here by quadrature of the
inner products of fine and coarse basis functions over each child element.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .assemble import Grid, _COO, block_inverse_diag
from .basis import ref_basis, tensor_gauss


def prolongation(fine: Grid, coarse: Grid, q: int):
    """Scalar injection matrix I (fine dofs x coarse dofs), element-major."""
    d, p, h = fine.d, fine.p, fine.h
    pts, w = tensor_gauss(q, d)
    Bf = ref_basis(p, pts) * h ** (-d / 2)
    blocks = {}
    for o in range(2 ** d):
        off = np.array([(o >> j) & 1 for j in range(d)], dtype=float)
        Bc = ref_basis(p, (off[None, :] + pts) / 2.0) * (2.0 * h) ** (-d / 2)
        blocks[o] = np.einsum("q,qf,qc->fc", w * h ** d, Bf, Bc)
    parent = coarse.index(fine.ijk // 2)
    child = ((fine.ijk % 2) * (2 ** np.arange(d))[None, :]).sum(axis=1)
    nq = fine.nq
    ar = np.arange(nq)
    rows = (np.arange(fine.NE)[:, None, None] * nq + ar[None, :, None])
    cols = (parent[:, None, None] * nq + ar[None, None, :])
    rows, cols = np.broadcast_arrays(rows, cols)
    vals = np.stack([blocks[c] for c in child])
    return sp.csr_matrix((vals.ravel(), (rows.ravel(), cols.ravel())),
                         shape=(fine.NE * nq, coarse.NE * nq))


def frobenius_blend(Emu, Erho, nq):
    """eq. (Etimedep): per element-pair block,
    E_ij = (|Erho_ij| / (|Emu_ij| + |Erho_ij|))^2 Emu_ij
         + (|Emu_ij|  / (|Emu_ij| + |Erho_ij|))^2 Erho_ij   (Frobenius norms);
    a block where both norms vanish is zero."""
    S = Emu.shape[0]
    NE = S // nq

    def blocks_of(A):
        Ab = sp.csr_matrix(A).tobsr(blocksize=(nq, nq))
        out = {}
        for r in range(NE):
            for k in range(Ab.indptr[r], Ab.indptr[r + 1]):
                out[(r, int(Ab.indices[k]))] = Ab.data[k]
        return out

    bm, br = blocks_of(Emu), blocks_of(Erho)
    zero = np.zeros((nq, nq))
    coo = _COO(S, nq)
    keys = sorted(set(bm) | set(br))
    rows, cols, vals = [], [], []
    for key in keys:
        a, b = bm.get(key, zero), br.get(key, zero)
        na, nb = np.linalg.norm(a), np.linalg.norm(b)
        if na + nb == 0.0:
            continue
        rows.append(key[0])
        cols.append(key[1])
        vals.append((nb / (na + nb)) ** 2 * a + (na / (na + nb)) ** 2 * b)
    if vals:
        coo.add(np.array(rows), np.array(cols), np.stack(vals))
    return coo.csr()


def coarsen(ops, prob, unsteady: bool):
    """One application of Algorithm 2 (steady) or Algorithm 3 (unsteady)."""
    fine = ops["grid"]
    coarse = Grid(fine.d, fine.n // 2, fine.p, fine.bc, prob.phases, h=2.0 * fine.h)
    I = prolongation(fine, coarse, prob.q_op)
    out = coarsen_components(ops, I, fine.nq, unsteady)
    out.update(n=coarse.n, h=coarse.h, grid=coarse)
    return out


def coarsen_components(ops, I, nq, unsteady: bool):
    """Algorithm 2 / 3 for a given scalar injection I (any nested mesh pair)."""
    It = I.T.tocsr()
    M = ops["M"]
    M2 = (It @ M @ I).tocsr()                                   # M_2h
    Mmu2 = (It @ ops["Mmu"] @ I).tocsr()                        # M_mu,2h
    M2inv = block_inverse_diag(M2, nq)
    G2 = [(M2inv @ It @ M @ Gk @ I).tocsr() for Gk in ops["G"]]  # G_2h
    Et2 = (0.5 * (It @ ops["Et"] @ I)).tocsr()                  # velocity penalty, factor 1/2
    out = dict(M=M2, Mmu=Mmu2, G=G2, Et=Et2, I=I)
    if unsteady:
        out["Mrho"] = (It @ ops["Mrho"] @ I).tocsr()            # M_rho,2h
        out["Emu"] = (2.0 * (It @ ops["Emu"] @ I)).tocsr()      # factor 2
        out["Erho"] = (0.5 * (It @ ops["Erho"] @ I)).tocsr()    # factor 1/2
        out["E"] = frobenius_blend(out["Emu"], out["Erho"], nq)
    else:
        out["E"] = (2.0 * (It @ ops["E"] @ I)).tocsr()          # pressure penalty, factor 2
    return out
