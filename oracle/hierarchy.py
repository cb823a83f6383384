"""The multigrid hierarchy of section 3: levels, transfers, smoother data and
the bottom solver.

* Levels: the finest operator by quadrature, coarser ones by Algorithms 2/3.
* Transfers: injection I per field; restriction by I^T (Algorithm 1 and
  its footnote on the transpose of interpolation).
* Smoother data: the diagonal element blocks A_EE of every smoothed level,
  factorised once (section 3, "precompute a ... factorisation"); here an LU
  with partial pivoting of the Jacobi-equilibrated block, turned into an
  explicit inverse.
* Colours: multi-coloured element ordering (section 3), colour of element
  i = (i_0 .. i_{d-1}): red-black sum(i) mod 2, parity sum (i_k mod 2) 2^k,
  mod-3 sum (i_k mod 3) 3^k; colours are swept in increasing order.
* Bottom: symmetric eigendecomposition of the coarsest operator with the
  k0 eigenvalues of smallest magnitude snapped to zero (the bottom-solver
  footnote), k0 = dimension of the trivial kernel.  Reading: the
  decomposition is taken of the Jacobi-equilibrated operator D A D,
  D = |diag A|^{-1/2}, whose near-zero eigenvalues are separated from the
  rest by many orders of magnitude even where A itself is badly scaled
  (unsteady problems with large rho/delta); the bottom solve is then
  x = D (D A D)^+ D r, a generalized inverse of A that solves A x = r for
  every r in range(A) and differs from A^+ r only along the kernel.
* Optional diagonal (alpha, beta) scaling of the multi-phase section: every
  level's operator is replaced by D A D with D = mu_E^{-1/2} on velocity and
  mu_E^{1/2} on pressure, mu_E the element mean of mu.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from synth import kernel_dimension
from .assemble import fine_operators, stokes_system, field_to_element_major
from .coarsen import coarsen


def colour_of(ijk, scheme):
    ijk = np.asarray(ijk)
    d = ijk.shape[1]
    if scheme == "rb":
        return ijk.sum(axis=1) % 2
    if scheme == "parity":
        return ((ijk % 2) * (2 ** np.arange(d))[None, :]).sum(axis=1)
    if scheme == "mod3":
        return ((ijk % 3) * (3 ** np.arange(d))[None, :]).sum(axis=1)
    raise ValueError(scheme)


def n_colours(scheme, d):
    return {"rb": 2, "parity": 2 ** d, "mod3": 3 ** d}[scheme]


def diagonal_blocks(A, nb):
    """(NE, nb, nb) diagonal element blocks of an element-major matrix."""
    NE = A.shape[0] // nb
    Ab = sp.csr_matrix(A).tobsr(blocksize=(nb, nb))
    out = np.zeros((NE, nb, nb))
    for r in range(NE):
        for k in range(Ab.indptr[r], Ab.indptr[r + 1]):
            if Ab.indices[k] == r:
                out[r] += Ab.data[k]
    return out


def equilibrated_inverse(blocks, rcond_min=1e-14):
    """Explicit inverses of A_EE via LU with partial pivoting of D A D,
    D = diag(|A_jj|^{-1/2}); inv(A) = D inv(D A D) D.  Raises if a scaled
    block is numerically singular."""
    dg = np.abs(np.einsum("eii->ei", blocks))
    if np.any(dg == 0.0):
        raise np.linalg.LinAlgError("zero diagonal entry in an element block")
    D = 1.0 / np.sqrt(dg)
    S = D[:, :, None] * blocks * D[:, None, :]
    Sinv = np.linalg.inv(S)
    cond = np.linalg.norm(S, 1, axis=(1, 2)) * np.linalg.norm(Sinv, 1, axis=(1, 2))
    if np.any(1.0 / cond < rcond_min):
        raise np.linalg.LinAlgError("singular element block")
    return D[:, :, None] * Sinv * D[:, None, :]


class Level:
    pass


class Hierarchy:
    """All levels of one problem.  ``levels[0]`` is the finest."""

    def __init__(self, prob, levels, k0):
        self.prob = prob
        self.levels = levels
        self.k0 = k0

    @property
    def fine(self):
        return self.levels[0]

    def kernel_basis(self):
        """Orthonormal basis (N, k0) of the trivial kernel of the unscaled fine
        operator, as coefficient vectors in the orthonormal basis: constant
        velocity components (periodic steady) and constant pressure; with
        stress walls the constant velocity components and (viscous-stress
        form) the rigid rotations (x_a - 1/2) e_b - (x_b - 1/2) e_a, a < b."""
        lv = self.fine
        prob = self.prob
        nq, nb, NE = lv.nq, lv.nb, lv.NE
        if all(b == "stress" for b in prob.bc):
            return self._rigid_modes()
        fields = [prob.dim] if self.k0 == 1 else list(range(prob.dim + 1))
        K = np.zeros((NE * nb, len(fields)))
        for c, f in enumerate(fields):
            K[np.arange(NE) * nb + f * nq, c] = 1.0 / np.sqrt(NE)
        return K

    def _rigid_modes(self):
        """Rigid motions as coefficient vectors: the L2 projection (exact for
        these linear fields) of each mode onto the element basis, by Gauss
        quadrature; orthonormalised (the centred modes are already mutually
        orthogonal, QR only normalises them)."""
        from .assemble import FineAssembly
        prob = self.prob
        d = prob.dim
        lv = self.fine
        NE, nq, nb = lv.NE, lv.nq, lv.nb
        fa = FineAssembly(prob)
        X = fa.element_points()                                   # (NE, Q, d)
        W = fa.B * fa.vol_w[:, None]                              # (Q, nq)
        modes = []
        for i in range(d):
            F = np.zeros(X.shape)
            F[..., i] = 1.0
            modes.append(F)
        if prob.gamma and not prob.unsteady:
            for a in range(d):
                for b in range(a + 1, d):
                    F = np.zeros(X.shape)
                    F[..., b] = X[..., a] - 0.5
                    F[..., a] = -(X[..., b] - 0.5)
                    modes.append(F)
        if prob.unsteady:
            modes = []
        K = np.zeros((NE * nb, len(modes)))
        for c, F in enumerate(modes):
            coef = np.einsum("qa,eqi->eia", W, F)                  # (NE, d, nq)
            v = np.zeros((NE, nb))
            v[:, :d * nq] = coef.reshape(NE, d * nq)
            K[:, c] = v.ravel()
        if K.shape[1]:
            K, _ = np.linalg.qr(K)
        return K

    def project_kernel(self, v):
        K = self.kernel_basis()
        return v - K @ (K.T @ v)


def build_hierarchy(prob):
    """Assemble every level of the V-cycle hierarchy (FP64)."""
    d = prob.dim
    nq = (prob.p + 1) ** d
    nb = (d + 1) * nq
    unsteady = prob.unsteady
    ops = fine_operators(prob)
    levels = []
    sizes = prob.levels()
    for li, n in enumerate(sizes):
        if li > 0:
            ops = coarsen(ops, prob, unsteady)
        lv = Level()
        lv.n, lv.h, lv.nq, lv.nb = n, ops["h"], nq, nb
        lv.NE = n ** d
        lv.ops = ops
        lv.grid = ops["grid"]
        A = stokes_system(ops, d, prob.gamma, nq, prob.delta if unsteady else None)
        if prob.diag_scaling:
            mu_e = np.array([ops["Mmu"][E * nq, E * nq] for E in range(lv.NE)])
            dvec = np.empty(lv.NE * nb)
            for E in range(lv.NE):
                dvec[E * nb:E * nb + d * nq] = mu_e[E] ** -0.5
                dvec[E * nb + d * nq:(E + 1) * nb] = mu_e[E] ** 0.5
            lv.dscale = dvec
            Ds = sp.diags(dvec)
            A = (Ds @ A @ Ds).tocsr()
        else:
            lv.dscale = None
        lv.A = A
        levels.append(lv)
    # system-level injection between consecutive levels
    for li in range(len(levels) - 1):
        Is = levels[li + 1].ops["I"]
        Ifb = sp.block_diag([Is] * (d + 1), format="csr")
        pf = field_to_element_major(levels[li].NE, d + 1, nq)
        pc = field_to_element_major(levels[li + 1].NE, d + 1, nq)
        levels[li].I = Ifb[pf][:, pc].tocsr()
    # smoother data on smoothed levels
    for lv in levels[:-1]:
        lv.colours = colour_of(lv.grid.ijk, prob.coloring)
        lv.ncol = n_colours(prob.coloring, d)
        lv.Ainv = equilibrated_inverse(diagonal_blocks(lv.A, nb))
    # bottom: eigendecomposition pseudo-inverse
    k0 = kernel_dimension(prob)
    bot = levels[-1]
    Ad = bot.A.toarray()
    dg = 1.0 / np.sqrt(np.abs(np.diag(Ad)))
    Bd = dg[:, None] * Ad * dg[None, :]
    lam, V = np.linalg.eigh(0.5 * (Bd + Bd.T))
    order = np.argsort(np.abs(lam))
    inv = np.zeros_like(lam)
    keep = order[k0:]
    if np.abs(lam[keep]).min() <= 1e-8 * np.abs(lam).max():
        raise np.linalg.LinAlgError("coarsest operator has more near-zero eigenvalues than the kernel")
    inv[keep] = 1.0 / lam[keep]
    bot.pinv = dg[:, None] * ((V * inv[None, :]) @ V.T) * dg[None, :]
    bot.eig = lam
    return Hierarchy(prob, levels, k0)
