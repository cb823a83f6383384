"""Fine-grid LDG operators, assembled by Gauss quadrature of the weak forms.

Follows appendix A of the paper:

* discrete gradient G = grad_h + L (eq. geqn summed into eq. gsum, with the
  lifting operator L and the numerical flux u-hat of eq. ustarflux),
* mu- and rho-weighted mass matrices (eq. sigmaresult, eq. timedep2),
* velocity penalty E-tilde (linear part of eq. Epenalty) and pressure
  penalty E (eq. eop with tau_p of eq. taueqn, or eq. taugeneral when the
  problem is unsteady),
* the saddle-point operator of eq. (stokessystem) with the viscous block of
  eq. (viscousop).

Faces carry the paper's orientation: intraphase faces point left to right,
interphase faces point from the lower phase index to the higher one, and
boundary faces point outward; u^- is the trace behind the normal and u^+ the
trace ahead of it.  The penalty constants are those of the appendix on
penalty parameters (tau_u,boundary = 10 p mu^- / h, tau_u,intraphase = 0 on
Cartesian grids, tau_u,interphase = 3 p min(mu^-, mu^+) / h) and lambda is
the viscosity-upwinded weight of eq. (viscosityupwind).

All operators act on one scalar field with element-major numbering
(element E, local basis index a) -> E * (p+1)^d + a.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .basis import ref_basis, tensor_gauss, face_gauss


class Grid:
    """Uniform Cartesian grid of n^d elements of width h on the unit cube."""

    def __init__(self, dim, n, p, bc, phases=None, h=None):
        self.d, self.n, self.p = dim, n, p
        self.m = p + 1
        self.nq = self.m ** dim
        self.NE = n ** dim
        self.h = 1.0 / n if h is None else h
        self.bc = tuple(bc)
        # multi-index of each element, axis 0 fastest
        self.ijk = np.array(np.unravel_index(np.arange(self.NE), (n,) * dim, order="F")).T
        centres = (self.ijk + 0.5) * self.h
        self.chi = np.ones(self.NE, dtype=int) if phases is None else phases.phase(centres)

    def index(self, ijk):
        ijk = np.atleast_2d(ijk)
        return np.ravel_multi_index(tuple(ijk.T), (self.n,) * self.d, order="F")

    def faces(self, axis):
        """Faces normal to ``axis``: arrays (L, R, anchor, side).  L / R are the
        elements below / above the face (-1 on the boundary); the face is the
        xi_axis = side face of the reference cell of element ``anchor``."""
        n = self.n
        R = np.arange(self.NE)
        jl = self.ijk.copy()
        jl[:, axis] = (self.ijk[:, axis] - 1) % n
        L = self.index(jl)
        anchor = R.copy()
        side = np.zeros(self.NE)
        if self.bc[axis] != "periodic":
            L[self.ijk[:, axis] == 0] = -1
            hi = np.nonzero(self.ijk[:, axis] == n - 1)[0]
            L = np.concatenate([L, hi])
            R = np.concatenate([R, -np.ones(hi.size, dtype=int)])
            anchor = np.concatenate([anchor, hi])
            side = np.concatenate([side, np.ones(hi.size)])
        return L, R, anchor, side


def _lam(mu_m, mu_p):
    """Viscosity-upwinded weight, eq. (viscosityupwind)."""
    return np.where(mu_m < mu_p, 0.0, np.where(mu_m > mu_p, 1.0, 0.5))


def interphase_mu(mu_m, mu_p):
    """Viscosity that scales the interphase velocity penalty: the smaller of
    the two sides (appendix on penalty parameters)."""
    return np.minimum(mu_m, mu_p)


class _COO:
    def __init__(self, size, nq):
        self.size, self.nq = size, nq
        self.r, self.c, self.v = [], [], []

    def add(self, rows_e, cols_e, blocks):
        rows_e = np.asarray(rows_e)
        cols_e = np.asarray(cols_e)
        if rows_e.size == 0:
            return
        nq = self.nq
        ar = np.arange(nq)
        r = rows_e[:, None, None] * nq + ar[None, :, None]
        c = cols_e[:, None, None] * nq + ar[None, None, :]
        r, c = np.broadcast_arrays(r, c)
        self.r.append(r.ravel())
        self.c.append(c.ravel())
        self.v.append(np.asarray(blocks).ravel())

    def csr(self):
        if not self.r:
            return sp.csr_matrix((self.size, self.size))
        A = sp.coo_matrix((np.concatenate(self.v), (np.concatenate(self.r), np.concatenate(self.c))),
                          shape=(self.size, self.size))
        A = A.tocsr()
        A.sum_duplicates()
        return A


class FineAssembly:
    """Quadrature assembly of the fine-grid scalar operators of one problem."""

    def __init__(self, prob, q=None):
        self.prob = prob
        self.q = prob.q_op if q is None else q
        self.grid = Grid(prob.dim, prob.n, prob.p, prob.bc, prob.phases)
        g = self.grid
        d, p, h = g.d, g.p, g.h
        self.S = g.NE * g.nq
        # volume quadrature
        self.qpts, qw = tensor_gauss(self.q, d)
        self.vol_w = qw * h ** d
        self.B = ref_basis(p, self.qpts) * h ** (-d / 2)
        self.dB = [ref_basis(p, self.qpts, deriv_axis=k) * h ** (-d / 2) / h for k in range(d)]
        # face quadrature (reference traces at xi_axis = 0 and 1)
        self.face = {}
        for k in range(d):
            pts0, fw = face_gauss(self.q, d, k, 0.0)
            pts1, _ = face_gauss(self.q, d, k, 1.0)
            self.face[k] = dict(w=fw * h ** (d - 1), pts0=pts0, pts1=pts1,
                                T0=ref_basis(p, pts0) * h ** (-d / 2),
                                T1=ref_basis(p, pts1) * h ** (-d / 2))

    # ------------------------------------------------------------------
    def element_points(self):
        g = self.grid
        return (g.ijk[:, None, :] + self.qpts[None, :, :]) * g.h

    def _coef(self, field, X, chi):
        """Evaluate a coefficient field at points X (F, Q, d); chi (F,) is the
        phase of the element each row of points belongs to."""
        shp = X.shape[:-1]
        chi_b = np.broadcast_to(np.asarray(chi)[:, None], shp)
        return field.value(X.reshape(-1, self.grid.d), chi_b.reshape(-1)).reshape(shp)

    def weighted_mass(self, field):
        """(M_c)_{ab} = int_E c phi_a phi_b, one block per element."""
        g = self.grid
        X = self.element_points()
        c = self._coef(field, X, g.chi)                         # (NE, Q)
        blocks = np.einsum("qa,eq,qb->eba", self.B, c * self.vol_w[None, :], self.B)
        coo = _COO(self.S, g.nq)
        E = np.arange(g.NE)
        coo.add(E, E, blocks)
        return coo.csr()

    def mass(self):
        g = self.grid
        blk = np.einsum("qa,q,qb->ba", self.B, self.vol_w, self.B)
        coo = _COO(self.S, g.nq)
        E = np.arange(g.NE)
        coo.add(E, E, np.broadcast_to(blk, (g.NE, g.nq, g.nq)))
        return coo.csr()

    # ------------------------------------------------------------------
    def face_data(self, axis):
        """Per face along ``axis``: minus/plus elements, the reference traces
        of each side, the normal sign s (n = s e_axis), physical points, the
        face type and lambda.  Types: 0 intraphase, 1 interphase, 2 Dirichlet
        boundary, 3 stress boundary (eq. govern3: u-hat = u- and sigma-hat the
        data, so the face adds nothing to the operator, eq. ustarflux and
        eq. qstarflux)."""
        g = self.grid
        fd = self.face[axis]
        L, R, anchor, side = g.faces(axis)
        nf = L.size
        minus = np.where(L >= 0, L, R)
        plus = np.where((L >= 0) & (R >= 0), R, -1)
        s = np.ones(nf)
        Tm_is_hi = L >= 0                       # minus trace at xi=1 when minus is the low element
        ftype = np.zeros(nf, dtype=int)
        both = (L >= 0) & (R >= 0)
        inter = both & (g.chi[np.maximum(L, 0)] != g.chi[np.maximum(R, 0)])
        ftype[inter] = 1
        ftype[~both] = 3 if g.bc[axis] == "stress" else 2
        # boundary faces: normal outward; a low-side boundary face has the
        # interior element above it, so n = -e_axis and the minus trace is at xi = 0
        s[(L < 0)] = -1.0
        # interphase faces: normal from the lower phase index to the higher
        flip = inter & (g.chi[np.maximum(L, 0)] > g.chi[np.maximum(R, 0)])
        minus = np.where(flip, R, minus)
        plus = np.where(flip, L, plus)
        s[flip] = -1.0
        Tm_is_hi = np.where(flip, False, Tm_is_hi)
        # physical face points, from the anchor element's reference cell
        pts_ref = np.where(side[:, None, None] > 0.5, fd["pts1"][None], fd["pts0"][None])
        X = (g.ijk[anchor][:, None, :] + pts_ref) * g.h
        X[:, :, axis] = np.mod(X[:, :, axis], 1.0) if g.bc[axis] == "periodic" else X[:, :, axis]
        chi_m = g.chi[minus]
        chi_p = g.chi[np.maximum(plus, 0)]
        mu_m = self._coef(self.prob.mu, X, chi_m)
        mu_p = self._coef(self.prob.mu, X, chi_p)
        lam = _lam(mu_m, mu_p)
        return dict(minus=minus, plus=plus, s=s, Tm_is_hi=Tm_is_hi, type=ftype, X=X,
                    chi_m=chi_m, chi_p=chi_p, mu_m=mu_m, mu_p=mu_p, lam=lam)

    def _traces(self, axis, is_hi):
        fd = self.face[axis]
        return np.where(np.asarray(is_hi)[:, None, None], fd["T1"][None], fd["T0"][None])

    def _fblock(self, axis, coef, Trow, Tcol):
        w = self.face[axis]["w"]
        return np.einsum("q,fq,fqb,fqa->fba", w, coef, Trow, Tcol)

    # ------------------------------------------------------------------
    def gradient(self, axis):
        """Discrete gradient component G_axis (eq. geqn with flux ustarflux).

        (G_k u, v) = sum_E int_E d_k u v
                     + int_intraphase (u+ - u-) v+ n_k
                     + int_interphase [(1-lam) v- + lam v+] (u+ - u-) n_k
                     - int_Dirichlet u- v- n_k
        (stress walls: u-hat = u-, no term)
        """
        g = self.grid
        coo = _COO(self.S, g.nq)
        vol = np.einsum("qa,q,qb->ba", self.dB[axis], self.vol_w, self.B)
        E = np.arange(g.NE)
        coo.add(E, E, np.broadcast_to(vol, (g.NE, g.nq, g.nq)))
        # faces normal to other axes have n_axis = 0 and do not contribute
        for k in (axis,):
            fd = self.face_data(k)
            Tm = self._traces(k, fd["Tm_is_hi"])
            Tp = self._traces(k, ~fd["Tm_is_hi"])
            s = fd["s"][:, None] * np.ones_like(fd["mu_m"])
            # intraphase
            sel = fd["type"] == 0
            if sel.any():
                c = s[sel]
                coo.add(fd["plus"][sel], fd["plus"][sel], self._fblock(k, c, Tp[sel], Tp[sel]))
                coo.add(fd["plus"][sel], fd["minus"][sel], self._fblock(k, -c, Tp[sel], Tm[sel]))
            # interphase
            sel = fd["type"] == 1
            if sel.any():
                lam = fd["lam"][sel]
                c_m = (1.0 - lam) * s[sel]
                c_p = lam * s[sel]
                mi, pl = fd["minus"][sel], fd["plus"][sel]
                coo.add(mi, pl, self._fblock(k, c_m, Tm[sel], Tp[sel]))
                coo.add(mi, mi, self._fblock(k, -c_m, Tm[sel], Tm[sel]))
                coo.add(pl, pl, self._fblock(k, c_p, Tp[sel], Tp[sel]))
                coo.add(pl, mi, self._fblock(k, -c_p, Tp[sel], Tm[sel]))
            # Dirichlet boundary faces
            sel = fd["type"] == 2
            if sel.any():
                mi = fd["minus"][sel]
                coo.add(mi, mi, self._fblock(k, -s[sel], Tm[sel], Tm[sel]))
        return coo.csr()

    def velocity_penalty(self):
        """Linear part of eq. (Epenalty): Dirichlet faces tau_b u- v-, interphase
        faces tau_ij [u][v]; the intraphase penalty is zero on Cartesian grids."""
        g, prob = self.grid, self.prob
        coo = _COO(self.S, g.nq)
        for k in range(g.d):
            fd = self.face_data(k)
            Tm = self._traces(k, fd["Tm_is_hi"])
            Tp = self._traces(k, ~fd["Tm_is_hi"])
            sel = fd["type"] == 2
            if sel.any():
                tau_b = prob.tau_u_bdry_C * prob.p * fd["mu_m"][sel] / g.h
                mi = fd["minus"][sel]
                coo.add(mi, mi, self._fblock(k, tau_b, Tm[sel], Tm[sel]))
            sel = fd["type"] == 1
            if sel.any():
                tau_i = prob.tau_u_inter_C * prob.p * interphase_mu(fd["mu_m"][sel], fd["mu_p"][sel]) / g.h
                self._jump_jump(coo, k, fd, sel, tau_i, Tm, Tp)
        return coo.csr()

    def _jump_jump(self, coo, k, fd, sel, tau, Tm, Tp):
        """Adds int tau [u][v] with [u] = u- - u+ over the selected faces."""
        mi, pl = fd["minus"][sel], fd["plus"][sel]
        coo.add(mi, mi, self._fblock(k, tau, Tm[sel], Tm[sel]))
        coo.add(pl, pl, self._fblock(k, tau, Tp[sel], Tp[sel]))
        coo.add(mi, pl, self._fblock(k, -tau, Tm[sel], Tp[sel]))
        coo.add(pl, mi, self._fblock(k, -tau, Tp[sel], Tm[sel]))

    def pressure_penalty(self, which="net"):
        """eq. (eop): int_{Gamma_0} tau_p [p][q] over intraphase faces (periodic
        wrap faces included).  ``which``: "net" uses eq. (taueqn), or eq.
        (taugeneral) for unsteady problems; "mu" uses tau h / mu and "rho" uses
        tau_0 delta / (h rho) (the two parts coarsened separately by Algorithm 3)."""
        g, prob = self.grid, self.prob
        coo = _COO(self.S, g.nq)
        for k in range(g.d):
            fd = self.face_data(k)
            sel = fd["type"] == 0
            if not sel.any():
                continue
            Tm = self._traces(k, fd["Tm_is_hi"])
            Tp = self._traces(k, ~fd["Tm_is_hi"])
            mu = fd["mu_m"][sel]
            t_mu = prob.tau * g.h / mu
            if prob.unsteady:
                rho = self._coef(prob.rho, fd["X"][sel], fd["chi_m"][sel])
                t_rho = prob.tau0 * prob.delta / (g.h * rho)
            if which == "mu":
                tau = t_mu
            elif which == "rho":
                tau = t_rho
            elif prob.unsteady:
                tau = 1.0 / (g.h * rho / (prob.tau0 * prob.delta) + mu / (prob.tau * g.h))
            else:
                tau = t_mu
            self._jump_jump(coo, k, fd, sel, tau, Tm, Tp)
        return coo.csr()


def fine_operators(prob):
    """All scalar operators of the finest grid (dict of CSR matrices)."""
    fa = FineAssembly(prob)
    ops = dict(
        n=prob.n, h=fa.grid.h, grid=fa.grid,
        M=fa.mass(),
        Mmu=fa.weighted_mass(prob.mu),
        G=[fa.gradient(k) for k in range(prob.dim)],
        Et=fa.velocity_penalty(),
        E=fa.pressure_penalty("net"),
    )
    if prob.unsteady:
        ops["Mrho"] = fa.weighted_mass(prob.rho)
        ops["Emu"] = fa.pressure_penalty("mu")
        ops["Erho"] = fa.pressure_penalty("rho")
    return ops


def block_inverse_diag(M, nq):
    """Inverse of a block-diagonal matrix with nq x nq blocks."""
    S = M.shape[0]
    NE = S // nq
    Md = M.tobsr(blocksize=(nq, nq))
    out = np.zeros((NE, nq, nq))
    for r in range(NE):
        for k in range(Md.indptr[r], Md.indptr[r + 1]):
            if Md.indices[k] == r:
                out[r] = np.linalg.inv(Md.data[k])
    coo = _COO(S, nq)
    coo.add(np.arange(NE), np.arange(NE), out)
    return coo.csr()


def stokes_system(ops, dim, gamma, nq, delta=None):
    """eq. (stokessystem) with the viscous block of eq. (viscousop):

    [[A, M calG], [calG^T M, -E]] with A_ij = delta_ij (sum_k G_k^T M_mu G_k + Et
    (+ M_rho / delta)) + gamma G_j^T M_mu G_i and calG_i = -M^{-1} G_i^T M, so that
    M calG_i = -G_i^T M and calG_i^T M = -M G_i.

    Returned in element-major ordering (element, field, basis index), fields
    ordered u_1 .. u_d, p.
    """
    G, Mmu, M = ops["G"], ops["Mmu"], ops["M"]
    lap = sum(G[k].T @ Mmu @ G[k] for k in range(dim)) + ops["Et"]
    if delta is not None:
        lap = lap + ops["Mrho"] / delta
    blocks = [[None] * (dim + 1) for _ in range(dim + 1)]
    for i in range(dim):
        for j in range(dim):
            Aij = gamma * (G[j].T @ Mmu @ G[i])
            if i == j:
                Aij = Aij + lap
            blocks[i][j] = Aij
        blocks[i][dim] = -(G[i].T @ M)
        blocks[dim][i] = -(M @ G[i])
    blocks[dim][dim] = -ops["E"]
    Afb = sp.bmat(blocks, format="csr")
    perm = field_to_element_major(Afb.shape[0] // ((dim + 1) * nq), dim + 1, nq)
    return Afb[perm][:, perm].tocsr()


def field_to_element_major(NE, nfield, nq):
    """perm[new] = old for new = (E, f, a) element-major, old = (f, E, a)."""
    E, f, a = np.meshgrid(np.arange(NE), np.arange(nfield), np.arange(nq), indexing="ij")
    return (f * NE * nq + E * nq + a).ravel()
