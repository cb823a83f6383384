"""LDG operators, right-hand side, hierarchy and errors on an implicitly
defined mesh (2D, circular interface; section 5 "Curved domain geometry",
section 5.6 and appendix A).

TEST INFRASTRUCTURE ONLY (part of the oracle).

The weak forms are those of the Cartesian assembly (eq. geqn with the
fluxes of eq. ustarflux / qstarflux, eq. Epenalty, eq. eop), written for
faces of any shape: every face carries its own quadrature points and a unit
normal per point, and every element its own orthonormal basis.

* intraphase faces are pieces of grid edges; minus is the element below the
  edge, plus the element above, n = +e_axis (the lifting of the Cartesian
  grids, u-hat = u-);
* interphase faces are the pieces of the interface inside cut cells, minus
  in phase 1, n = grad phi / |grad phi| (into phase 2), lambda from
  eq. (viscosityupwind) pointwise;
* wall faces carry the Dirichlet data.

Penalties (appendix A, "Specification of penalty parameters"): walls
tau = 10 p mu- / h; interphase tau = C p min(mu-, mu+) / h with C = 8 on
implicitly defined meshes; intraphase tau_u,0 = 0.5 p mu / h (reading:
implicitly defined meshes count among the semi-unstructured meshes, for
which the appendix gives 0.5 p mu / h); pressure tau h / mu on intraphase
faces, eq. (taueqn).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .assemble import _lam, interphase_mu, stokes_system, field_to_element_major
from .coarsen import coarsen_components
from .hierarchy import Hierarchy, Level, diagonal_blocks, equilibrated_inverse
from .implicit_mesh import ImplicitMesh, coarsen_mesh, prolongation


class _Acc:
    """COO accumulator of nq x nq blocks."""

    def __init__(self, NE, nq):
        self.NE, self.nq = NE, nq
        self.r, self.c, self.v = [], [], []

    def add(self, E, F, blk):
        nq = self.nq
        ar = np.arange(nq)
        self.r.append(np.repeat(E * nq + ar, nq))
        self.c.append(np.tile(F * nq + ar, nq))
        self.v.append(np.asarray(blk).ravel())

    def csr(self):
        S = self.NE * self.nq
        if not self.v:
            return sp.csr_matrix((S, S))
        return sp.csr_matrix((np.concatenate(self.v), (np.concatenate(self.r), np.concatenate(self.c))),
                             shape=(S, S))


def _fb(w, coef, Trow, Tcol):
    """int coef * row_basis * col_basis over a face: (nq, nq), rows from Trow."""
    return (Trow * (w * coef)[:, None]).T @ Tcol


class ImplicitAssembly:
    def __init__(self, prob, mesh: ImplicitMesh):
        if prob.dim != 2 or any(b != "dirichlet" for b in prob.bc):
            raise ValueError("implicitly defined meshes: 2D problems with Dirichlet walls")
        self.prob, self.mesh = prob, mesh
        self.nq = mesh.nq
        self.h = mesh.h
        self.Psi = [mesh.basis(i, e.X) for i, e in enumerate(mesh.elements)]
        self.dPsi = [[mesh.basis(i, e.X, k) for k in range(2)] for i, e in enumerate(mesh.elements)]
        chi = mesh.chi()
        self.trace = []
        for f in mesh.faces:
            Tm = mesh.basis(f.minus, f.X)
            Tp = mesh.basis(f.plus, f.X) if f.plus >= 0 else None
            mu_m = prob.mu.value(f.X, np.full(f.w.size, chi[f.minus]))
            mu_p = prob.mu.value(f.X, np.full(f.w.size, chi[f.plus])) if f.plus >= 0 else None
            self.trace.append((Tm, Tp, mu_m, mu_p))

    def mass(self):
        acc = _Acc(self.mesh.NE, self.nq)
        for i, e in enumerate(self.mesh.elements):
            acc.add(i, i, (self.Psi[i] * e.w[:, None]).T @ self.Psi[i])
        return acc.csr()

    def weighted_mass(self, field):
        acc = _Acc(self.mesh.NE, self.nq)
        for i, e in enumerate(self.mesh.elements):
            c = field.value(e.X, np.full(e.w.size, e.phase))
            acc.add(i, i, (self.Psi[i] * (e.w * c)[:, None]).T @ self.Psi[i])
        return acc.csr()

    def gradient(self, k):
        """G_k (M = I in the orthonormal bases):
        (G_k u, v) = sum_E int_E d_k u v + int_intra (u+ - u-) v+ n_k
                     + int_inter [(1-lam) v- + lam v+] (u+ - u-) n_k - int_wall u- v- n_k."""
        acc = _Acc(self.mesh.NE, self.nq)
        for i, e in enumerate(self.mesh.elements):
            acc.add(i, i, (self.Psi[i] * e.w[:, None]).T @ self.dPsi[i][k])
        for f, (Tm, Tp, mu_m, mu_p) in zip(self.mesh.faces, self.trace):
            nk = f.normal[:, k]
            if not np.any(nk):
                continue
            m, p = f.minus, f.plus
            if f.kind == 0:
                acc.add(p, p, _fb(f.w, nk, Tp, Tp))
                acc.add(p, m, _fb(f.w, -nk, Tp, Tm))
            elif f.kind == 1:
                lam = _lam(mu_m, mu_p)
                acc.add(m, p, _fb(f.w, (1 - lam) * nk, Tm, Tp))
                acc.add(m, m, _fb(f.w, -(1 - lam) * nk, Tm, Tm))
                acc.add(p, p, _fb(f.w, lam * nk, Tp, Tp))
                acc.add(p, m, _fb(f.w, -lam * nk, Tp, Tm))
            else:
                acc.add(m, m, _fb(f.w, -nk, Tm, Tm))
        return acc.csr()

    def _jump(self, acc, f, tau, Tm, Tp):
        m, p = f.minus, f.plus
        acc.add(m, m, _fb(f.w, tau, Tm, Tm))
        acc.add(p, p, _fb(f.w, tau, Tp, Tp))
        acc.add(m, p, _fb(f.w, -tau, Tm, Tp))
        acc.add(p, m, _fb(f.w, -tau, Tp, Tm))

    def velocity_penalty(self):
        prob, h = self.prob, self.h
        acc = _Acc(self.mesh.NE, self.nq)
        for f, (Tm, Tp, mu_m, mu_p) in zip(self.mesh.faces, self.trace):
            if f.kind == 2:
                acc.add(f.minus, f.minus, _fb(f.w, prob.tau_u_bdry_C * prob.p * mu_m / h, Tm, Tm))
            elif f.kind == 1:
                self._jump(acc, f, prob.tau_u_inter_C * prob.p * interphase_mu(mu_m, mu_p) / h, Tm, Tp)
            elif prob.tau_u_intra_C > 0.0:
                self._jump(acc, f, prob.tau_u_intra_C * prob.p * mu_m / h, Tm, Tp)
        return acc.csr()

    def pressure_penalty(self, which="net"):
        """eq. (eop) on intraphase faces: tau h / mu (eq. taueqn), or for
        unsteady problems eq. (taugeneral) ("net") and its two limits "mu"
        (tau h / mu) and "rho" (tau_0 delta / (h rho)), coarsened separately
        by Algorithm 3."""
        prob, h = self.prob, self.h
        acc = _Acc(self.mesh.NE, self.nq)
        chi = self.mesh.chi()
        for f, (Tm, Tp, mu_m, mu_p) in zip(self.mesh.faces, self.trace):
            if f.kind != 0:
                continue
            t_mu = prob.tau * h / mu_m
            if prob.unsteady:
                rho = prob.rho.value(f.X, np.full(f.w.size, chi[f.minus]))
                t_rho = prob.tau0 * prob.delta / (h * rho)
            if which == "mu" or not prob.unsteady:
                tau = t_mu
            elif which == "rho":
                tau = t_rho
            else:
                tau = 1.0 / (h * rho / (prob.tau0 * prob.delta) + mu_m / (prob.tau * h))
            self._jump(acc, f, tau, Tm, Tp)
        return acc.csr()


def implicit_mesh(prob):
    return ImplicitMesh(prob.n, prob.p, prob.phases, prob.q_op, prob.q_cut,
                        void_outside=getattr(prob.phases, "void_outside", False))


def implicit_fine_operators(prob, mesh=None):
    mesh = mesh or implicit_mesh(prob)
    fa = ImplicitAssembly(prob, mesh)
    ops = dict(n=prob.n, h=mesh.h, mesh=mesh, asm=fa, M=fa.mass(), Mmu=fa.weighted_mass(prob.mu),
               G=[fa.gradient(k) for k in range(2)], Et=fa.velocity_penalty(), E=fa.pressure_penalty("net"))
    if prob.unsteady:
        ops["Mrho"] = fa.weighted_mass(prob.rho)
        ops["Emu"] = fa.pressure_penalty("mu")
        ops["Erho"] = fa.pressure_penalty("rho")
    return ops


# ---------------------------------------------------------------------------
# right-hand side
# ---------------------------------------------------------------------------
def _interface_data(src, X, nrm):
    """(g, h) = ([u], [sigma n]) across the interface, phase 1 minus phase 2."""
    if hasattr(src, "interface_jumps"):
        return src.interface_jumps(X, nrm)
    one = np.ones(X.shape[0], dtype=int)
    g = src.velocity(X, one) - src.velocity(X, 2 * one)
    S = src.stress(X, one) - src.stress(X, 2 * one)
    return g, np.einsum("qik,qk->qi", S, nrm)


def implicit_rhs(prob, ops):
    """Right-hand side of eq. (stokessystem) on the implicit mesh (the terms of
    the Cartesian assembly, with pointwise normals); element-major."""
    mesh, fa = ops["mesh"], ops["asm"]
    d, nq, NE = 2, mesh.nq, mesh.NE
    S = NE * nq
    src = prob.rhs_source()
    Pf = np.zeros((d, NE, nq))
    Pfd = np.zeros((NE, nq))
    for i, e in enumerate(mesh.elements):
        chi = np.full(e.w.size, e.phase)
        f = src.forcing(e.X, chi)
        Pf[:, i] = ((fa.Psi[i] * e.w[:, None]).T @ f).T
        Pfd[i] = (fa.Psi[i] * e.w[:, None]).T @ src.forcing_div(e.X, chi)
    Jg = np.zeros((d, d, NE, nq))
    Jh = np.zeros((d, NE, nq))
    pen = np.zeros((d, NE, nq))
    Jgn = np.zeros((NE, nq))
    chi_e = mesh.chi()
    for f, (Tm, Tp, mu_m, mu_p) in zip(mesh.faces, fa.trace):
        m, p, n, w = f.minus, f.plus, f.normal, f.w
        if f.kind == 2:
            g = src.velocity(f.X, np.full(w.size, chi_e[m]))
            tau = prob.tau_u_bdry_C * prob.p * mu_m / mesh.h
            for i in range(d):
                for k in range(d):
                    Jg[i, k, m] += Tm.T @ (w * g[:, i] * n[:, k])
                pen[i, m] += Tm.T @ (w * tau * g[:, i])
            Jgn[m] += Tm.T @ (w * (g * n).sum(axis=1))
        elif f.kind == 1:
            g, hj = _interface_data(src, f.X, n)
            lam = _lam(mu_m, mu_p)
            tau = prob.tau_u_inter_C * prob.p * interphase_mu(mu_m, mu_p) / mesh.h
            for i in range(d):
                for k in range(d):
                    Jg[i, k, m] += Tm.T @ (w * (1 - lam) * g[:, i] * n[:, k])
                    Jg[i, k, p] += Tp.T @ (w * lam * g[:, i] * n[:, k])
                Jh[i, m] += Tm.T @ (w * lam * hj[:, i])
                Jh[i, p] += Tp.T @ (w * (1 - lam) * hj[:, i])
                pen[i, m] += Tm.T @ (w * tau * g[:, i])
                pen[i, p] -= Tp.T @ (w * tau * g[:, i])
            gn = (g * n).sum(axis=1)
            Jgn[m] += Tm.T @ (w * (1 - lam) * gn)
            Jgn[p] += Tp.T @ (w * lam * gn)
    G, Mmu = ops["G"], ops["Mmu"]
    bu = []
    for i in range(d):
        v = (Pf[i] + Jh[i] + pen[i]).ravel()
        for j in range(d):
            v = v - G[j].T @ (Mmu @ (Jg[i, j] + prob.gamma * Jg[j, i]).ravel())
        bu.append(v)
    bp = (Pfd + Jgn).ravel()
    fields = np.stack(bu + [bp])
    return fields.reshape(d + 1, NE, nq).transpose(1, 0, 2).ravel()


# ---------------------------------------------------------------------------
# hierarchy
# ---------------------------------------------------------------------------
def greedy_colours(A, nb):
    """Greedy colouring of the element-block graph of A: elements in index
    order, each taking the smallest colour no earlier neighbour holds."""
    NE = A.shape[0] // nb
    Ab = sp.csr_matrix(A).tobsr(blocksize=(nb, nb))
    nbrs = [set() for _ in range(NE)]
    for r in range(NE):
        for k in range(Ab.indptr[r], Ab.indptr[r + 1]):
            c = int(Ab.indices[k])
            if c != r and np.any(Ab.data[k]):
                nbrs[r].add(c)
                nbrs[c].add(r)
    col = -np.ones(NE, dtype=int)
    for E in range(NE):
        used = {col[F] for F in nbrs[E] if col[F] >= 0}
        c = 0
        while c in used:
            c += 1
        col[E] = c
    return col


class ImplicitHierarchy(Hierarchy):
    def kernel_basis(self):
        """The constant pressure (Dirichlet walls, steady), as coefficients in
        the orthonormal bases: sqrt(|E|) on each element's first function."""
        lv = self.fine
        K = np.zeros((lv.NE * lv.nb, 1))
        areas = np.array([e.area for e in lv.mesh.elements])
        K[np.arange(lv.NE) * lv.nb + 2 * lv.nq, 0] = np.sqrt(areas)
        return K / np.linalg.norm(K)


def build_implicit_hierarchy(prob):
    """Every level of the V-cycle on the implicit mesh: fine operators by
    quadrature, coarser ones by Algorithm 2 with the implicit-mesh injection,
    greedy colours, block inverses and the bottom pseudo-inverse (the same
    steps as the Cartesian hierarchy)."""
    d, nq = 2, (prob.p + 1) ** 2
    nb = (d + 1) * nq
    ops = implicit_fine_operators(prob)
    mesh = ops["mesh"]
    levels = []
    sizes = prob.levels()
    for li, n in enumerate(sizes):
        if li > 0:
            cmesh, parent = coarsen_mesh(mesh)
            I = prolongation(mesh, cmesh, parent)
            ops = coarsen_components(ops, I, nq, prob.unsteady)
            ops.update(n=cmesh.n, h=cmesh.h, mesh=cmesh)
            mesh = cmesh
        lv = Level()
        lv.n, lv.h, lv.nq, lv.nb = n, mesh.h, nq, nb
        lv.NE = mesh.NE
        lv.ops = ops
        lv.mesh = mesh
        A = stokes_system(ops, d, prob.gamma, nq, prob.delta if prob.unsteady else None)
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
    for li in range(len(levels) - 1):
        Is = levels[li + 1].ops["I"]
        Ifb = sp.block_diag([Is] * (d + 1), format="csr")
        pf = field_to_element_major(levels[li].NE, d + 1, nq)
        pc = field_to_element_major(levels[li + 1].NE, d + 1, nq)
        levels[li].I = Ifb[pf][:, pc].tocsr()
    for lv in levels[:-1]:
        lv.colours = greedy_colours(lv.A, nb)
        lv.ncol = int(lv.colours.max()) + 1
        lv.Ainv = equilibrated_inverse(diagonal_blocks(lv.A, nb))
    k0 = 1
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
    return ImplicitHierarchy(prob, levels, k0)


# ---------------------------------------------------------------------------
# errors
# ---------------------------------------------------------------------------
def implicit_solution_errors(prob, mesh, x):
    """L2 and max-norm errors of (u, p) over the elements' quadrature points;
    the constant-pressure component of the error is removed (its kernel)."""
    d, nq, nb = 2, mesh.nq, 3 * mesh.nq
    xr = x.reshape(mesh.NE, d + 1, nq)
    errs, ws = [], []
    for i, e in enumerate(mesh.elements):
        B = mesh.basis(i, e.X)
        uh = B @ xr[i].T                                    # (Q, 3)
        chi = np.full(e.w.size, e.phase)
        ue = prob.exact.velocity(e.X, chi)
        pe = prob.exact.pressure(e.X, chi)
        errs.append(np.concatenate([ue, pe[:, None]], axis=1) - uh)
        ws.append(e.w)
    err = np.concatenate(errs)
    w = np.concatenate(ws)
    err[:, d] -= (err[:, d] * w).sum() / w.sum()
    l2 = np.sqrt((err ** 2 * w[:, None]).sum(axis=0))
    linf = np.abs(err).max(axis=0)
    return dict(u_l2=float(np.sqrt((l2[:d] ** 2).sum())), p_l2=float(l2[d]),
                u_max=float(linf[:d].max()), p_max=float(linf[d]))
