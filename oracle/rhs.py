"""Right-hand side of eq. (stokessystem), from eq. (appstokes1)-(appstokes2)
multiplied by M.

Momentum row i:
    b_u,i = int f_i phi
            - sum_j G_j^T M_mu (J_g,ij + gamma J_g,ji)
            + J_h,i
            + int_Dirichlet tau_b g_i phi^-  + int_interphase tau_ij g_ij,i [phi]
Constraint row:
    b_p   = int f phi + J_{g.n}

J_g, J_h and J_{g.n} are the data vectors defined after eq. (gsum), after
eq. (wworkings) and after eq. (ewv).  The last two momentum terms are
-E_{u,g}(0) of eq. (Epenalty).

Reading of the printed equations: eq. (wform) and eq. (appstokes1) print
M^{-1} G_j^T (J_g,ij + gamma J_g,ji); substituting eq. (sigmaresult) into the
adjoint form of w_i gives M^{-1} G_j^T M_mu (J_g,ij + gamma J_g,ji), which is
used here (the two agree when mu = 1).
"""
from __future__ import annotations

import numpy as np

from . import assemble as _asm
from .assemble import FineAssembly


def _scatter(S, nq, elems, vals):
    out = np.zeros(S)
    np.add.at(out.reshape(-1, nq), elems, vals)
    return out


def assemble_rhs(prob, ops):
    fa = FineAssembly(prob, q=prob.q_rhs)
    g = fa.grid
    d, nq, S = g.d, g.nq, fa.S
    src = prob.rhs_source()
    X = fa.element_points()
    NE, Q = X.shape[:2]
    chi_pts = np.broadcast_to(g.chi[:, None], (NE, Q)).reshape(-1)
    f = src.forcing(X.reshape(-1, d), chi_pts).reshape(NE, Q, d)
    fdiv = src.forcing_div(X.reshape(-1, d), chi_pts).reshape(NE, Q)
    Pf = [np.einsum("qa,eq->ea", fa.B, f[..., i] * fa.vol_w[None, :]).ravel() for i in range(d)]
    Pfd = np.einsum("qa,eq->ea", fa.B, fdiv * fa.vol_w[None, :]).ravel()

    Jg = np.zeros((d, d, S))
    Jh = np.zeros((d, S))
    pen = np.zeros((d, S))
    Jgn = np.zeros(S)
    exact = prob.exact
    for k in range(d):
        fd = fa.face_data(k)
        w = fa.face[k]["w"]
        Tm = fa._traces(k, fd["Tm_is_hi"])
        Tp = fa._traces(k, ~fd["Tm_is_hi"])
        s = fd["s"]
        # Dirichlet boundary faces: u-hat = g, normal outward
        sel = fd["type"] == 2
        if sel.any():
            if exact is None:
                raise ValueError("Dirichlet data needs an exact solution")
            Xf = fd["X"][sel]
            F = Xf.shape[0]
            chi = np.broadcast_to(fd["chi_m"][sel][:, None], Xf.shape[:2]).reshape(-1)
            gv = exact.velocity(Xf.reshape(-1, d), chi).reshape(F, -1, d)
            tau_b = prob.tau_u_bdry_C * prob.p * fd["mu_m"][sel] / g.h
            mi = fd["minus"][sel]
            ss = s[sel][:, None]
            for i in range(d):
                Jg[i, k] += _scatter(S, nq, mi, np.einsum("q,fq,fqa->fa", w, gv[..., i] * ss, Tm[sel]))
                pen[i] += _scatter(S, nq, mi, np.einsum("q,fq,fqa->fa", w, tau_b * gv[..., i], Tm[sel]))
            Jgn += _scatter(S, nq, mi, np.einsum("q,fq,fqa->fa", w, gv[..., k] * ss, Tm[sel]))
        # stress boundary faces: sigma-hat = h n with h = sigma(exact) n, n
        # outward; the data enter through J_h (the face has no operator terms)
        sel = fd["type"] == 3
        if sel.any():
            if exact is None:
                raise ValueError("stress data needs an exact solution")
            Xf = fd["X"][sel]
            F = Xf.shape[0]
            chi = np.broadcast_to(fd["chi_m"][sel][:, None], Xf.shape[:2]).reshape(-1)
            sig = exact.stress(Xf.reshape(-1, d), chi).reshape(F, -1, d, d)
            hb = sig[..., :, k] * s[sel][:, None, None]          # h_i = sigma_ik n_k
            mi = fd["minus"][sel]
            for i in range(d):
                Jh[i] += _scatter(S, nq, mi, np.einsum("q,fq,fqa->fa", w, hb[..., i], Tm[sel]))
        # interphase faces: jump data g_ij = [u], h_ij = [sigma n], lambda-weighted
        sel = fd["type"] == 1
        if sel.any():
            Xf = fd["X"][sel]
            F = Xf.shape[0]
            cm = np.broadcast_to(fd["chi_m"][sel][:, None], Xf.shape[:2]).reshape(-1)
            cp = np.broadcast_to(fd["chi_p"][sel][:, None], Xf.shape[:2]).reshape(-1)
            xr = Xf.reshape(-1, d)
            gij = (exact.velocity(xr, cm) - exact.velocity(xr, cp)).reshape(F, -1, d)
            sig = (exact.stress(xr, cm) - exact.stress(xr, cp)).reshape(F, -1, d, d)
            ss = s[sel][:, None]
            hij = sig[..., :, k] * ss[..., None]
            lam = fd["lam"][sel]
            tau_i = prob.tau_u_inter_C * prob.p * _asm.interphase_mu(fd["mu_m"][sel], fd["mu_p"][sel]) / g.h
            mi, pl = fd["minus"][sel], fd["plus"][sel]
            for i in range(d):
                Jg[i, k] += _scatter(S, nq, mi, np.einsum("q,fq,fqa->fa", w, (1 - lam) * gij[..., i] * ss, Tm[sel]))
                Jg[i, k] += _scatter(S, nq, pl, np.einsum("q,fq,fqa->fa", w, lam * gij[..., i] * ss, Tp[sel]))
                Jh[i] += _scatter(S, nq, mi, np.einsum("q,fq,fqa->fa", w, lam * hij[..., i], Tm[sel]))
                Jh[i] += _scatter(S, nq, pl, np.einsum("q,fq,fqa->fa", w, (1 - lam) * hij[..., i], Tp[sel]))
                pen[i] += _scatter(S, nq, mi, np.einsum("q,fq,fqa->fa", w, tau_i * gij[..., i], Tm[sel]))
                pen[i] -= _scatter(S, nq, pl, np.einsum("q,fq,fqa->fa", w, tau_i * gij[..., i], Tp[sel]))
            Jgn += _scatter(S, nq, mi, np.einsum("q,fq,fqa->fa", w, (1 - lam) * gij[..., k] * ss, Tm[sel]))
            Jgn += _scatter(S, nq, pl, np.einsum("q,fq,fqa->fa", w, lam * gij[..., k] * ss, Tp[sel]))

    G, Mmu = ops["G"], ops["Mmu"]
    bu = []
    for i in range(d):
        v = Pf[i] + Jh[i] + pen[i]
        for j in range(d):
            v = v - G[j].T @ (Mmu @ (Jg[i, j] + prob.gamma * Jg[j, i]))
        bu.append(v)
    bp = Pfd + Jgn
    fields = np.stack(bu + [bp])                      # (d+1, S)
    return fields.reshape(d + 1, g.NE, nq).transpose(1, 0, 2).ravel()
