"""Discretisation errors, as in the grid-convergence appendix: the error
(u - u_h, p - p_h) with its components along the trivial kernel (constant
fields; the rigid motions of the velocity with stress walls) removed by
Gram-Schmidt, measured in L2 and at a fine Gauss grid per
element (max norm)."""
from __future__ import annotations

import numpy as np

from .basis import ref_basis, tensor_gauss
from .assemble import Grid


def solution_errors(prob, x, k0):
    d, p, n = prob.dim, prob.p, prob.n
    g = Grid(d, n, p, prob.bc, prob.phases)
    nq = g.nq
    pts, w = tensor_gauss(prob.q_err, d)
    B = ref_basis(p, pts) * g.h ** (-d / 2)
    X = (g.ijk[:, None, :] + pts[None]) * g.h
    NE, Q = X.shape[:2]
    chi = np.broadcast_to(g.chi[:, None], (NE, Q)).reshape(-1)
    xr = x.reshape(NE, d + 1, nq)
    uh = np.einsum("qa,efa->eqf", B, xr)                     # (NE, Q, d+1)
    ue = prob.exact.velocity(X.reshape(-1, d), chi).reshape(NE, Q, d)
    pe = prob.exact.pressure(X.reshape(-1, d), chi).reshape(NE, Q)
    err = np.concatenate([ue, pe[..., None]], axis=2) - uh
    wq = w[None, :] * g.h ** d
    vol = NE * wq.sum()                                      # measure of the domain
    if all(b == "stress" for b in prob.bc):
        # rigid motions of the velocity (the stress-wall kernel), removed by
        # Gram-Schmidt in L2 over the domain
        modes = []
        for i in range(d):
            F = np.zeros((NE, Q, d + 1))
            F[..., i] = 1.0
            modes.append(F)
        if prob.gamma and not prob.unsteady:
            for a in range(d):
                for b in range(a + 1, d):
                    F = np.zeros((NE, Q, d + 1))
                    F[..., b] = X[..., a] - 0.5
                    F[..., a] = -(X[..., b] - 0.5)
                    modes.append(F)
        if prob.unsteady:
            modes = []
        basis = []
        for F in modes:
            for Bm in basis:
                F = F - (F * Bm * wq[..., None]).sum() * Bm
            F = F / np.sqrt((F * F * wq[..., None]).sum())
            basis.append(F)
        for Bm in basis:
            err = err - (err * Bm * wq[..., None]).sum() * Bm
    else:
        fields = [d] if k0 == 1 else list(range(d + 1))
        for f in fields:                                         # remove constants
            err[..., f] -= (err[..., f] * wq).sum() / vol
    l2 = np.sqrt((err ** 2 * wq[..., None]).sum(axis=(0, 1)))
    linf = np.abs(err).max(axis=(0, 1))
    return dict(u_l2=float(np.sqrt((l2[:d] ** 2).sum())), p_l2=float(l2[d]),
                u_max=float(linf[:d].max()), p_max=float(linf[d]))
