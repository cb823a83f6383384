"""Outer iterations around the V-cycle.

* stationary: x_{k+1} = V(b, x_k) from x_0 = 0 (section 3: the V-cycle "can be
  used as a standalone iterative solver");
* iterative refinement: r = b - A x in FP64, z = V(r) from zero in the cycle's
  precision, x += z;
* FGMRES(m), right-preconditioned by one V-cycle from zero, modified
  Gram-Schmidt and Givens rotations in FP64 (the paper uses left-
  preconditioned GMRES without restarts; a flexible right-preconditioned
  variant is needed once the preconditioner is inexact);
* the convergence metric rho of eq. (rho): left-preconditioned GMRES with
  b = 0 and a random initial guess, run until the preconditioned residual
  has dropped by 1e8.

Relative residuals are ||b - A x||_2 / ||b||_2 recomputed explicitly in FP64
on the unscaled fine-grid operator.  b is first projected onto the range of
A by removing its components along the known kernel.
"""
from __future__ import annotations

import numpy as np

from .multigrid import Precision, apply_vcycle


class Solver:
    def __init__(self, hier):
        self.hier = hier
        fine = hier.fine
        self.d = fine.dscale if fine.dscale is not None else np.ones(fine.A.shape[0])
        Dinv = 1.0 / self.d
        # unscaled fine operator A = D^{-1} (D A D) D^{-1}
        import scipy.sparse as sp
        self.A = (sp.diags(Dinv) @ fine.A @ sp.diags(Dinv)).tocsr()
        self.P = {(np.float64, False): Precision(hier, np.float64)}

    def prec(self, dtype, inv_bf16=False):
        key = (dtype, inv_bf16)
        if key not in self.P:
            self.P[key] = Precision(self.hier, dtype, inv_bf16)
        return self.P[key]

    def vcycle_unscaled(self, b, x=None, dtype=np.float64, inv_bf16=False):
        """One V-cycle for A x = b in unscaled variables (inv_bf16: block
        inverses stored as bfloat16, float32 arithmetic)."""
        P = self.prec(dtype, inv_bf16)
        bs = (self.d * b).astype(dtype)
        xs = None if x is None else (x / self.d).astype(dtype)
        return self.d * apply_vcycle(P, bs, xs).astype(np.float64)

    def relres(self, b, x):
        return np.linalg.norm(b - self.A @ x) / np.linalg.norm(b)

    def stationary(self, b, maxit, tol=0.0, dtype=np.float64, inv_bf16=False):
        b = self.hier.project_kernel(np.asarray(b, dtype=np.float64))
        x = np.zeros_like(b)
        hist = [self.relres(b, x)]
        for _ in range(maxit):
            x = self.vcycle_unscaled(b, x, dtype, inv_bf16)
            hist.append(self.relres(b, x))
            if hist[-1] <= tol:
                break
        return x, np.array(hist)

    def refinement(self, b, tol=1e-10, maxit=50, dtype=np.float32, inv_bf16=False):
        b = self.hier.project_kernel(np.asarray(b, dtype=np.float64))
        x = np.zeros_like(b)
        hist = [1.0]
        for _ in range(maxit):
            r = b - self.A @ x
            if np.linalg.norm(r) / np.linalg.norm(b) <= tol:
                break
            x = x + self.vcycle_unscaled(r, None, dtype, inv_bf16)
            hist.append(self.relres(b, x))
        return x, np.array(hist)

    def fgmres(self, b, tol=1e-10, m=30, maxit=200, dtype=np.float64):
        b = self.hier.project_kernel(np.asarray(b, dtype=np.float64))
        nb = np.linalg.norm(b)
        x = np.zeros_like(b)
        hist = [1.0]
        its = 0
        while its < maxit:
            r = b - self.A @ x
            beta = np.linalg.norm(r)
            if beta / nb <= tol:
                break
            V = [r / beta]
            Z = []
            H = np.zeros((m + 1, m))
            cs, sn = np.zeros(m), np.zeros(m)
            g = np.zeros(m + 1)
            g[0] = beta
            j_done = 0
            for j in range(m):
                z = self.vcycle_unscaled(V[j], None, dtype)
                Z.append(z)
                w = self.A @ z
                for i in range(j + 1):
                    H[i, j] = np.dot(w, V[i])
                    w = w - H[i, j] * V[i]
                H[j + 1, j] = np.linalg.norm(w)
                V.append(w / H[j + 1, j] if H[j + 1, j] > 0 else w)
                for i in range(j):
                    t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                    H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                    H[i, j] = t
                den = np.hypot(H[j, j], H[j + 1, j])
                cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
                H[j, j] = den
                H[j + 1, j] = 0.0
                g[j + 1] = -sn[j] * g[j]
                g[j] = cs[j] * g[j]
                its += 1
                j_done = j + 1
                hist.append(abs(g[j + 1]) / nb)
                if abs(g[j + 1]) / nb <= tol or its >= maxit:
                    break
            y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
            x = x + np.stack(Z[:j_done], axis=1) @ y
        return x, np.array(hist)

    def rho_metric(self, seed=0, reduction=1e-8, maxit=100, return_history=False):
        """eq. (rho): average reduction per iteration of the left-preconditioned
        GMRES residual ||V A x_n - V b|| with b = 0 and a random x_0 (x_0 from
        PCG64(seed), kernel removed).  With return_history, also the ratios
        ||V A x_k|| / ||V A x_0||, k = 0..n."""
        rng = np.random.Generator(np.random.PCG64(seed))
        x0 = self.hier.project_kernel(rng.standard_normal(self.A.shape[0]))

        def VA(v):
            return self.vcycle_unscaled(self.A @ v, None, np.float64)

        r0 = -VA(x0)
        beta = np.linalg.norm(r0)
        V = [r0 / beta]
        H = np.zeros((maxit + 1, maxit))
        res = [beta]
        for j in range(maxit):
            w = VA(V[j])
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            V.append(w / H[j + 1, j])
            e1 = np.zeros(j + 2)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)
            res.append(np.linalg.norm(e1 - H[:j + 2, :j + 1] @ y))
            if res[-1] <= reduction * beta:
                break
        n = len(res) - 1
        rho = float(np.exp(np.log(res[-1] / res[0]) / n))
        if return_history:
            return rho, n, np.array(res) / res[0]
        return rho, n
