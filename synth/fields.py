"""Closed-form coefficient fields, manufactured solutions and forcings.

Every object evaluates pointwise on an array of points ``x`` of shape
``(N, d)`` with coordinates in the unit cube.  Nothing here discretises
anything: these are the PDE data of the Stokes problems of the paper,
eq. (govern1)-(govern3) and its unsteady variant eq. (timedep1).
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * math.pi


# ---------------------------------------------------------------------------
# Coefficient fields (viscosity mu, density rho)
# ---------------------------------------------------------------------------
@dataclass
class ConstField:
    """mu(x) = c."""
    c: float = 1.0
    kind: str = "const"

    def value(self, x, chi=None):
        return np.full(x.shape[0], float(self.c))

    def grad(self, x, chi=None):
        return np.zeros_like(x, dtype=float)

    def params(self):
        return np.array([self.c], dtype=float)


@dataclass
class SinProductField:
    """mu(x) = a + b * prod_j sin(2 pi k x_j)  (the C2 viscosity has a=1, b=0.9, k=1)."""
    a: float = 1.0
    b: float = 0.9
    k: float = 1.0
    kind: str = "sinsin"

    def value(self, x, chi=None):
        return self.a + self.b * np.prod(np.sin(TWO_PI * self.k * x), axis=1)

    def grad(self, x, chi=None):
        s = np.sin(TWO_PI * self.k * x)
        c = np.cos(TWO_PI * self.k * x)
        d = x.shape[1]
        g = np.empty_like(x, dtype=float)
        for j in range(d):
            others = np.prod(np.delete(s, j, axis=1), axis=1)
            g[:, j] = self.b * TWO_PI * self.k * c[:, j] * others
        return g

    def params(self):
        return np.array([self.a, self.b, self.k], dtype=float)


@dataclass
class PhaseField:
    """Piecewise-constant field on two phases of the square/cube inclusion.

    Phase 1 is the open box (lo, hi)^d, phase 2 its complement (the paper's
    square inclusion test).  ``values[chi-1]`` is the value in phase chi.
    """
    values: tuple = (1.0e4, 1.0)
    lo: float = 0.25
    hi: float = 0.75
    kind: str = "phase"

    def phase(self, x):
        inside = np.all((x > self.lo) & (x < self.hi), axis=1)
        return np.where(inside, 1, 2)

    def value(self, x, chi=None):
        if chi is None:
            chi = self.phase(x)
        vals = np.asarray(self.values, dtype=float)
        return vals[np.asarray(chi) - 1]

    def grad(self, x, chi=None):
        return np.zeros_like(x, dtype=float)

    def params(self):
        return np.array([self.values[0], self.values[1], self.lo, self.hi], dtype=float)


@dataclass
class LogNormalRFF:
    """mu(x) = 10**g(x), g = sqrt(2/K) sum_m cos(k_m . x + phi_m).

    Random Fourier features of a unit-variance Gaussian field with squared
    exponential covariance of correlation length ``ell``: k_m ~ N(0, ell^-2 I),
    phi_m ~ U[0, 2 pi), drawn from numpy's PCG64 with the given seed.
    """
    kvecs: np.ndarray = field(default_factory=lambda: np.zeros((1, 3)))
    phases: np.ndarray = field(default_factory=lambda: np.zeros(1))
    kind: str = "lognormal_rff"

    @staticmethod
    def from_seed(seed: int, dim: int, K: int = 256, ell: float = 0.1):
        rng = np.random.Generator(np.random.PCG64(seed))
        kvecs = rng.normal(0.0, 1.0 / ell, size=(K, dim))
        phases = rng.uniform(0.0, TWO_PI, size=K)
        return LogNormalRFF(kvecs=kvecs, phases=phases)

    def _eval(self, x, want_grad):
        """g (and its gradient) at the points x, evaluated in row blocks on a
        thread pool (numpy releases the interpreter lock inside the products
        and the trigonometric functions)."""
        K = self.kvecs.shape[0]
        x = np.asarray(x, dtype=float)
        n = x.shape[0]
        g = np.empty(n)
        dg = np.empty_like(x) if want_grad else None
        sc = math.sqrt(2.0 / K)

        def block(lo, hi):
            arg = x[lo:hi] @ self.kvecs.T + self.phases[None, :]
            g[lo:hi] = sc * np.cos(arg).sum(axis=1)
            if want_grad:
                dg[lo:hi] = -sc * (np.sin(arg) @ self.kvecs)

        step = 8192
        if n <= step:
            block(0, n)
        else:
            from concurrent.futures import ThreadPoolExecutor
            with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
                list(ex.map(lambda lo: block(lo, min(lo + step, n)), range(0, n, step)))
        return g, dg

    def value(self, x, chi=None):
        g, _ = self._eval(x, False)
        return 10.0 ** g

    def grad(self, x, chi=None):
        g, dg = self._eval(x, True)
        return (10.0 ** g)[:, None] * math.log(10.0) * dg

    def params(self):
        return np.concatenate([self.kvecs.ravel(), self.phases])


# ---------------------------------------------------------------------------
# Manufactured solutions built from products of shifted sines
# ---------------------------------------------------------------------------
@dataclass
class AmplitudeField:
    """mu_a(x) = mu(x)^a for a positive field mu: for the log-normal field,
    10^(a g(x)), the same field with its log-amplitude scaled by a."""
    base: object
    a: float
    kind: str = "callback"

    def value(self, x, chi=None):
        return self.base.value(x, chi) ** self.a

    def grad(self, x, chi=None):
        m = self.base.value(x, chi)
        return (self.a * m ** (self.a - 1.0))[:, None] * self.base.grad(x, chi)


@dataclass
class SinProd:
    """c * prod_j sin(2 pi (x_j + s_j)), with value, gradient and Hessian."""
    c: float
    shifts: tuple

    def _sc(self, x):
        arg = TWO_PI * (x + np.asarray(self.shifts)[None, :])
        return np.sin(arg), np.cos(arg)

    def value(self, x):
        s, _ = self._sc(x)
        return self.c * np.prod(s, axis=1)

    def grad(self, x):
        s, co = self._sc(x)
        d = x.shape[1]
        g = np.empty_like(x, dtype=float)
        for j in range(d):
            f = TWO_PI * co[:, j]
            for l in range(d):
                if l != j:
                    f = f * s[:, l]
            g[:, j] = self.c * f
        return g

    def hess(self, x):
        s, co = self._sc(x)
        d = x.shape[1]
        H = np.empty((x.shape[0], d, d))
        for j in range(d):
            for l in range(d):
                f = np.full(x.shape[0], self.c)
                for r in range(d):
                    if r == j and r == l:
                        f = f * (-(TWO_PI ** 2) * s[:, r])
                    elif r == j or r == l:
                        f = f * (TWO_PI * co[:, r])
                    else:
                        f = f * s[:, r]
                H[:, j, l] = f
        return H


@dataclass
class ExactSolution:
    """Exact (u, p) per phase, with the forcing it induces for a given mu.

    ``u[chi]`` is a list of d SinProd components and ``p[chi]`` a SinProd, for
    each phase chi present.  ``forcing`` evaluates eq. (govern1):
    f = -div(mu (grad u + gamma grad u^T)) + grad p and f_div = -div u, with
    the term (rho / delta) u of eq. (timedep1) added when rho_delta > 0.
    """
    dim: int
    gamma: int
    mu: object
    u: dict
    p: dict
    rho_delta: object = 0.0     # rho / delta of eq. (timedep1): a number, or {phase: value}; 0: steady

    def _phases(self, chi, n):
        if chi is None:
            return np.ones(n, dtype=int) * min(self.u.keys())
        return np.asarray(chi)

    def _per_phase(self, x, chi, fn):
        chi = self._phases(chi, x.shape[0])
        out = None
        for c in np.unique(chi):
            sel = chi == c
            val = fn(x[sel], int(c))
            if out is None:
                out = np.zeros((x.shape[0],) + val.shape[1:])
            out[sel] = val
        return out

    def velocity(self, x, chi=None):
        return self._per_phase(x, chi, lambda y, c: np.stack([f.value(y) for f in self.u[c]], axis=1))

    def grad_velocity(self, x, chi=None):
        """(N, d, d) with [i, j] = d u_i / d x_j."""
        return self._per_phase(x, chi, lambda y, c: np.stack([f.grad(y) for f in self.u[c]], axis=1))

    def pressure(self, x, chi=None):
        return self._per_phase(x, chi, lambda y, c: self.p[c].value(y))

    def stress(self, x, chi=None):
        """sigma = mu (grad u + gamma grad u^T) - p I."""
        gu = self.grad_velocity(x, chi)
        mu = self.mu.value(x, chi)
        s = mu[:, None, None] * (gu + self.gamma * np.transpose(gu, (0, 2, 1)))
        s -= self.pressure(x, chi)[:, None, None] * np.eye(self.dim)[None]
        return s

    def forcing(self, x, chi=None):
        def f(y, c):
            d = self.dim
            mu = self.mu.value(y, np.full(y.shape[0], c))
            dmu = self.mu.grad(y, np.full(y.shape[0], c))
            gu = np.stack([q.grad(y) for q in self.u[c]], axis=1)       # [n, i, j]
            Hu = np.stack([q.hess(y) for q in self.u[c]], axis=1)       # [n, i, j, l]
            gp = self.p[c].grad(y)
            out = np.empty((y.shape[0], d))
            for i in range(d):
                acc = np.zeros(y.shape[0])
                for j in range(d):
                    acc += dmu[:, j] * (gu[:, i, j] + self.gamma * gu[:, j, i])
                    acc += mu * (Hu[:, i, j, j] + self.gamma * Hu[:, j, i, j])
                rd = self.rho_delta[c] if isinstance(self.rho_delta, dict) else self.rho_delta
                out[:, i] = -acc + gp[:, i] + rd * np.stack([q.value(y) for q in self.u[c]], axis=1)[:, i]
            return out
        return self._per_phase(x, chi, f)

    def forcing_div(self, x, chi=None):
        def f(y, c):
            gu = np.stack([q.grad(y) for q in self.u[c]], axis=1)
            return -np.einsum("nii->n", gu)
        return self._per_phase(x, chi, f)


def make_exact_c1(mu=None):
    """u = (sin2pi x cos2pi y, -cos2pi x sin2pi y), p = cos2pi x cos2pi y (2D)."""
    mu = mu or ConstField(1.0)
    u = {1: [SinProd(1.0, (0.0, 0.25)), SinProd(-1.0, (0.25, 0.0))]}
    p = {1: SinProd(1.0, (0.25, 0.25))}
    return ExactSolution(dim=2, gamma=0, mu=mu, u=u, p=p)


def make_exact_paper(dim, gamma, mu, phases=(1,), mu_chi=None):
    """The paper's manufactured solution (grid-convergence appendix):

    u_i = prod_j sin 2pi(x_j - 0.2 i - 0.25 (chi-1)),
    p   = mu_chi prod_j sin 2pi(x_j + 0.2 - 0.25 (chi-1)),  i = 1..d.
    """
    mu_chi = mu_chi or {c: 1.0 for c in phases}
    u, p = {}, {}
    for chi in phases:
        off = -0.25 * (chi - 1)
        u[chi] = [SinProd(1.0, tuple([-0.2 * i + off] * dim)) for i in range(1, dim + 1)]
        p[chi] = SinProd(float(mu_chi[chi]), tuple([0.2 + off] * dim))
    return ExactSolution(dim=dim, gamma=gamma, mu=mu, u=u, p=p)


def projected_coeffs(exact, dim, n, p, q=None):
    """Coefficients of the element-wise L2 projection of a single-phase sine
    product solution (u_i and p each a SinProd) onto the orthonormal tensor
    Legendre basis of the n^d grid (element-major, axis 0 fastest; fields
    u_1..u_d, p; tensor-lexicographic coefficients).  A product of functions
    of one coordinate projects as the product of their 1D projections, so
    only n (p+1) one-dimensional integrals per factor are formed (Gauss rule
    of q = p + 6 points)."""
    from numpy.polynomial.legendre import leggauss
    q = q or p + 6
    m = p + 1
    h = 1.0 / n
    t, w = leggauss(q)
    xi, wq = 0.5 * (t + 1.0), 0.5 * w                         # Gauss rule on [0, 1]
    # l_a(xi) = sqrt(2a+1) P_a(2 xi - 1)
    L = np.stack([np.sqrt(2 * a + 1) * np.polynomial.legendre.legval(2 * xi - 1, [0] * a + [1]) for a in range(m)])
    X = (np.arange(n)[:, None] + xi[None, :]) * h              # (n, q) points per cell

    def proj1d(sp, j):
        # int over cell c of sin(2 pi (x + s_j)) h^{-1/2} l_a((x - c h)/h) dx
        f = np.sin(TWO_PI * (X + sp.shifts[j]))
        return (f * wq[None, :]) @ L.T * np.sqrt(h)           # (n, m)

    fields = [exact.u[1][i] for i in range(dim)] + [exact.p[1]]
    out = np.empty((n ** dim, dim + 1, m ** dim))
    for fi, sp in enumerate(fields):
        P = [proj1d(sp, j) for j in range(dim)]
        if dim == 2:
            # element (c0, c1), axis 0 fastest; coefficient (a0, a1), a0 fastest
            T = np.einsum("xa,yb->yxba", P[0], P[1])
        else:
            T = np.einsum("xa,yb,zc->zyxcba", P[0], P[1], P[2])
        out[:, fi, :] = sp.c * T.reshape(n ** dim, m ** dim)
    return out.ravel()


@dataclass
class FourierForcing:
    """Seeded smooth Gaussian-random forcing.

    f_c(x) = s_c sum_{k in {0..kmax-1}^d, k != 0} a_{c,k} cos 2pi k.x + b_{c,k} sin 2pi k.x
    with a, b ~ N(0, 1) from PCG64(seed) and s_c chosen so that each component
    has unit root-mean-square over the unit cube.  f_div = 0.
    """
    dim: int
    kmodes: np.ndarray      # (M, d) integer wave vectors
    a: np.ndarray           # (d, M)
    b: np.ndarray           # (d, M)

    @staticmethod
    def from_seed(seed: int, dim: int, kmax: int = 8):
        grids = np.meshgrid(*[np.arange(kmax)] * dim, indexing="ij")
        kmodes = np.stack([g.ravel() for g in grids], axis=1)
        kmodes = kmodes[np.any(kmodes != 0, axis=1)]
        rng = np.random.Generator(np.random.PCG64(seed))
        a = rng.normal(size=(dim, kmodes.shape[0]))
        b = rng.normal(size=(dim, kmodes.shape[0]))
        rms = np.sqrt(0.5 * (a ** 2 + b ** 2).sum(axis=1))
        return FourierForcing(dim=dim, kmodes=kmodes, a=a / rms[:, None], b=b / rms[:, None])

    def forcing_direct(self, x):
        arg = TWO_PI * (x @ self.kmodes.T)
        return np.cos(arg) @ self.a.T + np.sin(arg) @ self.b.T

    def forcing(self, x, chi=None):
        """Same sum, evaluated axis by axis: a cos(2pi k.x) + b sin(2pi k.x) is
        Re[(a - i b) prod_j exp(2 pi i k_j x_j)], and the wave vectors fill a
        tensor grid, so the sum contracts one axis at a time."""
        x = np.asarray(x, dtype=float)
        n, d = x.shape
        km = int(self.kmodes.max()) + 1
        C = np.zeros((self.dim,) + (km,) * d, dtype=complex)
        C[(slice(None),) + tuple(self.kmodes[:, j] for j in range(d))] = (self.a - 1j * self.b)
        m = np.arange(km)
        out = np.empty((n, self.dim))
        Cm = C.reshape(-1, km).T

        def block(lo, hi):
            xs = x[lo:hi]
            nb = xs.shape[0]
            Z = [np.exp(2j * np.pi * xs[:, j:j + 1] * m[None, :]) for j in range(d)]
            T = Z[d - 1] @ Cm                                   # (nb, dim * km^(d-1)), last axis contracted
            for j in range(d - 2, -1, -1):
                T = (T.reshape(nb, -1, km) * Z[j][:, None, :]).sum(axis=2)
            out[lo:hi] = T.real.reshape(nb, self.dim)

        step = 8192
        if n <= step:
            block(0, n)
        else:
            from concurrent.futures import ThreadPoolExecutor
            with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
                list(ex.map(lambda lo: block(lo, min(lo + step, n)), range(0, n, step)))
        return out

    def forcing_div(self, x, chi=None):
        return np.zeros(x.shape[0])


# ---------------------------------------------------------------------------
# Circular interface (implicitly defined meshes)
# ---------------------------------------------------------------------------
@dataclass
class CirclePhaseField:
    """Two phases separated by a circle: phase 1 the open disk |x - c| < r,
    phase 2 the rest of the unit square.  The level set is the signed
    distance phi(x) = |x - c| - r (negative in phase 1), its gradient the unit
    normal pointing from phase 1 into phase 2, its curvature 1 / r.
    ``values[chi-1]`` is the field's value in phase chi."""
    values: tuple = (1.0e4, 1.0)
    centre: tuple = (0.5, 0.5)
    radius: float = 0.3
    kind: str = "circle"
    void_outside: bool = False      # True: the domain is the disk alone (curved domain)

    def levelset(self, x):
        x = np.atleast_2d(x)
        return np.sqrt(((x - np.asarray(self.centre)[None, :]) ** 2).sum(axis=1)) - self.radius

    def levelset_grad(self, x):
        x = np.atleast_2d(x)
        v = x - np.asarray(self.centre)[None, :]
        return v / np.sqrt((v ** 2).sum(axis=1))[:, None]

    def curvature(self):
        return 1.0 / self.radius

    def box_range(self, lo, hi):
        """Exact minimum and maximum of phi over the box [lo, hi]."""
        c = np.asarray(self.centre, dtype=float)
        lo, hi = np.asarray(lo, dtype=float), np.asarray(hi, dtype=float)
        near = np.clip(c, lo, hi)
        far = np.where(np.abs(lo - c) > np.abs(hi - c), lo, hi)
        return (float(np.sqrt(((near - c) ** 2).sum())) - self.radius,
                float(np.sqrt(((far - c) ** 2).sum())) - self.radius)

    def phase(self, x):
        return np.where(self.levelset(x) < 0.0, 1, 2)

    def value(self, x, chi=None):
        if chi is None:
            chi = self.phase(x)
        vals = np.asarray(self.values, dtype=float)
        return vals[np.asarray(chi) - 1]

    def grad(self, x, chi=None):
        return np.zeros_like(np.atleast_2d(x), dtype=float)

    def params(self):
        return np.array([self.values[0], self.values[1], self.centre[0], self.centre[1],
                         self.radius], dtype=float)


@dataclass
class BubbleForcing:
    """A static bubble: gravity rho_chi g (g = (0, -1)) in each phase, no-slip
    walls, no velocity jump across the interface, and the stress jump of
    surface tension: with jumps taken phase 1 (the bubble) minus phase 2, as
    in the interface conditions of eq. (govern2), n the unit normal from
    phase 1 into phase 2 and kappa = 1 / r, [sigma n] = -sigma_st kappa n, so
    that at rest (sigma = -p I) phase 1's pressure exceeds phase 2's by
    sigma_st kappa (the Young-Laplace balance)."""
    rho: tuple = (1.0, 1.0e-3)
    sigma_st: float = 1.0
    kappa: float = 1.0 / 0.3
    dim: int = 2

    def forcing(self, x, chi=None):
        x = np.atleast_2d(x)
        chi = np.ones(x.shape[0], dtype=int) if chi is None else np.asarray(chi)
        out = np.zeros((x.shape[0], self.dim))
        out[:, self.dim - 1] = -np.asarray(self.rho, dtype=float)[chi - 1]
        return out

    def forcing_div(self, x, chi=None):
        return np.zeros(np.atleast_2d(x).shape[0])

    def velocity(self, x, chi=None):
        return np.zeros((np.atleast_2d(x).shape[0], self.dim))

    def interface_jumps(self, x, normal):
        """(g, h) = ([u], [sigma n]) at points x with unit normals ``normal``."""
        g = np.zeros_like(np.atleast_2d(x), dtype=float)
        return g, -self.sigma_st * self.kappa * np.atleast_2d(normal)
