"""Orthonormal tensor-product Legendre basis and Gauss quadrature on [0,1]^d.

The paper leaves the basis of Q_p open (section 2); this oracle uses the
orthonormal shifted Legendre polynomials l_m(xi) = sqrt(2m+1) P_m(2 xi - 1),
so that the element mass matrix M is the identity.  Element basis functions
are phi_a(x) = h^{-d/2} prod_k l_{a_k}((x_k - x_{E,k}) / h) with the multi-
index a = sum_k a_k (p+1)^k (axis 0 fastest).
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from numpy.polynomial import legendre as npleg


def gauss01(q: int):
    """q-point Gauss-Legendre nodes and weights on [0, 1]."""
    x, w = npleg.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def leg_values(p: int, xi):
    """(len(xi), p+1) values of l_m at xi."""
    xi = np.asarray(xi, dtype=float)
    out = np.empty((xi.size, p + 1))
    for m in range(p + 1):
        c = np.zeros(m + 1)
        c[m] = 1.0
        out[:, m] = math.sqrt(2 * m + 1) * npleg.legval(2.0 * xi - 1.0, c)
    return out


def leg_derivs(p: int, xi):
    """(len(xi), p+1) derivatives d l_m / d xi at xi."""
    xi = np.asarray(xi, dtype=float)
    out = np.empty((xi.size, p + 1))
    for m in range(p + 1):
        c = np.zeros(m + 1)
        c[m] = 1.0
        out[:, m] = math.sqrt(2 * m + 1) * 2.0 * npleg.legval(2.0 * xi - 1.0, npleg.legder(c))
    return out


def multi_indices(p: int, d: int):
    """List of (a_0, ..., a_{d-1}) in storage order (axis 0 fastest)."""
    m = p + 1
    return [tuple((a // m ** j) % m for j in range(d)) for a in range(m ** d)]


def ref_basis(p: int, pts, deriv_axis=None):
    """Reference basis prod_j l_{a_j}(xi_j) at points (Q, d); optionally its
    derivative along ``deriv_axis`` (with respect to the reference coordinate)."""
    pts = np.atleast_2d(pts)
    Q, d = pts.shape
    vals = [leg_values(p, pts[:, j]) for j in range(d)]
    ders = [leg_derivs(p, pts[:, j]) for j in range(d)]
    idx = multi_indices(p, d)
    out = np.ones((Q, len(idx)))
    for a, digits in enumerate(idx):
        for j in range(d):
            tab = ders[j] if j == deriv_axis else vals[j]
            out[:, a] *= tab[:, digits[j]]
    return out


def tensor_gauss(q: int, d: int):
    """Tensor Gauss points (Q, d) and weights (Q,) on [0,1]^d, axis 0 fastest."""
    x, w = gauss01(q)
    pts, wts = [], []
    for tup in itertools.product(range(q), repeat=d):
        ids = tup[::-1]  # itertools varies the last entry fastest; store axis 0 fastest
        pts.append([x[i] for i in ids])
        wts.append(np.prod([w[i] for i in ids]))
    return np.array(pts), np.array(wts)


def face_gauss(q: int, d: int, axis: int, side: float):
    """Gauss points (Q, d) on the reference face xi_axis = side and weights."""
    if d == 1:
        return np.array([[side]]), np.array([1.0])
    tp, tw = tensor_gauss(q, d - 1)
    pts = np.insert(tp, axis, side, axis=1)
    return pts, tw
