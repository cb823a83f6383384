"""Quadrature on rectangles cut by a level set (2D), for implicitly defined
meshes (section 5, "Curved domain geometry": elements and faces whose shape
is defined by a level set need quadrature schemes of their own, computed by
the high-order algorithm the paper cites).

TEST INFRASTRUCTURE ONLY (part of the oracle).

The method restated here is the dimension-reduction scheme of Saye (SIAM J.
Sci. Comput. 37, 2015) specialised to two dimensions:

* a height axis k is chosen along which phi is monotone on the box (the
  axis of the largest |d phi / d x_k| at the box centre; if d phi / d x_k
  changes sign on the box, the box is halved along its longer side and each
  half treated the same way);
* the base interval (the other axis) is split at the roots of phi on the two
  bounding lines x_k = lo_k and x_k = hi_k; on each piece q Gauss points;
* at each base point the height line meets phi = 0 at most once; the line is
  split there and each part receives q Gauss points and the phase of its
  midpoint; the root itself is a point of the interface rule, with weight
  w_base |grad phi| / |d phi / d x_k| and normal grad phi / |grad phi|.

Roots of phi along a line are bracketed by the sign changes of ``NSAMP + 1``
equally spaced samples and refined with Brent's method.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq

from .basis import gauss01

NSAMP = 32


def line_roots(f, a, b):
    """Roots of the scalar function f on [a, b] (sign changes of samples)."""
    s = np.linspace(a, b, NSAMP + 1)
    v = np.array([f(t) for t in s])
    out = []
    for i in range(NSAMP):
        if v[i] == 0.0:
            if 0 < i:
                out.append(s[i])
        elif v[i] * v[i + 1] < 0.0:
            out.append(brentq(f, s[i], s[i + 1], xtol=1e-16, rtol=1e-15, maxiter=200))
    return out


def _point(k, t_base, t_height):
    x = np.empty(2)
    x[k] = t_height
    x[1 - k] = t_base
    return x


def _monotone(ls, lo, hi, k):
    """True when d phi / d x_k keeps one strict sign on the box (sampled)."""
    s0 = np.linspace(lo[0], hi[0], 9)
    s1 = np.linspace(lo[1], hi[1], 9)
    X = np.array([[a, b] for a in s0 for b in s1])
    g = ls.levelset_grad(X)[:, k]
    return bool(np.all(g > 0.0) or np.all(g < 0.0))


def cut_box_rules(ls, lo, hi, q):
    """Quadrature rules on the box [lo, hi]:

    returns dict(vol={1: (X, w), 2: (X, w)}, surf=(X, w, normals)) with the
    volume rules of phase 1 (phi < 0) and phase 2 (phi > 0) and the rule of
    the interface phi = 0 inside the box."""
    lo = np.asarray(lo, dtype=float)
    hi = np.asarray(hi, dtype=float)
    centre = 0.5 * (lo + hi)
    gc = ls.levelset_grad(centre[None, :])[0]
    k = int(np.argmax(np.abs(gc)))
    if not _monotone(ls, lo, hi, k):
        ax = int(np.argmax(hi - lo))
        mid = 0.5 * (lo[ax] + hi[ax])
        hi1 = hi.copy()
        hi1[ax] = mid
        lo2 = lo.copy()
        lo2[ax] = mid
        r1 = cut_box_rules(ls, lo, hi1, q)
        r2 = cut_box_rules(ls, lo2, hi, q)
        return _join(r1, r2)
    j = 1 - k
    phi = lambda x: float(ls.levelset(x[None, :])[0])
    brk = [lo[j], hi[j]]
    for side in (lo[k], hi[k]):
        brk += line_roots(lambda t: phi(_point(k, t, side)), lo[j], hi[j])
    brk = np.unique(np.array(brk))
    xg, wg = gauss01(q)
    vol = {1: ([], []), 2: ([], [])}
    sX, sw, sn = [], [], []
    for a, b in zip(brk[:-1], brk[1:]):
        if b - a <= 0.0:
            continue
        for t, wb in zip(a + (b - a) * xg, (b - a) * wg):
            f = lambda s: phi(_point(k, t, s))
            fa, fb = f(lo[k]), f(hi[k])
            cuts = [lo[k]]
            if fa * fb < 0.0:
                r = brentq(f, lo[k], hi[k], xtol=1e-16, rtol=1e-15, maxiter=200)
                cuts.append(r)
                xr = _point(k, t, r)
                gr = ls.levelset_grad(xr[None, :])[0]
                sX.append(xr)
                sw.append(wb * np.linalg.norm(gr) / abs(gr[k]))
                sn.append(gr / np.linalg.norm(gr))
            cuts.append(hi[k])
            for c, e in zip(cuts[:-1], cuts[1:]):
                if e - c <= 0.0:
                    continue
                chi = 1 if f(0.5 * (c + e)) < 0.0 else 2
                for s, wh in zip(c + (e - c) * xg, (e - c) * wg):
                    vol[chi][0].append(_point(k, t, s))
                    vol[chi][1].append(wb * wh)
    out = dict(vol={}, surf=None)
    for chi in (1, 2):
        X, w = vol[chi]
        out["vol"][chi] = (np.array(X).reshape(-1, 2), np.array(w))
    out["surf"] = (np.array(sX).reshape(-1, 2), np.array(sw), np.array(sn).reshape(-1, 2))
    return out


def _join(r1, r2):
    out = dict(vol={}, surf=None)
    for chi in (1, 2):
        out["vol"][chi] = (np.concatenate([r1["vol"][chi][0], r2["vol"][chi][0]]),
                           np.concatenate([r1["vol"][chi][1], r2["vol"][chi][1]]))
    out["surf"] = tuple(np.concatenate([a, b]) for a, b in zip(r1["surf"], r2["surf"]))
    return out


def segment_rules(ls, fixed_axis, fixed_value, a, b, q):
    """Rules on the segment {x_fixed_axis = fixed_value, a <= x_other <= b}
    for each phase: {1: (X, w), 2: (X, w)} (empty arrays for an absent phase)."""
    k = fixed_axis
    phi = lambda t: float(ls.levelset(_point(k, t, fixed_value)[None, :])[0])
    brk = np.unique(np.array([a, b] + line_roots(phi, a, b)))
    xg, wg = gauss01(q)
    out = {1: ([], []), 2: ([], [])}
    for c, e in zip(brk[:-1], brk[1:]):
        if e - c <= 0.0:
            continue
        chi = 1 if phi(0.5 * (c + e)) < 0.0 else 2
        for t, w in zip(c + (e - c) * xg, (e - c) * wg):
            out[chi][0].append(_point(k, t, fixed_value))
            out[chi][1].append(w)
    return {chi: (np.array(X).reshape(-1, 2), np.array(w)) for chi, (X, w) in out.items()}
