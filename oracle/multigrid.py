"""Element-block Gauss-Seidel smoothing and the V-cycle (Algorithm 1).

Bottom solve (footnote to the bottom solver in section 3): the least-squares
solution with the eigendecomposition pseudo-inverse, near-zero eigenvalues
snapped to zero (built in hierarchy.py on the equilibrated operator).
Reading: the solve is that solution computed to working accuracy, i.e. the
pseudo-inverse applied with one refinement step; the pseudo-inverse alone
has a backward error of order eps * cond(A_c).

Block Gauss-Seidel (section 3): for element i of the current colour,
x_i <- A_ii^{-1} (b_i - sum_{j != i} A_ij x_j).  Elements of one colour are
updated together from the iterate as it stood at the start of the colour
pass; for a colouring in which no two same-coloured elements are coupled
this is the sequential sweep in colour order.  The update is carried out in
the algebraically identical correction form x_i <- x_i + A_ii^{-1} r_i with
r = b - A x, which is what both the paper's formula and this form compute in
exact arithmetic.
"""
from __future__ import annotations

import numpy as np


def blocks_all_equal(Ainv):
    """True when every element's block is the same matrix (to 1e-12 of its
    largest entry): constant coefficients on a translation-invariant grid."""
    B = np.asarray(Ainv)
    return bool(np.abs(B - B[0]).max() <= 1e-12 * np.abs(B[0]).max())


class Precision:
    """Operator copies in one floating-point type (float64, or float32 to
    emulate the mixed-precision V-cycle).  inv_bf16: the block inverses held
    as bfloat16 values (the symmetric part of each FP64 inverse rounded to
    float32, then to the nearest bfloat16), the arithmetic in float32; a
    level whose blocks are all one matrix keeps that one inverse in the
    working precision (storing a single block in bfloat16 saves nothing)."""

    def __init__(self, hier, dtype=np.float64, inv_bf16=False):
        self.hier = hier
        self.dtype = dtype
        self.A = [lv.A.astype(dtype) for lv in hier.levels]
        self.I = [lv.I.astype(dtype) if hasattr(lv, "I") else None for lv in hier.levels]
        self.Ainv = []
        for lv in hier.levels:
            if not hasattr(lv, "Ainv"):
                self.Ainv.append(None)
            elif inv_bf16 and not blocks_all_equal(lv.Ainv):
                from .learned import bf16
                sym = 0.5 * (lv.Ainv + np.transpose(lv.Ainv, (0, 2, 1)))
                self.Ainv.append(bf16(sym.astype(np.float32)).astype(dtype))
            else:
                self.Ainv.append(lv.Ainv.astype(dtype))


def colour_pass(A, Ainv, x, b, elems, nb):
    """One colour: x_E += A_EE^{-1} (b - A x)_E for every E in ``elems``."""
    r = b - A @ x
    rE = r.reshape(-1, nb)[elems]
    upd = np.einsum("eij,ej->ei", Ainv[elems], rE)
    xv = x.reshape(-1, nb)
    xv[elems] += upd
    return x


def smooth(P, li, x, b, sweeps):
    lv = P.hier.levels[li]
    A, Ainv = P.A[li], P.Ainv[li]
    for _ in range(sweeps):
        for c in range(lv.ncol):
            elems = np.nonzero(lv.colours == c)[0]
            if elems.size:
                colour_pass(A, Ainv, x, b, elems, lv.nb)
    return x


def vcycle(P, li, x, b):
    """Algorithm 1 on level ``li`` (0 = finest); returns the updated x."""
    hier = P.hier
    prob = hier.prob
    if li == len(hier.levels) - 1:
        lv = hier.levels[li]
        # bottom solve in FP64 (cast in and out for reduced-precision cycles):
        # the least-squares solution A_c^+ b of the bottom-solver footnote,
        # applied with one step of iterative refinement so that it is
        # computed to working accuracy
        b64 = b.astype(np.float64)
        x = lv.pinv @ b64
        x = x + lv.pinv @ (b64 - lv.A @ x)
        return x.astype(P.dtype)
    smooth(P, li, x, b, prob.nu1)
    r2 = P.I[li].T @ (b - P.A[li] @ x)
    x2 = vcycle(P, li + 1, np.zeros_like(r2), r2)
    x += P.I[li] @ x2
    smooth(P, li, x, b, prob.nu2)
    return x


def apply_vcycle(P, b, x=None):
    """One V-cycle on the (possibly scaled) finest-level system from x (default 0)."""
    b = np.asarray(b, dtype=P.dtype)
    x = np.zeros_like(b) if x is None else np.array(x, dtype=P.dtype)
    return vcycle(P, 0, x, b)
