"""Pins of the oracle's two-phase, scaling, divergence, unsteady and 3D parts
against what the paper states, plus planted mistakes that must fail them.

* The error measure of the grid-convergence appendix removes the trivial
  kernel (constant fields) by an L2-orthogonal projection over the whole
  domain: checked on the L2 projection of the exact solution.
* Two phases, square inclusion (section 5.6): velocity of order p+1,
  pressure p+1/2 in L2 and p in the max norm; 7 to 10 GMRES iterations per
  1e8 reduction across viscosity ratios.
* The (alpha, beta) diagonal scaling (section 5.6) leaves the V-cycle's
  iterates unchanged when the viscosity is constant on every coarse
  element: block Gauss-Seidel is invariant under block-diagonal scaling,
  and the scaling then commutes with injection.
* The constraint row of eq. (appstokes2): the computed solution satisfies
  it, its data is compatible with the constant-pressure kernel, and for a
  divergence-free exact velocity sum_i G_i u_i tends to zero.
* The unsteady operator of eq. (timedep2) at Re ~ 1e4, delta = 0.1 h
  (section 6.1): velocity and pressure both of order p+1.
* 3D velocity Dirichlet problem with variable viscosity (sections 5.2, 5.4).
"""
import dataclasses
import math
import os

import numpy as np
import pytest

from synth import Problem, ConstField, SinProductField, PhaseField, c1_periodic_standard, \
    c2_dirichlet_varmu, c4a_square_inclusion
from synth.fields import make_exact_paper
from oracle import build_hierarchy
from oracle.assemble import Grid
from oracle.basis import ref_basis, tensor_gauss
from oracle.rhs import assemble_rhs
from oracle.solvers import Solver
from oracle.errors import solution_errors

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_orders(case):
    out = {}
    with open(os.path.join(GOLDEN, "convergence_orders.txt")) as fh:
        for line in fh:
            f = line.split()
            if f and not f[0].startswith("#") and f[0] == case:
                out[f[1]] = float(f[2])
    assert out, case
    return out


def _l2_projection(prob, q=8):
    """Coefficients of the L2 projection of the exact (u, p) onto the
    element-wise orthonormal basis (M = I: coefficient = inner product)."""
    d, p, n = prob.dim, prob.p, prob.n
    g = Grid(d, n, p, prob.bc, prob.phases)
    pts, w = tensor_gauss(q, d)
    B = ref_basis(p, pts) * g.h ** (-d / 2)
    X = (g.ijk[:, None, :] + pts[None]) * g.h
    NE, Q = X.shape[:2]
    chi = np.broadcast_to(g.chi[:, None], (NE, Q)).reshape(-1)
    u = prob.exact.velocity(X.reshape(-1, d), chi).reshape(NE, Q, d)
    pr = prob.exact.pressure(X.reshape(-1, d), chi).reshape(NE, Q)
    vals = np.concatenate([u, pr[..., None]], axis=2)            # (NE, Q, d+1)
    coef = np.einsum("qa,q,eqf->efa", B, w * g.h ** d, vals)
    return coef.ravel(), g


def _solve(prob, tol=1e-12):
    H = build_hierarchy(prob)
    b = assemble_rhs(prob, H.fine.ops)
    S = Solver(H)
    x, hist = S.fgmres(b, tol=tol, m=40, maxit=200)
    assert hist[-1] <= tol * 10, hist[-1]
    return H, x


def _orders(mk, ns):
    errs = []
    for n in ns:
        prob = mk(n)
        H, x = _solve(prob)
        errs.append(solution_errors(prob, H.project_kernel(x), H.k0))
    return {k: math.log2(errs[0][k] / errs[1][k]) for k in errs[0]}


def _check_orders(o, case, p):
    for q, off in _golden_orders(case).items():
        assert o[q] >= p + off - 0.3, (case, q, o[q])


# ---------------------------------------------------------- error measure --
@pytest.mark.parametrize("mk,k0", [(lambda n: c4a_square_inclusion(n=n, p=2), 1),
                                   (lambda n: c1_periodic_standard(n=n, p=2), 3)])
def test_error_measure_removes_kernel_constants(mk, k0):
    """Adding kernel modes (constant pressure; constant velocities on the
    periodic grid) to a coefficient vector leaves the measured error
    unchanged, and the L2 projection of the exact solution has errors of
    order p+1 (the two-phase exact pressure has a non-zero mean, so a wrong
    normalisation of the constant shows)."""
    errs = []
    for n in (8, 16):
        prob = mk(n)
        x, g = _l2_projection(prob)
        e0 = solution_errors(prob, x, k0)
        y = x.reshape(g.NE, prob.dim + 1, g.nq).copy()
        fields = [prob.dim] if k0 == 1 else list(range(prob.dim + 1))
        for f in fields:
            y[:, f, 0] += 3.7 * g.h ** (prob.dim / 2)       # the constant 3.7 in the orthonormal basis
        e1 = solution_errors(prob, y.ravel(), k0)
        for k in e0:
            assert abs(e1[k] - e0[k]) <= 1e-9 * max(e0[k], 1e-30) + 1e-12, k
        errs.append(e0)
    for k in ("u_l2", "p_l2"):
        assert math.log2(errs[0][k] / errs[1][k]) >= 3 - 0.3, (k, errs)


# ---------------------------------------------------------------- phases --
def test_two_phase_square_orders():
    """Section 5.6 / grid-convergence appendix: velocity order p+1 (max
    norm), pressure p+1/2 in L2 and p in the max norm, viscosity 1e4 inside
    the square (1/4, 3/4)^2 and 1 outside, Dirichlet walls."""
    o = _orders(lambda n: c4a_square_inclusion(n=n, p=2), [16, 32])
    _check_orders(o, "two_phase_square", 2)


def _square(mu_in, bc):
    ph = PhaseField(values=(mu_in, 1.0))
    return Problem(name="sq", dim=2, n=16, p=2, gamma=1, bc=(bc, bc), mu=ph, phases=ph,
                   coloring="mod3" if bc == "dirichlet" else "auto", diag_scaling=True)


@pytest.mark.parametrize("mu_in,bc", [(1e-3, "periodic"), (1e3, "periodic"), (1e4, "dirichlet")])
def test_square_inclusion_gmres_iterations_in_paper_band(mu_in, bc):
    """Section 5.6: with viscosity-upwinded fluxes and the diagonal scaling,
    7-10 iterations of V-cycle-preconditioned GMRES reduce the residual by
    1e8 across the viscosity ratios (eq. rho metric, V(3,3))."""
    rho, its = Solver(build_hierarchy(_square(mu_in, bc))).rho_metric()
    assert its <= 10, (rho, its)


def test_planted_flipped_lambda_leaves_the_band(monkeypatch):
    """Planted mistake: lambda of eq. (viscosityupwind) flipped (u-hat biased
    to the less viscous phase).  The band above must catch it."""
    import oracle.assemble as A
    monkeypatch.setattr(A, "_lam", lambda mm, mp: np.where(mm < mp, 1.0, np.where(mm > mp, 0.0, 0.5)))
    rho, its = Solver(build_hierarchy(_square(1e3, "periodic"))).rho_metric()
    assert its > 10, (rho, its)


def test_p12_scaling_leaves_iterates_unchanged():
    """For a viscosity constant on every element of every level (phases
    aligned with the coarsest grid), the scaled and unscaled V-cycles give
    the same iterates up to rounding."""
    p1 = c4a_square_inclusion(n=16, p=2)
    p0 = dataclasses.replace(p1, diag_scaling=False)
    H1, H0 = build_hierarchy(p1), build_hierarchy(p0)
    S1, S0 = Solver(H1), Solver(H0)
    b = H1.project_kernel(assemble_rhs(p1, H1.fine.ops))
    x1 = x0 = None
    for k in range(6):
        x1, x0 = S1.vcycle_unscaled(b, x1), S0.vcycle_unscaled(b, x0)
        assert np.linalg.norm(x1 - x0) <= 1e-10 * np.linalg.norm(x0), k
    assert S0.relres(b, x0) < 1e-5


def test_p12_planted_inconsistent_coarse_scaling_changes_iterates():
    """Planted mistake: the first coarse level scaled by a viscosity other
    than its own (a further element-wise congruence S A S).  Its smoother is
    invariant under that, its coarse-grid correction is not, so the pin
    above must see different iterates."""
    from oracle.hierarchy import diagonal_blocks, equilibrated_inverse
    import scipy.sparse as sp
    p1 = c4a_square_inclusion(n=16, p=2)
    p0 = dataclasses.replace(p1, diag_scaling=False)
    H1, H0 = build_hierarchy(p1), build_hierarchy(p0)
    lv = H1.levels[1]
    rng = np.random.default_rng(3)
    s = np.repeat(np.exp(rng.uniform(-1.0, 1.0, lv.NE)), lv.nb)
    lv.A = (sp.diags(s) @ lv.A @ sp.diags(s)).tocsr()
    lv.Ainv = equilibrated_inverse(diagonal_blocks(lv.A, lv.nb))
    S1, S0 = Solver(H1), Solver(H0)
    b = H1.project_kernel(assemble_rhs(p1, H1.fine.ops))
    x1, x0 = S1.vcycle_unscaled(b), S0.vcycle_unscaled(b)
    assert np.linalg.norm(x1 - x0) > 1e-6 * np.linalg.norm(x0)


# ------------------------------------------------------------ divergence --
def test_s23_constraint_row_and_discrete_divergence():
    """eq. (appstokes2): -sum_i G_i u_i - E p = b_p.  The converged solution
    satisfies the constraint row, b_p is orthogonal to the constant pressure,
    and for the divergence-free exact velocity of the periodic standard-form
    problem sum_i G_i u_i tends to zero under refinement (here at order > p:
    it equals -E p - b_p with b_p = 0 and tau_p [p] small)."""
    norms = []
    for n in (8, 16):
        prob = c1_periodic_standard(n=n, p=2)
        H = build_hierarchy(prob)
        b = assemble_rhs(prob, H.fine.ops)
        S = Solver(H)
        x, hist = S.stationary(b, 60, tol=1e-13)
        d, nq = prob.dim, H.fine.nq
        X, Bv = x.reshape(-1, d + 1, nq), b.reshape(-1, d + 1, nq)
        r = (b - S.A @ x).reshape(-1, d + 1, nq)
        assert np.linalg.norm(r[:, d]) <= 1e-12 * np.linalg.norm(b)
        assert abs(Bv[:, d, 0].sum()) <= 1e-12 * max(np.linalg.norm(Bv[:, d]), np.linalg.norm(b))
        G = H.fine.ops["G"]
        norms.append(np.linalg.norm(sum(G[i] @ X[:, i, :].ravel() for i in range(d))))
    assert norms[0] / norms[1] >= 2 ** prob.p, norms
    # compatibility of the constraint data with a non-zero b_p (Dirichlet
    # walls): the boundary flux of g balances the integral of f_div
    prob = c2_dirichlet_varmu(n=8, p=2)
    H = build_hierarchy(prob)
    Bv = assemble_rhs(prob, H.fine.ops).reshape(-1, prob.dim + 1, H.fine.nq)
    assert abs(Bv[:, prob.dim, 0].sum()) <= 1e-10 * np.linalg.norm(Bv[:, prob.dim])


# -------------------------------------------------------------- unsteady --
def _unsteady(n, bc, p=2):
    h = 1.0 / n
    mu = ConstField(1e-4)
    delta = 0.1 * h
    ex = make_exact_paper(2, 0, mu)
    ex.rho_delta = 1.0 / delta
    return Problem(name="u", dim=2, n=n, p=p, gamma=0, bc=(bc, bc), mu=mu, rho=ConstField(1.0),
                   delta=delta, exact=ex)


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_unsteady_high_reynolds_orders(bc):
    """Section 6.1: rho = 1, mu = 1e-4, delta = 0.1 h (Re ~ 1e4): velocity and
    pressure both of order p+1 (the mass term (rho / delta) M_rho and the
    pressure penalty of eq. taugeneral enter every row)."""
    o = _orders(lambda n: _unsteady(n, bc), [8, 16])
    _check_orders(o, "unsteady_re1e4", 2)


def test_planted_wrong_power_of_delta_spoils_unsteady_orders(monkeypatch):
    """Planted mistake: M_rho / delta^2 in place of M_rho / delta."""
    import oracle.hierarchy as Hm
    orig = Hm.stokes_system

    def bad(ops, dim, gamma, nq, delta=None):
        return orig(ops, dim, gamma, nq, None if delta is None else delta * delta)
    monkeypatch.setattr(Hm, "stokes_system", bad)
    errs = []
    for n in (8, 16):
        prob = _unsteady(n, "periodic")
        H = build_hierarchy(prob)
        b = assemble_rhs(prob, H.fine.ops)
        x, _ = Solver(H).fgmres(b, tol=1e-12, m=40, maxit=200)
        errs.append(solution_errors(prob, H.project_kernel(x), H.k0))
    assert math.log2(errs[0]["u_l2"] / errs[1]["u_l2"]) < 3 - 0.3 or errs[1]["u_l2"] > 1e-2


# -------------------------------------------------------------------- 3D --
@pytest.mark.slow
def test_dirichlet_3d_variable_viscosity_orders():
    """3D viscous-stress form, velocity Dirichlet walls, the viscosity of
    eq. (mu): velocity order p+1, pressure p+1/2 in L2, p in the max norm."""
    mu = SinProductField(1.0, 0.5, 2.0)
    o = _orders(lambda n: Problem(name="d3", dim=3, n=n, p=2, gamma=1, bc=("dirichlet",) * 3, mu=mu,
                                  exact=make_exact_paper(3, 1, mu)), [4, 8])
    _check_orders(o, "dirichlet_3d", 2)
