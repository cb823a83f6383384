"""Stress boundary conditions (eq. govern3 on every wall, viscous-stress form;
sections 5.3 and 5.4) in the oracle, pinned to facts outside it:

* the trivial kernel is the rigid motions of the velocity (the bottom-solver
  footnote): d translations and d(d-1)/2 rotations, annihilated to rounding;
  a constant pressure is not in it (the walls fix the pressure);
* the operator stays symmetric;
* the manufactured right-hand side is orthogonal to the kernel (the
  grid-convergence appendix notes this holds for manufactured solutions);
* orders under refinement: velocity p+1 in L2 and in the maximum norm,
  pressure p+1/2 in L2 (section 5.3);
* planted mistakes fail: the Dirichlet lift applied on the stress walls
  (the rotations leave the kernel), and the stress data J_h dropped (the
  velocity error stops converging).
"""
import numpy as np
import pytest

from synth import stress_walls, SinProductField


def _solve(prob):
    from oracle import build_hierarchy
    from oracle.rhs import assemble_rhs
    from oracle.solvers import Solver
    H = build_hierarchy(prob)
    S = Solver(H)
    b = H.project_kernel(assemble_rhs(prob, H.fine.ops))
    x, hist = S.fgmres(b, tol=1e-12, m=100, maxit=300)
    assert hist[-1] <= 1e-12
    return H, S, x


@pytest.mark.parametrize("dim,n,p", [(2, 8, 2), (3, 4, 2)])
def test_stress_kernel_is_the_rigid_motions(dim, n, p):
    from oracle import build_hierarchy
    from oracle.rhs import assemble_rhs
    from oracle.solvers import Solver
    prob = stress_walls(dim=dim, n=n, p=p)
    H = build_hierarchy(prob)
    A = Solver(H).A
    K = H.kernel_basis()
    assert K.shape[1] == H.k0 == dim + dim * (dim - 1) // 2
    scale = abs(A).max()
    assert np.abs(A @ K).max() <= 1e-13 * scale
    assert abs(A - A.T).max() <= 1e-13 * scale
    pc = np.zeros(A.shape[0])
    pc[np.arange(H.fine.NE) * H.fine.nb + dim * H.fine.nq] = 1.0
    assert np.abs(A @ pc).max() > 1e-4 * scale
    b = assemble_rhs(prob, H.fine.ops)
    assert np.abs(K.T @ b).max() <= 1e-12 * np.abs(b).max()


def _orders(probs):
    from oracle.errors import solution_errors
    errs = []
    for prob in probs:
        H, S, x = _solve(prob)
        errs.append(solution_errors(prob, H.project_kernel(x), H.k0))
    return [{k: np.log2(a[k] / c[k]) for k in a} for a, c in zip(errs, errs[1:])], errs


def test_stress_orders_2d():
    orders, errs = _orders([stress_walls(dim=2, n=n, p=2) for n in (8, 16, 32)])
    print(errs, orders)
    for o in orders:
        assert o["u_l2"] >= 2.8 and o["u_max"] >= 2.8        # p + 1 = 3
    assert orders[-1]["p_l2"] >= 2.0                          # p + 1/2 = 2.5 (approached from below)


def test_stress_orders_variable_viscosity_2d():
    """Section 5.4: eq. (mu) with stress walls, same orders."""
    mu = SinProductField(1.0, 0.5, 2.0)
    orders, errs = _orders([stress_walls(dim=2, n=n, p=2, mu=mu) for n in (8, 16, 32)])
    print(errs, orders)
    for o in orders:
        assert o["u_l2"] >= 2.7
    assert orders[-1]["p_l2"] >= 1.9


def test_planted_dirichlet_lift_on_stress_walls_breaks_the_kernel(monkeypatch):
    from oracle import assemble
    from oracle import build_hierarchy
    from oracle.solvers import Solver
    orig = assemble.FineAssembly.face_data

    def as_dirichlet(self, axis):
        fd = orig(self, axis)
        fd["type"] = np.where(fd["type"] == 3, 2, fd["type"])
        return fd

    monkeypatch.setattr(assemble.FineAssembly, "face_data", as_dirichlet)
    prob = stress_walls(dim=2, n=8, p=2)
    H = build_hierarchy(prob)
    A = Solver(H).A
    assert np.abs(A @ H.kernel_basis()).max() > 1e-3 * abs(A).max()


def test_planted_missing_stress_data_stops_convergence(monkeypatch):
    from synth.fields import ExactSolution
    from oracle.errors import solution_errors
    monkeypatch.setattr(ExactSolution, "stress", lambda self, x, chi=None: np.zeros((x.shape[0], self.dim, self.dim)))
    errs = []
    for n in (8, 16):
        prob = stress_walls(dim=2, n=n, p=2)
        H, S, x = _solve(prob)
        errs.append(solution_errors(prob, H.project_kernel(x), H.k0)["u_l2"])
    assert errs[1] > 0.5 * errs[0]
