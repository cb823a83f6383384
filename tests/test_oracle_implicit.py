"""The oracle on implicitly defined meshes (a circle cutting a Cartesian
grid; section 5 "Curved domain geometry", section 5.6, appendix A), pinned
to facts outside it:

* quadrature: the disk's area, perimeter and second moment in closed form,
  and the divergence theorem on every cut piece (volume rule, interface rule
  with its weights and normals, and the edge rules must agree);
* the mesh: every element holds at least a quarter of a cell, each phase's
  total area is the disk's (or its complement's);
* with the interface outside the square the operators reduce to those of
  the Cartesian assembly (a separately pinned code path);
* the operator is symmetric, the mass matrix the identity, the constant
  pressure in its kernel (to quadrature accuracy);
* the injection reproduces coarse polynomials on fine elements exactly and
  its transpose is a left inverse (L2 projection);
* orders under refinement for the paper's two-phase manufactured solution
  with viscosity ratio 1e4: velocity p + 1, pressure about p + 1/2 in L2;
* the V-cycle contracts at a Cartesian-like rate;
* planted mistakes (interface normals reversed, the interface weight
  factor |grad phi| / |d_k phi| dropped) fail the pins above.
"""
import numpy as np
import pytest

from synth import c4_circle, CirclePhaseField
from oracle.implicit_quad import cut_box_rules, segment_rules


def _cut_cells(ls, n):
    h = 1.0 / n
    for i1 in range(n):
        for i0 in range(n):
            lo = np.array([i0, i1]) * h
            mn, mx = ls.box_range(lo, lo + h)
            yield lo, lo + h, mn < 0.0 < mx, mx <= 0.0


@pytest.mark.parametrize("n", [8, 16])
def test_disk_area_perimeter_moment(n):
    ls = CirclePhaseField()
    r = ls.radius
    area = per = mom = 0.0
    h = 1.0 / n
    for lo, hi, cut, inside in _cut_cells(ls, n):
        if cut:
            q = cut_box_rules(ls, lo, hi, 8)
            X, w = q["vol"][1]
            area += w.sum()
            mom += (w * (X[:, 0] - 0.5) ** 2).sum()
            per += q["surf"][1].sum()
        elif inside:
            area += h * h
            mom += h * ((hi[0] - 0.5) ** 3 - (lo[0] - 0.5) ** 3) / 3.0
    tol = 1e-10 if n == 8 else 1e-13
    assert abs(area - np.pi * r * r) <= tol
    assert abs(per - 2 * np.pi * r) <= 10 * tol
    assert abs(mom - np.pi * r ** 4 / 4) <= tol


def _field():
    def F(X):
        x, y = X[:, 0], X[:, 1]
        return np.stack([x ** 3 * y + 2 * y ** 2, x * y ** 3 - x ** 2], axis=1)

    def dF(X):
        x, y = X[:, 0], X[:, 1]
        out = np.zeros((X.shape[0], 2, 2))
        out[:, 0, 0] = 3 * x ** 2 * y
        out[:, 0, 1] = x ** 3 + 4 * y
        out[:, 1, 0] = y ** 3 - 2 * x
        out[:, 1, 1] = 3 * x * y ** 2
        return out
    return F, dF


def test_divergence_theorem_on_every_cut_piece():
    ls = CirclePhaseField()
    F, dF = _field()
    worst = 0.0
    for lo, hi, cut, _ in _cut_cells(ls, 16):
        if cut:
            worst = max(worst, abs(_defect_with(cut_box_rules, ls, lo, hi, F, dF)))
    assert worst <= 1e-14


def test_planted_weight_factor_dropped_fails_divergence(monkeypatch):
    from oracle import implicit_quad as iq
    orig = iq.cut_box_rules

    def no_factor(ls, lo, hi, q):
        r = orig(ls, lo, hi, q)
        S, sw, sn = r["surf"]
        k = np.argmax(np.abs(sn), axis=1)
        r["surf"] = (S, sw * np.abs(sn[np.arange(sn.shape[0]), k]), sn)
        return r

    monkeypatch.setattr(iq, "cut_box_rules", no_factor)
    ls = CirclePhaseField()
    F, dF = _field()
    worst = 0.0
    for lo, hi, cut, _ in _cut_cells(ls, 16):
        if cut:
            worst = max(worst, abs(_defect_with(iq.cut_box_rules, ls, lo, hi, F, dF)))
    assert worst > 1e-6


def _defect_with(rulefn, ls, lo, hi, F, dF):
    """int_piece div F - int_boundary F . n for the phase-1 piece of a box, F
    a polynomial vector field (boundary: the interface inside the box and the
    box edges where phi < 0)."""
    rules = rulefn(ls, lo, hi, 8)
    X, w = rules["vol"][1]
    vol = (w * (dF(X)[:, 0, 0] + dF(X)[:, 1, 1])).sum()
    S, sw, sn = rules["surf"]
    bnd = (sw * (F(S) * sn).sum(axis=1)).sum()
    for axis in (0, 1):
        for val, sgn in ((lo[axis], -1.0), (hi[axis], 1.0)):
            Y, wy = segment_rules(ls, axis, val, lo[1 - axis], hi[1 - axis], 8)[1]
            if wy.size:
                bnd += sgn * (wy * F(Y)[:, axis]).sum()
    return vol - bnd


@pytest.fixture(scope="module")
def c16():
    from oracle.implicit_assemble import implicit_fine_operators
    prob = c4_circle(n=16, p=2, rhs="exact")
    return prob, implicit_fine_operators(prob)


def test_mesh_fractions_and_areas(c16):
    prob, ops = c16
    mesh = ops["mesh"]
    h = mesh.h
    r = prob.phases.radius
    areas = np.array([e.area for e in mesh.elements])
    assert areas.min() >= 0.25 * h * h
    chi = mesh.chi()
    assert abs(areas[chi == 1].sum() - np.pi * r * r) <= 1e-13
    assert abs(areas[chi == 2].sum() - (1 - np.pi * r * r)) <= 1e-13
    assert len(mesh.merged) > 0                       # the pin exercises merging
    assert all(mesh.elem_of[k] is not None for k in mesh.pieces)


def test_operator_symmetric_mass_identity_kernel(c16):
    from oracle.assemble import stokes_system
    prob, ops = c16
    mesh = ops["mesh"]
    assert abs(ops["M"] - np.eye(ops["M"].shape[0])).max() <= 1e-10
    A = stokes_system(ops, 2, 1, mesh.nq)
    scale = abs(A).max()
    assert abs(A - A.T).max() <= 1e-15 * scale
    K = np.zeros(A.shape[0])
    K[np.arange(mesh.NE) * 27 + 18] = np.sqrt([e.area for e in mesh.elements])
    assert np.abs(A @ K).max() <= 1e-18 * scale


def test_planted_reversed_interface_normal_breaks_kernel(monkeypatch):
    from oracle import implicit_mesh as im
    from oracle.implicit_assemble import implicit_fine_operators
    from oracle.assemble import stokes_system
    orig = im.ImplicitMesh._faces

    def flipped(self):
        faces = orig(self)
        for f in faces:
            if f.kind == 1:
                f.normal = -f.normal
        return faces

    monkeypatch.setattr(im.ImplicitMesh, "_faces", flipped)
    prob = c4_circle(n=8, p=2, rhs="exact")
    ops = implicit_fine_operators(prob)
    mesh = ops["mesh"]
    A = stokes_system(ops, 2, 1, mesh.nq)
    K = np.zeros(A.shape[0])
    K[np.arange(mesh.NE) * 27 + 18] = np.sqrt([e.area for e in mesh.elements])
    assert np.abs(A @ K).max() > 1e-12 * abs(A).max()          # unplanted: <= 1e-18


def test_reduces_to_cartesian_without_interface():
    from synth.problems import Problem
    from synth.fields import SinProductField, make_exact_paper
    from oracle.implicit_assemble import implicit_fine_operators
    from oracle.assemble import fine_operators
    mu = SinProductField(1.0, 0.9, 1.0)
    far = CirclePhaseField(values=(1.0, 1.0), centre=(5.0, 5.0), radius=0.3)
    kw = dict(dim=2, n=8, p=2, gamma=1, bc=("dirichlet", "dirichlet"), mu=mu, exact=make_exact_paper(2, 1, mu))
    oi = implicit_fine_operators(Problem(name="i", phases=far, coloring="greedy", **kw))
    oc = fine_operators(Problem(name="c", coloring="parity", **kw))
    for key in ("M", "Mmu", "Et", "E"):
        assert abs(oi[key] - oc[key]).max() <= 1e-12 * max(1.0, abs(oc[key]).max())
    for k in range(2):
        assert abs(oi["G"][k] - oc["G"][k]).max() <= 1e-12 * abs(oc["G"][k]).max()


def test_injection_exact_and_projection(c16):
    from oracle.implicit_mesh import coarsen_mesh, prolongation
    prob, ops = c16
    mesh = ops["mesh"]
    cm, parent = coarsen_mesh(mesh)
    I = prolongation(mesh, cm, parent).toarray()
    nq = mesh.nq
    # (rounding amplified by the conditioning of a coarse basis orthonormalised
    # over a single small child: about 1e-10)
    assert abs(I.T @ I - np.eye(I.shape[1])).max() <= 1e-9
    rng = np.random.default_rng(3)
    for f in rng.choice(mesh.NE, 12, replace=False):
        e = mesh.elements[f]
        c = parent[f]
        Bc = cm.basis(c, e.X)
        Bf = mesh.basis(f, e.X)
        blk = I[f * nq:(f + 1) * nq, c * nq:(c + 1) * nq]
        assert abs(Bf @ blk - Bc).max() <= 1e-10 * abs(Bc).max()


def test_orders_two_phase_circle():
    """Section 5.6 / grid-convergence appendix: velocity order p + 1 in L2 and
    (about) in the maximum norm, pressure p + 1/2 in L2, viscosity ratio 1e4."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    from oracle.implicit_assemble import implicit_fine_operators, implicit_rhs, implicit_solution_errors
    from oracle.assemble import stokes_system
    errs = []
    for n in (8, 16, 32):
        prob = c4_circle(n=n, p=2, rhs="exact")
        ops = implicit_fine_operators(prob)
        mesh = ops["mesh"]
        A = stokes_system(ops, 2, 1, mesh.nq)
        b = implicit_rhs(prob, ops)
        K = np.zeros(A.shape[0])
        K[np.arange(mesh.NE) * 27 + 18] = np.sqrt([e.area for e in mesh.elements])
        K /= np.linalg.norm(K)
        assert abs(K @ b) <= 1e-10 * np.abs(b).max()
        Ab = sp.bmat([[A, sp.csr_matrix(K[:, None])], [sp.csr_matrix(K[None, :]), None]]).tocsc()
        x = spl.spsolve(Ab, np.concatenate([b, [0.0]]))[:-1]
        errs.append(implicit_solution_errors(prob, mesh, x))
    o = [{k: np.log2(a[k] / c[k]) for k in a} for a, c in zip(errs, errs[1:])]
    print(errs, o)
    for oo in o:
        assert oo["u_l2"] >= 2.9
        assert oo["u_max"] >= 2.5
    assert o[-1]["p_l2"] >= 2.4


def test_vcycle_contracts_on_implicit_mesh():
    from oracle.implicit_assemble import build_implicit_hierarchy, implicit_rhs
    from oracle.solvers import Solver
    prob = c4_circle(n=16, p=2, rhs="bubble")
    H = build_implicit_hierarchy(prob)
    for lv in H.levels[:-1]:
        # greedy colours are proper: no block couples two elements of one colour
        Ab = lv.A.tobsr(blocksize=(lv.nb, lv.nb))
        for r in range(lv.NE):
            for k in range(Ab.indptr[r], Ab.indptr[r + 1]):
                c = Ab.indices[k]
                if c != r and np.any(Ab.data[k]):
                    assert lv.colours[c] != lv.colours[r]
    S = Solver(H)
    b = implicit_rhs(prob, H.fine.ops)
    x, hist = S.stationary(b, maxit=12)
    rates = hist[1:] / hist[:-1]
    assert rates.max() < 0.4
    x, h2 = S.fgmres(b, tol=1e-10, m=40, maxit=60)
    assert h2[-1] <= 1e-10 and len(h2) - 1 <= 14


@pytest.mark.parametrize("water", [True, False])
def test_bubble_orders_and_rate(water):
    """Section 6, multi-phase time-dependent test: water (gas) bubble in gas
    (water), rho 1 / 0.001, mu 1 / 0.0002, delta = 0.1 h.  The paper states
    velocity order p + 1 in the maximum norm and pressure p + 1/2 in L2; the
    manufactured solution carries rho / delta u in its forcing per phase.
    The V-cycle contracts."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    from synth import bubble_unsteady
    from oracle.implicit_assemble import (implicit_fine_operators, implicit_rhs, implicit_solution_errors,
                                          build_implicit_hierarchy)
    from oracle.assemble import stokes_system
    from oracle.solvers import Solver
    errs = []
    for n in (8, 16, 32):
        prob = bubble_unsteady(n=n, p=2, water_inside=water)
        ops = implicit_fine_operators(prob)
        mesh = ops["mesh"]
        A = stokes_system(ops, 2, 1, mesh.nq, prob.delta)
        b = implicit_rhs(prob, ops)
        K = np.zeros(A.shape[0])
        K[np.arange(mesh.NE) * 27 + 18] = np.sqrt([e.area for e in mesh.elements])
        K /= np.linalg.norm(K)
        assert np.abs(A @ K).max() <= 1e-12 * abs(A).max()
        Ab = sp.bmat([[A, sp.csr_matrix(K[:, None])], [sp.csr_matrix(K[None, :]), None]]).tocsc()
        x = spl.spsolve(Ab, np.concatenate([b, [0.0]]))[:-1]
        errs.append(implicit_solution_errors(prob, mesh, x))
    o = [{k: np.log2(a[k] / c[k]) for k in a} for a, c in zip(errs, errs[1:])]
    print(errs, o)
    for oo in o:
        assert oo["u_l2"] >= 2.9 and oo["u_max"] >= 2.6
    assert o[-1]["p_l2"] >= 2.4
    H = build_implicit_hierarchy(bubble_unsteady(n=16, p=2, water_inside=water))
    S = Solver(H)
    bb = H.project_kernel(np.random.default_rng(2).standard_normal(H.fine.A.shape[0]))
    x, hist = S.stationary(bb, maxit=10)
    assert (hist[3:] / hist[2:-1]).max() < 0.4


def test_disk_domain_orders_and_rate():
    """Section 5, curved domain: Stokes in standard form on the unit-diameter
    disk, velocity Dirichlet data on the circle (the interface of the
    implicit mesh becomes the domain's wall).  The disk's area is exact, the
    constant pressure is in the kernel, velocity order p + 1 (L2), pressure
    about p + 1/2 (L2); the V-cycle contracts (the paper: efficient rates)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    from synth import disk_domain
    from oracle.implicit_assemble import (implicit_fine_operators, implicit_rhs, implicit_solution_errors,
                                          build_implicit_hierarchy)
    from oracle.assemble import stokes_system
    from oracle.solvers import Solver
    errs = []
    for n in (8, 16, 32):
        prob = disk_domain(n=n, p=2)
        ops = implicit_fine_operators(prob)
        mesh = ops["mesh"]
        assert abs(sum(e.area for e in mesh.elements) - np.pi / 4) <= 1e-13
        assert all(f.kind in (0, 2) for f in mesh.faces)
        A = stokes_system(ops, 2, 0, mesh.nq)
        b = implicit_rhs(prob, ops)
        K = np.zeros(A.shape[0])
        K[np.arange(mesh.NE) * 27 + 18] = np.sqrt([e.area for e in mesh.elements])
        K /= np.linalg.norm(K)
        assert np.abs(A @ K).max() <= 1e-15 * abs(A).max()
        Ab = sp.bmat([[A, sp.csr_matrix(K[:, None])], [sp.csr_matrix(K[None, :]), None]]).tocsc()
        x = spl.spsolve(Ab, np.concatenate([b, [0.0]]))[:-1]
        errs.append(implicit_solution_errors(prob, mesh, x))
    o = [{k: np.log2(a[k] / c[k]) for k in a} for a, c in zip(errs, errs[1:])]
    print(errs, o)
    for oo in o:
        assert oo["u_l2"] >= 2.9 and oo["u_max"] >= 2.6
        assert oo["p_l2"] >= 2.2
    H = build_implicit_hierarchy(disk_domain(n=32, p=2))
    S = Solver(H)
    bb = H.project_kernel(np.random.default_rng(3).standard_normal(H.fine.A.shape[0]))
    x, hist = S.stationary(bb, maxit=10)
    assert (hist[3:] / hist[2:-1]).max() < 0.2
