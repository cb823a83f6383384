"""Pins of the oracle's learned correction (network, BF16 rounding, Adam and
the guarded refinement) against facts that do not come from the oracle:
exactly representable bfloat16 rounding cases, central differences of the
loss, a pure-Python patch convolution on a tiny grid, translation
equivariance on a periodic grid, positive homogeneity of the correction,
properties of Adam's first step, the zero-output network reproducing the
plain iteration exactly, and the guard switching a harmful correction off."""
import numpy as np
import pytest

from synth import c1_periodic_standard, c2_dirichlet_varmu
from oracle import build_hierarchy
from oracle.solvers import Solver
from oracle import learned as L


# ------------------------------------------------------------ bf16 -------
def test_bf16_rounding_cases():
    u = 2.0 ** -7                                     # spacing of bfloat16 in [1, 2)
    cases = [
        (1.0, 1.0),
        (1.0 + u / 2, 1.0),                           # tie, even neighbour below
        (1.0 + 1.5 * u, 1.0 + 2 * u),                 # tie, even neighbour above
        (1.0 + u / 2 + 2.0 ** -20, 1.0 + u),          # just above the tie
        (1.0 + u / 2 - 2.0 ** -20, 1.0),              # just below the tie
        (-(1.0 + 1.5 * u), -(1.0 + 2 * u)),
        (3.0 * 2.0 ** -130, 3.0 * 2.0 ** -130),       # subnormal with few bits
        (0.0, 0.0),
    ]
    x = np.array([c[0] for c in cases], dtype=np.float32)
    want = np.array([c[1] for c in cases], dtype=np.float32)
    assert np.array_equal(L.bf16(x), want)
    assert np.isnan(L.bf16(np.array([np.nan], dtype=np.float32)))[0]
    # every output has its low 16 bits clear
    r = L.bf16(np.random.default_rng(0).standard_normal(1000).astype(np.float32))
    assert not np.any(r.view(np.uint32) & 0xFFFF)


# ------------------------------------------------------- gradients -------
def test_p13_central_differences_match_backward():
    rng = np.random.default_rng(3)
    d, nb, H, N = 2, 12, 8, 40
    params = L.init_params(d, nb, H, seed=1)
    for k in ("b1", "b2", "b3"):
        params[k] = 0.1 * rng.standard_normal(params[k].shape)
    X = rng.standard_normal((N, 9 * (nb + 1)))
    T = rng.standard_normal((N, nb))
    _, g = L.loss_and_grad(params, X, T)
    h = 1e-6
    for name in params:
        flat = params[name].ravel()
        for idx in rng.choice(flat.size, size=min(flat.size, 12), replace=False):
            p_plus = {k: v.copy() for k, v in params.items()}
            p_minus = {k: v.copy() for k, v in params.items()}
            p_plus[name].ravel()[idx] += h
            p_minus[name].ravel()[idx] -= h
            fd = (L.loss_and_grad(p_plus, X, T)[0] - L.loss_and_grad(p_minus, X, T)[0]) / (2 * h)
            an = g[name].ravel()[idx]
            assert abs(fd - an) <= 1e-6 * max(abs(an), np.abs(g[name]).max()), (name, idx)


def test_bf16_emulated_gradients_close_to_fp64():
    rng = np.random.default_rng(4)
    params = L.init_params(2, 12, 16, seed=2)
    X = rng.standard_normal((200, 9 * 13))
    T = rng.standard_normal((200, 12))
    _, g64 = L.loss_and_grad(params, X, T)
    _, g16 = L.loss_and_grad(params, X, T, emulate_bf16=True)
    # a handful of first-layer ReLU decisions flip under BF16 rounding, so the
    # first-layer weight gradient differs most
    for k in g64:
        a, b = g64[k].ravel(), np.asarray(g16[k], dtype=np.float64).ravel()
        assert np.linalg.norm(a - b) <= 0.1 * np.linalg.norm(a), k
        assert a @ b >= 0.995 * np.linalg.norm(a) * np.linalg.norm(b), k


# ---------------------------------------------------------- patches ------
@pytest.mark.parametrize("periodic", [(True, True), (False, False), (True, False)])
def test_patch_convolution_matches_explicit_loops(periodic):
    """First-layer pre-activations from explicit coordinate loops."""
    rng = np.random.default_rng(5)
    n0, n1, C, H = 4, 3, 5, 3
    Z = rng.standard_normal((n0 * n1, C))
    W = rng.standard_normal((H, 9 * C))
    X = L.patches(Z, (n0, n1), periodic)
    got = X @ W.T
    for j in range(n1):
        for i in range(n0):
            acc = np.zeros(H)
            for oj in (-1, 0, 1):
                for oi in (-1, 0, 1):
                    slot = (oi + 1) + 3 * (oj + 1)
                    ii, jj = i + oi, j + oj
                    if periodic[0]:
                        ii %= n0
                    if periodic[1]:
                        jj %= n1
                    if not (0 <= ii < n0 and 0 <= jj < n1):
                        continue
                    for c in range(C):
                        acc += W[:, slot * C + c] * Z[jj * n0 + ii, c]
            assert np.allclose(got[j * n0 + i], acc, atol=1e-12)


def _grid_and_net(prob, H=8, seed=0):
    hier = build_hierarchy(prob)
    g = L.grid_of(hier)
    params = L.init_params(prob.dim, g.nb, H, seed)
    rng = np.random.default_rng(seed + 10)
    for k in ("b1", "b2", "b3"):
        params[k] = 0.1 * rng.standard_normal(params[k].shape)
    return hier, g, params


def test_correction_is_translation_equivariant_on_periodic_grids():
    prob = c1_periodic_standard(n=8, p=1)
    hier, g, params = _grid_and_net(prob)
    rng = np.random.default_rng(7)
    r = rng.standard_normal(hier.fine.NE * g.nb)
    dx = L.correction(params, (0.5, 2.0), g, r).reshape(g.n, g.n, g.nb)
    rs = np.roll(r.reshape(g.n, g.n, g.nb), 3, axis=1).ravel()      # shift along axis 0
    dxs = L.correction(params, (0.5, 2.0), g, rs).reshape(g.n, g.n, g.nb)
    assert np.allclose(np.roll(dx, 3, axis=1), dxs, atol=1e-13)


@pytest.mark.parametrize("emulate", [False, True])
def test_correction_is_positively_homogeneous(emulate):
    prob = c2_dirichlet_varmu(n=8, p=1)
    hier, g, params = _grid_and_net(prob)
    r = np.random.default_rng(8).standard_normal(hier.fine.NE * g.nb)
    a = L.correction(params, (0.3, 1.7), g, r, emulate)
    b = L.correction(params, (0.3, 1.7), g, 4.0 * r, emulate)
    assert np.allclose(4.0 * a, b, rtol=1e-12, atol=0)


def test_bf16_correction_close_to_fp64():
    prob = c2_dirichlet_varmu(n=8, p=2)
    hier, g, params = _grid_and_net(prob, H=16)
    r = np.random.default_rng(9).standard_normal(hier.fine.NE * g.nb)
    a = L.correction(params, (0.3, 1.7), g, r)
    b = L.correction(params, (0.3, 1.7), g, r, True)
    assert np.linalg.norm(a - b) <= 2e-2 * np.linalg.norm(a)


# ------------------------------------------------------------- Adam -------
def test_adam_first_step_moves_each_weight_by_lr_against_the_gradient():
    rng = np.random.default_rng(11)
    p0 = {"w": rng.standard_normal(50)}
    g = {"w": rng.standard_normal(50) * 10.0 ** rng.uniform(-3, 3, 50)}
    p1 = L.Adam(p0, lr=1e-3).step({"w": p0["w"].copy()}, g)
    step = p1["w"] - p0["w"]
    assert np.allclose(np.abs(step), 1e-3, rtol=1e-4)
    assert np.all(np.sign(step) == -np.sign(g["w"]))
    # invariant to a uniform rescaling of the gradient
    p2 = L.Adam(p0, lr=1e-3).step({"w": p0["w"].copy()}, {"w": 1e3 * g["w"]})
    assert np.allclose(p2["w"], p1["w"], atol=1e-9)


# ------------------------------------------------ guarded refinement -------
def test_p13_zero_output_network_reproduces_plain_history_exactly():
    prob = c2_dirichlet_varmu(n=8, p=2)
    hier, g, params = _grid_and_net(prob)
    params["W3"][:] = 0.0
    params["b3"][:] = 0.0
    S = Solver(hier)
    b = np.random.default_rng(12).standard_normal(hier.fine.A.shape[0])
    _, h_plain = S.refinement(b, tol=1e-10, maxit=30)
    _, h_learn, ev = L.refinement_learned(S, b, params, (1.0, 1.0), g, tol=1e-10, maxit=30)
    assert ev == 0
    assert np.array_equal(h_plain, h_learn)


def test_guard_switches_a_harmful_correction_off():
    prob = c2_dirichlet_varmu(n=8, p=2)
    hier, g, params = _grid_and_net(prob)
    params["b3"][:] = 50.0                      # a correction far larger than the error
    S = Solver(hier)
    b = np.random.default_rng(13).standard_normal(hier.fine.A.shape[0])
    _, h_plain = S.refinement(b, tol=1e-10, maxit=40)
    # the full step (w = 1): the minimal-residual step would shrink it away
    x, h, ev = L.refinement_learned(S, b, params, (1.0, 1.0), g, tol=1e-10, maxit=40, minres=False)
    assert ev == 1
    assert h[-1] <= 1e-10
    # the triggering step is replaced by the plain step: identical histories
    assert np.array_equal(h, h_plain)


def test_crop_matches_patch_neighbourhood():
    rng = np.random.default_rng(14)
    shape, C = (8, 8), 4
    F = rng.standard_normal((64, 3))
    c = L.crop(F, shape, (False, True), (6, 7), C, 1)
    m = C + 2
    # element (origin - 1) along axis 0 at local (0, 1): global (5, 7)
    assert np.allclose(c[1 * m + 0], F[7 * 8 + 5])
    # local (3, 2) -> global (8, 8 mod 8 = 0): outside the wall on axis 0
    assert np.allclose(c[2 * m + 3], 0.0)
    # local (1, 2) -> global (6, 0) via the periodic wrap on axis 1
    assert np.allclose(c[2 * m + 1], F[0 * 8 + 6])


def test_training_reduces_the_loss_on_collected_pairs():
    prob = c2_dirichlet_varmu(n=8, p=1)
    hier = build_hierarchy(prob)
    S = Solver(hier)
    g = L.grid_of(hier)
    rng = np.random.default_rng(15)
    X, T = [], []
    for s in range(3):
        xstar = hier.project_kernel(rng.standard_normal(hier.fine.A.shape[0]))
        for r, e in L.collect_pairs(S, xstar, 3):
            Z, sc = L.element_channels(r, g.logmu, g.d, g.nq)
            X.append(L.patches(Z, (g.n,) * g.d, g.periodic))
            E = e.reshape(-1, g.nb).copy()
            E[:, :g.d * g.nq] /= sc[0]
            E[:, g.d * g.nq:] /= sc[1]
            T.append(E)
    X, T = np.concatenate(X), np.concatenate(T)
    params = L.init_params(g.d, g.nb, 16, seed=3)
    opt = L.Adam(params, lr=1e-3)
    l0 = L.loss_and_grad(params, X, T)[0]
    for _ in range(300):
        _, gr = L.loss_and_grad(params, X, T)
        params = opt.step(params, gr)
    assert L.loss_and_grad(params, X, T)[0] < 0.5 * l0


# ------------------------------------------------ minimal-residual step -------
def _step_case(seed=15):
    prob = c2_dirichlet_varmu(n=8, p=2)
    hier, g, params = _grid_and_net(prob)
    S = Solver(hier)
    rng = np.random.default_rng(seed)
    v = hier.project_kernel(rng.standard_normal(hier.fine.A.shape[0]))
    z = S.vcycle_unscaled(v, None, np.float64)
    return S, g, params, v, z


def test_minres_step_is_the_residual_projection():
    """In FP64 the corrected residual v - A(z + w dx) is orthogonal to A dx
    (w minimises its norm over the line), never longer than v - A z, and
    shorter than with the full step for a correction of the wrong size."""
    S, g, params, v, z = _step_case()
    params["b3"][:] = 3.0
    out, w = L.minres_step(S, v, z, params, (1.0, 1.0), g, np.float64, emulate_bf16=False)
    full, _ = L.minres_step(S, v, z, params, (1.0, 1.0), g, np.float64, emulate_bf16=False, minres=False)
    dx = full - z
    q = S.A @ dx
    r_plain = v - S.A @ z
    r_new = v - S.A @ out
    assert abs(np.dot(r_new, q)) <= 1e-12 * np.linalg.norm(r_new) * np.linalg.norm(q)
    assert np.linalg.norm(r_new) <= np.linalg.norm(r_plain)
    assert np.linalg.norm(r_new) < np.linalg.norm(v - S.A @ full)
    assert w != 1.0


def test_minres_step_is_invariant_to_the_output_scale():
    """Scaling the network's output constants by 4 scales dx by 4 and w by
    1/4: the corrected result is unchanged (a misplaced power of the step
    formula breaks this)."""
    S, g, params, v, z = _step_case(16)
    a, wa = L.minres_step(S, v, z, params, (0.3, 0.5), g, np.float64, emulate_bf16=False)
    b, wb = L.minres_step(S, v, z, params, (1.2, 2.0), g, np.float64, emulate_bf16=False)
    assert abs(wa / wb - 4.0) <= 1e-12 * 4.0
    assert np.allclose(a, b, rtol=0, atol=1e-13 * np.abs(a).max())


def test_zero_network_minres_fgmres_is_plain_fgmres():
    """With a zero-output network w = 0 and the flexible GMRES directions are
    the plain V-cycle results: the same iteration estimates as the oracle's
    plain FGMRES, run without a restart."""
    prob = c2_dirichlet_varmu(n=8, p=2)
    hier, g, params = _grid_and_net(prob)
    params["W3"][:] = 0.0
    params["b3"][:] = 0.0
    S = Solver(hier)
    b = np.random.default_rng(17).standard_normal(hier.fine.A.shape[0])
    _, h_plain = S.fgmres(b, tol=1e-10, m=60, maxit=60, dtype=np.float64)
    _, h_learn, ws = L.fgmres_learned(S, b, params, (1.0, 1.0), g, tol=1e-10, m=60, maxit=60, dtype=np.float64,
                                      emulate_bf16=False)
    assert all(w == 0.0 for w in ws)
    assert len(h_plain) == len(h_learn)
    assert np.array_equal(h_plain[:-1], h_learn[:-1])
    assert h_learn[-1] <= 1e-10
