"""GPU parity at the sizes and launch configurations of the benchmark.

Launches with at least 4096 elements run one wavefront per element; smaller
ones (every grid the oracle can assemble quickly) run several.  Two checks
cover the large-grid configuration:

* tiling: a periodic, constant-viscosity operator is translation invariant,
  and with the orthonormal basis its blocks scale as h^-2 (velocity-velocity),
  h^-1 (velocity-pressure) and h^0 (pressure penalty, tau_p = tau h / mu), so
  A(h') = S A(h) S with S = h / h' on velocity and 1 on pressure.  On a 128^2
  grid a field that repeats with period 16 elements therefore gives the 16^2
  oracle's result, scaled and repeated (operator, colour passes, fused
  residual + restriction);
* invariants at the full benchmark size (256^2, Q_3, variable mu, Dirichlet):
  after a colour pass the residual of that colour vanishes to rounding, and
  the FP32 colour pass agrees with the FP64 one to FP32 accuracy.
"""
import numpy as np
import pytest

from synth import Problem, c2_dirichlet_varmu

pytestmark = pytest.mark.gpu


def _tile(v, n_small, n_big, nb, d=2):
    V = v.reshape((n_small,) * d + (nb,))              # numpy axes (axis1, axis0, nb)
    reps = n_big // n_small
    return np.tile(V, (reps,) * d + (1,)).ravel()


def _dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("p", [2, 3])
def test_tiled_periodic_matches_oracle_on_large_grid(p):
    from oracle import build_hierarchy
    from oracle.multigrid import colour_pass
    from paper_1911_05888_amd import Context
    small = Problem(name="ps", dim=2, n=16, p=p, gamma=1, bc=("periodic", "periodic"))
    big = Problem(name="pb", dim=2, n=128, p=p, gamma=1, bc=("periodic", "periodic"))
    print(f"[scale] tiled periodic p={p}", flush=True)
    H = build_hierarchy(small)
    lv = H.fine
    nb = lv.nb
    ctx = Context(big)
    n_l, _, ncol = ctx.level_info(0)
    assert n_l == 128 and (128 * 128) // ncol >= 4096
    nvel = 2 * lv.nq
    ratio = 128 / 16                                   # h_small / h_big

    def S(v, f):                                       # scale the velocity entries by f
        w = v.reshape(-1, nb).copy()
        w[:, :nvel] *= f
        return w.ravel()

    rng = np.random.Generator(np.random.PCG64(41))
    x = rng.standard_normal(lv.A.shape[0])
    b = rng.standard_normal(lv.A.shape[0])
    xb = _tile(S(x, 1 / ratio), 16, 128, nb)           # x' = S^-1 x
    bb = _tile(S(b, ratio), 16, 128, nb)               # b' = S b
    # operator: A' x' = S A x
    y = _dev(np.zeros(128 * 128 * nb))
    ctx.level_apply(0, _dev(xb), y)
    assert _rel(_host(y), _tile(S(lv.A @ x, ratio), 16, 128, nb)) <= 1e-12
    # residual + restriction to the 64^2 level (oracle: 16^2 -> 8^2): S I^T r
    rc = _dev(np.zeros(64 * 64 * nb))
    ctx.level_residual_restrict(0, _dev(bb), _dev(xb), rc)
    want = lv.I.T @ (b - lv.A @ x)
    assert _rel(_host(rc), _tile(S(want, ratio), 8, 64, nb)) <= 1e-12
    # colour passes commute with the scaling: x'_new = S^-1 x_new
    xo = x.copy()
    xg = _dev(xb)
    bg = _dev(bb)
    for c in range(lv.ncol):
        colour_pass(lv.A, lv.Ainv, xo, b, np.nonzero(lv.colours == c)[0], nb)
        ctx.level_smooth_colour(0, c, bg, xg)
        assert _rel(_host(xg), _tile(S(xo, 1 / ratio), 16, 128, nb)) <= 1e-11, c


def test_full_size_colour_pass_invariants():
    import torch
    from paper_1911_05888_amd import Context, V_FP32
    prob = c2_dirichlet_varmu(n=256, p=3)
    print("[scale] full-size C2 colour passes", flush=True)
    ctx = Context(prob, vprec=0, build_precisions=(1 << V_FP32))
    n_l, _, ncol = ctx.level_info(0)
    nb = prob.nb
    N = ctx.ndof
    rng = np.random.Generator(np.random.PCG64(42))
    x0 = rng.standard_normal(N)
    b = rng.standard_normal(N)
    bg = _dev(b)
    colours = (np.arange(n_l)[None, :] % 2) + 2 * (np.arange(n_l)[:, None] % 2)   # parity colouring
    colours = colours.ravel()
    x64 = _dev(x0)
    for c in range(ncol):
        ctx.level_smooth_colour(0, c, bg, x64)
        r = _dev(np.zeros(N))
        ctx.level_apply(0, x64, r)
        ax = _host(r).reshape(-1, nb)
        res = b.reshape(-1, nb) - ax
        el = np.nonzero(colours == c)[0]
        # zero up to the rounding of b - A x, eps |A| |x|: the velocity blocks
        # grow like h^-2 = 65536 here, so |A| |x| exceeds |b| + |A x| (the
        # scale used) by several orders of magnitude for a random x
        scale = np.linalg.norm(b.reshape(-1, nb)[el]) + np.linalg.norm(ax[el])
        print(f"[scale] colour {c}: |r_c| / scale = {np.linalg.norm(res[el]) / scale:.2e}", flush=True)
        assert np.linalg.norm(res[el]) <= 1e-7 * scale, c
    # FP32 colour passes agree with FP64 to FP32 accuracy
    x32 = torch.tensor(x0, dtype=torch.float32, device="cuda")
    b32 = torch.tensor(b, dtype=torch.float32, device="cuda")
    x64 = _dev(x0)
    for c in range(ncol):
        ctx.level_smooth_colour(0, c, bg, x64)
        ctx.level_smooth_colour_f32(0, c, V_FP32, b32, x32)
    d = _host(x32.double()) - _host(x64)
    e = np.linalg.norm(d) / np.linalg.norm(_host(x64))
    print(f"[scale] FP32 vs FP64 colour passes: relative difference {e:.2e}", flush=True)
    assert e <= 1e-4


SMALL_CASES = {
    "c4a_n16_p2": lambda: __import__("synth").c4a_square_inclusion(n=16, p=2),
    "c2_n16_p3": lambda: c2_dirichlet_varmu(n=16, p=3),
    "per3d_n8_p2": lambda: Problem(name="per3d", dim=3, n=8, p=2, gamma=1, bc=("periodic",) * 3),
}


@pytest.mark.parametrize("name", list(SMALL_CASES))
def test_one_wavefront_kernels_match_oracle(name, monkeypatch):
    """The launch threshold lowered to 1 element (LDGS_SMALL_GRID, read at
    setup): every element kernel runs its one-wavefront variant, compared with
    the oracle directly (interphase variant included)."""
    from oracle import build_hierarchy
    from oracle.multigrid import colour_pass
    from paper_1911_05888_amd import Context
    monkeypatch.setenv("LDGS_SMALL_GRID", "1")
    prob = SMALL_CASES[name]()
    print(f"[scale] one-wavefront kernels {name}", flush=True)
    H = build_hierarchy(prob)
    ctx = Context(prob)
    rng = np.random.Generator(np.random.PCG64(43))
    for l, lv in enumerate(H.levels[:-1]):
        x = rng.standard_normal(lv.A.shape[0])
        b = rng.standard_normal(lv.A.shape[0])
        y = _dev(np.zeros_like(x))
        ctx.level_apply(l, _dev(x), y)
        assert _rel(_host(y), lv.A @ x) <= 1e-12, (name, l)
        rc = _dev(np.zeros(H.levels[l + 1].A.shape[0]))
        ctx.level_residual_restrict(l, _dev(b), _dev(x), rc)
        assert _rel(_host(rc), lv.I.T @ (b - lv.A @ x)) <= 1e-12, (name, l)
        xo = x.copy()
        xg = _dev(x)
        bg = _dev(b)
        for c in range(lv.ncol):
            colour_pass(lv.A, lv.Ainv, xo, b, np.nonzero(lv.colours == c)[0], lv.nb)
            ctx.level_smooth_colour(l, c, bg, xg)
            assert _rel(_host(xg), xo) <= 1e-11, (name, l, c)


def test_shared_inverse_matches_per_element_inverses(monkeypatch):
    """3D unsteady periodic workload at 32^3 (colours of 4096 elements, the
    one-wavefront-per-element launches): colour passes with the level's one
    inverse agree with those that stream a copy per element (the shared path
    turned off with LDGS_SHARED_INVERSE=0), in FP64 and FP32."""
    import torch
    from paper_1911_05888_amd import Context, V_FP32
    from synth import c3_unsteady_periodic
    prob = c3_unsteady_periodic(n=32, p=2, re_eff=10.0, h_ref=1.0 / 64)
    print("[scale] shared vs per-element inverses, 3D unsteady 32^3 Q_2", flush=True)
    ctxs = []
    for flag in ("1", "0"):
        monkeypatch.setenv("LDGS_SHARED_INVERSE", flag)
        ctxs.append(Context(prob, build_precisions=(1 << V_FP32)))
    shared, plain = ctxs
    assert shared.level_shared_inverse(0) and not plain.level_shared_inverse(0)
    N = shared.ndof
    rng = np.random.Generator(np.random.PCG64(44))
    x0 = rng.standard_normal(N)
    b = rng.standard_normal(N)
    _, _, ncol = shared.level_info(0)
    xs, xp, bg = _dev(x0), _dev(x0), _dev(b)
    for c in range(ncol):
        shared.level_smooth_colour(0, c, bg, xs)
        plain.level_smooth_colour(0, c, bg, xp)
        assert _rel(_host(xs), _host(xp)) <= 1e-12, c
    xs = torch.tensor(x0, dtype=torch.float32, device="cuda")
    xp = xs.clone()
    b32 = torch.tensor(b, dtype=torch.float32, device="cuda")
    for c in range(ncol):
        shared.level_smooth_colour_f32(0, c, V_FP32, b32, xs)
        plain.level_smooth_colour_f32(0, c, V_FP32, b32, xp)
    e = _rel(_host(xs.double()), _host(xp.double()))
    print(f"[scale] FP32 shared vs per-element: {e:.2e}", flush=True)
    assert e <= 1e-4


SU_CASES = {
    # 12 x 12 blocks (2D Q_1, standard form, red-black): colours of 8192 and
    # 32768 elements take the 16-elements-per-thread tiles of the vector-ALU
    # update, 336 elements per tile (more than the work-group's threads)
    "per2d_n128_p1": lambda: Problem(name="per2d", dim=2, n=128, p=1, gamma=0, bc=("periodic", "periodic")),
    "per2d_n256_p1": lambda: Problem(name="per2d", dim=2, n=256, p=1, gamma=0, bc=("periodic", "periodic")),
    # 27 x 27 blocks, colours of 8192 elements
    "per2d_n128_p2": lambda: Problem(name="per2d", dim=2, n=128, p=2, gamma=0, bc=("periodic", "periodic")),
}


@pytest.mark.parametrize("name", list(SU_CASES))
def test_shared_inverse_large_colours_match_per_element_inverses(name, monkeypatch):
    """FP64 colour passes and a V-cycle from zero (first pass included) with
    the level's one inverse against per-element inverses
    (LDGS_SHARED_INVERSE=0) on colours of 8192 elements and more."""
    import torch
    from paper_1911_05888_amd import Context
    prob = SU_CASES[name]()
    print(f"[scale] shared update, large colours {name}", flush=True)
    ctxs = []
    for flag in ("1", "0"):
        monkeypatch.setenv("LDGS_SHARED_INVERSE", flag)
        ctxs.append(Context(prob))
    shared, plain = ctxs
    assert shared.level_shared_inverse(0) and not plain.level_shared_inverse(0)
    N = shared.ndof
    rng = np.random.Generator(np.random.PCG64(48))
    x0, b = rng.standard_normal(N), rng.standard_normal(N)
    _, _, ncol = shared.level_info(0)
    xs, xp, bg = _dev(x0), _dev(x0), _dev(b)
    for c in range(ncol):
        shared.level_smooth_colour(0, c, bg, xs)
        plain.level_smooth_colour(0, c, bg, xp)
        assert _rel(_host(xs), _host(xp)) <= 1e-12, c
    shared.project_kernel(bg)
    ys = []
    for ctx in (shared, plain):
        y = torch.zeros_like(bg)
        ctx.vcycle(bg, y)
        ys.append(_host(y))
    assert _rel(ys[0], ys[1]) <= 1e-12


FULL_CASES = {
    # 3D unsteady periodic, 64^3 Q_2: every level on the one-inverse path,
    # two-wavefront launches of the 3D evaluation
    "c3_n64_p2": lambda: __import__("synth").c3_unsteady_periodic(n=64, p=2, re_eff=10.0),
    # square inclusion, 512^2 Q_2: interphase faces, mod-3 colouring, regular /
    # extended-stencil split of the large colours, diagonal scaling
    "c4a_n512_p2": lambda: __import__("synth").c4a_square_inclusion(n=512, p=2),
}


@pytest.mark.parametrize("name", list(FULL_CASES))
def test_full_size_colour_pass_invariants_other_configurations(name):
    """At the full sizes the benchmark measures for the other configurations:
    after an FP64 colour pass the residual of every element the pass changed
    vanishes to rounding (scale |b_E| + |(A x)_E|, as for the 256^2 case)."""
    import torch
    from paper_1911_05888_amd import Context
    prob = FULL_CASES[name]()
    print(f"[scale] full-size colour passes {name}", flush=True)
    ctx = Context(prob)
    nb = prob.nb
    N = ctx.ndof
    _, _, ncol = ctx.level_info(0)
    g = torch.Generator(device="cuda").manual_seed(45)
    x = torch.randn(N, dtype=torch.float64, device="cuda", generator=g)
    b = torch.randn(N, dtype=torch.float64, device="cuda", generator=g)
    for c in range(min(ncol, 3)):
        x0 = x.clone()
        ctx.level_smooth_colour(0, c, b, x)
        ax = torch.zeros_like(x)
        ctx.level_apply(0, x, ax)
        changed = (x != x0).view(-1, nb).any(dim=1)
        assert int(changed.sum()) > 0
        res = (b - ax).view(-1, nb)[changed]
        scale = torch.linalg.norm(b.view(-1, nb)[changed]) + torch.linalg.norm(ax.view(-1, nb)[changed])
        rel = float(torch.linalg.norm(res) / scale)
        print(f"[scale] {name} colour {c}: {int(changed.sum())} elements, |r_c| / scale = {rel:.2e}", flush=True)
        assert rel <= 1e-7, (name, c, rel)


MFMA_CASES = {
    # colours of 32768 elements, 108 x 108 inverse (the 3D unsteady workload)
    "c3_n64_p2": (lambda: __import__("synth").c3_unsteady_periodic(n=64, p=2, re_eff=10.0), None),
    # colours of 16384 elements, 48 x 48 inverse
    "per2d_n256_p3": (lambda: Problem(name="per2d", dim=2, n=256, p=3, gamma=1, bc=("periodic", "periodic")), None),
    # every colour on the matrix cores (threshold lowered): 64 elements per
    # colour on the finest level (two 32-element tiles), 8 on the next (one
    # partial tile), 108 x 108 inverse
    "per3d_n8_p2_all": (lambda: Problem(name="per3d", dim=3, n=8, p=2, gamma=1, bc=("periodic",) * 3), "1"),
}


@pytest.mark.parametrize("name", list(MFMA_CASES))
def test_shared_inverse_update_on_matrix_cores(name, monkeypatch):
    """FP32 and FP64 colour passes on a one-inverse level with colours of at
    least 8192 elements (or of any size, with the threshold lowered): the
    update on the matrix cores (FP32 / FP64 MFMA) against the same update on
    the vector ALUs (LDGS_MFMA=0), the first pass from a zero guess (inside
    V-cycles) included, and FP32 against FP64."""
    import torch
    from paper_1911_05888_amd import Context, V_FP32
    make, mfma_min = MFMA_CASES[name]
    prob = make()
    print(f"[scale] matrix-core shared update {name}", flush=True)
    if mfma_min:
        monkeypatch.setenv("LDGS_MFMA_MIN", mfma_min)
    ctxs = []
    for flag in ("1", "0"):
        monkeypatch.setenv("LDGS_MFMA", flag)
        ctxs.append(Context(prob, build_precisions=(1 << V_FP32)))
    mf, va = ctxs
    assert mf.level_shared_inverse(0)
    N = mf.ndof
    _, _, ncol = mf.level_info(0)
    g = torch.Generator(device="cuda").manual_seed(46)
    x0 = torch.randn(N, dtype=torch.float64, device="cuda", generator=g)
    b = torch.randn(N, dtype=torch.float64, device="cuda", generator=g)
    xm = x0.float()
    xv = x0.float()
    x64 = x0.clone()
    x64v = x0.clone()
    b32 = b.float()
    for c in range(ncol):
        mf.level_smooth_colour_f32(0, c, V_FP32, b32, xm)
        va.level_smooth_colour_f32(0, c, V_FP32, b32, xv)
        mf.level_smooth_colour(0, c, b, x64)
        va.level_smooth_colour(0, c, b, x64v)
        e = float(torch.linalg.norm((xm - xv).double()) / torch.linalg.norm(xv.double()))
        e64 = float(torch.linalg.norm(xm.double() - x64) / torch.linalg.norm(x64))
        # FP64: the same products summed in another order (rounding only)
        d64 = float(torch.linalg.norm(x64 - x64v) / torch.linalg.norm(x64v))
        print(f"[scale] {name} colour {c}: MFMA vs VALU {e:.2e} (FP32) {d64:.2e} (FP64), FP32 vs FP64 {e64:.2e}",
              flush=True)
        assert e <= 1e-5 and e64 <= 1e-4 and d64 <= 1e-12, (c, e, e64, d64)
    # whole V-cycles (first pass from a zero guess through the matrix cores)
    from paper_1911_05888_amd import V_FP64
    bp = b.clone()
    mf.project_kernel(bp)
    for vp, tol in ((V_FP32, 1e-5), (V_FP64, 1e-11)):
        ys = []
        for ctx in (mf, va):
            ctx.set_vprec(vp)
            y = torch.zeros_like(bp)
            ctx.vcycle(bp, y)
            ys.append(y)
        e = float(torch.linalg.norm(ys[0] - ys[1]) / torch.linalg.norm(ys[1]))
        print(f"[scale] {name} V-cycle ({'FP64' if vp == V_FP64 else 'FP32'}): MFMA vs VALU {e:.2e}", flush=True)
        assert e <= tol


FUSED_SHARED_CASES = {
    # 2D, red-black colouring, colours of 128 elements, 27 x 27 inverse
    "c1_n16_p2": lambda: __import__("synth").c1_periodic_standard(n=16, p=2),
    # 3D parity colouring, colours of 512 elements, 108 x 108 inverse
    "c3_n16_p2": lambda: __import__("synth").c3_unsteady_periodic(n=16, p=2, re_eff=10.0),
}


@pytest.mark.parametrize("name", list(FUSED_SHARED_CASES))
def test_one_launch_passes_on_one_inverse_levels(name, monkeypatch):
    """Small colours of one-inverse levels run as one launch (the element
    evaluation and the product with the level's inverse, stored once in the
    symmetric tile layout) instead of a residual launch and an update launch
    (LDGS_FUSE_SHARED_MAX=0): the same colour passes and V-cycles up to the
    order of the sums, in FP64, FP32 and with BF16 inverses."""
    import torch
    from paper_1911_05888_amd import Context, V_FP64, V_FP32, V_FP32_BF16BLK
    prob = FUSED_SHARED_CASES[name]()
    print(f"[scale] one-launch one-inverse passes {name}", flush=True)
    ctxs = []
    for flag in ("8192", "0"):
        monkeypatch.setenv("LDGS_FUSE_SHARED_MAX", flag)
        ctxs.append(Context(prob, build_precisions=(1 << V_FP32) | (1 << V_FP32_BF16BLK)))
    fused, split = ctxs
    assert fused.level_shared_inverse(0)
    N = fused.ndof
    _, _, ncol = fused.level_info(0)
    g = torch.Generator(device="cuda").manual_seed(47)
    x0 = torch.randn(N, dtype=torch.float64, device="cuda", generator=g)
    b = torch.randn(N, dtype=torch.float64, device="cuda", generator=g)
    xf, xs = x0.clone(), x0.clone()
    xf32, xs32 = x0.float(), x0.float()
    for c in range(ncol):
        fused.level_smooth_colour(0, c, b, xf)
        split.level_smooth_colour(0, c, b, xs)
        fused.level_smooth_colour_f32(0, c, V_FP32, b.float(), xf32)
        split.level_smooth_colour_f32(0, c, V_FP32, b.float(), xs32)
        d64 = float(torch.linalg.norm(xf - xs) / torch.linalg.norm(xs))
        d32 = float(torch.linalg.norm((xf32 - xs32).double()) / torch.linalg.norm(xs32.double()))
        print(f"[scale] {name} colour {c}: one launch vs two, FP64 {d64:.2e}, FP32 {d32:.2e}", flush=True)
        assert d64 <= 1e-12 and d32 <= 1e-5, (c, d64, d32)
    bp = b.clone()
    fused.project_kernel(bp)
    for vp, tol in ((V_FP64, 1e-11), (V_FP32, 1e-5), (V_FP32_BF16BLK, 1e-5)):
        ys = []
        for ctx in (fused, split):
            ctx.set_vprec(vp)
            y = torch.zeros_like(bp)
            for _ in range(2):
                ctx.vcycle(bp, y)
            ys.append(y)
        e = float(torch.linalg.norm(ys[0] - ys[1]) / torch.linalg.norm(ys[1]))
        print(f"[scale] {name} two V-cycles (vprec {vp}): one launch vs two {e:.2e}", flush=True)
        assert e <= tol, (vp, e)
