"""V-cycles replayed from captured HIP graphs against direct launches.

Every V-cycle of a context is captured into a graph on first use and replayed
afterwards (LDGS_GRAPH=0 turns this off).  The kernels are deterministic, so
each replay must reproduce the directly launched cycle bit for bit.  The
replays are interleaved with other work of the program on the same stream
(stage entry points, residuals, other precisions) and host synchronisations,
and every replay is checked, in every precision and for the one-inverse and
interphase paths.
"""
import numpy as np
import pytest

from synth import Problem, c2_dirichlet_varmu, c4a_square_inclusion

pytestmark = pytest.mark.gpu

CASES = {
    "c2_n32_p3": lambda: c2_dirichlet_varmu(n=32, p=3),
    "per3d_n8_p2": lambda: Problem(name="per3d", dim=3, n=8, p=2, gamma=1, bc=("periodic",) * 3),
    "c4a_n16_p2": lambda: c4a_square_inclusion(n=16, p=2),
}


def _contexts(prob, monkeypatch):
    from paper_1911_05888_amd import Context, V_FP32, V_FP32_BF16BLK
    out = []
    for flag in ("0", "1"):
        monkeypatch.setenv("LDGS_GRAPH", flag)
        out.append(Context(prob, build_precisions=(1 << V_FP32) | (1 << V_FP32_BF16BLK)))
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_graph_replays_match_direct_launches(name, monkeypatch):
    import torch
    from paper_1911_05888_amd import V_FP64, V_FP32, V_FP32_BF16BLK
    prob = CASES[name]()
    print(f"[graph] {name}", flush=True)
    direct, graph = _contexts(prob, monkeypatch)
    rng = np.random.Generator(np.random.PCG64(7))
    b_host = rng.standard_normal(direct.ndof)
    for vp in (V_FP64, V_FP32, V_FP32_BF16BLK):
        xs = []
        for ctx in (direct, graph):
            ctx.set_vprec(vp)
            b = torch.tensor(b_host, dtype=torch.float64, device="cuda")
            ctx.project_kernel(b)
            x = torch.zeros_like(b)
            seq = []
            for it in range(4):
                ctx.vcycle(b, x)
                torch.cuda.synchronize()
                seq.append(x.cpu().numpy().copy())
                # other work on the stream between replays
                y = torch.zeros_like(x)
                ctx.level_apply(0, x, y)
                torch.cuda.synchronize()
            xs.append(seq)
        for it in range(4):
            assert np.array_equal(xs[0][it], xs[1][it]), (name, vp, it)
    # the graph context did capture its cycles (one graph per precision, for
    # cycles from a given x); the direct one launched them
    assert direct.graph_count() == 0
    assert graph.graph_count() == 3


@pytest.mark.parametrize("name", ["c2_n32_p3"])
def test_graph_solve_history_matches_direct(name, monkeypatch):
    import torch
    from paper_1911_05888_amd import V_FP32, IR
    prob = CASES[name]()
    direct, graph = _contexts(prob, monkeypatch)
    hists = []
    for ctx in (direct, graph):
        ctx.set_vprec(V_FP32)
        for rep in range(2):                       # capture, then replays
            b = ctx.assemble_rhs(prob.rhs_source())
            x = torch.zeros_like(b)
            st, info = ctx.solve(b, x, tol=1e-10, maxit=40, outer=IR)
            assert st == 0
            hists.append((np.asarray(info["history"]), x.cpu().numpy()))
    for k in (1, 2, 3):
        assert np.array_equal(hists[0][0], hists[k][0])
        assert np.array_equal(hists[0][1], hists[k][1])
    assert direct.graph_count() == 0 and graph.graph_count() == 1


def test_graph_profiling_counts_timed_passes(monkeypatch):
    """Timed cycles are launched directly (events inside a captured graph
    cannot be timed): with timing on, a graph context counts the same timed
    passes as a direct one and captures no further graph."""
    import torch
    from paper_1911_05888_amd import V_FP32, IR
    prob = CASES["c2_n32_p3"]()
    direct, graph = _contexts(prob, monkeypatch)
    counts = []
    assert graph.graph_count() == 0
    for ctx in (direct, graph):
        ctx.set_vprec(V_FP32)
        b = ctx.assemble_rhs(prob.rhs_source())
        ctx.solve(b.clone(), torch.zeros_like(b), tol=1e-10, maxit=40, outer=IR)
        ctx.profile(2)
        st, info = ctx.solve(b.clone(), torch.zeros_like(b), tol=1e-10, maxit=40, outer=IR)
        ms, n = ctx.profile_read()
        ctx.profile(0)
        assert st == 0 and ms > 0.0
        counts.append((n, info["iters"]))
    # 6 sweeps of 4 colour passes per cycle on the finest level; the sweep
    # that starts from the zero guess is not timed, every second one of the
    # other 5 is (3 and 2 sweeps in alternate cycles)
    for n, iters in counts:
        assert n % 4 == 0 and 8 * iters <= n <= 12 * iters, (n, iters)
    assert counts[0] == counts[1]
    # only the untimed cycles were captured
    assert direct.graph_count() == 0 and graph.graph_count() == 1


@pytest.mark.parametrize("name", ["circle_n32_p2", "water_bubble_n16_p2"])
def test_graph_replays_on_implicit_meshes(name, monkeypatch):
    """Implicitly defined meshes (explicit element blocks): FP64 and FP32
    cycles replayed from graphs reproduce direct launches bit for bit,
    interleaved with other work on the stream; the solve history too."""
    import torch
    from paper_1911_05888_amd import Context, V_FP64, V_FP32, FGMRES
    from synth import c4_circle, bubble_unsteady
    prob = {"circle_n32_p2": lambda: c4_circle(n=32, p=2, rhs="bubble"),
            "water_bubble_n16_p2": lambda: bubble_unsteady(n=16, p=2)}[name]()
    print(f"[graph] {name}", flush=True)
    ctxs = []
    for flag in ("0", "1"):
        monkeypatch.setenv("LDGS_GRAPH", flag)
        ctxs.append(Context(prob, build_precisions=1 << V_FP32))
    direct, graph = ctxs
    rng = np.random.Generator(np.random.PCG64(8))
    b_host = rng.standard_normal(direct.ndof)
    for vp in (V_FP64, V_FP32):
        xs = []
        for ctx in (direct, graph):
            ctx.set_vprec(vp)
            b = torch.tensor(b_host, dtype=torch.float64, device="cuda")
            ctx.project_kernel(b)
            x = torch.zeros_like(b)
            seq = []
            for it in range(4):
                ctx.vcycle(b, x)
                torch.cuda.synchronize()
                seq.append(x.cpu().numpy().copy())
                y = torch.zeros_like(x)
                ctx.level_apply(0, x, y)
                torch.cuda.synchronize()
            xs.append(seq)
        for it in range(4):
            assert np.array_equal(xs[0][it], xs[1][it]), (name, vp, it)
    hists = []
    for ctx in (direct, graph):
        ctx.set_vprec(V_FP64)
        b = ctx.assemble_rhs(prob.rhs_source())
        x = torch.zeros_like(b)
        st, info = ctx.solve(b, x, tol=1e-10, maxit=40, outer=FGMRES, fgmres_m=40)
        assert st == 0
        hists.append((np.asarray(info["history"]), x.cpu().numpy()))
    assert np.array_equal(hists[0][0], hists[1][0]) and np.array_equal(hists[0][1], hists[1][1])
    assert direct.graph_count() == 0 and graph.graph_count() >= 2


OVERLAP_CASES = {
    # Dirichlet walls: a chunk's residuals wait only for the previous
    # colour's products up to the next chunk
    "c5_n16_p2": lambda: __import__("synth").c5_lognormal(n=16, p=2),
    # periodic on every axis, variable viscosity (per-element inverses): the
    # slowest axis wraps, so every chunk waits for all previous products
    "per3d_n16_p2_mu": lambda: Problem(name="per3d_n16_p2_mu", dim=3, n=16, p=2, gamma=1, bc=("periodic",) * 3,
                                       mu=__import__("synth").SinProductField(1.0, 0.5, 1.0)),
}


@pytest.mark.parametrize("name,chunks", [("c5_n16_p2", "3"), ("c5_n16_p2", "8"), ("per3d_n16_p2_mu", "4")])
def test_overlapped_colour_passes_match_single_launches(name, chunks, monkeypatch):
    """3D colour passes split into chunks (the residuals of chunk k + 1 on the
    library's stream beside the product of chunk k on a second stream), with
    and without chaining across colours (the next colour's first residual
    chunks start while the last products still run), give the same iterates
    bit for bit as one residual launch and one product launch per colour,
    launched directly and replayed from graphs, in every precision; colours of
    512 elements into 3, 4 or 8 chunks (a ragged last chunk with 3)."""
    import torch
    from paper_1911_05888_amd import Context, V_FP64, V_FP32, V_FP32_BF16BLK
    prob = OVERLAP_CASES[name]()
    print(f"[overlap] {name} chunks={chunks}", flush=True)
    ctxs = {}
    for label, ov, chain, graph in (("single", "1", "1", "1"), ("direct", chunks, "0", "0"),
                                    ("graph", chunks, "0", "1"), ("chained_direct", chunks, "1", "0"),
                                    ("chained_graph", chunks, "1", "1")):
        monkeypatch.setenv("LDGS_OVERLAP", ov)
        monkeypatch.setenv("LDGS_OVERLAP_MIN", "1")
        monkeypatch.setenv("LDGS_OVERLAP_CHAIN", chain)
        monkeypatch.setenv("LDGS_GRAPH", graph)
        ctxs[label] = Context(prob, build_precisions=(1 << V_FP32) | (1 << V_FP32_BF16BLK))
    assert not ctxs["single"].level_shared_inverse(0)   # per-element inverses: the split pass
    rng = np.random.Generator(np.random.PCG64(11))
    b_host = rng.standard_normal(ctxs["single"].ndof)
    for vp in (V_FP64, V_FP32, V_FP32_BF16BLK):
        seqs = {}
        for label, ctx in ctxs.items():
            ctx.set_vprec(vp)
            b = torch.tensor(b_host, dtype=torch.float64, device="cuda")
            ctx.project_kernel(b)
            x = torch.zeros_like(b)
            seq = []
            for it in range(3):
                ctx.vcycle(b, x)
                torch.cuda.synchronize()
                seq.append(x.cpu().numpy().copy())
                y = torch.zeros_like(x)
                ctx.level_apply(0, x, y)
                torch.cuda.synchronize()
            seqs[label] = seq
        for label in ctxs:
            for it in range(3):
                assert np.array_equal(seqs["single"][it], seqs[label][it]), (name, chunks, vp, label, it)
    for label in ("direct", "chained_direct"):
        assert ctxs[label].graph_count() == 0
    for label in ("graph", "chained_graph"):
        assert ctxs[label].graph_count() == 3
