"""The oracle's reduced-precision emulation, pinned to facts outside it.

* bfloat16 inverses: every stored entry is a bfloat16 value (low 16 bits of
  its float32 pattern zero), the stored block is exactly symmetric, and each
  entry is within half a bfloat16 unit (2^-8 relative: 8 significant bits) of the symmetric part
  of the FP64 inverse.  A dropped symmetrisation or a truncating rounding
  fails one of these.
* A periodic constant-coefficient level (all blocks one matrix) keeps its
  inverse in float32; the blocks-equal test itself is checked on a level
  that is translation invariant and on one that is not.
* Iterative refinement with a float32 cycle converges to 1e-10 in the FP64
  residual (the residual is formed in FP64), with per-cycle contraction
  within a small margin of the FP64 cycle's: the classical bound for mixed-
  precision refinement adds only O(u_32 cond) to the contraction.
"""
import numpy as np

from synth import c2_dirichlet_varmu


def _hier():
    from oracle import build_hierarchy
    return build_hierarchy(c2_dirichlet_varmu(n=8, p=2))


def test_bf16_inverses_are_rounded_symmetric_parts():
    from oracle.multigrid import Precision, blocks_all_equal
    H = _hier()
    P = Precision(H, np.float32, inv_bf16=True)
    for lv, Ai in zip(H.levels[:-1], P.Ainv[:-1]):
        assert not blocks_all_equal(lv.Ainv)            # Dirichlet walls, varying mu
        assert Ai.dtype == np.float32
        bits = Ai.view(np.uint32)
        assert np.all((bits & 0xFFFF) == 0)
        assert np.array_equal(Ai, np.transpose(Ai, (0, 2, 1)))
        sym = 0.5 * (lv.Ainv + np.transpose(lv.Ainv, (0, 2, 1)))
        big = np.abs(sym) > 1e-30
        assert np.all(np.abs(Ai[big] - sym[big]) <= 2.0 ** -8 * np.abs(sym[big]) * (1 + 1e-6))


def test_float32_refinement_converges_like_fp64():
    from oracle.solvers import Solver
    H = _hier()
    S = Solver(H)
    rng = np.random.Generator(np.random.PCG64(3))
    b = rng.standard_normal(H.fine.A.shape[0])
    _, h64 = S.refinement(b, tol=1e-10, maxit=40, dtype=np.float64)
    for bf in (False, True):
        x, h32 = S.refinement(b, tol=1e-10, maxit=40, dtype=np.float32, inv_bf16=bf)
        bp = H.project_kernel(b)
        assert np.linalg.norm(bp - S.A @ x) <= 1e-10 * np.linalg.norm(bp)
        assert len(h32) <= len(h64) + (3 if bf else 1)


def test_uniform_levels_keep_float32_inverse():
    from oracle import build_hierarchy
    from oracle.multigrid import Precision, blocks_all_equal
    from synth import Problem
    H = build_hierarchy(Problem(name="per", dim=2, n=8, p=2, gamma=1, bc=("periodic", "periodic")))
    assert all(blocks_all_equal(lv.Ainv) for lv in H.levels[:-1])
    P = Precision(H, np.float32, inv_bf16=True)
    for lv, Ai in zip(H.levels[:-1], P.Ainv[:-1]):
        assert np.array_equal(Ai, lv.Ainv.astype(np.float32))
