"""GPU residual histories against the oracle, cycle by cycle.

* Scaled norm: for the diagonally scaled problems (the (alpha, beta) scaling
  of section 5.6) the residual is also measured as ||D (b - A x)||, the norm
  of the system the cycle works on.  In the unscaled norm the first cycle of
  the inclusion problem raises the residual by about the viscosity contrast
  (1e4), which makes the per-cycle bar of the next step 1e4 times looser; in
  the scaled norm the rise is a few units.  Both sides run single V-cycles
  from x_0 = 0; the scaled residual of each iterate is computed on the host
  in FP64 for both; bar 1e-11 max(1, rho_{k-1}, rho_k).
* Reduced precision: iterative refinement (residual in FP64, V-cycle in
  float32, block inverses in float32 or bfloat16) against the oracle's
  float32 emulation of the same cycle.  Two float32 evaluations of one cycle
  differ from each other by about as much as either differs from the FP64
  cycle, so the bar is stated against that difference: per-cycle
  contractions c_k = rho_k / rho_{k-1} agree to (3 s + 1e-6) c_k, with s
  the largest relative |c_k(float32 arithmetic) - c_k(FP64 arithmetic)| of
  the oracle's cycle with the same stored inverses (the triangle inequality
  gives 2 s when the library's float32 cycle is no less accurate than the
  emulation's; the third s is margin for a different summation order).
  For the bfloat16 inverses the emulation rounds the same FP64 symmetric
  parts to float32 and then to bfloat16 (nearest, ties to even) as the
  library does; both sides hold the same bfloat16 values, so their
  remaining difference is float32 arithmetic, and s is taken between the
  float32 and the FP64 arithmetic of the cycle with those bfloat16 values.
  Levels whose blocks are all one matrix keep their single inverse in
  float32 in both.  The log-normal
  case diverges as a stationary iteration (eq. (rho) is measured with
  GMRES there); with bfloat16 inverses it passes the library's blow-up
  guard (residual 1e10) after three cycles, so it is compared over three.
* Full size: the 2D viscous-stress benchmark problem at 256^2 elements, Q_3
  (3,145,728 unknowns), 13 FP64 stationary cycles against the history the
  committed script tests/golden/make_c2_history.py wrote from the oracle;
  bar 1e-11 max(1, rho_{k-1}, rho_k).
"""
import os

import numpy as np
import pytest

from test_gpu_parity import dev, host, setup_case

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_n256_p3_history.txt")


def _per_cycle_scale(h):
    """max(1, rho_{k-1}, rho_k) for each k."""
    h = np.asarray(h)
    return np.maximum(np.maximum(1.0, h), np.concatenate([[1.0], h[:-1]]))


@pytest.mark.parametrize("name", ["c4a_n16_p2", "c4a_n32_p1", "c5_n8_p2_scaled"])
def test_history_scaled_norm(name):
    from oracle.solvers import Solver
    prob, H, ctx = setup_case(name)
    S = Solver(H)
    assert H.fine.dscale is not None
    d = S.d
    rng = np.random.Generator(np.random.PCG64(17))
    b = H.project_kernel(rng.standard_normal(H.fine.A.shape[0]))
    nb = np.linalg.norm(d * b)
    xo = np.zeros_like(b)
    bg = dev(b)
    xg = dev(np.zeros_like(b))
    ho, hg = [1.0], [1.0]
    for k in range(8):
        xo = S.vcycle_unscaled(b, xo)
        ctx.vcycle(bg, xg)
        xh = host(xg)
        ho.append(np.linalg.norm(d * (b - S.A @ xo)) / nb)
        hg.append(np.linalg.norm(d * (b - S.A @ xh)) / nb)
    ho, hg = np.array(ho), np.array(hg)
    print(name, "scaled rho_k gpu", hg, "oracle", ho, flush=True)
    if name.startswith("c4a"):
        # the first cycle raises the scaled residual by a few units, not by
        # the viscosity contrast; the later cycles contract
        assert ho[1] < 10.0 and np.all(ho[2:] < ho[1:-1])
    assert np.all(np.abs(hg - ho) <= 1e-11 * _per_cycle_scale(ho)), np.abs(hg - ho)


@pytest.mark.parametrize("vprec", [1, 2], ids=["fp32", "fp32_bf16_inverses"])
@pytest.mark.parametrize("name", ["c2_n32_p3", "per3d_n8_p2", "mu3d_n8_p2", "c4a_n16_p2", "c5_n8_p2"])
def test_reduced_precision_refinement(name, vprec):
    from oracle.solvers import Solver
    from paper_1911_05888_amd import IR
    prob, H, ctx = setup_case(name, vprec=vprec)
    S = Solver(H)
    rng = np.random.Generator(np.random.PCG64(18))
    b = H.project_kernel(rng.standard_normal(H.fine.A.shape[0]))
    its = 3 if name.startswith("c5") else 8
    bf = vprec == 2
    _, h64 = S.refinement(b, tol=0.0, maxit=its, dtype=np.float64, inv_bf16=bf)
    _, he = S.refinement(b, tol=0.0, maxit=its, dtype=np.float32, inv_bf16=bf)
    st, info = ctx.solve(dev(b), dev(np.zeros_like(b)), tol=0.0, maxit=its, outer=IR)
    hg = info["history"]
    assert len(hg) == len(he) == its + 1
    c64, ce, cg = (h[1:] / h[:-1] for h in (h64, he, hg))
    s = (np.abs(ce - c64) / c64).max()
    print(name, vprec, "contractions gpu", cg, "emulation", ce, "FP64 arithmetic", c64, "s", s, flush=True)
    assert np.all(np.abs(cg - ce) <= (3 * s + 1e-6) * ce), (np.abs(cg - ce) / ce, s)
    if bf and not all(ctx.level_shared_inverse(l) for l in range(len(H.levels) - 1)):
        # the bfloat16 inverses are in use: the cycle differs from the one
        # with float32 inverses by more than the float32 arithmetic does
        c32 = (lambda h: h[1:] / h[:-1])(S.refinement(b, tol=0.0, maxit=its, dtype=np.float32)[1])
        assert (np.abs(ce - c32) / c32).max() > 3 * s


def test_full_size_c2_history():
    """256^2 elements, Q_3: the FP64 stationary history against the oracle's
    stored one (right-hand side assembled by each side from the same source)."""
    import torch
    from paper_1911_05888_amd import Context
    from synth import c2_dirichlet_varmu
    if not os.path.exists(GOLDEN):
        pytest.skip("golden history not written (tests/golden/make_c2_history.py)")
    ref = np.loadtxt(GOLDEN)
    ho = ref[:, 1]
    prob = c2_dirichlet_varmu(n=256, p=3)
    print("[history] c2 n=256 p=3 setup", flush=True)
    ctx = Context(prob)
    b = ctx.assemble_rhs(prob.rhs_source())
    x = torch.zeros_like(b)
    st, info = ctx.solve(b, x, tol=0.0, maxit=len(ho) - 1)
    hg = info["history"]
    print("rho_k gpu", hg, "oracle", ho, flush=True)
    assert len(hg) == len(ho)
    assert np.all(np.abs(hg - ho) <= 1e-11 * _per_cycle_scale(ho)), np.abs(hg - ho)
