"""The library's host setup of implicitly defined meshes (a circle cutting
the grid) against the oracle, on the CPU (host-only contexts): every
level's operator (explicit element blocks, after Algorithm 2 with the
implicit-mesh injection), the greedy colours, the block inverses, the
bottom pseudo-inverse and the right-hand side, for the manufactured and the
bubble data.  Element numbering is (host cell, phase) on both sides."""
import numpy as np
import pytest

from synth import c4_circle, bubble_unsteady, disk_domain

pytestmark = pytest.mark.filterwarnings("ignore")


def _ldgs():
    from paper_1911_05888_amd import ldgs
    return ldgs


@pytest.mark.parametrize("n,rhs", [(16, "exact"), (32, "bubble"), (16, "water"), (16, "gas"), (16, "disk"),
                                   (32, "disk_vs")])
def test_host_levels_match_oracle(n, rhs):
    """(water / gas: the unsteady bubbles of section 6, with the rho-weighted
    mass, eq. (taugeneral) and Algorithm 3's coarsening)"""
    from oracle.implicit_assemble import build_implicit_hierarchy, implicit_rhs
    ldgs = _ldgs()
    if rhs in ("water", "gas"):
        prob = bubble_unsteady(n=n, p=2, water_inside=rhs == "water")
    elif rhs.startswith("disk"):
        # the curved domain of section 5 (standard and viscous-stress form)
        prob = disk_domain(n=n, p=2, gamma=1 if rhs == "disk_vs" else 0)
    else:
        prob = c4_circle(n=n, p=2, rhs=rhs)
    H = build_implicit_hierarchy(prob)
    ctx = ldgs.Context(prob, host_only=True)
    assert ctx.n_levels == len(H.levels)
    rng = np.random.default_rng(n)
    for l, lv in enumerate(H.levels):
        assert ctx.level_elements(l) == lv.NE
        x = rng.standard_normal(lv.A.shape[0])
        y = ctx.host_level_apply(l, x)
        yo = lv.A @ x
        assert np.abs(y - yo).max() <= 1e-11 * np.abs(yo).max(), l
        if hasattr(lv, "Ainv"):
            assert ctx.level_info(l)[2] == lv.ncol
            for e in rng.choice(lv.NE, 6, replace=False):
                inv = ctx.level_block_inverse(l, int(e))
                assert np.abs(inv - lv.Ainv[e]).max() <= 1e-11 * np.abs(lv.Ainv[e]).max()
    pinv, eig = ctx.bottom_info()
    assert np.abs(pinv - H.levels[-1].pinv).max() <= 1e-7 * np.abs(H.levels[-1].pinv).max()
    b = ctx.assemble_rhs(prob.rhs_source())
    bo = implicit_rhs(prob, H.fine.ops)
    assert np.abs(b - bo).max() <= 1e-12 * np.abs(bo).max()


def test_circle_argument_errors():
    ldgs = _ldgs()
    from synth.problems import Problem
    prob = c4_circle(n=16, p=2)
    prob.bc = ("periodic", "periodic")
    with pytest.raises(ldgs.LdgsError):
        ldgs.Context(prob, host_only=True)
    prob = c4_circle(n=16, p=2)
    with pytest.raises(ldgs.LdgsError):
        ldgs.Context(prob, host_only=True, vprec=ldgs.V_FP32_BF16BLK)
