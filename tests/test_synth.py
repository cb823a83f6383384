"""Input generators: the fast evaluations of the seeded fields equal their
defining sums."""
import math

import numpy as np

from synth import FourierForcing, LogNormalRFF


def test_fourier_forcing_separable_evaluation_equals_the_sum():
    for d in (2, 3):
        f = FourierForcing.from_seed(3, d)
        x = np.random.default_rng(d).random((20000, d))   # above one evaluation block
        assert np.allclose(f.forcing(x), f.forcing_direct(x), rtol=0, atol=1e-12)


def test_lognormal_threaded_evaluation_equals_the_sum():
    f = LogNormalRFF.from_seed(1001, 3)
    x = np.random.default_rng(0).random((20000, 3))
    K = f.kvecs.shape[0]
    arg = x @ f.kvecs.T + f.phases[None, :]
    g = math.sqrt(2.0 / K) * np.cos(arg).sum(axis=1)
    dg = -math.sqrt(2.0 / K) * (np.sin(arg) @ f.kvecs)
    assert np.allclose(f.value(x), 10.0 ** g, rtol=1e-13, atol=0)
    assert np.allclose(f.grad(x), (10.0 ** g)[:, None] * math.log(10.0) * dg, rtol=1e-12, atol=1e-300)


def test_projected_coeffs_equal_quadrature_projection():
    """The separable projection of the manufactured solution equals the L2
    projection by a full tensor Gauss rule (2D and 3D)."""
    import numpy as np
    from synth.fields import projected_coeffs, make_exact_paper
    from oracle.assemble import Grid
    from oracle.basis import ref_basis, tensor_gauss
    from synth import ConstField
    for d, n, p in ((2, 4, 2), (3, 2, 2), (2, 3, 3)):
        ex = make_exact_paper(d, 1, ConstField(1.0))
        x = projected_coeffs(ex, d, n, p)
        g = Grid(d, n, p, ("dirichlet",) * d)
        pts, w = tensor_gauss(p + 6, d)
        B = ref_basis(p, pts) * g.h ** (-d / 2)
        X = (g.ijk[:, None, :] + pts[None]) * g.h
        NE, Q = X.shape[:2]
        vals = np.concatenate([ex.velocity(X.reshape(-1, d)).reshape(NE, Q, d),
                               ex.pressure(X.reshape(-1, d)).reshape(NE, Q, 1)], axis=2)
        ref = np.einsum("qa,q,eqf->efa", B, w * g.h ** d, vals).ravel()
        assert np.abs(x - ref).max() <= 1e-13 * np.abs(ref).max(), (d, n, p)
