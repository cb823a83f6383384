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
