"""Host check of the position bound behind chained chunked colour passes.

Under parity colouring the elements of colour c are numbered by their
half-grid coordinates, idx = sum_k i_k (n/2)^k with element coordinate
e_k = 2 i_k + bit_k(c).  The chained passes let the residuals of chunk q of
one colour wait only for the previous colour's products up to the chunk that
holds position (q+1) ch - 1 + H, H = 2 (n/2)^(d-1), and for all of them when
the slowest axis is periodic.  That is safe if every stencil neighbour F of
an element E (offsets in {-1, 0, 1}^d: the faces, and the E + e_k - e_j pairs
of the viscous-stress form) sits at a position within H of E's, whatever the
two colours, with walls or with periodic wrap on the axes below the slowest.
This test enumerates every element and neighbour on small grids.
"""
import itertools

import numpy as np
import pytest


def positions(n, d):
    """idx of every element (by full coordinates) under parity colouring,
    and its colour."""
    h = n // 2
    coords = np.array(list(itertools.product(range(n), repeat=d)))[:, ::-1]   # axis 0 fastest
    half = coords // 2
    idx = sum(half[:, k] * h ** k for k in range(d))
    col = sum((coords[:, k] % 2) << k for k in range(d))
    return coords, idx, col


def stencil(d):
    return [o for o in itertools.product((-1, 0, 1), repeat=d) if any(o) and sum(map(abs, o)) <= 2]


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("n", [4, 8, 16])
@pytest.mark.parametrize("periodic_low", [False, True])
def test_neighbour_positions_within_bound(d, n, periodic_low):
    coords, idx, col = positions(n, d)
    lookup = {tuple(c): (i, k) for c, i, k in zip(coords, idx, col)}
    H = 2 * (n // 2) ** (d - 1)
    worst = 0
    for c, i, k in zip(coords, idx, col):
        for o in stencil(d):
            f = c + np.array(o)
            if periodic_low:
                f[:d - 1] %= n            # wrap on the axes below the slowest
            if np.any(f < 0) or np.any(f >= n):
                continue                  # a wall: no neighbour
            j, kf = lookup[tuple(f)]
            assert kf != k                # parity colouring is proper for this stencil
            worst = max(worst, abs(int(j) - int(i)))
    assert worst <= H, (d, n, periodic_low, worst, H)


@pytest.mark.parametrize("d", [2, 3])
def test_periodic_slowest_axis_needs_full_wait(d):
    """With the slowest axis periodic the bound fails (neighbours across the
    wrap sit a whole grid of positions away), which is why those passes wait
    for every product of the previous colour."""
    n = 8
    coords, idx, col = positions(n, d)
    lookup = {tuple(c): i for c, i in zip(coords, idx)}
    H = 2 * (n // 2) ** (d - 1)
    c = np.zeros(d, dtype=int)
    f = c.copy()
    f[d - 1] = n - 1                      # the wrap neighbour of the first plane
    assert abs(lookup[tuple(f)] - lookup[tuple(c)]) > H
