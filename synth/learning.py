"""Seeded inputs of the learned-correction experiments: random smooth
coefficient fields x* (the exact solutions of the training systems), crop
origins, minibatch orders, and random crop arrays for gradient checks.

Input synthesis only; no discretisation or solver arithmetic.
"""
from __future__ import annotations

import numpy as np


def random_smooth_coeffs(seed, dim, n, p, kmax=3, tail=0.05, out=None):
    """Element-major coefficient vector (n^d elements, d+1 fields, (p+1)^d
    coefficients each, axis 0 fastest): the mean coefficient of every element
    and field is a random trigonometric polynomial of degree kmax evaluated at
    the element centre; the other coefficients are independent normal values
    scaled by tail * 2^-(total degree).  out: a float64 array of n^d (d+1)
    (p+1)^d entries to fill (reused across calls, it saves the first touch of
    fresh memory on large grids)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nq = (p + 1) ** dim
    nb = (dim + 1) * nq
    ne = n ** dim
    ks = np.array(np.meshgrid(*[np.arange(-kmax, kmax + 1)] * dim, indexing="ij")).reshape(dim, -1).T
    m = 2 * kmax + 1
    # e^{2 pi i c k} on the element centres c = (i + 1/2) / n of one axis
    E1 = np.exp(2j * np.pi * np.outer((np.arange(n) + 0.5) / n, np.arange(-kmax, kmax + 1)))
    x = np.empty((ne, nb)) if out is None else out.reshape(ne, nb)
    deg = np.indices((p + 1,) * dim).reshape(dim, -1)[::-1].sum(axis=0)
    scale = tail * 2.0 ** -deg[1:]
    rows = 8192
    for f in range(dim + 1):
        a = rng.standard_normal(len(ks)) / (1.0 + (ks ** 2).sum(axis=1))
        ph = rng.uniform(0.0, 2.0 * np.pi, len(ks))
        # sum_k a_k cos(2 pi c.k + ph_k) = Re sum_k a_k e^{i ph_k} prod_j e^{2 pi i c_j k_j},
        # contracted one axis at a time (ks[:, 0] varies slowest)
        T = (a * np.exp(1j * ph)).reshape((m,) * dim)
        for _ in range(dim):
            T = np.tensordot(T, E1, axes=([0], [1]))   # the contracted axis moves to the end
        # T[i_0, ..., i_{d-1}] with i_j the coordinate of axis j; axis 0 fastest
        x[:, f * nq] = T.real.transpose(tuple(range(dim))[::-1]).ravel()
        # the same draws as one (ne, nq - 1) block, taken a few rows at a time
        for r0 in range(0, ne, rows):
            blk = rng.standard_normal((min(ne, r0 + rows) - r0, nq - 1))
            blk *= scale
            x[r0:r0 + blk.shape[0], f * nq + 1:(f + 1) * nq] = blk
    return x.ravel()


def crop_origins(seed, ncycles, ncrops, dim, n, crop, periodic):
    """Random crop origins (ncycles, ncrops, dim); on non-periodic axes the
    crop stays inside the grid."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.zeros((ncycles, ncrops, dim), dtype=np.int32)
    for k in range(dim):
        hi = n if periodic[k] else n - crop + 1
        out[:, :, k] = rng.integers(0, hi, size=(ncycles, ncrops))
    return out


def batch_order(seed, steps, batch, ncrops):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, ncrops, size=(steps, batch)).astype(np.int32)


def bf16_grid_values(rng, shape, scale=1.0):
    """Normal values that are exactly representable in bfloat16 (low 16 bits
    of the float32 pattern cleared), returned as (float32 values, uint16 bits)."""
    v = (scale * rng.standard_normal(shape)).astype(np.float32)
    bits = (v.view(np.uint32) >> 16).astype(np.uint16)
    return (bits.astype(np.uint32) << 16).view(np.float32), bits
