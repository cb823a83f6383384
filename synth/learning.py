"""Seeded inputs of the learned-correction experiments: random smooth
coefficient fields x* (the exact solutions of the training systems), crop
origins, minibatch orders, and random crop arrays for gradient checks.

Input synthesis only; no discretisation or solver arithmetic.
"""
from __future__ import annotations

import numpy as np


def random_smooth_coeffs(seed, dim, n, p, kmax=3, tail=0.05):
    """Element-major coefficient vector (n^d elements, d+1 fields, (p+1)^d
    coefficients each, axis 0 fastest): the mean coefficient of every element
    and field is a random trigonometric polynomial of degree kmax evaluated at
    the element centre; the other coefficients are independent normal values
    scaled by tail * 2^-(total degree)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nq = (p + 1) ** dim
    nb = (dim + 1) * nq
    ne = n ** dim
    idx = np.indices((n,) * dim).reshape(dim, -1)[::-1]          # idx[k] = coordinate along axis k
    centre = (idx.T + 0.5) / n                                   # (ne, dim)
    ks = np.array(np.meshgrid(*[np.arange(-kmax, kmax + 1)] * dim, indexing="ij")).reshape(dim, -1).T
    x = np.zeros((ne, nb))
    deg = np.indices((p + 1,) * dim).reshape(dim, -1)[::-1].sum(axis=0)
    for f in range(dim + 1):
        a = rng.standard_normal(len(ks)) / (1.0 + (ks ** 2).sum(axis=1))
        ph = rng.uniform(0.0, 2.0 * np.pi, len(ks))
        x[:, f * nq] = np.cos(2.0 * np.pi * centre @ ks.T + ph) @ a
        x[:, f * nq + 1:(f + 1) * nq] = tail * rng.standard_normal((ne, nq - 1)) * 2.0 ** -deg[None, 1:]
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
