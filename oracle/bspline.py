"""Quadratic B-spline interpolation on the cell-centred grid (Section 4.2: N_i(x) =
N(x - x_i) with x_i at cell centres, the kernel of Stomakhin et al. 2013).

1D kernel: N(u) = 3/4 - u^2 for |u| < 1/2, (3/2 - |u|)^2 / 2 for 1/2 <= |u| < 3/2, else 0,
with u = (x - x_i)/dx; in d dimensions N_i(x) = prod_a N((x_a - x_ia)/dx).

Parity: pinned by the closed-form identities in tests/test_oracle_bspline.py (partition
of unity, linear reproduction, sum of gradients, sum x_i (x) grad N_i = I, and the
quadratic-moment identity sum N_i (x_i-x)(x_i-x)^T = dx^2/4 I used by the APIC inertia).
"""
from __future__ import annotations

import itertools

import numpy as np


class DomainError(ValueError):
    """A point's 3^d stencil leaves the grid (the point must lie in [dx, 1-dx)^d)."""


def kernel_1d(u):
    """The 1D quadratic B-spline N(u) and its derivative dN/du, written from the
    piecewise definition."""
    a = np.abs(u)
    N = np.where(a < 0.5, 0.75 - a * a, np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0))
    dN = np.where(a < 0.5, -2.0 * u, np.where(a < 1.5, -(1.5 - a) * np.sign(u), 0.0))
    return N, dN


def offsets(dim):
    """The 3^d stencil offsets k in {0,1,2}^d, k_0 varying fastest."""
    return np.array([k[::-1] for k in itertools.product(range(3), repeat=dim)], dtype=np.int64)


def stencil(x, dx, n):
    """For points x (P, d): the 3^d nodes whose support contains x, their weights and
    weight gradients.

    Returns idx (P, 3^d) natural linear node indices, N (P, 3^d), G (P, 3^d, d) with
    G[p, j, a] = dN_j/dx_a (x_p).  The nodes are base + k with base = floor(x/dx - 1),
    which covers every node with |x_a - x_ia| < 3/2 dx."""
    x = np.asarray(x, np.float64)
    P, dim = x.shape
    base = np.floor(x / dx - 1.0).astype(np.int64)
    if P and (base.min() < 0 or base.max() + 2 > n - 1):
        raise DomainError("point outside [dx, 1-dx)^d")
    K = offsets(dim)
    nodes = base[:, None, :] + K[None, :, :]                  # (P, 3^d, d)
    xi = (nodes + 0.5) * dx
    u = (x[:, None, :] - xi) / dx                             # (P, 3^d, d)
    w1, dw1 = kernel_1d(u)
    N = np.prod(w1, axis=2)
    G = np.empty_like(u)
    for a in range(dim):
        others = np.prod(np.delete(w1, a, axis=2), axis=2)
        G[:, :, a] = dw1[:, :, a] / dx * others
    mult = n ** np.arange(dim)
    idx = nodes @ mult
    return idx, N, G


def node_positions(n, dim):
    """Positions (n^d, d) of all nodes in natural order."""
    g = (np.arange(n) + 0.5) / n
    mesh = np.meshgrid(*([g] * dim)[::-1], indexing="ij")[::-1]
    return np.stack([m.ravel() for m in mesh], axis=1)


def node_multi_index(idx, n, dim):
    out = np.empty((len(idx), dim), np.int64)
    r = np.asarray(idx, np.int64)
    for a in range(dim):
        out[:, a] = r % n
        r = r // n
    return out
