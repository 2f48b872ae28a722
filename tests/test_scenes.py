"""The scene generators' lattices: points per cell, particle volumes and the seeded jitter
(inputs shared by the oracle and the GPU path)."""
import numpy as np

import mpm_scenes as sc


def _cell_counts(x, n):
    c = np.floor(x * n).astype(np.int64)
    key = c[:, 0] + n * (c[:, 1] + (n * c[:, 2] if c.shape[1] == 3 else 0))
    return np.unique(key, return_counts=True)[1]


def test_meltslab_four_particles_per_cell():
    """The 4-ppc slab: four particles in every interior cell, each a quarter of the cell's
    volume, half the particles of the 8-ppc slab on the same grid, and the same
    jitter stream for the same seed."""
    n = 32
    S4 = sc.meltslab3d(n=n, ppc=4)
    S8 = sc.meltslab3d(n=n)
    P4, P8 = S4["particles"], S8["particles"]
    cnt = _cell_counts(P4["x"], n)
    assert cnt.max() == 4 and np.median(cnt) == 4
    assert np.allclose(P4["V0"], (1.0 / n) ** 3 / 4)
    assert abs(len(P4["m"]) / len(P8["m"]) - 0.5) < 0.02
    assert np.array_equal(sc.meltslab3d(n=n, ppc=4)["particles"]["x"], P4["x"])
    # total mass: the slab's volume times the density either way
    assert abs(P4["m"].sum() / P8["m"].sum() - 1) < 0.02
