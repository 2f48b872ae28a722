"""Pins of the surface sampler (Section 4.1.1): the counter-based generator against its
published test vector, the isocontour against exact planes and spheres, and the
area bookkeeping of the samples."""
import os

import numpy as np
import pytest

import mpm_scenes as sc
from oracle import sampler

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_vector():
    vals = [int(l) for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt")) if l.strip() and not l.startswith("#")]
    state = 1234567
    for v in vals:
        state = (state + sampler.GAMMA) & sampler.MASK64
        assert int(sampler.splitmix64(np.array([state], np.uint64))[0]) == v


def test_counter_uniform_is_uniform():
    u = sampler.counter_uniform(sampler.stream_key(3, 1), np.arange(20000), np.arange(20000) % 7)
    assert u.min() >= 0 and u.max() < 1
    hist = np.histogram(u, bins=10, range=(0, 1))[0]
    assert np.all(np.abs(hist - 2000) < 200)
    # different keys give different streams
    v = sampler.counter_uniform(sampler.stream_key(3, 2), np.arange(20000), np.arange(20000) % 7)
    assert not np.allclose(u, v)


def _linear_phi(n, dim, a, c):
    pos = np.stack(np.meshgrid(*([(np.arange(n) + 0.5) / n] * dim)[::-1], indexing="ij")[::-1], -1).reshape(-1, dim)
    return pos @ np.asarray(a) - c


def test_plane_isocontour_exact():
    n = 16
    a = np.array([1.0, 0.3, 0.2])
    phi = _linear_phi(n, 3, a, 0.7)
    ids, verts, orient = sampler.isocontour(phi, n, 3)
    nhat, area = sampler.element_normals(verts, orient)
    keep = area > 0
    assert np.allclose(nhat[keep], a / np.linalg.norm(a), atol=1e-12)
    # the plane x = 0.7 - 0.3 y - 0.2 z stays inside the node box for y,z in the box
    L = (n - 1) / n
    assert area.sum() == pytest.approx(L * L * np.linalg.norm(a) / a[0], rel=1e-12)
    # every vertex lies on the plane
    assert np.allclose(verts.reshape(-1, 3) @ a - 0.7, 0, atol=1e-14)


def test_line_isocontour_exact_2d():
    n = 32
    a = np.array([0.4, 1.0])
    phi = _linear_phi(n, 2, a, 0.55)
    ids, verts, orient = sampler.isocontour(phi, n, 2)
    nhat, length = sampler.element_normals(verts, orient)
    keep = length > 0
    assert np.allclose(nhat[keep], a / np.linalg.norm(a), atol=1e-12)
    L = (n - 1) / n
    assert length.sum() == pytest.approx(L * np.linalg.norm(a) / a[1], rel=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_sphere_isocontour_converges(dim):
    R = 0.3
    errs = []
    for n in (16, 32, 64):
        pos = np.stack(np.meshgrid(*([(np.arange(n) + 0.5) / n] * dim)[::-1], indexing="ij")[::-1], -1).reshape(-1, dim)
        phi = np.linalg.norm(pos - 0.5, axis=1) - R
        ids, verts, orient = sampler.isocontour(phi, n, dim)
        nhat, meas = sampler.element_normals(verts, orient)
        exact = 4 * np.pi * R * R if dim == 3 else 2 * np.pi * R
        errs.append(abs(meas.sum() - exact) / exact)
        cen = verts.mean(1) - 0.5
        assert np.all(np.sum(nhat * cen, axis=1) > 0)        # outward
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.01


@pytest.mark.parametrize("dim", [2, 3])
def test_samples_area_and_placement(dim):
    S = sc.droplet3d(16, 7, 0.05, [0, 0, 0]) if dim == 3 else sc.square2d(n=32)
    P, p = S["particles"], S["params"]
    surf = sampler.sample_surface(P["x"], p)
    area = np.linalg.norm(surf["dA"], axis=1)
    assert area.sum() == pytest.approx(surf["area"], rel=1e-12)
    # deterministic
    surf2 = sampler.sample_surface(P["x"], p)
    assert np.array_equal(surf["s"], surf2["s"]) and np.array_equal(surf["dA"], surf2["dA"])
    # each sample lies outside every particle's sphere by no more than a cube diagonal,
    # and on the zero set of the piecewise-linear interpolant (close to the sphere union)
    from scipy.spatial import cKDTree
    d, _ = cKDTree(P["x"]).query(surf["s"])
    r = p["ls_radius"]
    assert np.all(np.abs(d - r) < 0.5 * p["dx"])
    # density: every element gets max(1, floor(rho A + u)) samples
    ntri = len(np.unique(surf["tri"]))
    assert p["sample_density"] * surf["area"] - ntri <= len(surf["s"]) <= p["sample_density"] * surf["area"] + ntri
