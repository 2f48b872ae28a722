"""Pins of the quadratic B-spline (Section 4.2) against closed-form identities."""
import numpy as np
import pytest

from oracle import bspline


def test_kernel_values_from_definition():
    N, dN = bspline.kernel_1d(np.array([0.0, 0.5, 1.0, 1.5, -1.0, 2.0, 0.25]))
    assert np.allclose(N, [0.75, 0.5, 0.125, 0.0, 0.125, 0.0, 0.75 - 0.0625], atol=0, rtol=0)
    h = 1e-6
    u = np.array([-1.3, -0.7, -0.2, 0.1, 0.6, 1.2])
    fd = (bspline.kernel_1d(u + h)[0] - bspline.kernel_1d(u - h)[0]) / (2 * h)
    assert np.allclose(bspline.kernel_1d(u)[1], fd, atol=1e-8)


@pytest.mark.parametrize("dim", [2, 3])
def test_reproduction_identities(dim):
    n = 16
    dx = 1.0 / n
    rng = np.random.default_rng(dim)
    x = rng.uniform(1.01 * dx, 1 - 1.01 * dx, size=(200, dim))
    idx, N, G = bspline.stencil(x, dx, n)
    xi = (bspline.node_multi_index(idx.ravel(), n, dim).reshape(idx.shape + (dim,)) + 0.5) * dx
    assert np.allclose(N.sum(1), 1.0, rtol=0, atol=1e-14)
    assert np.allclose(np.einsum("pj,pja->pa", N, xi), x, rtol=0, atol=1e-14)
    assert np.allclose(G.sum(1), 0.0, atol=1e-12)
    outer = np.einsum("pja,pjb->pab", xi, G)
    assert np.allclose(outer, np.eye(dim)[None], atol=1e-12)
    r = xi - x[:, None, :]
    inertia = np.einsum("pj,pja,pjb->pab", N, r, r)
    assert np.allclose(inertia, dx * dx / 4 * np.eye(dim)[None], atol=1e-16)


def test_gradient_matches_finite_difference():
    n, dim = 16, 3
    dx = 1.0 / n
    x = np.array([[0.33, 0.41, 0.57]])
    idx, N, G = bspline.stencil(x, dx, n)
    h = 1e-7
    for a in range(3):
        e = np.zeros(3); e[a] = h
        ip, Np, _ = bspline.stencil(x + e, dx, n)
        im, Nm, _ = bspline.stencil(x - e, dx, n)
        assert np.array_equal(ip, idx) and np.array_equal(im, idx)
        assert np.allclose((Np - Nm) / (2 * h), G[:, :, a], atol=1e-5)


def test_domain_check():
    with pytest.raises(bspline.DomainError):
        bspline.stencil(np.array([[0.5 / 16, 0.5]]), 1.0 / 16, 16)
