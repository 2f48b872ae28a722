"""Pins of the discrete energy, forces and Hessian-vector product (Section 4.3.1):
central finite differences, symmetry and semidefiniteness, translation and rotation
invariance of the forces (eq. fe), and closed forms at the undeformed state."""
import numpy as np
import pytest

import mpm_scenes as sc
from oracle import bspline, energy, resample, transfer


def _ctx(dim, seed, mask=7, hess_mode=1, count=30, nsurf=25, vel=0.5):
    S = sc.random_scene(dim, 8 if dim == 3 else 16, count, seed, box=(0.35, 0.65),
                        mu0=0.7, mu_k=0.01, mu_T0=300.0, g0=0.3, g1=0.004, gT0=300.0,
                        term_mask=mask, hess_mode=hess_mode, dt=2e-3, vel=vel)
    P, p = S["particles"], S["params"]
    surf = sc.random_surface(P, nsurf, seed, dx=p["dx"], spread=0.7)
    sp = resample.split(P, surf)
    g = transfer.p2g(P, surf, sp, p)
    st = transfer.grid_setup(P, surf, sp, g, p)
    ctx = energy.Context(P, surf, g, st, p)
    rng = np.random.default_rng(seed + 99)
    vhat = np.where(st["dof"][:, None], rng.normal(size=ctx.vn.shape) * 3.0, 0.0)
    return ctx, vhat, rng, P, surf, p


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("mask", [1, 2, 4, 7])
def test_gradient_finite_difference(dim, mask):
    ctx, vhat, rng, *_ = _ctx(dim, 3 + mask, mask=mask)
    g = ctx.grad_Phi(vhat)
    d = rng.normal(size=vhat.shape) * ctx.dof[:, None]
    h = 1e-6
    fd = (ctx.Phi(vhat + h * d) - ctx.Phi(vhat - h * d)) / (2 * h)
    an = float(np.sum(g * d))
    assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-300) + 1e-14


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("mask", [1, 2, 4, 7])
def test_hessvec_finite_difference(dim, mask):
    ctx, vhat, rng, *_ = _ctx(dim, 30 + mask, mask=mask, hess_mode=1)
    w = rng.normal(size=vhat.shape) * ctx.dof[:, None]
    h = 1e-6
    fd = (ctx.grad_Phi(vhat + h * w) - ctx.grad_Phi(vhat - h * w)) / (2 * h)
    hv = ctx.hessvec(vhat, w)
    err = np.linalg.norm(fd - hv) / np.linalg.norm(hv)
    assert err < 1e-6


@pytest.mark.parametrize("dim", [2, 3])
def test_hessian_symmetric_and_psd(dim):
    ctx, vhat, rng, *_ = _ctx(dim, 50, hess_mode=1)
    u = rng.normal(size=vhat.shape) * ctx.dof[:, None]
    w = rng.normal(size=vhat.shape) * ctx.dof[:, None]
    a, b = np.sum(u * ctx.hessvec(vhat, w)), np.sum(w * ctx.hessvec(vhat, u))
    assert a == pytest.approx(b, rel=1e-12)
    # PSD mode: the surface part alone is positive semidefinite, and symmetric
    ctx2, vhat2, rng2, *_ = _ctx(dim, 51, mask=2, hess_mode=0)
    for _ in range(5):
        w = rng2.normal(size=vhat2.shape) * ctx2.dof[:, None]
        assert np.sum(w * ctx2.psi_hessvec(vhat2, w)) >= -1e-14
    u = rng2.normal(size=vhat2.shape) * ctx2.dof[:, None]
    assert np.sum(u * ctx2.psi_hessvec(vhat2, w)) == pytest.approx(np.sum(w * ctx2.psi_hessvec(vhat2, u)), rel=1e-12)


def test_J_hessian_independent_of_linearization():
    ctx, vhat, rng, *_ = _ctx(3, 60, mask=1)
    w = rng.normal(size=vhat.shape)
    assert np.allclose(ctx.psi_hessvec(vhat, w), ctx.psi_hessvec(0 * vhat, w), rtol=0, atol=0)


def test_surface_2d_has_no_indefinite_part():
    ctx, vhat, rng, *_ = _ctx(2, 61, mask=2, hess_mode=1)
    w = rng.normal(size=vhat.shape)
    ctx2, *_ = _ctx(2, 61, mask=2, hess_mode=0)
    assert np.allclose(ctx.psi_hessvec(vhat, w), ctx2.psi_hessvec(vhat, w), rtol=0, atol=0)


@pytest.mark.parametrize("dim", [2, 3])
def test_surface_gradient_at_identity(dim):
    rng = np.random.default_rng(4)
    N = rng.normal(size=(20, dim))
    G = np.repeat(np.eye(dim)[None], 20, 0)
    Q = energy.surface_grad(G, N)
    nrm = np.linalg.norm(N, axis=1)
    nh = N / nrm[:, None]
    ref = nrm[:, None, None] * (np.eye(dim)[None] - nh[:, :, None] * nh[:, None, :])
    assert np.allclose(Q, ref, atol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_force_invariances(dim):
    ctx, vhat, rng, P, surf, p = _ctx(dim, 70, mask=3)
    gp = ctx.psi_grad(vhat)                       # dt * de/dy at y = x + dt v^
    assert np.allclose(gp.sum(0), 0, atol=1e-13 * np.abs(gp).sum())
    xi = bspline.node_positions(p["n"], dim)
    y = xi + ctx.dt * vhat
    ctx_s = energy.Context(P, surf, dict(m=ctx.m), dict(k=ctx.k, Vn=ctx.Vn, mu=ctx.mu, vn=ctx.vn, dof=ctx.dof, free=ctx.free), dict(p, term_mask=2))
    gs = ctx_s.psi_grad(vhat)
    if dim == 3:
        torque = np.cross(y, gs).sum(0)
    else:
        torque = np.sum(y[:, 0] * gs[:, 1] - y[:, 1] * gs[:, 0])
    assert np.allclose(torque, 0, atol=1e-13 * np.abs(gs).sum())
    ctx_j = energy.Context(P, surf, dict(m=ctx.m), dict(k=ctx.k, Vn=ctx.Vn, mu=ctx.mu, vn=ctx.vn, dof=ctx.dof, free=ctx.free), dict(p, term_mask=1))
    gj = ctx_j.psi_grad(0 * vhat)
    if dim == 3:
        torque = np.cross(xi, gj).sum(0)
    else:
        torque = np.sum(xi[:, 0] * gj[:, 1] - xi[:, 1] * gj[:, 0])
    assert np.allclose(torque, 0, atol=1e-13 * np.abs(gj).sum() + 1e-300)


def test_surface_energy_at_rest_is_k_times_area():
    ctx, vhat, rng, P, surf, p = _ctx(3, 80, mask=2)
    eJ, es, D = ctx.psi_terms(0 * vhat)
    assert es == pytest.approx(np.sum(ctx.k * np.linalg.norm(surf["dA"], axis=1)), rel=1e-14)
