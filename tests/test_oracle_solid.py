"""Pins of the fixed-corotated solid and the phase change (Sections 3.2.1 and 3.5): the
energy's values and invariances in closed form, its Piola stress and exact stress
differential against central differences, the definiteness fix's symmetry and sign,
the discrete energy's gradient and Hessian with solid particles against finite
differences, the F update of G2P under an affine velocity, and the resets at T_melt."""
import numpy as np
import pytest

import mpm_scenes as sc
from oracle import energy, resample, step, transfer


def _rot(dim, rng, k):
    Q, _ = np.linalg.qr(rng.normal(size=(k, dim, dim)))
    Q[np.linalg.det(Q) < 0, :, 0] *= -1.0
    return Q


def _F(dim, rng, k, spread=0.3):
    return np.eye(dim)[None] + spread * rng.normal(size=(k, dim, dim))


@pytest.mark.parametrize("dim", [2, 3])
def test_corotated_values_and_invariance(dim):
    rng = np.random.default_rng(dim)
    mu, lam = np.full(6, 3.0), np.full(6, 7.0)
    R = _rot(dim, rng, 6)
    assert np.allclose(energy.corotated_psi(R, mu, lam), 0.0, atol=1e-24)
    assert np.allclose(energy.corotated_P(R, mu, lam), 0.0, atol=1e-13)
    F = _F(dim, rng, 6)
    F = F[np.linalg.det(F) > 0.2][:4]
    Q = _rot(dim, rng, len(F))
    assert np.allclose(energy.corotated_psi(Q @ F, mu[:len(F)], lam[:len(F)]),
                       energy.corotated_psi(F, mu[:len(F)], lam[:len(F)]), rtol=1e-12)
    # diagonal stretch: psi = mu sum (s - 1)^2 + lam/2 (J - 1)^2, P = 2 mu (S - I) + lam (J-1) J S^-1
    s = np.array([1.3, 0.8, 1.1])[:dim]
    D = np.diag(s)[None]
    J = np.prod(s)
    assert energy.corotated_psi(D, mu[:1], lam[:1])[0] == pytest.approx(3.0 * np.sum((s - 1) ** 2) + 3.5 * (J - 1) ** 2,
                                                                       rel=1e-13)
    Pd = 2 * 3.0 * (np.diag(s) - np.eye(dim)) + 7.0 * (J - 1) * J * np.diag(1 / s)
    assert np.allclose(energy.corotated_P(D, mu[:1], lam[:1])[0], Pd, rtol=0, atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_corotated_stress_and_differential_finite_differences(dim):
    rng = np.random.default_rng(10 + dim)
    F = _F(dim, rng, 8)
    F = F[np.linalg.det(F) > 0.3]
    k = len(F)
    mu, lam = rng.uniform(1, 4, k), rng.uniform(2, 9, k)
    dF = rng.normal(size=F.shape)
    h = 1e-6
    fd = (energy.corotated_psi(F + h * dF, mu, lam) - energy.corotated_psi(F - h * dF, mu, lam)) / (2 * h)
    an = np.sum(energy.corotated_P(F, mu, lam) * dF, axis=(1, 2))
    assert np.allclose(fd, an, rtol=1e-6, atol=1e-10)
    fdP = (energy.corotated_P(F + h * dF, mu, lam) - energy.corotated_P(F - h * dF, mu, lam)) / (2 * h)
    dP = energy.corotated_dP(F, mu, lam, dF, exact=True)
    assert np.linalg.norm(fdP - dP) <= 1e-6 * np.linalg.norm(dP)
    # the definiteness fix: symmetric and positive semidefinite, and different from EXACT
    dG = rng.normal(size=F.shape)
    a = np.sum(dG * energy.corotated_dP(F, mu, lam, dF, exact=False), axis=(1, 2))
    b = np.sum(dF * energy.corotated_dP(F, mu, lam, dG, exact=False), axis=(1, 2))
    assert np.allclose(a, b, rtol=1e-12)
    assert np.all(np.sum(dF * energy.corotated_dP(F, mu, lam, dF, exact=False), axis=(1, 2)) >= 0)
    assert np.linalg.norm(energy.corotated_dP(F, mu, lam, dF, exact=False) - dP) > 1e-3 * np.linalg.norm(dP)


def _solid_ctx(dim, seed, hess_mode=1):
    S = sc.random_scene(dim, 8 if dim == 3 else 16, 40, seed, box=(0.35, 0.65),
                        mu0=0.7, mu_k=0.01, mu_T0=300.0, g0=0.3, g1=0.004, gT0=300.0,
                        hess_mode=hess_mode, dt=2e-3, vel=0.5,
                        T_melt=315.0, muh0=50.0, lamh0=120.0, kh=0.01, Th0=300.0)
    P, p = S["particles"], S["params"]
    rng = np.random.default_rng(seed)
    P["F"] = _F(dim, rng, len(P["m"]), 0.1)
    surf = sc.random_surface(P, 25, seed, dx=p["dx"], spread=0.7)
    sp = resample.split(P, surf)
    g = transfer.p2g(P, surf, sp, p)
    st = transfer.grid_setup(P, surf, sp, g, p)
    ctx = energy.Context(P, surf, g, st, p)
    vhat = np.where(st["dof"][:, None], rng.normal(size=ctx.vn.shape) * 3.0, 0.0)
    return ctx, vhat, rng, P, p


@pytest.mark.parametrize("dim", [2, 3])
def test_discrete_energy_with_solids_finite_differences(dim):
    ctx, vhat, rng, P, p = _solid_ctx(dim, 40 + dim)
    assert 0 < ctx.solid.sum() < len(ctx.solid)
    g = ctx.grad_Phi(vhat)
    d = rng.normal(size=vhat.shape) * ctx.dof[:, None]
    h = 1e-6
    fd = (ctx.Phi(vhat + h * d) - ctx.Phi(vhat - h * d)) / (2 * h)
    assert fd == pytest.approx(float(np.sum(g * d)), rel=1e-6)
    w = rng.normal(size=vhat.shape) * ctx.dof[:, None]
    fdg = (ctx.grad_Phi(vhat + h * w) - ctx.grad_Phi(vhat - h * w)) / (2 * h)
    hv = ctx.hessvec(vhat, w)
    assert np.linalg.norm(fdg - hv) <= 1e-6 * np.linalg.norm(hv)
    # PSD mode: symmetric, positive semidefinite on the solid term alone
    ctx0, vhat0, rng0, *_ = _solid_ctx(dim, 40 + dim, hess_mode=0)
    ctx0.mask = 1
    ctx0.V0 = ctx0.V0 * 0.0          # the fluid's J term off: the solid term alone
    u = rng0.normal(size=vhat0.shape) * ctx0.dof[:, None]
    a = float(np.sum(u * ctx0.psi_hessvec(vhat0, w)))
    b = float(np.sum(w * ctx0.psi_hessvec(vhat0, u)))
    assert a == pytest.approx(b, rel=1e-10)
    assert float(np.sum(w * ctx0.psi_hessvec(vhat0, w))) >= 0


@pytest.mark.parametrize("dim", [2, 3])
def test_g2p_updates_F_under_affine_velocity(dim):
    """v^_i = B x_i + c gives grad v^ = B at every particle, so a solid's F becomes
    (I + dt B) F exactly and J = det F; liquids keep the trace form."""
    S = sc.random_scene(dim, 16, 200, 7, box=(0.3, 0.7), T_melt=300.0, dt=3e-3)
    P, p = S["particles"], S["params"]
    rng = np.random.default_rng(1)
    P["T"] = rng.uniform(280, 320, len(P["m"]))
    P["F"] = _F(dim, rng, len(P["m"]), 0.1)
    surf = sc.random_surface(P, 50, 7, dx=p["dx"], spread=0.7)
    sp = resample.split(P, surf)
    B = rng.normal(size=(dim, dim))
    c = rng.normal(size=dim)
    from oracle import bspline
    xi = bspline.node_positions(p["n"], dim)
    vhat = xi @ B.T + c
    out = transfer.g2p(P, surf, sp, vhat, np.zeros(p["n"] ** dim), p)
    sol = P["T"] < 300.0
    assert 0 < sol.sum() < len(sol)
    Fexp = (np.eye(dim) + p["dt"] * B)[None] @ P["F"][sol]
    assert np.allclose(out["F"][sol], Fexp, rtol=0, atol=1e-13)
    assert np.allclose(out["J"][sol], np.linalg.det(Fexp), rtol=1e-13)
    assert np.allclose(out["F"][~sol], P["F"][~sol])
    assert np.allclose(out["J"][~sol], (1 + p["dt"] * np.trace(B)) * P["J"][~sol], rtol=1e-13)


def test_phase_change_resets():
    """Melting (T crosses T_melt upward) sets J = 1 and F = I; freezing sets F = I (J = 1);
    particles that stay in their phase keep their state."""
    p = sc.make_params(dim=2, n=16, T_melt=300.0)
    F = np.tile(np.array([[1.2, 0.1], [0.0, 0.9]]), (4, 1, 1))
    P = dict(T=np.array([310.0, 290.0, 305.0, 295.0]), J=np.array([0.9, 1.1, 0.95, 1.05]), F=F)
    T_old = np.array([290.0, 310.0, 301.0, 299.0])     # melt, freeze, stay liquid, stay solid
    out = transfer.phase_change(T_old, dict(P), p)
    assert np.allclose(out["J"], [1.0, 1.0, 0.95, 1.05])
    assert np.allclose(out["F"][0], np.eye(2)) and np.allclose(out["F"][1], np.eye(2))
    assert np.allclose(out["F"][2:], F[2:])


def test_solid_block_step_conserves_momentum():
    """A free solid-and-liquid mixture (no walls, no gravity) steps with its total linear
    momentum conserved to round-off by the translation correction."""
    S = sc.random_scene(2, 16, 300, 11, box=(0.3, 0.7), T_melt=310.0, muh0=80.0, lamh0=200.0, dt=2e-3,
                        g0=0.05, vel=0.3)
    P, p = S["particles"], dict(S["params"], heat=0)
    rng = np.random.default_rng(3)
    P["T"] = rng.uniform(290, 330, len(P["m"]))
    P["F"] = _F(2, rng, len(P["m"]), 0.05)
    mom0 = (P["m"][:, None] * P["v"]).sum(0)
    newP, info = step.step(P, p, implicit=True)
    assert info["converged"]
    mom1 = (P["m"][:, None] * newP["v"]).sum(0)
    assert np.allclose(mom0, mom1, rtol=0, atol=1e-14 * np.abs(P["m"][:, None] * P["v"]).sum())
