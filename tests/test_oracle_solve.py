"""Pins of the implicit heat update (Section 4.3.2), the Newton momentum solve
(Section 4.3.1) and the end-to-end conservation claims (Section 6.1)."""
import numpy as np
import pytest

import mpm_scenes as sc
from oracle import bspline, resample, sampler, solve, step, transfer


def _heat(dim, seed, **kw):
    S = sc.random_scene(dim, 16, 40, seed, cp=2.0, K=0.3, h=4.0, T_amb=350.0, b=7.0, heat=1, dt=1e-3, **kw)
    P, p = S["particles"], S["params"]
    surf = sc.random_surface(P, 30, seed, dx=p["dx"], spread=0.7)
    sp = resample.split(P, surf)
    g = transfer.p2g(P, surf, sp, p)
    st = transfer.grid_setup(P, surf, sp, g, p)
    return solve.Heat(P, surf, g, st, p), P, surf, sp, g, st, p


@pytest.mark.parametrize("dim", [2, 3])
def test_heat_operator_symmetric_positive(dim):
    H, *_ = _heat(dim, 1)
    rng = np.random.default_rng(2)
    u = rng.normal(size=H.nn) * H.dof
    w = rng.normal(size=H.nn) * H.dof
    assert np.sum(u * H.apply(w)) == pytest.approx(np.sum(w * H.apply(u)), rel=1e-12)
    assert np.sum(u * H.apply(u)) > 0


@pytest.mark.parametrize("dim", [2, 3])
def test_heat_uniform_ambient_is_fixed_point(dim):
    H, P, surf, sp, g, st, p = _heat(dim, 3)
    P2 = dict(P, T=np.full(len(P["T"]), 350.0), gradT=np.zeros_like(P["gradT"]))
    g2 = transfer.p2g(P2, surf, sp, p)
    st2 = transfer.grid_setup(P2, surf, sp, g2, p)
    H2 = solve.Heat(P2, surf, g2, st2, dict(p, b=0.0))
    T, info = H2.solve(dict(p, heat_tol=1e-14))
    assert np.allclose(T[H2.dof], 350.0, rtol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_heat_balance_law(dim):
    """1^T L = 0, so sum_i c_p m_i (T^_i - T^n_i)/dt equals the Robin flux
    sum_r |dA_r| (h (T_amb - T^(s_r)) + b)."""
    H, P, surf, sp, g, st, p = _heat(dim, 4)
    T, info = H.solve(dict(p, heat_tol=1e-14))
    lhs = np.sum(H.c * H.m * (T - st["Tn"]) * H.dof)
    Ts = np.sum(H.sN * T[H.sidx], axis=1)
    rhs = np.sum(H.area * (p["h"] * (p["T_amb"] - Ts) + p["b"]))
    assert lhs == pytest.approx(rhs, rel=1e-9)


def test_newton_solution_is_stationary_and_conserves_momentum():
    S = sc.square2d(n=32)
    P, p = S["particles"], dict(S["params"], newton_tol=1e-12)
    rng = np.random.default_rng(5)
    P["v"] = rng.normal(size=P["v"].shape) * 0.05
    newP, info = step.step(P, p)
    assert info["converged"]
    ctx = step.prepare(P, p, info["surf"])[-1]
    g = ctx.project(ctx.grad_Phi(info["vhat"]))
    assert np.linalg.norm(g) <= 1e-9 * info["g0"]
    mom0 = (P["m"][:, None] * P["v"]).sum(0)
    mom1 = (P["m"][:, None] * newP["v"]).sum(0)
    assert np.allclose(mom0, mom1, rtol=0, atol=1e-15 * np.abs(P["m"][:, None] * P["v"]).sum())


def ellipse2d(cfl=0.0):
    S = sc.ellipse2d(cfl=cfl)
    return S["particles"], S["params"]


def test_explicit_steps_conserve_momentum_and_centre_of_mass():
    """Section 6.1: with the conservative split, total linear and angular momentum and
    the centre of mass are conserved to round-off under explicit stepping."""
    P, p = ellipse2d()
    xi = None
    mom = []
    L = []
    com = []
    for k in range(6):
        mom.append((P["m"][:, None] * P["v"]).sum(0))
        L.append(np.sum(P["m"] * (P["x"][:, 0] * P["v"][:, 1] - P["x"][:, 1] * P["v"][:, 0]))
                 + np.sum(P["m"] * (P["A"][:, 1, 0] - P["A"][:, 0, 1])) * p["dx"] ** 2 / 4)
        com.append((P["m"][:, None] * P["x"]).sum(0) / P["m"].sum())
        P, info = step.step(P, p, implicit=False, step_index=k)
    scale = np.abs(P["m"][:, None] * P["v"]).sum()
    assert scale > 0
    assert np.allclose(mom, 0, atol=1e-14 * scale)
    assert np.allclose(L, 0, atol=1e-14 * scale)
    assert np.allclose(com, com[0], rtol=0, atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_droplet_surface_energy_converges(dim):
    """A resting droplet of radius R: e_sigma = gamma * (mesh area) approaches gamma 4 pi R^2
    (2 pi R in 2D) under refinement; the offset is O(dx) because the union of spheres
    sits outside the particles."""
    R, gamma = 0.2, 0.07
    errs = []
    for n in ((32, 64, 128) if dim == 2 else (16, 32, 64)):
        c = np.full(dim, 0.5)
        x = sc.lattice(n, dim, lambda q: np.sum((q - c) ** 2, 1) < R * R, seed=n)
        p = sc.make_params(dim=dim, n=n, g0=gamma)
        surf = sampler.sample_surface(x, p)
        es = gamma * np.linalg.norm(surf["dA"], axis=1).sum()
        exact = gamma * (4 * np.pi * R * R if dim == 3 else 2 * np.pi * R)
        errs.append(abs(es - exact) / exact)
        if R * n >= 16:
            assert errs[-1] < 0.10
    assert errs[0] > errs[1] > errs[2]


def _sym_system(n, seed, indefinite):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    ev = rng.uniform(0.5, 4.0, size=n)
    if indefinite:
        ev[: n // 3] *= -1.0
    A = (Q * ev) @ Q.T
    b = rng.normal(size=n)
    d = np.abs(np.diag(A)) + rng.uniform(0.5, 1.5, size=n)      # an SPD (diagonal) preconditioner
    return A, b, d


@pytest.mark.parametrize("indefinite", [False, True])
def test_minres_solves_symmetric_systems(indefinite):
    """MINRES (Paige-Saunders) on dense symmetric systems, definite and indefinite: the
    solution of np.linalg.solve, and the same iterate count behaviour as SciPy's MINRES."""
    from scipy.sparse.linalg import minres as sp_minres
    A, b, d = _sym_system(40, 3 + indefinite, indefinite)
    x, it, phibar = solve.minres(lambda v: A @ v, b, d, 1e-12, 400)
    ref = np.linalg.solve(A, b)
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)
    xs, info = sp_minres(A, b, M=np.diag(1.0 / d), rtol=1e-12, maxiter=400)
    assert info == 0 and np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(ref)


def test_minres_tracks_the_preconditioned_residual():
    """After every iteration k, the tracked phibar equals |b - A x_k| in the norm of the
    inverse preconditioner, and it never increases (the defining property of MINRES)."""
    A, b, d = _sym_system(30, 7, True)
    prev = np.inf
    for k in range(1, 31):
        x, it, phibar = solve.minres(lambda v: A @ v, b, d, 0.0, k)
        r = b - A @ x
        true = np.sqrt(np.sum(r * r / d))
        assert it == k
        assert abs(phibar - true) <= 1e-9 * np.sqrt(np.sum(b * b / d)), (k, phibar, true)
        assert phibar <= prev * (1 + 1e-12)
        prev = phibar


def test_newton_with_minres_and_exact_hessian():
    """Newton with the exact surface Hessian, each step solved by MINRES: the solution is
    stationary and conserves momentum with the translation correction."""
    S = sc.square2d(n=32)
    P, p = S["particles"], dict(S["params"], newton_tol=1e-10, hess_mode=1, krylov=1)
    rng = np.random.default_rng(8)
    P["v"] = rng.normal(size=P["v"].shape) * 0.05
    newP, info = step.step(P, p)
    assert info["converged"] and info["cg"] > 0
    ctx = step.prepare(P, p, info["surf"])[-1]
    g = ctx.project(ctx.grad_Phi(info["vhat"]))
    assert np.linalg.norm(g) <= 1e-9 * info["g0"]
    mom0 = (P["m"][:, None] * P["v"]).sum(0)
    mom1 = (P["m"][:, None] * newP["v"]).sum(0)
    assert np.allclose(mom0, mom1, rtol=0, atol=1e-15 * np.abs(P["m"][:, None] * P["v"]).sum())


def _cfl_scene(seed):
    S = sc.random_scene(3, 16, 200, seed, cfl=0.5, dt_min=1e-6, dt_max=10.0, bulk=1e4)
    return S["particles"], S["params"]


@pytest.mark.parametrize("implicit", [True, False])
def test_cfl_dt_limits_the_fastest_crossing(implicit):
    """CFL-limited dt (Section 6: dt restricted to a range by the CFL condition): unclamped,
    the fastest particle (plus, explicit, the pressure wave sqrt(lambda/rho)) crosses
    exactly cfl dx; the result does not depend on the particle order."""
    P, p = _cfl_scene(21)
    dt = step.cfl_dt(P, p, implicit)
    assert p["dt_min"] < dt < p["dt_max"]
    vmax = np.max(np.linalg.norm(P["v"], axis=1))
    c = 0.0 if implicit else np.sqrt(p["bulk"] / np.min(P["m"] / P["V0"]))
    assert (vmax + c) * dt == pytest.approx(p["cfl"] * p["dx"], rel=1e-14)
    perm = np.random.default_rng(3).permutation(len(P["m"]))
    assert step.cfl_dt({k: v[perm] for k, v in P.items()}, p, implicit) == dt


def test_cfl_dt_clamps():
    P, p = _cfl_scene(22)
    P0 = dict(P, v=np.zeros_like(P["v"]))
    assert step.cfl_dt(P0, p, True) == p["dt_max"]
    Pf = dict(P, v=P["v"] * 1e9)
    assert step.cfl_dt(Pf, p, True) == p["dt_min"]
    assert step.cfl_dt(Pf, p, False) == p["dt_min"]


def test_ellipse_conservation_with_cfl_steps():
    """Section 6.1 at its parameters with CFL-limited explicit steps over 120 steps: total
    linear and angular momentum (APIC spin included) and the centre of mass stay at their
    initial values to round-off; the CFL rule, not a clamp, sets the steps."""
    P, p = ellipse2d(cfl=0.01)
    com0 = (P["m"][:, None] * P["x"]).sum(0) / P["m"].sum()
    dts = []
    for k in range(120):
        P, info = step.step(P, p, implicit=False, step_index=k)
        dts.append(info["dt"])
    m, x, v, A = P["m"], P["x"], P["v"], P["A"]
    scale = np.abs(m[:, None] * v).sum()
    mom = (m[:, None] * v).sum(0)
    L = np.sum(m * (x[:, 0] * v[:, 1] - x[:, 1] * v[:, 0])) + np.sum(m * (A[:, 1, 0] - A[:, 0, 1])) * p["dx"] ** 2 / 4
    com = (m[:, None] * x).sum(0) / m.sum()
    assert scale > 0 and p["dt_min"] < min(dts) and max(dts) < p["dt_max"]
    assert np.all(np.abs(mom) <= 1e-13 * scale)
    assert abs(L) <= 1e-13 * scale
    assert np.allclose(com, com0, rtol=0, atol=1e-13)


@pytest.mark.parametrize("sign", [1, -1])
def test_cavity_marangoni_flow_direction(sign):
    """Lid-driven cavity (Section 6.4): the free surface moves toward higher surface
    tension.  With k = 1 - T (hot left wall) the top layer flows to +x and its speed grows;
    with k = T the flow reverses.  The wall samples carry no energy, so nothing else drives
    the flow."""
    S = sc.cavity2d(n=32)
    P, p = S["particles"], dict(S["params"])
    if sign < 0:
        p.update(g0=0.0, g1=1.0)
    ux = []
    for k in range(6):
        P, info = step.step(P, p, implicit=True, step_index=k)
        assert info["converged"]
        y = P["x"][:, 1]
        top = y > y.max() - 2 * p["dx"]
        ux.append(float(np.mean(P["v"][top, 0])))
    ux = np.array(ux) * sign
    assert np.all(ux > 0) and ux[-1] > 2 * ux[0]


def test_ramp_friction_orders_the_slide():
    """A 2D droplet landing on a 5.5 degree ramp slides down-slope (-x); with more Coulomb
    friction it slides slower: mean u_x ordered mu = 0 < 0.2 < 5 in magnitude after 40
    steps, all negative."""
    ux = []
    for mu in (0.0, 0.2, 5.0):
        S = sc.ramp2d(mu=mu, v0=-3.0)
        P, p = S["particles"], S["params"]
        for k in range(40):
            P, info = step.step(P, p, implicit=True, step_index=k)
        ux.append(float(np.sum(P["m"] * P["v"][:, 0]) / P["m"].sum()))
    assert ux[0] < ux[1] < ux[2] < 0, ux
