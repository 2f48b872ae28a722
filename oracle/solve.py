"""Implicit grid updates (Section 4.3).

Momentum (Section 4.3.1): backward Euler solved with Newton's method.  The paper names
Newton's method and defers the linear algebra and the definiteness fix to earlier work,
so the solver details are chosen here: Jacobi-preconditioned CG on the projected Newton
system (or, for the exact and possibly indefinite surface Hessian, Jacobi-preconditioned
MINRES with the same relative reduction in the preconditioned residual norm), Armijo
backtracking on Phi (a trial is accepted when Phi does not exceed the Armijo bound by
more than the round-off of Phi, 8 eps |Phi|, eps the unit round-off of the arithmetic:
near convergence the Newton decrement falls below that round-off and the comparison
would otherwise be decided by summation order), and an optional exact minimization of
Phi along rigid translations (e and D are translation invariant, so Phi restricted to
v^ - c 1 is a quadratic whose minimizer is c = [sum m (v^ - v^n) - dt g sum m] / sum m).

Temperature (Section 4.3.2): with the surface samples as quadrature points of the Robin
term and interior particles as quadrature points of the conduction term,
    [c_p/dt diag(m) + L + R] T^ = c_p/dt m o T^n + sum_r N_i(s_r)(h T_amb + b)|dA_r|
                                  + sum_p N_i(x_p) H V^n_p
    L_ij = sum_p K V^n_p grad N_i(x_p) . grad N_j(x_p),   R_ij = sum_r h |dA_r| N_i(s_r) N_j(s_r)
over the nodes with mass (the heat mass is the momentum mass m_i, split mass included;
the stray factor h printed on the source term is dropped).  Solved with Jacobi-preconditioned CG from the initial guess T^n.

Parity pins: symmetry and definiteness of the heat operator, the ambient fixed point,
the balance law, Newton stationarity, explicit conservation (tests/test_oracle_solve.py);
the scale of L and R and of the right side's sources against a linear temperature
(tests/test_oracle_pins.py).
"""
from __future__ import annotations

import numpy as np

from . import bspline
from .transfer import _scatter


def pcg(apply, b, diag, tol_abs, maxit, x0=None):
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply(x) if x0 is not None else b.copy()
    z = r / diag
    p = z.copy()
    rz = float(np.sum(r * z))
    it = 0
    while it < maxit:
        if np.sqrt(np.sum(r * r)) <= tol_abs:
            break
        Ap = apply(p)
        pAp = float(np.sum(p * Ap))
        if pAp <= 0.0:
            if it == 0:
                x = z.copy()
            break
        alpha = rz / pAp
        x += alpha * p
        r -= alpha * Ap
        z = r / diag
        rz_new = float(np.sum(r * z))
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    return x, it, float(np.sqrt(np.sum(r * r)))


def minres(apply, b, diag, rel_tol, maxit):
    """Preconditioned MINRES (Paige and Saunders 1975) for a symmetric, possibly indefinite
    operator, with the SPD preconditioner diag(diag).  The Lanczos process on the
    preconditioned operator builds a tridiagonal matrix, which a sequence of Givens
    rotations reduces to upper triangular form one column at a time; the iterate is
    updated along the directions w_k that this triangular factor defines, so the
    preconditioned residual norm (tracked as phibar) never increases.  Stops when
    phibar <= rel_tol * phibar_0, or after maxit iterations.  Returns (x, iterations,
    phibar)."""
    x = np.zeros_like(b)
    r_prev = b.copy()                 # Lanczos residuals r_{k-1}, r_k (unpreconditioned)
    r_cur = b.copy()
    y = b / diag
    beta = float(np.sqrt(np.sum(b * y)))
    if beta == 0.0:
        return x, 0, 0.0
    beta_prev = 0.0
    phibar = beta
    tol = rel_tol * beta
    c, s = -1.0, 0.0                  # last Givens rotation
    dbar = eps_k = 0.0
    w = np.zeros_like(b)
    w_prev = np.zeros_like(b)
    it = 0
    while it < maxit and phibar > tol:
        v = y / beta                  # Lanczos vector
        y = apply(v)
        if it > 0:
            y = y - (beta / beta_prev) * r_prev
        alpha = float(np.sum(v * y))
        y = y - (alpha / beta) * r_cur
        r_prev, r_cur = r_cur, y
        y = r_cur / diag
        beta_prev = beta
        beta = float(np.sqrt(np.sum(r_cur * y)))
        # previous rotation applied to the new column (entries eps, delta, gbar), then the
        # rotation that annihilates the subdiagonal beta
        eps_prev = eps_k
        delta = c * dbar + s * alpha
        gbar = s * dbar - c * alpha
        eps_k = s * beta
        dbar = -c * beta
        gamma = max(float(np.hypot(gbar, beta)), np.finfo(np.float64).eps)
        c, s = gbar / gamma, beta / gamma
        phi = c * phibar
        phibar = s * phibar
        w_new = (v - eps_prev * w_prev - delta * w) / gamma
        w_prev, w = w, w_new
        x = x + phi * w
        it += 1
    return x, it, float(phibar)


def newton(ctx, params):
    P = ctx.project
    v = P(ctx.vn.copy())
    tol = params["newton_tol"]
    msum = float(np.sum(ctx.m[ctx.dof]))
    floor = 1e-14 * msum * ctx.dx / ctx.dt
    fix = params["momentum_fix"] and bool(np.all(ctx.free[ctx.dof]))
    diag = ctx.jacobi_diag()
    g = P(ctx.grad_Phi(v))
    g0 = float(np.linalg.norm(g))
    stats = dict(newton=0, cg=0, hessvec=0, energy=1, g0=g0, converged=False, line_search=0)
    gn = g0
    for it in range(params["newton_max"]):
        if gn <= max(tol * g0, floor):
            stats["converged"] = True
            break
        vl = v.copy()
        apply = lambda w: P(ctx.hessvec(vl, P(w)))
        cg_tol = max(params["cg_rel"] * gn, 0.1 * tol * g0)
        if params.get("krylov", 0) == 1:
            # MINRES for an indefinite (EXACT) Hessian: the same relative reduction, measured
            # in the preconditioned residual norm
            delta, cit, _ = minres(apply, -g, diag, cg_tol / gn, params["cg_max"])
        else:
            delta, cit, _ = pcg(apply, -g, diag, cg_tol, params["cg_max"])
        stats["cg"] += cit
        stats["hessvec"] += cit
        phi0 = ctx.Phi(v)
        slope = float(np.sum(g * delta))
        alpha = 1.0
        for ls in range(params["ls_max"]):
            stats["energy"] += 1
            phit = ctx.Phi(v + alpha * delta)
            noise = 8.0 * np.finfo(np.float64).eps * max(abs(phi0), abs(phit))
            if phit <= phi0 + params["ls_c1"] * alpha * slope + noise:
                break
            alpha *= 0.5
            stats["line_search"] += 1
        v = v + alpha * delta
        if fix:
            d = ctx.dof
            c = (np.sum(ctx.m[d, None] * (v[d] - ctx.vn[d]), axis=0)
                 - ctx.dt * ctx.g * msum) / msum
            v[d] -= c[None, :]
        g = P(ctx.grad_Phi(v))
        gn = float(np.linalg.norm(g))
        stats["newton"] = it + 1
        stats["energy"] += 1
    else:
        stats["converged"] = gn <= max(tol * g0, floor)
    stats["gnorm"] = gn
    return v, stats


def explicit_update(ctx):
    """q^ = 0 in eq. disc_force: forces at y = x; the viscous strain rate uses v^n."""
    f = ctx.psi_grad(np.zeros_like(ctx.vn))
    if ctx.mask & 4:
        # the viscous part of psi_grad at v^ = 0 vanishes; evaluate it at v^n instead
        from .energy import point_gradient, scatter_stress
        dv = point_gradient(ctx.vn, ctx.pidx, ctx.pG)
        eps = 0.5 * (dv + np.transpose(dv, (0, 2, 1)))
        f += scatter_stress(ctx.dt * (ctx.mu * ctx.Vn)[:, None, None] * eps, ctx.pidx, ctx.pG, ctx.nn)
    v = np.zeros_like(ctx.vn)
    d = ctx.dof
    # f above is dt * de/dy (+ dt * viscous); the update is v^n + (dt f_i + dt m g)/m
    v[d] = ctx.vn[d] - f[d] / ctx.m[d, None] + ctx.dt * ctx.g[None, :]
    return ctx.project(v)


def collide(vhat, params):
    """Static collision objects with Coulomb friction, applied to the grid velocity after
    the momentum update (the paper's ramps, Section 6.3, give only the friction
    coefficient; the rule here is the usual grid-node collision of MPM).  Object k is the
    half-space (x - o) . n < 0.  At a node x_i = (i + 1/2) dx with (x_i - o) . n <= 0
    (evaluated in FP64, products and sums in axis order) and v_n = v^ . n < 0, the
    normal part is removed and the tangential part v_t = v^ - v_n n keeps
    max(0, |v_t| + mu v_n) of its length.  Objects act one after another in index order."""
    planes = params.get("planes") or ()
    if not planes:
        return vhat
    dim, n, dx = params["dim"], params["n"], params["dx"]
    xi = (bspline.node_multi_index(np.arange(n ** dim), n, dim) + 0.5) * dx
    v = vhat.copy()
    for o, nrm, mu in planes:
        o = np.asarray(o, np.float64)[:dim]
        nr = np.asarray(nrm, np.float64)[:dim]
        phi = (xi[:, 0] - o[0]) * nr[0]
        vn = v[:, 0] * nr[0]
        for a in range(1, dim):
            phi = phi + (xi[:, a] - o[a]) * nr[a]
            vn = vn + v[:, a] * nr[a]
        hit = (phi <= 0) & (vn < 0)
        vt = v[hit] - vn[hit, None] * nr[None, :]
        tl = np.sqrt(np.sum(vt * vt, axis=1))
        keep = np.maximum(0.0, tl + mu * vn[hit])
        scale = np.where(tl > 0, keep / np.where(tl > 0, tl, 1.0), 0.0)
        v[hit] = vt * scale[:, None]
    return v


class Heat:
    def __init__(self, P, surf, grid, setup, params):
        dim, n, dx = params["dim"], params["n"], params["dx"]
        self.nn = n ** dim
        self.dof = setup["dof"]
        self.m = grid["m"]
        self.c = params["cp"] / params["dt"]
        self.K, self.h = params["K"], params["h"]
        self.pidx, self.pN, self.pG = bspline.stencil(P["x"], dx, n)
        self.sidx, self.sN, _ = bspline.stencil(surf["s"], dx, n)
        self.Vn = setup["Vn"]
        self.area = np.linalg.norm(surf["dA"], axis=1) if len(surf["s"]) else np.zeros(0)
        rhs = self.c * self.m * setup["Tn"]
        rhs += _scatter(self.sidx, self.sN * ((self.h * params["T_amb"] + params["b"]) * self.area)[:, None], self.nn)
        rhs += _scatter(self.pidx, self.pN * (params["H"] * self.Vn)[:, None], self.nn)
        self.rhs = np.where(self.dof, rhs, 0.0)
        self.Tn = setup["Tn"]

    def apply(self, T):
        out = self.c * self.m * T
        gT = np.einsum("pj,pja->pa", T[self.pidx], self.pG)
        out += _scatter(self.pidx, np.einsum("pa,pja->pj", gT, self.pG) * (self.K * self.Vn)[:, None], self.nn)
        if len(self.area):
            Ts = np.sum(self.sN * T[self.sidx], axis=1)
            out += _scatter(self.sidx, self.sN * (self.h * self.area * Ts)[:, None], self.nn)
        return np.where(self.dof, out, 0.0)

    def diag(self):
        d = self.c * self.m
        d = d + _scatter(self.pidx, np.sum(self.pG ** 2, axis=2) * (self.K * self.Vn)[:, None], self.nn)
        if len(self.area):
            d = d + _scatter(self.sidx, self.sN ** 2 * (self.h * self.area)[:, None], self.nn)
        return np.where(self.dof, d, 1.0)

    def solve(self, params):
        bn = float(np.linalg.norm(self.rhs))
        x0 = np.where(self.dof, self.Tn, 0.0)
        T, it, res = pcg(self.apply, self.rhs, self.diag(), params["heat_tol"] * bn, params["heat_max"], x0=x0)
        return T, dict(heat_cg=it, heat_res=res, heat_rhs=bn)
