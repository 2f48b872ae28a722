"""Discrete energy, forces and their linearization for the backward-Euler grid update
(Section 4.3.1).

With y = x + dt v^ (x the unmoved node positions) the discrete potential is
    e(y) = sum_p lambda/2 (J_p(y) - 1)^2 V^0_p  +  sum_r k_r |J^_r F^_r^{-T} dA_r|
where, in displacement form (identical to the printed form in exact arithmetic because
sum_i x_i (x) grad N_i = I, and four digits more accurate in FP32),
    J_p(y) = (1 + dt sum_i v^_i . grad N_i(x_p)) J^n_p,     F^_r = I + dt sum_i v^_i (x) grad N_i(s_r),
and J^ F^^{-T} = cof(F^) (the cofactor matrix, det(F) F^{-T}).  The linear viscous force
of eq. disc_force, -mu sum_p eps(v^; x_p) grad N_i(x_p) V^n_p with eps the symmetric
velocity gradient, is the negative gradient of the dissipation
    D(v^) = sum_p mu_p / 2 V^n_p eps_p : eps_p.
The backward-Euler update m (v^ - v^n)/dt = f(x + dt v^) + m g is the stationarity
condition of
    Phi(v^) = 1/2 sum_i m_i |v^_i - v^n_i|^2 - dt sum_i m_i g . v^_i + e(x + dt v^) + dt D(v^),
whose gradient and Hessian (M + dt^2 d2e/dy2 + dt C) drive Newton's method.

Surface term: f(G) = |cof(G) N| with N = dA_r.  Its first derivative (the force of
eq. fe, read as evaluated at the surface sample s_r, the quadrature point of e_sigma) and second derivative are
written with the cross-product form of the cofactor (3D: column m of cof(G) is
g_{m+1} x g_{m+2}) or the rotated normal (2D: |cof(G) N| = |G tau|, tau = (N_1, -N_0)).
The second derivative splits into a positive semidefinite part Q1 (the change of the
unit normal) and an indefinite part Q2 (3D only); the "definiteness fix" the paper
refers to is read as dropping Q2 (hess_mode PSD).  EXACT keeps it.

Parity pins: central finite differences of Phi and of grad Phi, Hessian symmetry,
translation/rotation invariance of the forces, the closed form at F^ = I
(tests/test_oracle_energy.py); each term's value and first moment of its force under an
affine velocity field, which fixes the scale of e_J, e_sigma and D and the
symmetrization of the strain rate (tests/test_oracle_pins.py).
"""
from __future__ import annotations

import numpy as np

from . import bspline, transfer
from .transfer import _scatter

TERM_J, TERM_SURF, TERM_VISC = 1, 2, 4


def cof_normal_definition(G, N):
    """a = det(G) G^{-T} N, written as the paper writes it (J^ F^^{-T} dA)."""
    det = np.linalg.det(G)
    inv_t = np.transpose(np.linalg.inv(G), (0, 2, 1))
    return det[:, None] * np.einsum("rab,rb->ra", inv_t, N)


def _col(G, m):
    return G[:, :, m % 3]


def surface_grad(G, N):
    """Q = d|cof(G) N| / dG  (R, d, d)."""
    dim = G.shape[1]
    if dim == 2:
        tau = np.stack([N[:, 1], -N[:, 0]], 1)
        c = np.einsum("rab,rb->ra", G, tau)
        ch = c / np.linalg.norm(c, axis=1, keepdims=True)
        return ch[:, :, None] * tau[:, None, :]
    a = cof_normal_definition(G, N)
    ah = a / np.linalg.norm(a, axis=1, keepdims=True)
    Q = np.empty_like(G)
    for m in range(3):
        Q[:, :, m] = (N[:, (m + 2) % 3, None] * np.cross(_col(G, m + 1), ah)
                      + N[:, (m + 1) % 3, None] * np.cross(ah, _col(G, m + 2)))
    return Q


def surface_hessvec(G, N, dG, exact):
    """d/de Q(G + e dG) at e = 0 (EXACT), or its positive semidefinite part (PSD)."""
    dim = G.shape[1]
    if dim == 2:
        tau = np.stack([N[:, 1], -N[:, 0]], 1)
        c = np.einsum("rab,rb->ra", G, tau)
        cn = np.linalg.norm(c, axis=1, keepdims=True)
        ch = c / cn
        dc = np.einsum("rab,rb->ra", dG, tau)
        u = (dc - ch * np.sum(ch * dc, axis=1, keepdims=True)) / cn
        return u[:, :, None] * tau[:, None, :]
    a = cof_normal_definition(G, N)
    an = np.linalg.norm(a, axis=1, keepdims=True)
    ah = a / an
    da = np.zeros_like(a)
    for k in range(3):
        da += N[:, k, None] * (np.cross(_col(dG, k + 1), _col(G, k + 2))
                               + np.cross(_col(G, k + 1), _col(dG, k + 2)))
    u = (da - ah * np.sum(ah * da, axis=1, keepdims=True)) / an
    H = np.empty_like(G)
    for m in range(3):
        H[:, :, m] = (N[:, (m + 2) % 3, None] * np.cross(_col(G, m + 1), u)
                      + N[:, (m + 1) % 3, None] * np.cross(u, _col(G, m + 2)))
        if exact:
            H[:, :, m] += (N[:, (m + 2) % 3, None] * np.cross(_col(dG, m + 1), ah)
                           + N[:, (m + 1) % 3, None] * np.cross(ah, _col(dG, m + 2)))
    return H


# ---- fixed-corotated solid (Section 3.2.1) ---------------------------------------------
# psi^h(F) = mu^h sum_a (sigma_a - 1)^2 + lambda^h / 2 (J - 1)^2 = mu^h |F - R|^2 +
# lambda^h / 2 (J - 1)^2 with R the orthogonal polar factor of F (S = R^T F symmetric
# positive semidefinite, its eigenvalues the singular values).  Piola stress
# P = 2 mu (F - R) + lambda (J - 1) cof(F), cof(F) = J F^{-T}.

def polar(F):
    """Orthogonal polar factor R and S = R^T F (Q, d, d), from the SVD F = U Sigma V^T."""
    U, _, Vt = np.linalg.svd(F)
    R = U @ Vt
    return R, np.transpose(R, (0, 2, 1)) @ F


def cofactor(F):
    """det(F) F^{-T}."""
    return np.linalg.det(F)[:, None, None] * np.transpose(np.linalg.inv(F), (0, 2, 1))


def corotated_psi(F, mu, lam):
    R, _ = polar(F)
    J = np.linalg.det(F)
    return mu * np.sum((F - R) ** 2, axis=(1, 2)) + 0.5 * lam * (J - 1.0) ** 2


def corotated_P(F, mu, lam):
    R, _ = polar(F)
    J = np.linalg.det(F)
    return 2.0 * mu[:, None, None] * (F - R) + (lam * (J - 1.0))[:, None, None] * cofactor(F)


def corotated_dP(F, mu, lam, dF, exact):
    """dP = dP/dF : dF.  EXACT: the full derivative, with dR = R [w]x, w solving
    (tr(S) I - S) w = axial(R^T dF - dF^T R) (3D; 2D: w = (M_10 - M_01) / tr S), and
    d cof = (cof : dF) F^{-T} - cof dF^T F^{-T}.  PSD (the definiteness fix): the rotation
    held fixed and the (J - 1) d cof term dropped, 2 mu dF + lambda (cof : dF) cof, which
    is positive semidefinite."""
    C = cofactor(F)
    cdf = np.sum(C * dF, axis=(1, 2))
    out = 2.0 * mu[:, None, None] * dF + (lam * cdf)[:, None, None] * C
    if not exact:
        return out
    d = F.shape[1]
    R, S = polar(F)
    M = np.transpose(R, (0, 2, 1)) @ dF
    K = M - np.transpose(M, (0, 2, 1))
    trS = np.trace(S, axis1=1, axis2=2)
    if d == 2:
        w = K[:, 1, 0] / trS
        Om = np.zeros_like(F)
        Om[:, 0, 1] = -w
        Om[:, 1, 0] = w
    else:
        ax = np.stack([K[:, 2, 1], K[:, 0, 2], K[:, 1, 0]], axis=1)
        A = trS[:, None, None] * np.eye(3)[None] - S
        w = np.linalg.solve(A, ax[:, :, None])[:, :, 0]
        Om = np.zeros_like(F)
        Om[:, 0, 1], Om[:, 0, 2], Om[:, 1, 2] = -w[:, 2], w[:, 1], -w[:, 0]
        Om[:, 1, 0], Om[:, 2, 0], Om[:, 2, 1] = w[:, 2], -w[:, 1], w[:, 0]
    dR = R @ Om
    Finv_t = np.transpose(np.linalg.inv(F), (0, 2, 1))
    dC = cdf[:, None, None] * Finv_t - C @ np.transpose(dF, (0, 2, 1)) @ Finv_t
    J = np.linalg.det(F)
    return out - 2.0 * mu[:, None, None] * dR + (lam * (J - 1.0))[:, None, None] * dC


def point_gradient(field, idx, G):
    """sum_j field_j (x) grad N_j(x_q) for every quadrature point q: (Q, d, d)."""
    return np.einsum("qja,qjb->qab", field[idx], G)


def scatter_stress(S, idx, G, nn):
    """out_i = sum_q S_q grad N_i(x_q)."""
    return _scatter(idx, np.einsum("qab,qjb->qja", S, G), nn)


class Context:
    """Everything the momentum solve needs, frozen at the start of the step."""

    def __init__(self, P, surf, grid, setup, params):
        self.params = params
        self.dim, self.n, self.dx, self.dt = params["dim"], params["n"], params["dx"], params["dt"]
        self.nn = self.n ** self.dim
        self.pidx, self.pN, self.pG = bspline.stencil(P["x"], self.dx, self.n)
        self.sidx, self.sN, self.sG = bspline.stencil(surf["s"], self.dx, self.n)
        self.dA = surf["dA"]
        self.k = setup["k"]
        self.lam = params["bulk"]
        # solid particles (T below the melting point, with F given) take the fixed-corotated
        # term in place of the fluid's J term, and no viscosity
        self.solid = transfer.solid_mask(P["T"], params) if "F" in P else np.zeros(len(P["m"]), bool)
        liq = ~self.solid
        self.V0 = P["V0"] * liq
        self.V0s = P["V0"][self.solid]
        self.Fn = P["F"][self.solid] if "F" in P else np.zeros((0, params["dim"], params["dim"]))
        self.muh, self.lamh = transfer.lame_of_T(P["T"][self.solid], params)
        self.Jn = P["J"]
        self.Vn = setup["Vn"]
        self.mu = setup["mu"] * liq
        self.m = grid["m"]
        self.vn = setup["vn"]
        self.dof = setup["dof"]
        self.free = setup["free"]
        self.g = np.asarray(params["gravity"][: self.dim])
        self.mask = params["term_mask"]
        self.exact = params["hess_mode"] == 1

    # ---- energy ---------------------------------------------------------------
    def Jp(self, vhat):
        dv = point_gradient(vhat, self.pidx, self.pG)
        return (1.0 + self.dt * np.trace(dv, axis1=1, axis2=2)) * self.Jn

    def Fs(self, vhat):
        I = np.eye(self.dim)[None]
        return I + self.dt * point_gradient(vhat, self.sidx, self.sG)

    def Fsolid(self, vhat):
        """F_p = (I + dt grad v^(x_p)) F^n_p of the solid particles."""
        I = np.eye(self.dim)[None]
        sel = self.solid
        return (I + self.dt * point_gradient(vhat, self.pidx[sel], self.pG[sel])) @ self.Fn

    def psi_terms(self, vhat):
        """e_J, e_sigma and D at y = x + dt v^."""
        eJ = es = D = 0.0
        if self.mask & TERM_J:
            eJ = float(np.sum(0.5 * self.lam * (self.Jp(vhat) - 1.0) ** 2 * self.V0))
            if len(self.V0s):
                eJ += float(np.sum(self.V0s * corotated_psi(self.Fsolid(vhat), self.muh, self.lamh)))
        if self.mask & TERM_SURF and len(self.k):
            a = cof_normal_definition(self.Fs(vhat), self.dA)
            es = float(np.sum(self.k * np.linalg.norm(a, axis=1)))
        if self.mask & TERM_VISC:
            dv = point_gradient(vhat, self.pidx, self.pG)
            eps = 0.5 * (dv + np.transpose(dv, (0, 2, 1)))
            D = float(np.sum(0.5 * self.mu * self.Vn * np.sum(eps * eps, axis=(1, 2))))
        return eJ, es, D

    def Phi(self, vhat):
        eJ, es, D = self.psi_terms(vhat)
        d = self.dof
        kin = 0.5 * np.sum(self.m[d, None] * (vhat[d] - self.vn[d]) ** 2)
        grav = -self.dt * np.sum(self.m[d, None] * vhat[d] * self.g[None, :])
        return float(kin + grav + eJ + es + self.dt * D)

    # ---- gradient -------------------------------------------------------------
    def psi_grad(self, vhat):
        """d Psi / d v^ with Psi = e(x + dt v^) + dt D(v^), all nodes."""
        out = np.zeros((self.nn, self.dim))
        dt = self.dt
        I = np.eye(self.dim)[None]
        if self.mask & TERM_J:
            s = dt * self.lam * self.V0 * self.Jn * (self.Jp(vhat) - 1.0)
            out += scatter_stress(s[:, None, None] * I, self.pidx, self.pG, self.nn)
            if len(self.V0s):
                sel = self.solid
                Pk = corotated_P(self.Fsolid(vhat), self.muh, self.lamh)
                Sq = dt * self.V0s[:, None, None] * Pk @ np.transpose(self.Fn, (0, 2, 1))
                out += scatter_stress(Sq, self.pidx[sel], self.pG[sel], self.nn)
        if self.mask & TERM_SURF and len(self.k):
            Q = surface_grad(self.Fs(vhat), self.dA)
            out += scatter_stress(dt * self.k[:, None, None] * Q, self.sidx, self.sG, self.nn)
        if self.mask & TERM_VISC:
            dv = point_gradient(vhat, self.pidx, self.pG)
            eps = 0.5 * (dv + np.transpose(dv, (0, 2, 1)))
            out += scatter_stress(dt * (self.mu * self.Vn)[:, None, None] * eps, self.pidx, self.pG, self.nn)
        return out

    def grad_Phi(self, vhat):
        g = self.psi_grad(vhat)
        d = self.dof
        g[d] += self.m[d, None] * (vhat[d] - self.vn[d]) - self.dt * self.m[d, None] * self.g[None, :]
        return g

    # ---- Hessian-vector product -----------------------------------------------
    def psi_hessvec(self, vlin, w):
        out = np.zeros((self.nn, self.dim))
        dt = self.dt
        I = np.eye(self.dim)[None]
        if self.mask & TERM_J:
            dw = point_gradient(w, self.pidx, self.pG)
            s = dt * dt * self.lam * self.V0 * self.Jn ** 2 * np.trace(dw, axis1=1, axis2=2)
            out += scatter_stress(s[:, None, None] * I, self.pidx, self.pG, self.nn)
            if len(self.V0s):
                sel = self.solid
                dF = dt * dw[sel] @ self.Fn
                dP = corotated_dP(self.Fsolid(vlin), self.muh, self.lamh, dF, self.exact)
                Sq = dt * self.V0s[:, None, None] * dP @ np.transpose(self.Fn, (0, 2, 1))
                out += scatter_stress(Sq, self.pidx[sel], self.pG[sel], self.nn)
        if self.mask & TERM_SURF and len(self.k):
            dG = dt * point_gradient(w, self.sidx, self.sG)
            H = surface_hessvec(self.Fs(vlin), self.dA, dG, self.exact)
            out += scatter_stress(dt * self.k[:, None, None] * H, self.sidx, self.sG, self.nn)
        if self.mask & TERM_VISC:
            dw = point_gradient(w, self.pidx, self.pG)
            eps = 0.5 * (dw + np.transpose(dw, (0, 2, 1)))
            out += scatter_stress(dt * (self.mu * self.Vn)[:, None, None] * eps, self.pidx, self.pG, self.nn)
        return out

    def hessvec(self, vlin, w, alpha_mass=1.0):
        """alpha M w + d2Psi/dv^2 (v_lin) w over all nodes (no projection)."""
        out = self.psi_hessvec(vlin, w)
        d = self.dof
        out[d] += alpha_mass * self.m[d, None] * w[d]
        return out

    def project(self, v):
        out = np.where(self.free, v, 0.0)
        return out

    def jacobi_diag(self):
        """Diagonal of M + dt^2 d2e_J + dt C (the surface term is left out)."""
        dt = self.dt
        diag = np.zeros((self.nn, self.dim))
        if self.mask & TERM_J:
            c = dt * dt * self.lam * self.V0 * self.Jn ** 2
            diag += _scatter(self.pidx, c[:, None, None] * self.pG ** 2, self.nn)
        if self.mask & TERM_VISC:
            c = dt * self.mu * self.Vn
            g2 = np.sum(self.pG ** 2, axis=2, keepdims=True)
            diag += _scatter(self.pidx, c[:, None, None] * 0.5 * (g2 + self.pG ** 2), self.nn)
        diag[self.dof] += self.m[self.dof, None]
        return np.where(self.free, diag, 1.0)
