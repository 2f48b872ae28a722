"""Particle-grid transfers (Sections 4.2 and 5) and the grid set-up between them.

P2G (Section 4.2), over the split collection of each particle (x_p and, for r in Pi_p,
s_r and b_r), all with the parent's m~_p, v_p, A_p:
    m_i      = sum_q m~ N_i(x_q)
    (mv)_i   = sum_q m~ N_i(x_q) (v_p + A_p (x_i - x_q))
Temperature P2G uses the interior particles only with their unsplit mass; where no
interior particle reaches a node, the interior temperatures are extrapolated as
constants onto the split members (the paper's "constant extrapolation" remark):
    W_i  = sum_p m_p N_i(x_p),   WT_i = sum_p m_p N_i(x_p) (T_p + (x_i - x_p) . grad T_p)
    E_i  = sum_r m~_p(r) (N_i(s_r) + N_i(b_r)),   ET_i = same weights times T_p(r)
    T^n_i = WT_i / W_i where W_i > 0, else ET_i / E_i.

Grid set-up: the degrees of freedom are the nodes with mass (Section 4.1: only grid
nodes with mass carry the solution); v^n_i = (mv)_i / m_i; constrained components are
slip walls (node layers at the domain faces) and, optionally, the normal component of
nodes inside a static slab box; k_r = gamma(T^s_r) with T^s_r = sum_i N_i(s_r) T^n_i
(Section 4.3.1, last remark) or a per-label constant (Section 3.6); mu_p = mu(T_p);
V^n_p = J_p V^0_p.

G2P with merge (Section 5): for every interior particle,
    p_ip = m~_p [N_i(x_p) + sum_{r in Pi_p} (N_i(s_r) + N_i(b_r))] v^_i
    v_p  = (1/m_p) sum_i p_ip
    t_p  = sum_i p_ip (x_i - x_p)^T,   A_p = 4 / (m_p dx^2) t_p
    T_p  = sum_i N_i(x_p) T^_i,   grad T_p = sum_i T^_i grad N_i(x_p)
and (not stated in the paper, read as the trace form at the solution) J_p <- (1 + dt sum_i v^_i . grad N_i(x_p)) J_p, x_p <- x_p + dt v_p.

Parity pins: conservation of mass, momentum and APIC angular momentum through P2G and
G2P with split groups, the unsplit splat written out per particle, linear temperature
reproduction (tests/test_oracle_transfer.py); k_r of a linear temperature field, G2P of
an affine grid velocity in closed form (v, A with the split groups' second moments, J,
x), the slip-wall and slab masks and the label table on enumerated grids
(tests/test_oracle_pins.py).
"""
from __future__ import annotations

import numpy as np

from . import bspline


def _scatter(idx, vals, nn):
    """out[i] = sum over (p,j) with idx[p,j] = i of vals[p,j,...] (a plain bincount)."""
    flat = idx.ravel()
    if vals.ndim == 2:
        return np.bincount(flat, weights=vals.ravel(), minlength=nn)
    tail = vals.shape[2:]
    v = vals.reshape(vals.shape[0] * vals.shape[1], -1)
    out = np.stack([np.bincount(flat, weights=v[:, c], minlength=nn) for c in range(v.shape[1])], 1)
    return out.reshape((nn,) + tail)


def p2g(P, surf, split, params):
    dim, n, dx = params["dim"], params["n"], params["dx"]
    nn = n ** dim
    x, v, A, m, T, gT = P["x"], P["v"], P["A"], P["m"], P["T"], P["gradT"]
    mt = split["mtilde"]
    idx, N, _ = bspline.stencil(x, dx, n)
    xi = (bspline.node_multi_index(idx.ravel(), n, dim).reshape(idx.shape + (dim,)) + 0.5) * dx
    rel = xi - x[:, None, :]                                     # x_i - x_p
    vel = v[:, None, :] + np.einsum("pab,pjb->pja", A, rel)      # v_p + A_p (x_i - x_p)
    mass = _scatter(idx, mt[:, None] * N, nn)
    mom = _scatter(idx, (mt[:, None] * N)[..., None] * vel, nn)
    W = _scatter(idx, m[:, None] * N, nn)
    WT = _scatter(idx, m[:, None] * N * (T[:, None] + np.einsum("pja,pa->pj", rel, gT)), nn)
    E = np.zeros(nn)
    ET = np.zeros(nn)
    par = split["parent"]
    if len(par):
        for q in (surf["s"], split["b"]):
            qi, qN, _ = bspline.stencil(q, dx, n)
            qx = (bspline.node_multi_index(qi.ravel(), n, dim).reshape(qi.shape + (dim,)) + 0.5) * dx
            qvel = v[par][:, None, :] + np.einsum("pab,pjb->pja", A[par], qx - q[:, None, :])
            w = mt[par][:, None] * qN
            mass += _scatter(qi, w, nn)
            mom += _scatter(qi, w[..., None] * qvel, nn)
            E += _scatter(qi, w, nn)
            ET += _scatter(qi, w * T[par][:, None], nn)
    return dict(m=mass, mv=mom, W=W, WT=WT, E=E, ET=ET)


def constraint_mask(params, dof):
    """free[i, a] is True when velocity component a of node i is an unknown."""
    dim, n, dx = params["dim"], params["n"], params["dx"]
    nn = n ** dim
    mi = bspline.node_multi_index(np.arange(nn), n, dim)
    free = np.repeat(dof[:, None], dim, axis=1)
    L = params["wall_layers"]
    if L > 0:
        wall = (mi < L) | (mi >= n - L)
        free &= ~wall
    if params["slab"]:
        xi = (mi + 0.5) * dx
        lo = np.asarray(params["slab_lo"][:dim])
        hi = np.asarray(params["slab_hi"][:dim])
        inside = np.all((xi >= lo) & (xi < hi), axis=1)
        free[inside, params["slab_axis"]] = False
    return free


def gamma_of_T(T, params):
    return np.clip(params["g0"] + params["g1"] * (T - params["gT0"]), params["gmin"], params["gmax"])


def solid_mask(T, params):
    """Phase of each particle (Section 3.5): solid below the melting point."""
    return np.asarray(T) < params.get("T_melt", -np.inf)


def lame_of_T(T, params):
    """mu^h and lambda^h of the solid (Section 3.5 lets them vary with temperature without
    a form; read as the viscosity's form, (muh0, lamh0) exp(-kh (T - Th0)))."""
    f = np.exp(-params.get("kh", 0.0) * (np.asarray(T) - params.get("Th0", 0.0)))
    return params.get("muh0", 0.0) * f, params.get("lamh0", 0.0) * f


def mu_of_T(T, params):
    if params["mu0"] == 0.0:
        return np.zeros_like(T)
    return params["mu0"] * np.exp(-params["mu_k"] * (T - params["mu_T0"]))


def grid_setup(P, surf, split, grid, params):
    dim, n, dx = params["dim"], params["n"], params["dx"]
    m = grid["m"]
    dof = m > 0
    vn = np.zeros_like(grid["mv"])
    vn[dof] = grid["mv"][dof] / m[dof][:, None]
    Tn = np.zeros_like(m)
    hasW = grid["W"] > 0
    Tn[hasW] = grid["WT"][hasW] / grid["W"][hasW]
    useE = dof & ~hasW & (grid["E"] > 0)
    Tn[useE] = grid["ET"][useE] / grid["E"][useE]
    free = constraint_mask(params, dof)
    s = surf["s"]
    if params["gamma_by_label"] == 1:
        k = np.asarray(params["gamma_label"], np.float64)[surf["label"]]
    else:
        if len(s):
            si, sN, _ = bspline.stencil(s, dx, n)
            Ts = np.sum(sN * Tn[si], axis=1)
        else:
            Ts = np.zeros(0)
        k = gamma_of_T(Ts, params)
        if params["gamma_by_label"] == 2:
            # free surface (label 1) by temperature; samples against the container's
            # walls (label 0) take the constant gamma_label[0]
            k = np.where(surf["label"] == 1, k, params["gamma_label"][0])
    mu = mu_of_T(P["T"], params)
    Vn = P["J"] * P["V0"]
    return dict(dof=dof, free=free, vn=vn, Tn=Tn, k=k, mu=mu, Vn=Vn)


def g2p(P, surf, split, vhat, That, params):
    """Returns the new particle state (a new dict) after G2P, merge and advection."""
    dim, n, dx, dt = params["dim"], params["n"], params["dx"], params["dt"]
    x, m = P["x"], P["m"]
    mt = split["mtilde"]
    par = split["parent"]

    def moments(q, ref):
        """sum_i N_i(q) v^_i and sum_i N_i(q) v^_i (x_i - ref)^T."""
        qi, qN, _ = bspline.stencil(q, dx, n)
        xi = (bspline.node_multi_index(qi.ravel(), n, dim).reshape(qi.shape + (dim,)) + 0.5) * dx
        vv = vhat[qi]                                                # (Q, 3^d, d)
        mom = np.einsum("qj,qja->qa", qN, vv)
        aff = np.einsum("qj,qja,qjb->qab", qN, vv, xi - ref[:, None, :])
        return mom, aff

    mom, aff = moments(x, x)
    mom = mom * mt[:, None]
    aff = aff * mt[:, None, None]
    if len(par):
        for q in (surf["s"], split["b"]):
            qm, qa = moments(q, x[par])
            w = mt[par]
            np.add.at(mom, par, w[:, None] * qm)
            np.add.at(aff, par, w[:, None, None] * qa)
    vnew = mom / m[:, None]
    Anew = aff * (4.0 / (m * dx * dx))[:, None, None]
    idx, N, G = bspline.stencil(x, dx, n)
    Tnew = np.sum(N * That[idx], axis=1)
    gTnew = np.einsum("pj,pja->pa", That[idx], G)
    div = np.einsum("pja,pja->p", vhat[idx], G)
    Jnew = (1.0 + dt * div) * P["J"]
    out = dict(P)
    if "F" in P:
        # solids carry F: F <- (I + dt grad v^(x_p)) F, J = det F
        solid = solid_mask(P["T"], params)
        dv = np.einsum("pja,pjb->pab", vhat[idx][solid], G[solid])
        Fnew = P["F"].copy()
        Fnew[solid] = np.einsum("pab,pbc->pac", np.eye(dim)[None] + dt * dv, P["F"][solid])
        Jnew[solid] = np.linalg.det(Fnew[solid])
        out["F"] = Fnew
    out.update(v=vnew, A=Anew, T=Tnew, gradT=gTnew, J=Jnew, x=x + dt * vnew)
    return out


def phase_change(T_old, P, params):
    """Phase change at T_melt (Section 3.5): a solid particle whose temperature reaches
    T_melt becomes liquid with J = 1; a liquid particle that cools below it becomes solid
    with F = I (and J = det F = 1).  P is updated in place."""
    if "F" not in P:
        return P
    was = solid_mask(T_old, params)
    now = solid_mask(P["T"], params)
    flip = was != now
    if np.any(flip):
        P["J"] = P["J"].copy()
        P["F"] = P["F"].copy()
        P["J"][flip] = 1.0
        P["F"][flip] = np.eye(P["F"].shape[1])
    return P
