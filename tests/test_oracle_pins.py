"""Closed-form pins of oracle functions that the invariance and finite-difference tests
leave free (a dropped factor, a wrong argument or a missing symmetrization would pass
those).  Every pin states a value that follows from the paper's formulas and the
B-spline moment identities alone, and each is shown to fail on a planted mistake:

  k_r = gamma(T^s_r), T^s_r interpolated from the grid T^n (Section 4.3.1, last remark;
      Section 4.3.2 temperature transfer): a linear T_p with matching grad T_p puts
      T^n_i = T(x_i) wherever W_i > 0, so k_r = gamma(T(s_r)) exactly;
  G2P with merge (Section 5): an affine grid velocity v^_i = B x_i + c gives
      v_p = B x_p + c, A_p = B (I + 8/((2|Pi_p|+1) dx^2) sum_r d_r d_r^T) with
      d_r = s_r - x_p (b_r = x_p - d_r), J <- (1 + dt tr B) J and x <- x + dt v_p;
  the conduction matrix (Section 4.3.2): for T^_i = a . x_i + t0,
      sum_i x_i (L T^)_i = K a sum_p V^n_p, and the Robin matrix
      sum_i x_i (R T^)_i = sum_r h |dA_r| s_r T^(s_r);
  the viscous term (eq. disc_force): for v^_i = B x_i + c every eps_p = sym(B), so
      D = sum_p mu_p/2 V^n_p |sym B|^2 and sum_i (dD/dv^_i) x_i^T = (sum_p mu_p V^n_p) sym B;
      a rigid rotation gives D = 0 and no force;
  the J term and the surface term at the same affine field: sum_i (de/dy_i) x_i^T equals
      sum_p lambda V^0_p J^n_p (J_p - 1) I and sum_r k_r d|cof(G) dA_r|/dG at G = I + dt B
      (the latter against central differences of |det(G) G^-T dA| over G's nine entries);
  the slip-wall and slab constraints and the label -> gamma map, on enumerated small grids.
"""
import numpy as np
import pytest

import mpm_scenes as sc
from oracle import bspline, energy, resample, sampler, solve, transfer


def _affine(dim, seed):
    rng = np.random.default_rng(seed)
    B = rng.normal(size=(dim, dim)) * 2.0
    c = rng.normal(size=dim) * 0.3
    return B, c


def _state(dim, seed, count=None, nsurf=80, **kw):
    count = count or (2500 if dim == 3 else 1200)
    prm = dict(mu0=0.7, mu_k=0.01, mu_T0=300.0, g0=0.05, g1=-2e-4, gT0=300.0, gmin=0.0, gmax=1.0,
               heat=1, cp=2.0, K=0.3, h=4.0, T_amb=330.0, b=3.0, dt=2e-3)
    prm.update(kw)
    S = sc.random_scene(dim, 16, count, seed, box=(0.25, 0.75), **prm)
    P, p = S["particles"], S["params"]
    surf = sc.random_surface(P, nsurf, seed, dx=p["dx"], spread=0.8)
    return P, p, surf


def _prepare(P, p, surf):
    sp = resample.split(P, surf)
    g = transfer.p2g(P, surf, sp, p)
    st = transfer.grid_setup(P, surf, sp, g, p)
    return sp, g, st


# ---- k_r from the grid temperature ---------------------------------------------------

def _kr_case(dim, seed):
    P, p, surf = _state(dim, seed)
    a = np.array([30.0, -20.0, 10.0])[:dim]
    t0 = 310.0
    P["T"] = t0 + P["x"] @ a
    P["gradT"] = np.tile(a, (len(P["x"]), 1))
    sp, g, st = _prepare(P, p, surf)
    sidx, _, _ = bspline.stencil(surf["s"], p["dx"], p["n"])
    ok = np.all(g["W"][sidx] > 0, axis=1)           # every stencil node carries interior mass
    expect = np.clip(p["g0"] + p["g1"] * (t0 + surf["s"] @ a - p["gT0"]), p["gmin"], p["gmax"])
    return P, p, surf, sp, st, ok, expect


@pytest.mark.parametrize("dim", [2, 3])
def test_kr_is_gamma_of_interpolated_grid_temperature(dim):
    P, p, surf, sp, st, ok, expect = _kr_case(dim, 3 + dim)
    assert ok.sum() >= 40
    err = np.max(np.abs(st["k"][ok] - expect[ok]) / np.abs(expect[ok]))
    assert err < 1e-12, err


def test_kr_pin_fails_on_parent_temperature():
    """Planted mistake: k_r from the parent's T_p instead of the grid's T^n at s_r."""
    P, p, surf, sp, st, ok, expect = _kr_case(3, 5)
    planted = transfer.gamma_of_T(P["T"][sp["parent"]], p)
    assert np.max(np.abs(planted[ok] - expect[ok]) / np.abs(expect[ok])) > 1e-6


def test_kr_clamp_and_label_map():
    """gamma(T) = clamp(g0 + g1 (T - gT0), gmin, gmax), and the label table of Section 3.6:
    hand-built samples with labels (0, 1, 1, 0) take (gamma_0, gamma_1, gamma_1, gamma_0)."""
    p = sc.make_params(dim=2, n=16, g0=0.05, g1=-1e-3, gT0=300.0, gmin=0.01, gmax=0.07)
    T = np.array([300.0, 250.0, 400.0, 310.0])
    assert np.allclose(transfer.gamma_of_T(T, p), [0.05, 0.07, 0.01, 0.04], rtol=0, atol=1e-15)
    P = sc.particles_from_positions(np.array([[0.5, 0.5], [0.52, 0.5]]), 2, p["dx"])
    surf = dict(s=np.array([[0.48, 0.5], [0.53, 0.51], [0.5, 0.47], [0.51, 0.53]]),
                dA=np.full((4, 2), 0.01), label=np.array([0, 1, 1, 0], np.int32))
    p2 = dict(p, gamma_by_label=1, gamma_label=(0.072, 0.02, 0.0, 0.0))
    sp, g, st = _prepare(P, p2, surf)
    assert np.array_equal(st["k"], [0.072, 0.02, 0.02, 0.072])


@pytest.mark.parametrize("dim", [2, 3])
def test_kr_free_surface_and_wall_samples(dim):
    """gamma_by_label 2 (the cavity's container walls): samples labelled 1 take gamma of
    the interpolated grid temperature as in the pin above, the others gamma_label[0]."""
    P, p, surf, sp, st, ok, expect = _kr_case(dim, 7 + dim)
    lab = (np.arange(len(surf["s"])) % 3 == 0).astype(np.int32)
    surf2 = dict(surf, label=lab)
    p2 = dict(p, gamma_by_label=2, gamma_label=(0.013, 0.5, 0.0, 0.0))
    _, _, st2 = _prepare(P, p2, surf2)
    on = ok & (lab == 1)
    assert on.sum() >= 10 and (lab == 0).sum() >= 10
    assert np.max(np.abs(st2["k"][on] - expect[on]) / np.abs(expect[on])) < 1e-12
    assert np.all(st2["k"][lab == 0] == 0.013)


def test_sampler_labels_the_wetted_base():
    """Contact scene (Section 6.5 analog): samples on the cap's top are liquid-air (label 0),
    samples on the flat base resting on the slab are solid-liquid (label 1)."""
    S = sc.contact3d(n=64, radius=0.08)
    P, p = S["particles"], S["params"]
    surf = sampler.sample_surface(P["x"], p)
    y = surf["s"][:, 1]
    yb = 6.0 / 64
    top = y > yb + 0.04
    base = (y < yb) & (np.abs(surf["s"][:, 0] - 0.5) < 0.05) & (np.abs(surf["s"][:, 2] - 0.5) < 0.05)
    assert top.sum() > 100 and base.sum() > 20
    assert np.all(surf["label"][top] == 0)
    assert np.all(surf["label"][base] == 1)


# ---- G2P with merge under an affine grid velocity ------------------------------------

def _g2p_case(dim, seed):
    P, p, surf = _state(dim, seed, count=300 if dim == 3 else 200, nsurf=120)
    sp, g, st = _prepare(P, p, surf)
    B, c = _affine(dim, seed + 1)
    xi = bspline.node_positions(p["n"], dim)
    vhat = xi @ B.T + c
    out = transfer.g2p(P, surf, sp, vhat, st["Tn"], p)
    x, dx, dt = P["x"], p["dx"], p["dt"]
    v_exp = x @ B.T + c
    D = np.zeros((len(x), dim, dim))
    d = surf["s"] - x[sp["parent"]]
    np.add.at(D, sp["parent"], d[:, :, None] * d[:, None, :])
    fac = 8.0 / ((2 * sp["count"] + 1) * dx * dx)
    A_exp = np.einsum("ab,pbc->pac", B, np.eye(dim)[None] + fac[:, None, None] * D)
    J_exp = (1.0 + dt * np.trace(B)) * P["J"]
    x_exp = x + dt * v_exp
    return P, sp, out, v_exp, A_exp, J_exp, x_exp


@pytest.mark.parametrize("dim", [2, 3])
def test_g2p_affine_field_closed_form(dim):
    P, sp, out, v_exp, A_exp, J_exp, x_exp = _g2p_case(dim, 21 + dim)
    assert np.sum(sp["count"] > 0) >= 20 and np.sum(sp["count"] == 0) >= 20
    assert np.max(np.abs(out["v"] - v_exp)) <= 1e-13 * np.max(np.abs(v_exp))
    assert np.max(np.abs(out["A"] - A_exp)) <= 1e-12 * np.max(np.abs(A_exp))
    assert np.max(np.abs(out["J"] - J_exp)) <= 1e-14
    assert np.max(np.abs(out["x"] - x_exp)) <= 1e-15
    # unsplit particles: A_p = B exactly as in APIC
    un = sp["count"] == 0
    assert np.allclose(out["A"][un], A_exp[un][:1].repeat(un.sum(), 0), rtol=0, atol=1e-12 * np.abs(A_exp).max())


def test_g2p_pin_fails_on_planted_mistakes():
    P, sp, out, v_exp, A_exp, J_exp, x_exp = _g2p_case(3, 24)
    # J advanced without the factor J^n
    assert np.max(np.abs(out["J"] / P["J"] - J_exp)) > 1e-3
    # A_p normalized by the split mass m~_p instead of m_p
    wrong = out["A"] * (2 * sp["count"] + 1)[:, None, None]
    assert np.max(np.abs(wrong - A_exp)) > 1e-3 * np.abs(A_exp).max()
    # balance points left out of the merge: the split particles' A loses its d d^T term
    split = sp["count"] > 0
    assert np.max(np.abs(A_exp[split] - A_exp[~split][:1])) > 1e-3 * np.abs(A_exp).max()


# ---- heat: conduction and Robin matrices ---------------------------------------------

def _heat_case(dim, seed, **kw):
    P, p, surf = _state(dim, seed, count=400 if dim == 3 else 250, **kw)
    sp, g, st = _prepare(P, p, surf)
    return P, p, surf, solve.Heat(P, surf, g, st, p), st


@pytest.mark.parametrize("dim", [2, 3])
def test_conduction_matrix_scale(dim):
    P, p, surf, H, st = _heat_case(dim, 31 + dim, h=0.0)
    xi = bspline.node_positions(p["n"], dim)
    a = np.array([4.0, -3.0, 2.0])[:dim]
    T = xi @ a                      # no constant offset: c_p/dt m T would swamp L T in the difference
    LT = np.where(H.dof, H.apply(T) - H.c * H.m * T, 0.0)
    lhs = xi.T @ LT
    Vn = P["J"] * P["V0"]
    rhs = p["K"] * a * Vn.sum()
    assert np.allclose(lhs, rhs, rtol=1e-10, atol=0)
    assert abs(LT.sum()) <= 1e-11 * np.abs(LT).sum()
    # planted: V^0 in place of V^n (J != 1 here), or K/2
    assert np.max(np.abs(p["K"] * a * P["V0"].sum() - rhs)) > 1e-4 * np.abs(rhs).max()
    H2 = solve.Heat(P, surf, _prepare(P, p, surf)[1], st, dict(p, K=p["K"] / 2))
    LT2 = np.where(H2.dof, H2.apply(T) - H2.c * H2.m * T, 0.0)
    assert np.max(np.abs(xi.T @ LT2 - rhs)) > 0.4 * np.abs(rhs).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_robin_matrix_and_rhs_scale(dim):
    P, p, surf, H, st = _heat_case(dim, 41 + dim, K=0.0, H=5.0)
    xi = bspline.node_positions(p["n"], dim)
    a = np.array([4.0, -3.0, 2.0])[:dim]
    T = xi @ a + 305.0
    RT = np.where(H.dof, H.apply(T) - H.c * H.m * T, 0.0)
    area = np.linalg.norm(surf["dA"], axis=1)
    Ts = surf["s"] @ a + 305.0
    assert np.isclose(RT.sum(), np.sum(p["h"] * area * Ts), rtol=1e-12)
    assert np.allclose(xi.T @ RT, (p["h"] * area * Ts) @ surf["s"], rtol=1e-11)
    # right side: c_p/dt m T^n + (h T_amb + b)|dA| at the samples + H V^n at the particles
    Vn = P["J"] * P["V0"]
    src = H.rhs - np.where(H.dof, H.c * H.m * st["Tn"], 0.0)
    assert np.isclose(src.sum(), np.sum((p["h"] * p["T_amb"] + p["b"]) * area) + p["H"] * Vn.sum(), rtol=1e-12)
    assert np.allclose(xi.T @ src, ((p["h"] * p["T_amb"] + p["b"]) * area) @ surf["s"] + p["H"] * (Vn @ P["x"]),
                       rtol=1e-11)


# ---- momentum terms under an affine velocity field ------------------------------------

def _ctx(dim, seed, mask):
    P, p, surf = _state(dim, seed, count=300 if dim == 3 else 200, nsurf=60, term_mask=mask)
    sp, g, st = _prepare(P, p, surf)
    return P, p, surf, energy.Context(P, surf, g, st, p)


def _sym(B):
    return 0.5 * (B + B.T)


@pytest.mark.parametrize("dim", [2, 3])
def test_viscous_term_closed_form(dim):
    P, p, surf, ctx = _ctx(dim, 51 + dim, mask=4)
    xi = bspline.node_positions(p["n"], dim)
    B, c = _affine(dim, 52)
    v = xi @ B.T + c
    mu = p["mu0"] * np.exp(-p["mu_k"] * (P["T"] - p["mu_T0"]))
    Vn = P["J"] * P["V0"]
    _, _, D = ctx.psi_terms(v)
    assert np.isclose(D, 0.5 * np.sum(mu * Vn) * np.sum(_sym(B) ** 2), rtol=1e-12)
    g = ctx.psi_grad(v)                                     # dt dD/dv^
    assert np.allclose(g.T @ xi, p["dt"] * np.sum(mu * Vn) * _sym(B), rtol=1e-11, atol=0)
    # planted: strain rate without the symmetrization
    assert not np.isclose(0.5 * np.sum(mu * Vn) * np.sum(B ** 2), D, rtol=1e-3)
    # a rigid rotation dissipates nothing and exerts no viscous force
    W = B - B.T
    vr = xi @ W.T + c
    _, _, Dr = ctx.psi_terms(vr)
    gr = ctx.psi_grad(vr)
    assert abs(Dr) <= 1e-13 * abs(D)
    assert np.max(np.abs(gr)) <= 1e-12 * np.max(np.abs(g))


@pytest.mark.parametrize("dim", [2, 3])
def test_J_term_closed_form(dim):
    P, p, surf, ctx = _ctx(dim, 61 + dim, mask=1)
    xi = bspline.node_positions(p["n"], dim)
    B, c = _affine(dim, 62)
    B *= 0.1
    v = xi @ B.T + c
    Jp = (1.0 + p["dt"] * np.trace(B)) * P["J"]
    eJ, _, _ = ctx.psi_terms(v)
    assert np.isclose(eJ, np.sum(0.5 * p["bulk"] * (Jp - 1) ** 2 * P["V0"]), rtol=1e-12)
    g = ctx.psi_grad(v)
    s = np.sum(p["bulk"] * P["V0"] * P["J"] * (Jp - 1.0))
    assert np.allclose(g.T @ xi, p["dt"] * s * np.eye(dim), rtol=1e-11, atol=1e-12 * abs(p["dt"] * s))


def _cof_norm(G, N):
    return np.linalg.norm(np.linalg.det(G) * np.linalg.inv(G).T @ N)


@pytest.mark.parametrize("dim", [2, 3])
def test_surface_term_closed_form(dim):
    P, p, surf, ctx = _ctx(dim, 71 + dim, mask=2)
    xi = bspline.node_positions(p["n"], dim)
    B, c = _affine(dim, 72)
    B *= 20.0
    v = xi @ B.T + c
    G = np.eye(dim) + p["dt"] * B
    k, N = ctx.k, surf["dA"]
    _, es, _ = ctx.psi_terms(v)
    assert np.isclose(es, sum(k[r] * _cof_norm(G, N[r]) for r in range(len(k))), rtol=1e-12)
    # d|cof(G) N|/dG by central differences over the entries of G
    Q = np.zeros((dim, dim))
    h = 1e-6
    for a in range(dim):
        for b in range(dim):
            E = np.zeros((dim, dim))
            E[a, b] = h
            Q[a, b] = sum(k[r] * (_cof_norm(G + E, N[r]) - _cof_norm(G - E, N[r])) for r in range(len(k))) / (2 * h)
    g = ctx.psi_grad(v)
    assert np.allclose(g.T @ xi, p["dt"] * Q, rtol=1e-7, atol=1e-8 * np.abs(p["dt"] * Q).max())


# ---- constraints on enumerated grids --------------------------------------------------

def test_wall_layers_enumerated():
    """Slip walls, two node layers (R10): on n = 8 the component a is free exactly on
    i_a in {2, 3, 4, 5}."""
    p = sc.make_params(dim=3, n=8, wall_layers=2)
    free = transfer.constraint_mask(p, np.ones(8 ** 3, bool))
    mi = bspline.node_multi_index(np.arange(8 ** 3), 8, 3)
    for a in range(3):
        assert set(np.unique(mi[free[:, a], a])) == {2, 3, 4, 5}
        assert set(np.unique(mi[~free[:, a], a])) == {0, 1, 6, 7}
    assert np.sum(np.all(free, axis=1)) == 4 ** 3
    # planted: one layer too many fixes 2 more indices per axis
    p3 = dict(p, wall_layers=3)
    assert np.sum(np.all(transfer.constraint_mask(p3, np.ones(8 ** 3, bool)), axis=1)) != 4 ** 3


def test_slab_box_enumerated():
    """Static slab y in [2dx, 6dx), x, z in [2dx, 1-2dx) on n = 16: the nodes with
    i_0, i_2 in 2..13 and i_1 in 2..5 have v_y fixed; nothing else is constrained."""
    n = 16
    dx = 1.0 / n
    p = sc.make_params(dim=3, n=n, slab=1, slab_axis=1, slab_lo=(2 * dx, 2 * dx, 2 * dx),
                       slab_hi=(1 - 2 * dx, 6 * dx, 1 - 2 * dx))
    dof = np.ones(n ** 3, bool)
    dof[5] = False                                    # a node without mass is never free
    free = transfer.constraint_mask(p, dof)
    fixed = {(i0, i1, i2) for i0 in range(2, 14) for i1 in range(2, 6) for i2 in range(2, 14)}
    mi = bspline.node_multi_index(np.arange(n ** 3), n, 3)
    got = {tuple(m) for m in mi[~free[:, 1] & dof]}
    assert got == fixed
    assert np.all(free[dof][:, [0, 2]])
    assert not np.any(free[5])


def test_collision_plane_coulomb_closed_form():
    """Collision object y < 0.5 with friction mu (the ramps' mechanism, Section 6.3): a node
    inside moving in (v_n < 0) loses its normal part and its tangential part shrinks by
    mu |v_n| (to zero when that is not positive); nodes moving out, and nodes outside, keep
    v^.  Planted mistake: friction added with the wrong sign gives |v_t| + mu |v_n|."""
    p = sc.make_params(dim=2, n=16, planes=(((0.0, 0.5, 0.0), (0.0, 1.0, 0.0), 0.5),))
    xi = (np.stack(np.meshgrid(np.arange(16), np.arange(16), indexing="xy"), -1).reshape(-1, 2) + 0.5) / 16
    below = np.nonzero(xi[:, 1] < 0.5)[0]
    above = np.nonzero(xi[:, 1] > 0.5)[0]
    v = np.zeros((256, 2))
    cases = [(below[3], (1.0, -1.0), (0.5, 0.0)), (below[7], (0.3, -1.0), (0.0, 0.0)),
             (below[9], (-2.0, -2.0), (-1.0, 0.0)), (below[11], (1.0, 1.0), (1.0, 1.0)),
             (above[5], (1.0, -1.0), (1.0, -1.0))]
    for k, vin, _ in cases:
        v[k] = vin
    out = solve.collide(v, p)
    for k, _, vout in cases:
        assert np.allclose(out[k], vout, rtol=0, atol=1e-15), (k, out[k], vout)
    p0 = dict(p, planes=(((0.0, 0.5, 0.0), (0.0, 1.0, 0.0), 0.0),))
    assert np.allclose(solve.collide(v, p0)[below[3]], (1.0, 0.0), rtol=0, atol=1e-15)
    vt, vn, mu = 1.0, -1.0, 0.5
    assert abs((vt - mu * vn) - out[below[3]][0]) > 0.5   # the planted sign misses the pin
