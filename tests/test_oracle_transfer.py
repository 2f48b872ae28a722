"""Pins of the split (Sections 4.1.2-4.1.3), P2G (Section 4.2) and G2P/merge (Section 5):
eq. cons_mom, exact conservation of mass, linear and angular momentum, reduction to the
standard APIC splat when no particle is split, and linear temperature reproduction."""
import numpy as np
import pytest

import mpm_scenes as sc
from oracle import bspline, resample, transfer


def _scene(dim, seed, count=40, nsurf=30):
    S = sc.random_scene(dim, 16, count, seed)
    P, p = S["particles"], S["params"]
    surf = sc.random_surface(P, nsurf, seed, dx=p["dx"], spread=0.8)
    return P, p, surf


def cross_z(a, b):
    return a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]


def ang_mom(x, mv):
    if x.shape[1] == 2:
        return np.array([np.sum(cross_z(x, mv))])
    return np.cross(x, mv).sum(0)


def apic_spin(m, A, dx):
    """(dx^2/4) sum_p m_p (eps_abc A_p,cb)_a: the angular momentum of the affine modes."""
    if A.shape[1] == 2:
        return np.array([np.sum(m * (A[:, 1, 0] - A[:, 0, 1]))]) * dx * dx / 4
    s = np.stack([A[:, 2, 1] - A[:, 1, 2], A[:, 0, 2] - A[:, 2, 0], A[:, 1, 0] - A[:, 0, 1]], 1)
    return (m[:, None] * s).sum(0) * dx * dx / 4


def test_parents_match_bruteforce_and_ties():
    rng = np.random.default_rng(0)
    # particles on distinct points of a 1/64 lattice, so exact dyadic ties can be planted
    cells = rng.choice(40 ** 3, size=300, replace=False)
    x = (np.stack([cells % 40, (cells // 40) % 40, cells // 1600], 1) + 12) / 64.0
    s = rng.uniform(0.2, 0.8, size=(500, 3))
    h = 1.0 / 1024
    # tie partners: particle 300+k sits 2h from particle a_k; the sample between them is
    # exactly h from both, and no other particle is within 1/64 - 2h
    a = rng.choice(300, size=40, replace=False)
    partner = x[a] + np.array([2 * h, 0, 0])
    x = np.concatenate([x, partner])
    s[:40] = x[a] + np.array([h, 0, 0])
    # put half of the partners first in index order
    perm = np.arange(len(x))
    perm[a[:20]], perm[300:320] = 300 + np.arange(20), a[:20]
    inv = np.argsort(perm)
    x = x[inv]
    got = resample.parents(s, x)
    assert np.array_equal(got, resample.parents_bruteforce(s, x))
    ia = np.argsort(inv)[a]
    ib = np.argsort(inv)[300 + np.arange(40)]
    assert np.all(resample.dist2(x[ia], s[:40]) == resample.dist2(x[ib], s[:40]))
    assert np.array_equal(got[:40], np.minimum(ia, ib))


@pytest.mark.parametrize("dim", [2, 3])
def test_split_conserves_mass_and_centre(dim):
    P, p, surf = _scene(dim, 11)
    sp = resample.split(P, surf)
    par = sp["parent"]
    gm = sp["mtilde"] * (2 * sp["count"] + 1)
    assert np.allclose(gm, P["m"], rtol=1e-15, atol=0)
    com = sp["mtilde"][:, None] * P["x"]
    np.add.at(com, par, sp["mtilde"][par][:, None] * (surf["s"] + sp["b"]))
    assert np.allclose(com / P["m"][:, None], P["x"], rtol=0, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_p2g_conservation(dim):
    P, p, surf = _scene(dim, 12)
    sp = resample.split(P, surf)
    g = transfer.p2g(P, surf, sp, p)
    n = p["n"]
    xi = bspline.node_positions(n, dim)
    assert g["m"].sum() == pytest.approx(P["m"].sum(), rel=1e-13)
    assert np.allclose(g["mv"].sum(0), (P["m"][:, None] * P["v"]).sum(0), rtol=1e-12, atol=1e-15)
    L_grid = ang_mom(xi, g["mv"])
    L_part = ang_mom(P["x"], P["m"][:, None] * P["v"]) + apic_spin(P["m"], P["A"], p["dx"])
    assert np.allclose(L_grid, L_part, rtol=1e-11, atol=1e-15)
    assert g["W"].sum() == pytest.approx(P["m"].sum(), rel=1e-13)
    assert g["E"].sum() == pytest.approx(2 * np.sum(sp["mtilde"] * sp["count"]), rel=1e-13)


def test_p2g_unsplit_is_standard_apic():
    P, p, surf = _scene(3, 13, count=5, nsurf=0)
    surf = dict(s=np.zeros((0, 3)), dA=np.zeros((0, 3)), label=np.zeros(0, np.int32))
    sp = resample.split(P, surf)
    g = transfer.p2g(P, surf, sp, p)
    n, dx = p["n"], p["dx"]
    m_ref = np.zeros(n ** 3)
    mv_ref = np.zeros((n ** 3, 3))
    for q in range(len(P["x"])):         # per-particle loop written from the APIC splat
        for k in np.ndindex(3, 3, 3):
            base = np.floor(P["x"][q] / dx - 1).astype(int)
            node = base + np.array(k[::-1])
            xi = (node + 0.5) * dx
            Nw = np.prod([bspline.kernel_1d((P["x"][q][a] - xi[a]) / dx)[0] for a in range(3)])
            lin = node[0] + n * (node[1] + n * node[2])
            m_ref[lin] += P["m"][q] * Nw
            mv_ref[lin] += P["m"][q] * Nw * (P["v"][q] + P["A"][q] @ (xi - P["x"][q]))
    assert np.allclose(g["m"], m_ref, rtol=1e-14, atol=1e-20)
    assert np.allclose(g["mv"], mv_ref, rtol=1e-13, atol=1e-18)


@pytest.mark.parametrize("dim", [2, 3])
def test_g2p_after_p2g_conserves(dim):
    """With v^ = v^n (no grid update), G2P o P2G keeps total momentum and the APIC
    angular momentum, split groups included (Sections 4.1.3 and 5)."""
    P, p, surf = _scene(dim, 14)
    sp = resample.split(P, surf)
    g = transfer.p2g(P, surf, sp, p)
    st = transfer.grid_setup(P, surf, sp, g, p)
    newP = transfer.g2p(P, surf, sp, st["vn"], st["Tn"], dict(p, dt=0.0))
    mom0 = (P["m"][:, None] * P["v"]).sum(0)
    mom1 = (P["m"][:, None] * newP["v"]).sum(0)
    assert np.allclose(mom0, mom1, rtol=1e-12, atol=1e-16)
    L0 = ang_mom(P["x"], P["m"][:, None] * P["v"]) + apic_spin(P["m"], P["A"], p["dx"])
    L1 = ang_mom(P["x"], P["m"][:, None] * newP["v"]) + apic_spin(P["m"], newP["A"], p["dx"])
    assert np.allclose(L0, L1, rtol=1e-11, atol=1e-16)


@pytest.mark.parametrize("dim", [2, 3])
def test_temperature_linear_reproduction(dim):
    P, p, surf = _scene(dim, 15)
    a = np.array([3.0, -2.0, 1.5])[:dim]
    P["T"] = 300.0 + P["x"] @ a
    P["gradT"] = np.tile(a, (len(P["x"]), 1))
    sp = resample.split(P, surf)
    g = transfer.p2g(P, surf, sp, p)
    st = transfer.grid_setup(P, surf, sp, g, p)
    xi = bspline.node_positions(p["n"], dim)
    hasW = g["W"] > 0
    assert np.allclose(st["Tn"][hasW], 300.0 + xi[hasW] @ a, rtol=1e-13)
    That = 300.0 + xi @ a
    newP = transfer.g2p(P, surf, sp, st["vn"], That, dict(p, dt=0.0))
    assert np.allclose(newP["T"], P["T"], rtol=1e-13)
    assert np.allclose(newP["gradT"], P["gradT"], rtol=1e-11)
