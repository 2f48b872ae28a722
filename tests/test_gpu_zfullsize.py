"""Parity at full size: the 3D Marangoni droplet (128^3 grid, ~560k particles), every
operator and G2P against the vectorized oracle on the same inputs, in MIXED and FP64;
the contact-angle scene (192^3) and the melting slab (256^3, ~9.7M particles) through
properties that hold at any size; and MIXED at 256^3 from unrounded FP64 inputs against
the FP64 oracle, which measures what the absolute FP32 positions cost at that grid."""
import numpy as np
import pytest

import mpm_scenes as sc
from gpu_cases import GpuState, OracleState, check, log, rel, round_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full_case():
    from paper_2101_12408_amd import api
    S = sc.marangoni3d()
    P, p = S["particles"], S["params"]
    surf = api.sample_surface(P["x"], p)       # product sampler; pinned to the oracle's in CPU tests
    log(f"full-size marangoni3d: N={len(P['m'])} S={len(surf['s'])}")
    return P, surf, p


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_fullsize_operators(full_case, precision):
    P, surf, p = full_case
    P, surf = round_inputs(P, surf, precision)
    log(f"case fullsize {precision}: oracle set-up")
    o = OracleState(P, surf, p)
    log("  gpu p2g")
    g = GpuState(P, surf, p, precision)
    from paper_2101_12408_amd import _lib as L
    tolf = 1e-10 if precision == "fp64" else 2e-5
    assert np.array_equal(g.scene.view(L.F_PARENT).cpu().numpy(), o.split["parent"])
    for name, f, ref in (("m", L.F_MASS, o.grid["m"]), ("mv", L.F_MOM, o.grid["mv"]), ("Tn", L.F_TN, o.setup["Tn"])):
        check(name, g.to_natural(g.scene.view(f)), ref, tolf)
    rng = np.random.default_rng(3)
    dof = o.setup["dof"]
    v = o.setup["vn"] + rng.normal(size=o.ctx.vn.shape) * 0.01 * dof[:, None]
    if precision != "fp64":
        v = v.astype(np.float32).astype(np.float64)
    grad = g.scene.grid_vector()
    g.scene.energy_grad(g.from_natural(v), grad)
    check("energy_grad", g.to_natural(grad)[dof], o.ctx.project(o.ctx.grad_Phi(v))[dof],
          1e-10 if precision == "fp64" else 1e-4)
    w = rng.normal(size=o.ctx.vn.shape) * dof[:, None]
    if precision != "fp64":
        w = w.astype(np.float32).astype(np.float64)
    out = g.scene.grid_vector()
    g.scene.hessvec(g.from_natural(v), g.from_natural(w), 1.0, out)
    check("hessvec", g.to_natural(out)[dof], o.ctx.project(o.ctx.hessvec(v, o.ctx.project(w), 1.0))[dof],
          1e-10 if precision == "fp64" else 1e-4)
    T = (300 + rng.normal(size=o.setup["Tn"].shape)) * dof
    if precision != "fp64":
        T = T.astype(np.float32).astype(np.float64)
    out1 = g.scene.grid_vector(1)[0]
    g.scene.heat_apply(g.from_natural(T), out1)
    check("heat_apply", g.to_natural(out1)[dof], o.heat.apply(T)[dof], 1e-10 if precision == "fp64" else 1e-5)
    # G2P with merge and advection at full size (the launch configuration of the benchmark)
    from test_gpu_parity import g2p_compare
    vh = o.ctx.project(v)
    g2p_compare(o, g, P, vh, T, precision, 3)


def test_mixed_at_256_from_fp64_inputs():
    """The melting slab's grid (256^3, dx = 1/256) with a small slab near x = 0.75, where the
    FP32 spacing of absolute positions is largest (6e-8, 1.5e-5 dx): the MIXED path takes
    the unrounded FP64 inputs (it stores them as FP32 itself) and is compared with the FP64
    oracle.  Grid forces must stay within 1e-4, the MIXED force tolerance."""
    import mpm_scenes as sc
    from oracle import sampler
    from paper_2101_12408_amd import _lib as L
    S = sc.meltslab3d(n=256, lo=0.7, hi=0.78, height=0.04)
    P, p = S["particles"], S["params"]
    rng = np.random.default_rng(256)
    P["v"] = rng.normal(size=P["v"].shape) * 0.01
    surf = sampler.sample_surface(P["x"], p)
    log(f"case 256^3 absolute FP32 positions: N={len(P['m'])} S={len(surf['s'])}; oracle set-up")
    o = OracleState(P, surf, p)
    g = GpuState(P, surf, p, "mixed")
    par = g.scene.view(L.F_PARENT).cpu().numpy()
    flips = int(np.sum(par != o.split["parent"]))
    log(f"  parents that differ from the FP64 search: {flips} of {len(par)}")
    assert flips <= len(par) // 1000
    dof = o.setup["dof"]
    for name, f, ref in (("m", L.F_MASS, o.grid["m"]), ("mv", L.F_MOM, o.grid["mv"]), ("Tn", L.F_TN, o.setup["Tn"])):
        check(name, g.to_natural(g.scene.view(f)), ref, 1e-4)
    v = o.setup["vn"] + rng.normal(size=o.ctx.vn.shape) * 0.01 * dof[:, None]
    grad = g.scene.grid_vector()
    g.scene.energy_grad(g.from_natural(v), grad)
    check("energy_grad", g.to_natural(grad)[dof], o.ctx.project(o.ctx.grad_Phi(v))[dof], 1e-4)
    w = rng.normal(size=o.ctx.vn.shape) * dof[:, None]
    out = g.scene.grid_vector()
    g.scene.hessvec(g.from_natural(v), g.from_natural(w), 1.0, out)
    check("hessvec", g.to_natural(out)[dof], o.ctx.project(o.ctx.hessvec(v, o.ctx.project(w), 1.0))[dof], 1e-4)


def _sum64(t):
    return t.double().sum(dim=-1).cpu().numpy()


@pytest.mark.parametrize("case,precision", [("contact3d", "mixed"), ("meltslab3d", "fp64"), ("meltslab3d", "mixed")])
def test_fullsize_step_properties(case, precision):
    """The contact-angle scene (192^3) and the melting slab (256^3, ~9.7M particles) at full
    size, where the oracle cannot run whole: properties that hold at any size.  P2G
    conserves mass and momentum, Newton converges, G2P returns the grid momentum to the
    particles exactly, and (slab) the heat update satisfies the Robin balance law
    sum_i c_p m_i (T^_i - T^n_i) / dt = sum_r |dA_r| (h (T_amb - T^(s_r)) + b)."""
    import torch
    from oracle import bspline
    from paper_2101_12408_amd import _lib as L
    from paper_2101_12408_amd import api
    S = sc.contact3d() if case == "contact3d" else sc.meltslab3d()
    P, p = S["particles"], S["params"]
    rng = np.random.default_rng(7)
    P["v"] = rng.normal(size=P["v"].shape) * 0.01
    surf = api.sample_surface(P["x"], p)
    N, Ns = len(P["m"]), len(surf["s"])
    log(f"case fullsize {case} {precision}: N={N} S={Ns} n={p['n']}")
    s = api.Scene(p, cap_part=N, cap_surf=Ns, precision=precision)
    Pd, Sd = s.to_device(P, surf)
    s.p2g(Pd, Sd)
    m_grid = float(s.view(L.F_MASS).double().sum())
    mv_grid = _sum64(s.view(L.F_MOM))
    m_p = P["m"].astype(np.float64)
    tol = 1e-12 if precision == "fp64" else 2e-5
    log(f"  mass {m_grid:.9e} vs {m_p.sum():.9e}")
    assert abs(m_grid - m_p.sum()) <= tol * m_p.sum()
    mom_p = (m_p[:, None] * P["v"]).sum(0)
    scale = (m_p[:, None] * np.abs(P["v"])).sum()
    log(f"  momentum {mv_grid} vs {mom_p}")
    assert np.all(np.abs(mv_grid - mom_p) <= tol * scale)
    rc = s.step(Pd, Sd, check=False)
    assert s.status() == rc             # synchronizes and reads the grid momentum
    st = s.stats()
    log(f"  step rc {rc}: newton {st['newton_iters']} ({st['converged']}), cg {st['cg_iters']}, heat {st['heat_iters']}")
    assert rc == 0 and st["converged"] in (1, 2)
    # G2P: particle momentum = grid momentum sum_i m_i v^_i (exact in arithmetic)
    v_new = Pd["v"].double().cpu().numpy()
    m_new = Pd["m"].double().cpu().numpy()
    mom_new = (m_new[None, :] * v_new).sum(1)
    gmom = np.asarray(st["momentum"][:3])
    scale = (m_new[None, :] * np.abs(v_new)).sum()
    log(f"  particle momentum {mom_new} vs grid {gmom}")
    assert np.all(np.abs(mom_new - gmom) <= (1e-11 if precision == "fp64" else 1e-5) * scale)
    assert np.all(np.isfinite(Pd["x"].cpu().numpy())) and np.all(np.isfinite(Pd["T"].cpu().numpy()))
    if p["heat"] and p["h"] > 0:
        nat = torch.as_tensor(api.tiled_index(3, p["n"]), device=Pd["x"].device)
        m = s.view(L.F_MASS).double()[nat].cpu().numpy()
        Th = s.view(L.F_THAT).double()[nat].cpu().numpy()
        Tn = s.view(L.F_TN).double()[nat].cpu().numpy()
        dof = m > 0
        lhs_terms = p["cp"] * m[dof] * (Th[dof] - Tn[dof]) / p["dt"]
        idx, Nw, _ = bspline.stencil(surf["s"], p["dx"], p["n"])
        Ts = (Nw * Th[idx]).sum(1)
        area = np.linalg.norm(surf["dA"], axis=1)
        rhs_terms = area * (p["h"] * (p["T_amb"] - Ts) + p["b"])
        lhs, rhs = lhs_terms.sum(), rhs_terms.sum()
        scale = np.abs(lhs_terms).sum() + np.abs(rhs_terms).sum()
        # FP64: the solver tolerance; MIXED: T^ and T^n are stored in FP32, so each term
        # c_p m_i (T^_i - T^n_i)/dt carries up to 2 eps32 c_p m_i |T_i|/dt of round-off
        bound = 1e-7 * scale if precision == "fp64" else \
            2.0 * 2.0 ** -24 * np.sum(p["cp"] * m[dof] * np.abs(Th[dof])) / p["dt"]
        log(f"  heat balance: {lhs:.9e} vs {rhs:.9e} (scale {scale:.3e}, bound {bound:.3e})")
        assert abs(lhs - rhs) <= bound


def test_device_sampler_at_256_equals_host_stage():
    """The device sampler at the melting slab's full size (256^3, ~9.7M particles, FP32
    positions as the MIXED bench holds them): the host stage's samples bit for bit, and the
    oracle's sample for sample on a sub-slab small enough for it."""
    from paper_2101_12408_amd import api
    from oracle import sampler
    S = sc.meltslab3d()
    P, p = S["particles"], S["params"]
    P = {k: v.astype(np.float32).astype(np.float64) for k, v in P.items()}
    N = len(P["m"])
    host = api.sample_surface(P["x"], p, step=2)
    s = api.Scene(p, cap_part=N, cap_surf=len(host["s"]) + 1024, precision="mixed")
    Pd = s.to_device(P)
    got = s.sample_surface(Pd, step=2)
    log(f"  256^3 device sampler: {got['s'].shape[1]} samples (host {len(host['s'])})")
    assert got["s"].shape[1] == len(host["s"])
    assert np.array_equal(got["s"].cpu().numpy().T, host["s"].astype(np.float32))
    assert np.array_equal(got["dA"].cpu().numpy().T, host["dA"].astype(np.float32))
    assert np.array_equal(got["label"].cpu().numpy(), host["label"])
    # a sub-slab of the same grid against the oracle, FP64 outputs
    Sb = sc.meltslab3d(lo=0.44, hi=0.56, height=0.06)
    Pb, pb = Sb["particles"], Sb["params"]
    ref = sampler.sample_surface(Pb["x"], pb, step=2)
    sb = api.Scene(pb, cap_part=len(Pb["m"]), cap_surf=len(ref["s"]) + 1024, precision="fp64")
    gb = sb.sample_surface(sb.to_device(Pb), step=2)
    assert gb["s"].shape[1] == len(ref["s"])
    assert np.max(np.abs(gb["s"].cpu().numpy().T - ref["s"])) <= 1e-13
    assert np.max(np.abs(gb["dA"].cpu().numpy().T - ref["dA"])) <= 1e-15
