"""GPU parity: every ABI call against the oracle on identical seeded inputs.

FP64 mode: 1e-10 relative on every floating output, bit-exact on integer outputs
(parents, group sizes, degree-of-freedom and constraint masks).  MIXED mode: 1e-4
relative on the grid forces (energy gradient); the other outputs are checked at the FP32
level stated per test.  Every floating comparison bounds both the norm-wise error and the
worst element (max |a - b| / max |b|).

Cases: random clouds with random surface samples (2D, 3D), the 2D square droplet, the
Marangoni droplet at 32^3, the contact-angle scene at 48^3 (label table k_r, slab
constraint, gravity), the lid-driven cavity, random clouds with solid particles, and
clouds packed into one cell (one cell tile holds several chunks of points in every tile
kernel)."""
import numpy as np
import pytest

from gpu_cases import TOL_FP64, TOL_MIXED_FORCE, GpuState, OracleState, check, log, make_case, rel, round_inputs

pytestmark = pytest.mark.gpu

CASES = [("random", 2, 1), ("random", 3, 2), ("square2d", 2, 0), ("marangoni3d_small", 3, 0),
         ("contact3d_small", 3, 0), ("cavity2d", 2, 0), ("random_solid", 2, 3), ("random_solid", 3, 4),
         ("dense", 2, 5), ("dense", 3, 6)]

# fixed-corotated solids below T_melt = 300 K (the random scene's T is uniform in 280-320 K)
SOLID = dict(T_melt=300.0, muh0=50.0, lamh0=120.0, kh=0.01, Th0=300.0)


def _case(kind, dim, seed, precision, **kw):
    import mpm_scenes as sc
    from oracle import sampler
    if kind in ("marangoni3d_small", "contact3d_small"):
        S = sc.marangoni3d(n=32, radius=0.25) if kind == "marangoni3d_small" else sc.contact3d(n=48, radius=0.12)
        P, p = S["particles"], dict(S["params"], **kw)
        surf = sampler.sample_surface(P["x"], p)
        P, surf = round_inputs(P, surf, precision)
    elif kind == "square2d":
        P, surf, p = make_case("square2d", n=32, precision=precision, **kw)
    elif kind == "random_solid":
        P, surf, p = make_case("random", dim=dim, seed=seed, precision="fp64", **SOLID, **kw)
        rng = np.random.default_rng(seed + 100)
        P["F"] = np.eye(dim)[None] + 0.1 * rng.normal(size=(len(P["m"]), dim, dim))
        P, surf = round_inputs(P, surf, precision)
    else:
        P, surf, p = make_case(kind, dim=dim, seed=seed, precision=precision, **kw)
    return P, surf, p


def _p2g_checks(o, g, P, surf, p, tol):
    from paper_2101_12408_amd import _lib as L
    sc_ = g.scene
    dim = p["dim"]
    # integer outputs: bit-exact
    assert np.array_equal(sc_.view(L.F_PARENT).cpu().numpy(), o.split["parent"])
    assert np.array_equal(sc_.view(L.F_COUNT).cpu().numpy(), o.split["count"])
    free = g.to_natural(sc_.view(L.F_FREE))
    assert np.array_equal((free & 0x80) != 0, o.setup["dof"])
    for a in range(dim):
        assert np.array_equal(((free >> a) & 1) != 0, o.setup["free"][:, a])
    for name, f, ref in (("m", L.F_MASS, o.grid["m"]), ("mv", L.F_MOM, o.grid["mv"]), ("W", L.F_W, o.grid["W"]),
                         ("WT", L.F_WT, o.grid["WT"]), ("E", L.F_E, o.grid["E"]), ("ET", L.F_ET, o.grid["ET"]),
                         ("vn", L.F_VN, o.setup["vn"]), ("Tn", L.F_TN, o.setup["Tn"])):
        check(name, g.to_natural(sc_.view(f)), ref, tol)
    check("k_r", sc_.view(L.F_KSURF).cpu().numpy(), o.setup["k"], tol)
    # heat system: right side and diagonal; Newton diagonal
    dof = o.setup["dof"]
    check("heat rhs", g.to_natural(sc_.view(L.F_HEAT_RHS))[dof], o.heat.rhs[dof], tol)
    check("heat diag", g.to_natural(sc_.view(L.F_HEAT_DIAG))[dof], o.heat.diag()[dof], tol)
    md = g.to_natural(sc_.view(L.F_MOM_DIAG))
    check("momentum diag", md[o.setup["free"]], o.ctx.jacobi_diag()[o.setup["free"]], tol)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kind,dim,seed", CASES)
def test_p2g_parity(kind, dim, seed, precision):
    log(f"case p2g {kind} dim={dim} seed={seed} {precision}")
    P, surf, p = _case(kind, dim, seed, precision)
    o = OracleState(P, surf, p)
    g = GpuState(P, surf, p, precision)
    _p2g_checks(o, g, P, surf, p, TOL_FP64 if precision == "fp64" else 2e-5)
    if kind == "contact3d_small":
        # the scene exercises both label values and the slab constraint
        lab = surf["label"]
        assert 0 < lab.sum() < len(lab)
        assert np.any(o.setup["dof"] & ~o.setup["free"][:, 1]) and np.all(o.setup["free"][o.setup["dof"]][:, [0, 2]])


def _rand_field(o, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return rng.normal(size=o.ctx.vn.shape) * scale * o.setup["dof"][:, None]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kind,dim,seed", CASES)
def test_energy_grad_parity(kind, dim, seed, precision):
    log(f"case energy_grad {kind} dim={dim} seed={seed} {precision}")
    P, surf, p = _case(kind, dim, seed, precision)
    o = OracleState(P, surf, p)
    g = GpuState(P, surf, p, precision)
    v = o.setup["vn"] + _rand_field(o, seed + 5, 0.3)
    if precision != "fp64":
        v = v.astype(np.float32).astype(np.float64)
    vd = g.from_natural(v)
    grad = g.scene.grid_vector()
    e = g.scene.energy_grad(vd, grad)
    ref_g = o.ctx.project(o.ctx.grad_Phi(v))
    got_g = g.to_natural(grad)
    tol = TOL_FP64 if precision == "fp64" else TOL_MIXED_FORCE
    check("grad", got_g[o.setup["dof"]], ref_g[o.setup["dof"]], tol)
    phi = float(e.cpu().numpy()[0])
    ref_phi = o.ctx.Phi(v)
    log(f"  phi {phi:.12e} ref {ref_phi:.12e}")
    assert abs(phi - ref_phi) <= (TOL_FP64 if precision == "fp64" else 1e-5) * max(abs(ref_phi), 1e-300)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("hess_mode", [0, 1])
@pytest.mark.parametrize("kind,dim,seed", CASES)
def test_hessvec_parity(kind, dim, seed, precision, hess_mode):
    log(f"case hessvec {kind} dim={dim} seed={seed} {precision} mode={hess_mode}")
    if kind == "random_solid" and hess_mode == 1:
        pytest.skip("the EXACT Hessian is not available with solids on the device (rejected with MPM_EINVAL)")
    P, surf, p = _case(kind, dim, seed, precision, hess_mode=hess_mode)
    o = OracleState(P, surf, p)
    g = GpuState(P, surf, p, precision)
    vl = o.setup["vn"] + _rand_field(o, seed + 7, 0.3)
    w = _rand_field(o, seed + 8)
    if precision != "fp64":
        vl = vl.astype(np.float32).astype(np.float64)
        w = w.astype(np.float32).astype(np.float64)
    out = g.scene.grid_vector()
    for alpha in (1.0, 0.0):
        g.scene.hessvec(g.from_natural(vl), g.from_natural(w), alpha, out)
        ref = o.ctx.project(o.ctx.hessvec(vl, o.ctx.project(w), alpha))
        got = g.to_natural(out)
        check(f"hessvec alpha {alpha}", got[o.setup["dof"]], ref[o.setup["dof"]],
              TOL_FP64 if precision == "fp64" else 1e-4)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kind,dim,seed", CASES)
def test_heat_apply_parity(kind, dim, seed, precision):
    log(f"case heat_apply {kind} dim={dim} seed={seed} {precision}")
    P, surf, p = _case(kind, dim, seed, precision, heat=1, K=0.3, h=4.0)
    o = OracleState(P, surf, p)
    g = GpuState(P, surf, p, precision)
    rng = np.random.default_rng(seed + 11)
    T = (300 + rng.normal(size=o.setup["Tn"].shape) * 10) * o.setup["dof"]
    if precision != "fp64":
        T = T.astype(np.float32).astype(np.float64)
    out = g.scene.grid_vector(1)[0]
    g.scene.heat_apply(g.from_natural(T), out)
    ref = o.heat.apply(T)
    got = g.to_natural(out)
    check("heat_apply", got[o.setup["dof"]], ref[o.setup["dof"]], TOL_FP64 if precision == "fp64" else 1e-5)


def g2p_compare(o, g, P, vh, Th, precision, dim):
    """G2P on the GPU against the oracle (results mapped through MPM_F_PERM)."""
    from oracle import transfer
    from paper_2101_12408_amd import _lib as L
    ref = transfer.g2p(o.P, o.surf, o.split, vh, Th, o.p)
    ref = transfer.phase_change(o.P["T"], ref, o.p)       # G2P also takes the phase change
    g.scene.g2p(g.from_natural(vh), g.from_natural(Th), g.Pd)
    perm = g.scene.view(L.F_PERM).cpu().numpy()
    N = len(P["m"])
    d = dim
    # the library writes particles back in cell order: slot j holds input particle perm[j]
    got = dict(x=g.Pd["x"].cpu().numpy().T, v=g.Pd["v"].cpu().numpy().T,
               A=g.Pd["A"].cpu().numpy().T.reshape(N, d, d), J=g.Pd["J"].cpu().numpy(),
               T=g.Pd["T"].cpu().numpy(), gradT=g.Pd["gradT"].cpu().numpy().T)
    assert np.array_equal(np.sort(perm), np.arange(N))
    assert np.array_equal(g.Pd["m"].cpu().numpy(), P["m"][perm].astype(g.Pd["m"].cpu().numpy().dtype))
    ref = {k: v[perm] for k, v in ref.items() if isinstance(v, np.ndarray) and len(v) == N}
    P = {k: v[perm] for k, v in P.items()}
    tol = TOL_FP64 if precision == "fp64" else 1e-4
    if "F" in P:
        got["F"] = g.Pd["F"].cpu().numpy().T.reshape(N, d, d)
        check("F", got["F"] - P["F"], ref["F"] - P["F"], tol)
    for k in ("v", "A", "J", "T", "gradT", "x"):
        if k in ("x", "J") and precision == "fp64":
            check(k, got[k] - P[k], ref[k] - P[k], tol)      # the update, not the carried value
        elif k == "x":
            check(k, got[k], ref[k], tol)                    # float32 storage of x bounds the displacement error
        elif k == "J":
            check(k, got[k] - P["J"], ref[k] - P["J"], tol)
        else:
            check(k, got[k], ref[k], tol)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kind,dim,seed", CASES)
def test_g2p_parity(kind, dim, seed, precision):
    log(f"case g2p {kind} dim={dim} seed={seed} {precision}")
    P, surf, p = _case(kind, dim, seed, precision)
    o = OracleState(P, surf, p)
    g = GpuState(P, surf, p, precision)
    vh = o.ctx.project(o.setup["vn"] + _rand_field(o, seed + 13, 0.3))
    rng = np.random.default_rng(seed + 14)
    Th = (300 + rng.normal(size=o.setup["Tn"].shape)) * o.setup["dof"]
    if precision != "fp64":
        vh = vh.astype(np.float32).astype(np.float64)
        Th = Th.astype(np.float32).astype(np.float64)
    g2p_compare(o, g, P, vh, Th, precision, dim)


def test_meltslab_mixed_operators_n64():
    """The melting slab at 64^3 (151k particles, viscosity mu(T), Robin heating, gravity,
    slip floor) in MIXED precision: every operator against the oracle."""
    import mpm_scenes as sc
    from oracle import sampler
    log("case meltslab3d n=64 mixed: oracle set-up")
    S = sc.meltslab3d(n=64)
    P, p = S["particles"], S["params"]
    rng = np.random.default_rng(64)
    P["v"] = rng.normal(size=P["v"].shape) * 0.01
    P["T"] = 290.0 + 20.0 * rng.uniform(size=len(P["T"]))
    surf = sampler.sample_surface(P["x"], p)
    P, surf = round_inputs(P, surf, "mixed")
    o = OracleState(P, surf, p)
    log(f"  N={len(P['m'])} S={len(surf['s'])}; gpu p2g")
    g = GpuState(P, surf, p, "mixed")
    _p2g_checks(o, g, P, surf, p, 2e-5)
    dof = o.setup["dof"]
    v = (o.setup["vn"] + _rand_field(o, 65, 0.01)).astype(np.float32).astype(np.float64)
    grad = g.scene.grid_vector()
    e = g.scene.energy_grad(g.from_natural(v), grad)
    check("grad", g.to_natural(grad)[dof], o.ctx.project(o.ctx.grad_Phi(v))[dof], TOL_MIXED_FORCE)
    ref_phi = o.ctx.Phi(v)
    assert abs(float(e.cpu().numpy()[0]) - ref_phi) <= 1e-5 * abs(ref_phi)
    w = _rand_field(o, 66).astype(np.float32).astype(np.float64)
    out = g.scene.grid_vector()
    g.scene.hessvec(g.from_natural(v), g.from_natural(w), 1.0, out)
    check("hessvec", g.to_natural(out)[dof], o.ctx.project(o.ctx.hessvec(v, o.ctx.project(w), 1.0))[dof], 1e-4)
    T = ((300 + rng.normal(size=o.setup["Tn"].shape) * 10) * dof).astype(np.float32).astype(np.float64)
    out1 = g.scene.grid_vector(1)[0]
    g.scene.heat_apply(g.from_natural(T), out1)
    check("heat_apply", g.to_natural(out1)[dof], o.heat.apply(T)[dof], 1e-5)
    vh = o.ctx.project(v).astype(np.float32).astype(np.float64)
    g2p_compare(o, g, P, vh, T, "mixed", 3)


def test_determinism_bitwise():
    log("case determinism")
    P, surf, p = _case("random", 3, 4, "mixed")
    o = OracleState(P, surf, p)
    outs = []
    for rep in range(2):
        g = GpuState(P, surf, p, "mixed")
        w = g.from_natural(_rand_field(o, 3))
        out = g.scene.grid_vector()
        g.scene.hessvec(w, w, 1.0, out)
        from paper_2101_12408_amd import _lib as L
        outs.append((out.cpu().numpy().copy(), g.scene.view(L.F_MOM).cpu().numpy().copy()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_domain_error_is_reported():
    log("case domain error")
    from paper_2101_12408_amd import _lib as L
    P, surf, p = _case("random", 3, 5, "fp64")
    P = dict(P)
    P["x"] = P["x"].copy()
    P["x"][3] = [0.5 / p["n"], 0.5, 0.5]           # stencil would leave the grid
    from paper_2101_12408_amd import api
    sc_ = api.Scene(p, cap_part=len(P["m"]), cap_surf=len(surf["s"]))
    Pd, Sd = sc_.to_device(P, surf)
    sc_.p2g(Pd, Sd)
    assert sc_.status() == L.MPM_EDOMAIN
