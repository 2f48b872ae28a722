"""GPU end-to-end: one full step (split, P2G, Newton-CG, heat CG, G2P) against the oracle,
conservation under explicit stepping (Section 6.1), momentum with the translation
correction, and batch invariance of mpm_step.

End-to-end parity is bounded by the solver tolerances, not by the arithmetic: both
sides stop Newton at |g| <= tol |g0| with tol = 1e-12 here, so the velocities agree to
about 1e-8 relative.  The single operators are checked at 1e-10 in test_gpu_parity."""
import numpy as np
import pytest

import mpm_scenes as sc
from gpu_cases import log, rel, round_inputs
from oracle import sampler, step as ostep

pytestmark = pytest.mark.gpu


def _gpu_step(P, surf, p, precision="fp64", implicit=True):
    from paper_2101_12408_amd import api
    s = api.Scene(p, cap_part=len(P["m"]), cap_surf=max(1, len(surf["s"])), precision=precision)
    Pd, Sd = s.to_device(P, surf)
    rc = s.step(Pd, Sd, implicit=implicit, check=False)
    N, d = len(P["m"]), p["dim"]
    from paper_2101_12408_amd import _lib as L
    perm = s.view(L.F_PERM).cpu().numpy()
    inv = np.empty_like(perm)
    inv[perm] = np.arange(N)           # back to input order for the comparison
    out = dict(x=Pd["x"].cpu().numpy().T.astype(np.float64)[inv], v=Pd["v"].cpu().numpy().T.astype(np.float64)[inv],
               A=Pd["A"].cpu().numpy().T.reshape(N, d, d).astype(np.float64)[inv],
               J=Pd["J"].cpu().numpy().astype(np.float64)[inv], T=Pd["T"].cpu().numpy().astype(np.float64)[inv],
               gradT=Pd["gradT"].cpu().numpy().T.astype(np.float64)[inv], m=P["m"], V0=P["V0"])
    assert np.array_equal(Pd["m"].cpu().numpy().astype(np.float64)[inv], P["m"].astype(Pd["m"].cpu().numpy().dtype))
    return out, s.stats(), rc


TIGHT = dict(newton_tol=1e-12, cg_rel=1e-3, heat_tol=1e-13)


@pytest.mark.parametrize("case", ["square2d", "marangoni3d_small", "meltslab_small", "contact_small", "cavity2d"])
def test_implicit_step_matches_oracle_fp64(case):
    log(f"case step {case}")
    if case == "square2d":
        S = sc.square2d(n=32)
        rng = np.random.default_rng(1)
        S["particles"]["v"] = rng.normal(size=S["particles"]["v"].shape) * 0.05
    elif case == "marangoni3d_small":
        S = sc.marangoni3d(n=32, radius=0.25)
    elif case == "contact_small":
        # label table k_r, slab constraint on v_y, gravity, no translation correction
        S = sc.contact3d(n=48, radius=0.12)
    elif case == "cavity2d":
        # k = clamp(1 - T, 0, 1) on the free surface, none on the walls, four slip walls,
        # CFL-limited dt; a flow already under way
        S = sc.cavity2d(n=32)
        rng = np.random.default_rng(4)
        S["particles"]["v"] = rng.normal(size=S["particles"]["v"].shape) * 0.01
    else:
        S = sc.meltslab3d(n=32)
    P, p = S["particles"], dict(S["params"], **TIGHT)
    surf = sampler.sample_surface(P["x"], p)
    ref, info = ostep.step(P, p, surf)
    got, st, rc = _gpu_step(P, surf, p)
    log(f"  gpu newton {st['newton_iters']} cg {st['cg_iters']} heat {st['heat_iters']} rc {rc}; "
        f"oracle newton {info['newton']} cg {info['cg']} heat {info.get('heat_cg')}")
    assert rc == 0
    for k in ("v", "A", "J", "x", "T", "gradT"):
        if k in ("x", "J"):
            e = rel(got[k] - P[k], ref[k] - P[k])
        else:
            e = rel(got[k], ref[k])
        log(f"  {k}: rel {e:.3e}")
        assert e < 1e-7, k


def test_implicit_step_without_translation_correction():
    """With the translation correction off, the Newton decision and the next CG's start run
    as kernels of their own (not inside the correction's pass): FP64 step against the
    oracle at the same bar."""
    S = sc.marangoni3d(n=32, radius=0.25)
    P, p = S["particles"], dict(S["params"], momentum_fix=0, **TIGHT)
    surf = sampler.sample_surface(P["x"], p)
    ref, info = ostep.step(P, p, surf)
    got, st, rc = _gpu_step(P, surf, p)
    log(f"  no correction: gpu newton {st['newton_iters']} cg {st['cg_iters']}; oracle newton {info['newton']} "
        f"cg {info['cg']}")
    assert rc == 0
    assert st["newton_iters"] >= 2   # the queued next-iteration CG was taken at least once
    for k in ("v", "A", "J", "x", "T"):
        e = rel(got[k] - P[k], ref[k] - P[k]) if k in ("x", "J") else rel(got[k], ref[k])
        log(f"  {k}: rel {e:.3e}")
        assert e < 1e-7, k


def test_mixed_step_error_report():
    """MIXED mode step against the FP64 oracle: reported, bounded at the FP32 level."""
    S = sc.marangoni3d(n=32, radius=0.25)
    P, p = S["particles"], dict(S["params"], newton_tol=1e-6)
    surf = sampler.sample_surface(P["x"], p)
    P32, surf32 = round_inputs(P, surf, "mixed")
    ref, info = ostep.step(P32, p, surf32)
    got, st, rc = _gpu_step(P32, surf32, p, precision="mixed")
    assert rc == 0
    for k in ("v", "A", "T"):
        e = rel(got[k], ref[k])
        log(f"  mixed {k}: rel {e:.3e}")
        assert e < 1e-3, k


def _momenta(P, dx):
    m = P["m"]
    mom = (m[:, None] * P["v"]).sum(0)
    x, v, A = P["x"], P["v"], P["A"]
    L = np.sum(m * (x[:, 0] * v[:, 1] - x[:, 1] * v[:, 0])) + np.sum(m * (A[:, 1, 0] - A[:, 0, 1])) * dx * dx / 4
    com = (m[:, None] * x).sum(0) / m.sum()
    return mom, L, com


def test_explicit_steps_conserve_on_gpu():
    """Section 6.1 on the GPU path: 2D ellipse, explicit stepping, surface tension only;
    linear and angular momentum and the centre of mass are conserved to round-off."""
    from paper_2101_12408_amd import api
    p = sc.make_params(dim=2, n=64, dt=1e-5, bulk=4166.67, g0=0.1, seed=6)
    rng = np.random.default_rng(6)
    cells = np.stack(np.meshgrid(np.arange(16, 48), np.arange(16, 48), indexing="xy"), -1).reshape(-1, 2)
    x = (cells[:, None, :] + rng.uniform(0, 1, size=(len(cells), 8, 2))).reshape(-1, 2) / 64
    x = x[((x[:, 0] - 0.5) / 0.2) ** 2 + ((x[:, 1] - 0.5) / 0.12) ** 2 < 1]
    P = sc.particles_from_positions(x, 2, p["dx"], ppc=8)
    s = api.Scene(p, cap_part=len(x), cap_surf=20 * len(x), precision="fp64")
    Pd = s.to_device(P)
    hist = []
    for k in range(10):
        xh = Pd["x"].cpu().numpy().T.copy()
        surf = api.sample_surface(xh, p, step=k)
        Sd = s.to_device(S=surf)
        s.step(Pd, Sd, implicit=False)
        Q = dict(m=Pd["m"].cpu().numpy(), x=Pd["x"].cpu().numpy().T, v=Pd["v"].cpu().numpy().T,
                 A=Pd["A"].cpu().numpy().T.reshape(-1, 2, 2))
        hist.append(_momenta(Q, p["dx"]))
    scale = np.abs(P["m"][:, None] * Q["v"]).sum()
    log(f"  momentum scale {scale:.3e}; final mom {hist[-1][0]}, L {hist[-1][1]:.3e}")
    assert scale > 0
    for mom, L, com in hist:
        assert np.all(np.abs(mom) < 1e-13 * scale)
        assert abs(L) < 1e-13 * scale
        assert np.allclose(com, hist[0][2], rtol=0, atol=1e-13)


def _host_state(Pd, d):
    N = Pd["m"].shape[0]
    return dict(x=Pd["x"].cpu().numpy().T.astype(np.float64), v=Pd["v"].cpu().numpy().T.astype(np.float64),
                A=Pd["A"].cpu().numpy().T.reshape(N, d, d).astype(np.float64),
                J=Pd["J"].cpu().numpy().astype(np.float64), V0=Pd["V0"].cpu().numpy().astype(np.float64),
                m=Pd["m"].cpu().numpy().astype(np.float64), T=Pd["T"].cpu().numpy().astype(np.float64),
                gradT=Pd["gradT"].cpu().numpy().T.astype(np.float64))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("implicit", [True, False])
def test_cfl_dt_matches_oracle(implicit, precision):
    """CFL-limited step (Section 6): the device max-speed and min-density reduction and the
    host rule give the oracle's dt bit for bit from the same particle state (FP32-rounded
    in MIXED, where the reduction still runs in FP64)."""
    from paper_2101_12408_amd import api
    S = sc.ellipse2d(cfl=0.5)
    P, p = S["particles"], dict(S["params"])
    p["dt_max"] = 1e-3
    r = P["x"] - 0.5                 # rigid motion: spin 100 rad/s plus a drift
    P["v"] = np.stack([-100.0 * r[:, 1] + 3.0, 100.0 * r[:, 0] - 2.0], 1)
    if precision == "mixed":
        P = {k: v.astype(np.float32).astype(np.float64) for k, v in P.items()}
    want = ostep.cfl_dt(P, p, implicit)
    assert p["dt_min"] < want < p["dt_max"]
    s = api.Scene(p, cap_part=len(P["m"]), cap_surf=20 * len(P["m"]), precision=precision)
    Pd = s.to_device(P)
    Sd = s.to_device(S=api.sample_surface(P["x"], p, step=0))
    s.step(Pd, Sd, implicit=implicit)
    got = s.stats()["dt"]
    log(f"  cfl dt {got:.17g} oracle {want:.17g}")
    assert got == want


def test_ellipse_cfl_steps_on_gpu():
    """Section 6.1 over 120 CFL-limited explicit steps in FP64 on the device path: every
    step's dt is the oracle's rule applied to the state before it; linear and angular
    momentum and the centre of mass stay at their initial values to round-off; after 120
    steps the particles agree with the oracle's own 120 steps."""
    from paper_2101_12408_amd import api
    from paper_2101_12408_amd import _lib as L
    S = sc.ellipse2d(cfl=0.01)
    P, p = S["particles"], S["params"]
    N = len(P["m"])
    s = api.Scene(p, cap_part=N, cap_surf=20 * N, precision="fp64")
    Pd = s.to_device(P)
    order = np.arange(N)             # order[j]: input index of device particle j
    hist, dts = [], []
    for k in range(S["steps"]):
        Q = _host_state(Pd, 2)
        want = ostep.cfl_dt(Q, p, False)
        Sd = s.to_device(S=api.sample_surface(Q["x"], p, step=k))
        s.step(Pd, Sd, implicit=False)
        dts.append(s.stats()["dt"])
        assert dts[-1] == want, k
        order = order[s.view(L.F_PERM).cpu().numpy()]
        hist.append(_momenta(_host_state(Pd, 2), p["dx"]))
    Q = _host_state(Pd, 2)
    scale = np.abs(Q["m"][:, None] * Q["v"]).sum()
    log(f"  dt {min(dts):.4e}..{max(dts):.4e}; momentum scale {scale:.3e}; final mom {hist[-1][0]}, "
        f"L {hist[-1][1]:.3e}")
    assert scale > 0 and p["dt_min"] < min(dts) and max(dts) < p["dt_max"]
    com0 = (P["m"][:, None] * P["x"]).sum(0) / P["m"].sum()
    for mom, Lz, com in hist:
        assert np.all(np.abs(mom) < 1e-13 * scale)
        assert abs(Lz) < 1e-13 * scale
        assert np.allclose(com, com0, rtol=0, atol=1e-13)
    Po = P
    for k in range(S["steps"]):
        Po, info = ostep.step(Po, p, implicit=False, step_index=k)
    inv = np.empty_like(order)
    inv[order] = np.arange(N)
    ex, ev = np.max(np.abs(Q["x"][inv] - Po["x"])), rel(Q["v"][inv], Po["v"])
    log(f"  vs oracle after {S['steps']} steps: max |dx| {ex:.3e}, v rel {ev:.3e}")
    assert ex < 1e-12 and ev < 1e-9


EPS32 = 2.0 ** -24


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_implicit_momentum_fix_conserves(precision):
    """Implicit steps with the translation correction and no constraint conserve the total
    linear momentum to round-off of the arithmetic: 1e-14 of sum |m v| in FP64, 16 eps32
    of it in MIXED (particle state in FP32, the sums and the correction in FP64)."""
    from paper_2101_12408_amd import api
    S = sc.square2d(n=32)
    P, p = S["particles"], S["params"]
    rng = np.random.default_rng(2)
    P["v"] = rng.normal(size=P["v"].shape) * 0.05
    if precision == "mixed":
        P = {k: v.astype(np.float32).astype(np.float64) for k, v in P.items()}
    mom0 = (P["m"][:, None] * P["v"]).sum(0)
    s = api.Scene(p, cap_part=len(P["m"]), cap_surf=20 * len(P["m"]), precision=precision)
    Pd = s.to_device(P)
    for k in range(3):
        surf = api.sample_surface(Pd["x"].double().cpu().numpy().T.copy(), p, step=k)
        s.step(Pd, s.to_device(S=surf), implicit=True)
    v = Pd["v"].double().cpu().numpy().T
    mom = (Pd["m"].double().cpu().numpy()[:, None] * v).sum(0)
    scale = np.abs(P["m"][:, None] * v).sum()
    bound = (1e-14 if precision == "fp64" else 16 * EPS32) * scale
    log(f"  {precision}: momentum {mom0} -> {mom}, drift {np.abs(mom - mom0).max():.3e} (bound {bound:.3e})")
    assert np.all(np.abs(mom - mom0) <= bound)


def test_mixed_batched_steps_conserve_momentum():
    """Three droplets of uneven size stepped together through mpm_step in MIXED precision:
    each keeps its linear momentum to FP32 round-off (16 eps32 of sum |m v|) over two steps."""
    from paper_2101_12408_amd import api
    specs = [(16, 51, 0.05, [40, 0, 0]), (32, 52, 0.03, [0, 30, 10]), (24, 53, 0.07, [0, 0, 90])]
    objs, Ps, mom0, Ph = [], [], [], []
    rng = np.random.default_rng(5)
    for n, seed, g0, grad in specs:
        S = sc.droplet3d(n, seed, g0, grad)
        P, p = S["particles"], S["params"]
        P["v"] = (rng.normal(size=P["v"].shape) * 0.05).astype(np.float32).astype(np.float64)
        s = api.Scene(p, cap_part=len(P["m"]), cap_surf=20 * len(P["m"]), precision="mixed")
        objs.append(s)
        Ps.append(s.to_device(P))
        mom0.append((P["m"].astype(np.float32).astype(np.float64)[:, None] * P["v"]).sum(0))
    for k in range(2):
        Ss = [s.to_device(S=api.sample_surface(Pd["x"].double().cpu().numpy().T.copy(), s.params, step=k))
              for s, Pd in zip(objs, Ps)]
        assert api.mpm_step(objs, Ps, Ss) == 0
    for s, Pd, m0 in zip(objs, Ps, mom0):
        v = Pd["v"].double().cpu().numpy().T
        m = Pd["m"].double().cpu().numpy()
        mom = (m[:, None] * v).sum(0)
        scale = np.abs(m[:, None] * v).sum()
        log(f"  n={s.n}: drift {np.abs(mom - m0).max():.3e} of scale {scale:.3e}")
        assert np.all(np.abs(mom - m0) <= 16 * EPS32 * scale)


def test_batch_invariance_bitwise():
    """A scene stepped alone and inside a batch gives bitwise-identical results."""
    from paper_2101_12408_amd import api
    scenes = [sc.droplet3d(16, 11, 0.05, [40, 0, 0]), sc.droplet3d(32, 12, 0.03, [0, 30, 10])]
    runs = []
    for batch in (False, True):
        outs = []
        objs, Ps, Ss = [], [], []
        for S in scenes:
            P, p = S["particles"], S["params"]
            surf = api.sample_surface(P["x"], p)
            s = api.Scene(p, cap_part=len(P["m"]), cap_surf=len(surf["s"]), precision="mixed")
            Pd, Sd = s.to_device(P, surf)
            objs.append(s); Ps.append(Pd); Ss.append(Sd)
        if batch:
            api.mpm_step(objs, Ps, Ss)
        else:
            for s, Pd, Sd in zip(objs, Ps, Ss):
                s.step(Pd, Sd)
        runs.append([{k: v.cpu().numpy().copy() for k, v in Pd.items()} for Pd in Ps])
    for a, b in zip(runs[0], runs[1]):
        for k in a:
            assert np.array_equal(a[k], b[k]), k


def test_batch_concurrent_matches_sequential():
    """Scenes of uneven size stepped two at a time, four at a time and one after another
    give bitwise-identical particles (each scene on its own stream in the concurrent runs)."""
    from paper_2101_12408_amd import api
    specs = [(16, 21, 0.05, [40, 0, 0]), (32, 22, 0.03, [0, 30, 10]), (24, 23, 0.07, [0, 0, 90]),
             (16, 24, 0.02, [10, 10, 10]), (48, 25, 0.06, [-50, 0, 20])]
    runs = []
    try:
        for conc in (1, 2, 4):
            api.batch_config(conc)
            objs, Ps, Ss = [], [], []
            for n, seed, g0, grad in specs:
                S = sc.droplet3d(n, seed, g0, grad)
                P, p = S["particles"], S["params"]
                surf = api.sample_surface(P["x"], p)
                s = api.Scene(p, cap_part=len(P["m"]), cap_surf=len(surf["s"]), precision="mixed")
                Pd, Sd = s.to_device(P, surf)
                objs.append(s); Ps.append(Pd); Ss.append(Sd)
            for _ in range(2):
                api.mpm_step(objs, Ps, Ss)
            runs.append([{k: v.cpu().numpy().copy() for k, v in Pd.items()} for Pd in Ps])
            log(f"  concurrency {conc}: newton {[s.stats()['newton_iters'] for s in objs]}")
    finally:
        api.batch_config(8)
    for other in runs[1:]:
        for a, b in zip(runs[0], other):
            for k in a:
                assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("case", ["square2d", "marangoni3d_small", "contact_small"])
def test_minres_exact_step_matches_oracle_fp64(case):
    """krylov = MINRES with the exact (possibly indefinite) surface Hessian: one FP64 step
    against the oracle's Newton-MINRES step, at the bar of the CG step tests."""
    log(f"case minres step {case}")
    if case == "square2d":
        S = sc.square2d(n=32)
        rng = np.random.default_rng(3)
        S["particles"]["v"] = rng.normal(size=S["particles"]["v"].shape) * 0.05
    elif case == "marangoni3d_small":
        S = sc.marangoni3d(n=32, radius=0.25)
    else:
        S = sc.contact3d(n=48, radius=0.12)
    P, p = S["particles"], dict(S["params"], hess_mode=1, krylov=1, **TIGHT)
    surf = sampler.sample_surface(P["x"], p)
    ref, info = ostep.step(P, p, surf)
    got, st, rc = _gpu_step(P, surf, p)
    log(f"  gpu newton {st['newton_iters']} minres {st['cg_iters']} rc {rc}; oracle newton {info['newton']} "
        f"minres {info['cg']}")
    assert rc == 0 and st["converged"] == 1
    for k in ("v", "A", "J", "x", "T"):
        e = rel(got[k] - P[k], ref[k] - P[k]) if k in ("x", "J") else rel(got[k], ref[k])
        log(f"  {k}: rel {e:.3e}")
        assert e < 1e-7, k


def test_minres_mixed_step_error_report():
    """MINRES in MIXED precision against the FP64 oracle: bounded at the FP32 level."""
    S = sc.marangoni3d(n=32, radius=0.25)
    P, p = S["particles"], dict(S["params"], hess_mode=1, krylov=1, newton_tol=1e-6)
    surf = sampler.sample_surface(P["x"], p)
    P32, surf32 = round_inputs(P, surf, "mixed")
    ref, info = ostep.step(P32, p, surf32)
    got, st, rc = _gpu_step(P32, surf32, p, precision="mixed")
    log(f"  mixed minres: newton {st['newton_iters']} minres {st['cg_iters']} converged {st['converged']}")
    assert rc == 0
    for k in ("v", "A", "T"):
        e = rel(got[k], ref[k])
        log(f"  mixed {k}: rel {e:.3e}")
        assert e < 1e-3, k


@pytest.mark.parametrize("krylov", [0, 1])
def test_mixed_newton_stops_at_fp32_floor(krylov):
    """Large momentum against weak forces (the ellipse of Section 6.1 spinning at 100 rad/s
    with a drift, dt 3.5e-4): the FP32 gradient's round-off, about eps32 times the size of
    m v^, sits at a few percent of |g0|, so no relative tolerance is reachable in MIXED.
    Newton stops at that floor (converged = 2) instead of running to the iteration cap, and
    the step still agrees with the FP64 oracle at the FP32 level."""
    S = sc.ellipse2d()
    P, p = S["particles"], dict(S["params"], dt=3.5e-4, krylov=krylov)
    r = P["x"] - 0.5
    P["v"] = np.stack([-100.0 * r[:, 1] + 3.0, 100.0 * r[:, 0] - 2.0], 1)
    surf = sampler.sample_surface(P["x"], p)
    P32, surf32 = round_inputs(P, surf, "mixed")
    ref, info = ostep.step(P32, p, surf32)
    got, st, rc = _gpu_step(P32, surf32, p, precision="mixed")
    log(f"  mixed krylov={krylov}: newton {st['newton_iters']} inner {st['cg_iters']} converged {st['converged']} "
        f"|g| {st['gnorm']:.3e} of |g0| {st['g0']:.3e}")
    assert rc == 0 and st["converged"] in (1, 2)
    for k in ("x", "v", "A"):
        e = rel(got[k], ref[k])
        log(f"  mixed {k}: rel {e:.3e}")
        assert e < 1e-5, k


def test_cavity_marangoni_circulation_on_gpu():
    """The lid-driven Marangoni cavity (Section 6.4) at 64^2 over 300 CFL-limited implicit
    steps in FP64 with the device sampler: the free surface flows from the hot wall (k = 0) toward the cold one
    (k = 1), the fluid stays between the walls, no velocity crosses a wall's node layers,
    and the first 20 steps agree with the oracle's."""
    from paper_2101_12408_amd import api
    from paper_2101_12408_amd import _lib as L
    S = sc.cavity2d()
    P, p = S["particles"], dict(S["params"], **TIGHT)
    N = len(P["m"])
    s = api.Scene(p, cap_part=N, cap_surf=20 * N, precision="fp64")
    Pd = s.to_device(P)
    Po = P
    for k in range(20):
        Po, _ = ostep.step(Po, p, implicit=True, step_index=k)
    order = np.arange(N)
    top_ux = []
    for k in range(300):
        Sd = s.sample_surface(Pd, step=k)
        s.step(Pd, Sd)
        order = order[s.view(L.F_PERM).cpu().numpy()]
        if k == 19:
            Q = _host_state(Pd, 2)
            inv = np.empty_like(order)
            inv[order] = np.arange(N)
            ev = rel(Q["v"][inv], Po["v"])
            log(f"  after 20 steps vs oracle: v rel {ev:.3e}")
            assert ev < 1e-6
        if k % 50 == 49:
            Q = _host_state(Pd, 2)
            y = Q["x"][:, 1]
            top = y > y.max() - 2 * p["dx"]
            top_ux.append(float(np.mean(Q["v"][top, 0])))
            log(f"  step {k + 1}: dt {s.stats()['dt']:.2e}, top u_x {top_ux[-1]:+.3e}")
    Q = _host_state(Pd, 2)
    dx = p["dx"]
    assert np.all(Q["x"] >= dx) and np.all(Q["x"] < 1 - dx)
    assert all(u > 0 for u in top_ux) and top_ux[-1] > top_ux[0]
    vh = s.view(L.F_VHAT).cpu().numpy()
    ti = api.tiled_index(2, p["n"])
    nat = np.empty_like(vh)
    nat[:, :] = vh[:, ti]
    grid = nat.reshape(2, p["n"], p["n"])          # [a][i1][i0]
    assert np.all(grid[0][:, :2] == 0) and np.all(grid[0][:, -2:] == 0)
    assert np.all(grid[1][:2, :] == 0) and np.all(grid[1][-2:, :] == 0)


@pytest.mark.parametrize("case", ["ramp2d", "ramp3d_small"])
def test_collision_step_matches_oracle_fp64(case):
    """Collision objects with Coulomb friction (the ramps of Section 6.3): from a state in
    contact (the oracle's trajectory after the droplet lands), one FP64 step against the
    oracle's."""
    if case == "ramp2d":
        S, pre = sc.ramp2d(v0=-3.0), 22
    else:
        S, pre = sc.ramp3d(n=32, radius=0.15, v0=-3.0), 12
    P, p = S["particles"], dict(S["params"], **TIGHT)
    for k in range(pre):
        P, _ = ostep.step(P, p, implicit=True, step_index=k)
    o, nr, _ = p["planes"][0]
    phi = (P["x"] - np.asarray(o)[:p["dim"]]) @ np.asarray(nr)[:p["dim"]]
    assert phi.min() < 0.5 * p["dx"]       # the droplet's stencils reach into the object
    surf = sampler.sample_surface(P["x"], p, step=pre)
    ref, info = ostep.step(P, p, surf, step_index=pre)
    got, st, rc = _gpu_step(P, surf, p)
    assert rc == 0
    for k in ("v", "A", "J", "x"):
        e = rel(got[k] - P[k], ref[k] - P[k]) if k in ("x", "J") else rel(got[k], ref[k])
        log(f"  {case} {k}: rel {e:.3e}")
        assert e < 1e-7, k


def test_ramp3d_friction_on_gpu():
    """The 3D ramp at 64^3 over 60 implicit steps in MIXED with the device sampler: the
    landed droplet slides down-slope, slower with friction 0.2 than without, and no
    particle ends more than 1.5 cells inside the ramp (the collision acts on grid nodes,
    so a particle's velocity also draws on the free nodes of its 3-node stencil above the
    plane: a grid-node collision bounds the penetration by the stencil's reach, not by 0)."""
    from paper_2101_12408_amd import api
    ux = []
    for mu in (0.0, 0.2):
        S = sc.ramp3d(mu=mu, v0=-3.0)
        P, p = S["particles"], S["params"]
        N = len(P["m"])
        s = api.Scene(p, cap_part=N, cap_surf=20 * N, precision="mixed")
        Pd = s.to_device(P)
        for k in range(60):
            s.step(Pd, s.sample_surface(Pd, step=k))
        Q = _host_state(Pd, 3)
        o, nr, _ = p["planes"][0]
        phi = (Q["x"] - np.asarray(o)) @ np.asarray(nr)
        ux.append(float(np.sum(Q["m"] * Q["v"][:, 0]) / Q["m"].sum()))
        log(f"  mu {mu}: mean u_x {ux[-1]:+.4e}, deepest particle {phi.min() / p['dx']:+.2f} dx")
        assert phi.min() > -1.5 * p["dx"]
    assert ux[0] < ux[1] < 0


def test_autotune_picks_a_layout_and_leaves_results_unchanged():
    """mpm_autotune times the tile kernels at every run length and keeps the fastest; the
    run length only deals tiles to workgroups, so a step is bitwise the same under the
    tuned layout, the built-in rule and an extreme fixed one."""
    from paper_2101_12408_amd import api
    S = sc.marangoni3d(n=64, radius=0.25)
    P, p = S["particles"], S["params"]
    surf = sampler.sample_surface(P["x"], p)
    res = []
    for mode in ("rule", "tuned", "fixed64"):
        s = api.Scene(p, cap_part=len(P["m"]), cap_surf=len(surf["s"]), precision="mixed")
        Pd, Sd = s.to_device(P, surf)
        if mode == "tuned":
            s.p2g(Pd, Sd)
            t = s.autotune()
            log(f"  autotune: {t}")
            assert set(t) == {"energy", "hess", "heat"}
            for name, (run, times) in t.items():
                assert run in times and all(v > 0 for v in times.values())
                assert times[run] == min(times.values())
        elif mode == "fixed64":
            s.tuning_set((64, 64, 64))
        s.step(Pd, Sd)
        res.append({k: v.cpu().numpy().copy() for k, v in Pd.items()})
    for r in res[1:]:
        for k in r:
            assert np.array_equal(r[k], res[0][k]), k
