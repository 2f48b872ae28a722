"""Parity at the full size of the 3D Marangoni droplet (128^3 grid, ~560k particles, the
benchmark workload): every operator against the vectorized oracle on the same inputs,
in the precision and launch configuration the benchmark uses (MIXED) and in FP64."""
import numpy as np
import pytest

import mpm_scenes as sc
from gpu_cases import GpuState, OracleState, log, rel, round_inputs

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
    for f, ref in ((L.F_MASS, o.grid["m"]), (L.F_MOM, o.grid["mv"]), (L.F_TN, o.setup["Tn"])):
        e = rel(g.to_natural(g.scene.view(f)), ref)
        log(f"  field {f}: rel {e:.3e}")
        assert e < tolf
    rng = np.random.default_rng(3)
    dof = o.setup["dof"]
    v = o.setup["vn"] + rng.normal(size=o.ctx.vn.shape) * 0.01 * dof[:, None]
    if precision != "fp64":
        v = v.astype(np.float32).astype(np.float64)
    grad = g.scene.grid_vector()
    g.scene.energy_grad(g.from_natural(v), grad)
    e = rel(g.to_natural(grad)[dof], o.ctx.project(o.ctx.grad_Phi(v))[dof])
    log(f"  energy_grad rel {e:.3e}")
    assert e < (1e-10 if precision == "fp64" else 1e-4)
    w = rng.normal(size=o.ctx.vn.shape) * dof[:, None]
    if precision != "fp64":
        w = w.astype(np.float32).astype(np.float64)
    out = g.scene.grid_vector()
    g.scene.hessvec(g.from_natural(v), g.from_natural(w), 1.0, out)
    e = rel(g.to_natural(out)[dof], o.ctx.project(o.ctx.hessvec(v, o.ctx.project(w), 1.0))[dof])
    log(f"  hessvec rel {e:.3e}")
    assert e < (1e-10 if precision == "fp64" else 1e-4)
    T = (300 + rng.normal(size=o.setup["Tn"].shape)) * dof
    out1 = g.scene.grid_vector(1)[0]
    g.scene.heat_apply(g.from_natural(T), out1)
    e = rel(g.to_natural(out1)[dof], o.heat.apply(T)[dof])
    log(f"  heat_apply rel {e:.3e}")
    assert e < (1e-10 if precision == "fp64" else 1e-5)
