"""One time step of the method, in the order of the paper's step list (Section 4):
resample the boundary, P2G, grid momentum and temperature update, G2P.

step(P, params, surf=None) returns (new particle state, info).  When surf is None the
surface samples are drawn from the level set of the current particles (Section 4.1.1);
tests pass the samples explicitly so that both implementations see identical inputs.
implicit=False is the explicit variant (q^ = 0 in eq. disc_force), used to pin the
conservation claims of Section 6.1.  With params["cfl"] > 0 the step's dt comes from
cfl_dt (the CFL-limited time step of Section 6).
"""
from __future__ import annotations

import numpy as np

from . import energy, resample, sampler, solve, transfer


def cfl_dt(P, params, implicit=True):
    """The time step of the next step under a CFL limit (the paper restricts dt to a range
    by the CFL condition without stating the rule; read as the classic one): the fastest
    particle, plus in explicit steps the pressure-wave speed sqrt(lambda / rho) of the
    weakly compressible fluid, may cross cfl dx in one step; clamped to [dt_min, dt_max].
    Particle speeds |v_p| = sqrt((v0^2 + v1^2) + v2^2), rho_p = m_p / V0_p."""
    v = P["v"]
    sp2 = v[:, 0] * v[:, 0]
    for a in range(1, v.shape[1]):
        sp2 = sp2 + v[:, a] * v[:, a]
    vmax = float(np.sqrt(np.max(sp2))) if len(sp2) else 0.0
    speed = vmax
    if not implicit:
        rho_min = float(np.min(P["m"] / P["V0"]))
        speed = vmax + float(np.sqrt(params["bulk"] / rho_min))
    dt = params["cfl"] * params["dx"] / speed if speed > 0 else params["dt_max"]
    return float(min(max(dt, params["dt_min"]), params["dt_max"]))


def prepare(P, params, surf=None, step_index=0):
    if surf is None:
        surf = sampler.sample_surface(P["x"], params, step_index)
    split = resample.split(P, surf)
    grid = transfer.p2g(P, surf, split, params)
    setup = transfer.grid_setup(P, surf, split, grid, params)
    ctx = energy.Context(P, surf, grid, setup, params)
    return surf, split, grid, setup, ctx


def step(P, params, surf=None, implicit=True, step_index=0):
    if params.get("cfl", 0.0) > 0:
        params = dict(params, dt=cfl_dt(P, params, implicit))
    surf, split, grid, setup, ctx = prepare(P, params, surf, step_index)
    info = dict(surf=surf, split=split, grid=grid, setup=setup)
    if implicit:
        vhat, st = solve.newton(ctx, params)
        info.update(st)
    else:
        vhat = solve.explicit_update(ctx)
    vhat = solve.collide(vhat, params)
    if params["heat"]:
        heat = solve.Heat(P, surf, grid, setup, params)
        That, hst = heat.solve(params)
        info.update(hst)
    else:
        That = setup["Tn"]
    newP = transfer.g2p(P, surf, split, vhat, That, params)
    if not params["heat"]:
        newP["T"] = P["T"].copy()
        newP["gradT"] = P["gradT"].copy()
    newP = transfer.phase_change(P["T"], newP, params)
    info.update(vhat=vhat, That=That, dt=params["dt"])
    return newP, info
