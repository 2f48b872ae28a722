"""One time step of the method, in the order of the paper's step list (Section 4):
resample the boundary, P2G, grid momentum and temperature update, G2P.

step(P, params, surf=None) returns (new particle state, info).  When surf is None the
surface samples are drawn from the level set of the current particles (Section 4.1.1);
tests pass the samples explicitly so that both implementations see identical inputs.
implicit=False is the explicit variant (q^ = 0 in eq. disc_force), used to pin the
conservation claims of Section 6.1.
"""
from __future__ import annotations

from . import energy, resample, sampler, solve, transfer


def prepare(P, params, surf=None, step_index=0):
    if surf is None:
        surf = sampler.sample_surface(P["x"], params, step_index)
    split = resample.split(P, surf)
    grid = transfer.p2g(P, surf, split, params)
    setup = transfer.grid_setup(P, surf, split, grid, params)
    ctx = energy.Context(P, surf, grid, setup, params)
    return surf, split, grid, setup, ctx


def step(P, params, surf=None, implicit=True, step_index=0):
    surf, split, grid, setup, ctx = prepare(P, params, surf, step_index)
    info = dict(surf=surf, split=split, grid=grid, setup=setup)
    if implicit:
        vhat, st = solve.newton(ctx, params)
        info.update(st)
    else:
        vhat = solve.explicit_update(ctx)
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
    info.update(vhat=vhat, That=That)
    return newP, info
