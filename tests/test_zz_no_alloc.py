"""GPU: mpm_step_noalloc (the step on the library's static scratch, no context, no
workspace, nothing allocated) against mpm_step on a context over a caller workspace, on
the same inputs: the particle state after the step is bitwise the same.  Three calls in a
row, each smaller scene after a larger one (the scratch keeps the last call's contents,
so every call must clear what it needs), and a scene too large for the scratch is
refused with MPM_ENOMEM."""
import numpy as np
import pytest

import mpm_scenes as sc
from gpu_cases import log

pytestmark = pytest.mark.gpu


def _reference(S, precision, implicit=True):
    from paper_2101_12408_amd import api
    P, p = S["particles"], S["params"]
    surf = api.sample_surface(P["x"], p)
    s = api.Scene(p, cap_part=len(P["m"]), cap_surf=max(1, len(surf["s"])), precision=precision)
    Pd, Sd = s.to_device(P, surf)
    rc = s.step(Pd, Sd, implicit=implicit, check=False)
    out = {k: v.cpu().numpy().copy() for k, v in Pd.items()}
    s.close()
    return rc, out, surf


def _noalloc(S, surf, precision, implicit=True):
    from paper_2101_12408_amd import api
    P, p = S["particles"], S["params"]
    s = api.Scene(p, cap_part=1, cap_surf=1, precision=precision)    # only for to_device
    Pd, Sd = s.to_device(P, surf)
    rc, nb = api.step_noalloc(p, Pd, Sd, implicit=implicit, precision=precision, check=False)
    return rc, nb, {k: v.cpu().numpy().copy() for k, v in Pd.items()}


def test_noalloc_matches_mpm_step_on_consecutive_calls():
    rng = np.random.default_rng(9)
    cases = [("droplet32 mixed", sc.droplet3d(32, 71, 0.05, [40, 0, 0]), "mixed"),
             ("droplet16 mixed", sc.droplet3d(16, 72, 0.03, [0, 30, 10]), "mixed"),
             ("square2d32 fp64", sc.square2d(n=32), "fp64")]
    for name, S, prec in cases:
        S["particles"]["v"] = rng.normal(size=S["particles"]["v"].shape) * 0.02
        rc_ref, ref, surf = _reference(S, prec)
        rc, nb, got = _noalloc(S, surf, prec)
        log(f"  {name}: N={len(S['particles']['m'])} S={len(surf['s'])}: mpm_step rc {rc_ref}, "
            f"mpm_step_noalloc rc {rc} (scratch {nb >> 20} MiB)")
        assert rc_ref == 0 and rc == 0
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (name, k)


def test_noalloc_refuses_a_scene_larger_than_the_scratch():
    import torch
    from paper_2101_12408_amd import _lib as L
    from paper_2101_12408_amd import api
    S = sc.droplet3d(96, 73, 0.05, [0, 0, 0])
    P, p = S["particles"], S["params"]
    s = api.Scene(p, cap_part=1, cap_surf=1, precision="fp64")
    Pd = s.to_device(P)
    x0 = Pd["x"].clone()
    rc, nb = api.step_noalloc(p, Pd, None, precision="fp64", check=False)
    msg = L.load().mpm_last_error(None).decode()
    log(f"  droplet96 fp64: rc {rc}: {msg}")
    assert rc == L.MPM_ENOMEM and "scratch" in msg
    assert torch.equal(Pd["x"], x0)
