"""Degenerate inputs through the C ABI: a step with particles and no surface samples (the
surface term is absent, the rest of the step against the oracle in FP64) and a scene
without particles (every call returns MPM_OK and the step leaves nothing behind)."""
import numpy as np
import pytest

import mpm_scenes as sc
from gpu_cases import log, rel
from oracle import step as ostep
from test_gpu_step import TIGHT, _gpu_step

pytestmark = pytest.mark.gpu

NO_SURF = {2: dict(s=np.zeros((0, 2)), dA=np.zeros((0, 2)), label=np.zeros(0, np.int32)),
           3: dict(s=np.zeros((0, 3)), dA=np.zeros((0, 3)), label=np.zeros(0, np.int32))}


@pytest.mark.parametrize("dim", [2, 3])
def test_step_without_surface_samples_matches_oracle_fp64(dim):
    S = sc.random_scene(dim, 16 if dim == 3 else 32, 400, 20 + dim, box=(0.35, 0.65), mu0=0.5, heat=1,
                        cp=2.0, K=0.3, h=4.0, T_amb=330.0, dt=2e-3)
    P, p = S["particles"], dict(S["params"], **TIGHT)
    surf = NO_SURF[dim]
    log(f"case step without samples {dim}d")
    ref, info = ostep.step(P, p, surf)
    got, st, rc = _gpu_step(P, surf, p)
    log(f"  gpu newton {st['newton_iters']} cg {st['cg_iters']} rc {rc}; oracle newton {info['newton']} cg {info['cg']}")
    assert rc == 0
    for k in ("v", "A", "J", "x", "T", "gradT"):
        e = rel(got[k] - P[k], ref[k] - P[k]) if k in ("x", "J") else rel(got[k], ref[k])
        log(f"  {k}: rel {e:.3e}")
        assert e < 1e-7, k


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("implicit", [True, False])
def test_empty_scene_steps(precision, implicit):
    from paper_2101_12408_amd import api
    S = sc.square2d(n=32)
    p = S["params"]
    E = dict(x=np.zeros((0, 2)), v=np.zeros((0, 2)), A=np.zeros((0, 2, 2)), J=np.zeros(0), V0=np.zeros(0),
             m=np.zeros(0), T=np.zeros(0), gradT=np.zeros((0, 2)))
    log(f"case empty scene {precision} implicit={implicit}")
    s = api.Scene(p, cap_part=16, cap_surf=16, precision=precision)
    Pd, Sd = s.to_device(E, NO_SURF[2])
    for _ in range(2):
        rc = s.step(Pd, Sd, implicit=implicit, check=False)
        assert rc == 0, rc
    st = s.stats()
    log(f"  stats newton {st['newton_iters']} cg {st['cg_iters']}")
    assert st["cg_iters"] == 0
