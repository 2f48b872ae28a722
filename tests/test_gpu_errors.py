"""GPU: the error contract of the C ABI.  A latched device-side failure is returned by the
step that met it, its outputs are still written, and the other scenes of the same
mpm_step batch are unaffected (bitwise the same as stepped alone).

  MPM_ENONFINITE  a NaN velocity of one particle makes the scene's energy and gradient
                  NaN; Newton stops at its first check;
  MPM_ENOCONV     newton_max = 1 with a tolerance one Newton step cannot meet;
  MPM_EDOMAIN     (test_gpu_parity) a particle outside [dx, 1 - dx)^d.
"""
import numpy as np
import pytest

import mpm_scenes as sc
from gpu_cases import log

pytestmark = pytest.mark.gpu

SPECS = [(16, 61, 0.05, [40, 0, 0]), (24, 62, 0.03, [0, 30, 10]), (16, 63, 0.07, [0, 0, 90])]


def _scenes(precision, bad=None, **kw):
    from paper_2101_12408_amd import api
    out = []
    for i, (n, seed, g0, grad) in enumerate(SPECS):
        S = sc.droplet3d(n, seed, g0, grad)
        P, p = S["particles"], dict(S["params"], **kw)
        rng = np.random.default_rng(seed)
        P["v"] = rng.normal(size=P["v"].shape) * 0.02
        if i == bad:
            P["v"][5, 1] = np.nan
        surf = api.sample_surface(P["x"], p)
        s = api.Scene(p, cap_part=len(P["m"]), cap_surf=len(surf["s"]), precision=precision)
        Pd, Sd = s.to_device(P, surf)
        out.append((s, Pd, Sd))
    return out


def _host(Pd):
    return {k: v.cpu().numpy().copy() for k, v in Pd.items()}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_nonfinite_is_latched_and_isolated(precision):
    from paper_2101_12408_amd import _lib as L
    from paper_2101_12408_amd import api
    alone = {}
    for i, (s, Pd, Sd) in enumerate(_scenes(precision)):
        if i != 1:
            assert s.step(Pd, Sd, check=False) == L.MPM_OK
            alone[i] = _host(Pd)
    batch = _scenes(precision, bad=1)
    rc = api.mpm_step([b[0] for b in batch], [b[1] for b in batch], [b[2] for b in batch], check=False)
    st = [b[0].stats() for b in batch]
    log(f"  {precision}: batch rc {rc}, per-scene status {[x['status'] for x in st]}")
    assert rc == L.MPM_ENONFINITE
    assert st[1]["status"] == L.MPM_ENONFINITE and st[0]["status"] == L.MPM_OK and st[2]["status"] == L.MPM_OK
    assert batch[1][0].status() == L.MPM_ENONFINITE      # stays latched until the next p2g
    for i in (0, 2):
        got = _host(batch[i][1])
        for k in got:
            assert np.array_equal(got[k], alone[i][k]), (i, k)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noconv_is_reported_with_outputs_written(precision):
    from paper_2101_12408_amd import _lib as L
    from paper_2101_12408_amd import api
    good = _scenes(precision)
    capped = _scenes(precision, newton_max=1, newton_tol=1e-14)
    x0 = [Pd["x"].double().cpu().numpy().copy() for _, Pd, _ in capped]
    rc = api.mpm_step([b[0] for b in capped], [b[1] for b in capped], [b[2] for b in capped], check=False)
    st = [b[0].stats() for b in capped]
    log(f"  {precision}: rc {rc}, newton {[x['newton_iters'] for x in st]}, converged {[x['converged'] for x in st]}")
    assert rc == L.MPM_ENOCONV
    assert all(x["status"] == L.MPM_ENOCONV and x["newton_iters"] == 1 and x["converged"] == 0 for x in st)
    for (s, Pd, _), x in zip(capped, x0):
        xn = Pd["x"].double().cpu().numpy()
        assert np.all(np.isfinite(xn)) and not np.array_equal(np.sort(xn, axis=1), np.sort(x, axis=1))
    # the same scenes without the cap converge
    rc = api.mpm_step([b[0] for b in good], [b[1] for b in good], [b[2] for b in good], check=False)
    assert rc == L.MPM_OK
