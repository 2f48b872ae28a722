"""GPU surface sampler (mpm_sample_surface_dev, Section 4.1.1) against the oracle's sampler
and the host input stage: the same samples in the same order (counts exact, labels exact,
positions and area vectors within the round-off of the oracle's own normalization), bit
for bit equal to the host stage, and a step fed with the device samples equal to the
step fed with the host's."""
import numpy as np
import pytest

import mpm_scenes as sc
from gpu_cases import log
from oracle import sampler

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "square2d":
        return sc.square2d(n=32)
    if name == "ellipse2d":
        return sc.ellipse2d()
    if name == "droplet3d":
        return sc.droplet3d(16, 3, 0.05, [10, 0, 0])
    if name == "contact3d":
        return sc.contact3d(n=64, radius=0.08)
    if name == "marangoni3d":
        return sc.marangoni3d(n=128, radius=0.2)
    raise KeyError(name)


def _device_samples(P, p, precision, step):
    from paper_2101_12408_amd import api
    N = len(P["m"])
    s = api.Scene(p, cap_part=N, cap_surf=max(64, 4 * N), precision=precision)
    Pd = s.to_device(P)
    S = s.sample_surface(Pd, step=step)
    out = dict(s=S["s"].double().cpu().numpy().T, dA=S["dA"].double().cpu().numpy().T,
               label=S["label"].cpu().numpy())
    return out, s, Pd, S


@pytest.mark.parametrize("name", ["square2d", "ellipse2d", "droplet3d", "contact3d", "marangoni3d"])
def test_device_sampler_matches_oracle_fp64(name):
    S = _case(name)
    P, p = S["particles"], S["params"]
    log(f"  sampler {name}: {len(P['m'])} particles, n={p['n']}")
    ref = sampler.sample_surface(P["x"], p, step=3)
    got, *_ = _device_samples(P, p, "fp64", 3)
    log(f"  {len(got['s'])} samples (oracle {len(ref['s'])})")
    assert len(got["s"]) == len(ref["s"]) > 0
    assert np.max(np.abs(got["s"] - ref["s"])) <= 1e-13
    assert np.max(np.abs(got["dA"] - ref["dA"])) <= 1e-15
    assert np.array_equal(got["label"], ref["label"])
    if name == "contact3d":
        assert 0 < ref["label"].sum() < len(ref["label"])


@pytest.mark.parametrize("name", ["square2d", "droplet3d", "contact3d"])
def test_device_sampler_equals_host_stage_bitwise(name):
    """The device sampler and the host stage take every operation in the same order."""
    from paper_2101_12408_amd import api
    S = _case(name)
    P, p = S["particles"], S["params"]
    for step in (0, 7):
        host = api.sample_surface(P["x"], p, step=step)
        got, *_ = _device_samples(P, p, "fp64", step)
        assert len(got["s"]) == len(host["s"])
        assert np.array_equal(got["s"], host["s"])
        assert np.array_equal(got["dA"], host["dA"])
        assert np.array_equal(got["label"], host["label"])


def test_device_sampler_mixed_positions():
    """MIXED: the sampler reads FP32 positions and computes in FP64; its samples are the
    oracle's on those positions, rounded to FP32."""
    S = _case("contact3d")
    P, p = S["particles"], S["params"]
    P32 = {k: v.astype(np.float32).astype(np.float64) for k, v in P.items()}
    ref = sampler.sample_surface(P32["x"], p, step=1)
    got, *_ = _device_samples(P32, p, "mixed", 1)
    assert len(got["s"]) == len(ref["s"]) > 0
    eps32 = 2.0 ** -24
    assert np.all(np.abs(got["s"] - ref["s"]) <= eps32 * np.abs(ref["s"]) + 1e-13)
    assert np.all(np.abs(got["dA"] - ref["dA"]) <= eps32 * np.abs(ref["dA"]) + 1e-15)
    assert np.array_equal(got["label"], ref["label"])


def test_device_sampler_empty_and_small_cap():
    """No particles: no samples.  A buffer smaller than the count: nothing written, the
    count returned, and the wrapper's second call with the exact capacity succeeds."""
    from paper_2101_12408_amd import api
    S = _case("droplet3d")
    P, p = S["particles"], S["params"]
    N = len(P["m"])
    s = api.Scene(p, cap_part=N, cap_surf=16, precision="fp64")
    Pd = s.to_device(P)
    out = s.sample_surface(Pd, step=0, cap=16)
    host = api.sample_surface(P["x"], p, step=0)
    assert out["s"].shape[1] == len(host["s"]) > 16
    assert np.array_equal(out["s"].cpu().numpy().T, host["s"])
    empty = {k: v[:, :0].contiguous() if v.dim() == 2 else v[:0] for k, v in Pd.items()}
    assert s.sample_surface(empty, step=0)["s"].shape[1] == 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_step_with_device_samples_equals_host_samples(precision):
    """An implicit step fed with the device sampler's output is bitwise the step fed with
    the host stage's samples of the same positions."""
    from paper_2101_12408_amd import api
    S = sc.marangoni3d(n=32, radius=0.25)
    P, p = S["particles"], S["params"]
    if precision == "mixed":
        P = {k: v.astype(np.float32).astype(np.float64) for k, v in P.items()}
    N = len(P["m"])
    res = []
    for mode in ("host", "device"):
        s = api.Scene(p, cap_part=N, cap_surf=4 * N, precision=precision)
        Pd = s.to_device(P)
        for k in range(2):
            if mode == "host":
                xh = Pd["x"].double().cpu().numpy().T.copy()
                Sd = s.to_device(S=api.sample_surface(xh, p, step=k))
            else:
                Sd = s.sample_surface(Pd, step=k)
            s.step(Pd, Sd)
        res.append({k: v.cpu().numpy().copy() for k, v in Pd.items()})
    for k in res[0]:
        assert np.array_equal(res[0][k], res[1][k]), k
