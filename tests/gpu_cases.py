"""Shared set-up of the GPU parity tests: one seeded case evaluated by the oracle and by
the HIP library on identical inputs (in MIXED mode the inputs are rounded to float32
first and the oracle receives the rounded values)."""
from __future__ import annotations

import sys

import numpy as np

import mpm_scenes as sc
from oracle import energy, resample, sampler, solve, transfer

TOL_FP64 = 1e-10          # relative (norm-wise), FP64 mode
TOL_MIXED_FORCE = 1e-4    # relative, grid forces in MIXED mode


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / max(nb, 1e-300))


def rel_max(a, b):
    """Worst element: max_i |a_i - b_i| / max_i |b_i| (a norm-wise bound lets one element of
    a large array be off by sqrt(size) times the tolerance)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if b.size == 0:
        return 0.0
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def check(name, got, ref, tol, tol_max=None):
    """Norm-wise and element-wise relative error of got against ref, both below tol."""
    e, m = rel(got, ref), rel_max(got, ref)
    log(f"  {name}: rel {e:.3e}, worst element {m:.3e}")
    assert e < tol and m < (tol if tol_max is None else tol_max), (name, e, m)
    return e, m


def round_inputs(P, surf, precision):
    if precision == "fp64":
        return P, surf
    f = lambda a: np.asarray(a, np.float32).astype(np.float64)
    P2 = {k: (f(v) if v.dtype.kind == "f" else v) for k, v in P.items()}
    S2 = dict(surf, s=f(surf["s"]), dA=f(surf["dA"]))
    return P2, S2


def make_case(kind, dim=3, seed=0, precision="fp64", n=None, **kw):
    if kind in ("random", "dense"):
        # "dense": every particle in a box smaller than one cell, so that one cell tile holds
        # several chunks of points in every tile kernel (P2G 288 points per chunk in 3D, the
        # stress and heat kernels 576; 192 in 2D)
        n = n or (16 if dim == 3 else 32)
        count = kw.pop("count", 300 if kind == "random" else (1500 if dim == 3 else 1200))
        nsurf = kw.pop("nsurf", 200 if kind == "random" else 600)
        box = (0.3, 0.7) if kind == "random" else (0.5 + 0.1 / n, 0.5 + 0.9 / n)
        prm = dict(mu0=0.7, mu_k=0.01, mu_T0=300.0, g0=0.3, g1=0.004, gT0=300.0,
                   heat=1, cp=2.0, K=0.3, h=4.0, T_amb=330.0, b=3.0, dt=2e-3)
        prm.update(kw)
        S = sc.random_scene(dim, n, count, seed, box=box, **prm)
        P, p = S["particles"], S["params"]
        surf = sc.random_surface(P, nsurf, seed, dx=p["dx"], spread=0.8)
    else:
        S = sc.CONFIGS[kind](**({"n": n} if n else {}))
        P, p = S["particles"], dict(S["params"], **kw)
        surf = sampler.sample_surface(P["x"], p)
    P, surf = round_inputs(P, surf, precision)
    return P, surf, p


class OracleState:
    def __init__(self, P, surf, p):
        self.P, self.surf, self.p = P, surf, p
        self.split = resample.split(P, surf)
        self.grid = transfer.p2g(P, surf, self.split, p)
        self.setup = transfer.grid_setup(P, surf, self.split, self.grid, p)
        self.ctx = energy.Context(P, surf, self.grid, self.setup, p)
        self.heat = solve.Heat(P, surf, self.grid, self.setup, p)


class GpuState:
    def __init__(self, P, surf, p, precision="fp64"):
        from paper_2101_12408_amd import api
        self.api = api
        self.scene = api.Scene(p, cap_part=max(1, len(P["m"])), cap_surf=max(1, len(surf["s"])),
                               precision=precision)
        self.Pd, self.Sd = self.scene.to_device(P, surf)
        self.scene.p2g(self.Pd, self.Sd)
        self.tiled = api.tiled_index(p["dim"], p["n"])
        self.dim = p["dim"]

    def to_natural(self, t):
        """(ncomp, nn) or (nn,) tiled device tensor -> natural numpy (nn, ncomp) / (nn,)."""
        a = t.detach().cpu().numpy().astype(np.float64) if t.dtype.is_floating_point else t.cpu().numpy()
        if a.ndim == 2:
            return np.ascontiguousarray(a[:, self.tiled].T)
        return a[self.tiled]

    def from_natural(self, a):
        import torch
        a = np.asarray(a, np.float64)
        out = np.zeros((a.shape[1], a.shape[0])) if a.ndim == 2 else np.zeros(a.shape[0])
        if a.ndim == 2:
            out[:, self.tiled] = a.T
        else:
            out[self.tiled] = a
        return torch.from_numpy(out).to(device="cuda", dtype=self.scene.dtype).contiguous()
