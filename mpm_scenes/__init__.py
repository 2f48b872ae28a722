"""Seeded synthetic scene generators shared by the oracle, the tests and the benchmark.

This module only lays out inputs: particle lattices, jitter, initial fields and the
material / solver parameters of each workload.  It contains none of the method's
arithmetic (no B-splines, no surface sampling, no transfers, no solves), so both the
CPU oracle and the GPU path may consume what it returns.

Every array is float64, natural (particle-major) order.  Positions live in the unit
domain [0,1]^d; the background grid has n nodes per axis at cell centres with
spacing dx = 1/n (the paper's cell-centred quadratic B-spline grid, Section 4.2).

Workloads (the paper uses no dataset; every scene here is procedural):
  square2d     2D square droplet relaxing under constant surface tension (64^2)
  marangoni3d  3D droplet with a linear temperature field and gamma(T) (128^3)
  contact3d    3D hemisphere-cap droplet on a static slab, three surface energies (192^3)
  meltslab3d   3D slab heated by the ambient through the Robin term, mu(T) (256^3, 8 ppc;
               meltslab3d_4ppc: the same slab at 4 particles per cell)
  ellipse2d    2D ellipse under surface tension, explicit steps (64^2)
  cavity2d     2D lid-driven Marangoni cavity, k = clamp(1 - T, 0, 1) (64^2)
  ramp2d/3d    droplet landing on a 5.5 degree ramp with Coulomb friction (32^2 / 64^3)
  serving      stream of small droplet scenes (n in {16,32,48,64,96})
"""
from __future__ import annotations

import copy
import math

import numpy as np

# Parameter defaults.  Keys mirror the fields of the C struct mpm_params.
DEFAULT_PARAMS = dict(
    dim=3, n=64, dx=1.0 / 64, dt=1e-3,
    gravity=(0.0, 0.0, 0.0),
    bulk=1e4,                       # lambda^l of Psi^p(J) = lambda/2 (J-1)^2
    mu0=0.0, mu_k=0.0, mu_T0=0.0,   # mu(T) = mu0 * exp(-mu_k (T - mu_T0))
    g0=0.07, g1=0.0, gT0=0.0,       # gamma(T) = clamp(g0 + g1 (T - gT0), gmin, gmax)
    gmin=0.0, gmax=1e30,
    gamma_by_label=0, gamma_label=(0.0, 0.0, 0.0, 0.0),
    heat=0, cp=1.0, K=0.0, h=0.0, T_amb=0.0, b=0.0, H=0.0,
    wall_layers=0,
    slab=0, slab_lo=(0.0, 0.0, 0.0), slab_hi=(0.0, 0.0, 0.0), slab_axis=1,
    label_lo=(0.0, 0.0, 0.0), label_hi=(0.0, 0.0, 0.0),
    newton_tol=1e-8, newton_max=20, cg_rel=1e-2, cg_max=1000, ls_max=10, ls_c1=1e-4,
    heat_tol=1e-10, heat_max=1000,
    hess_mode=0,                    # 0 = PSD (definiteness fix), 1 = EXACT
    krylov=0,                       # 0 = CG, 1 = MINRES (for the indefinite EXACT Hessian)
    cfl=0.0, dt_min=0.0, dt_max=0.0,  # cfl > 0: dt chosen per step, clamped to [dt_min, dt_max]
    planes=(),                      # collision half-spaces ((o, n, mu), ...): solid where (x-o).n < 0
    T_melt=-1e300,                  # particles with T < T_melt are fixed-corotated solids
    muh0=0.0, lamh0=0.0, kh=0.0, Th0=0.0,  # mu^h, lambda^h = (muh0, lamh0) exp(-kh (T - Th0))
    momentum_fix=1,
    term_mask=7,                    # bit0 J-term, bit1 surface, bit2 viscosity
    ls_radius=None,                 # union-of-spheres radius; None -> 0.73 dx (2D) / 0.867 dx (3D)
    sample_density=None,            # samples per unit area (3D) / length (2D); None -> 8/dx^2, 4/dx
    seed=0,
)


def make_params(**kw):
    p = copy.deepcopy(DEFAULT_PARAMS)
    for k, v in kw.items():
        if k not in p:
            raise KeyError(f"unknown parameter {k}")
        p[k] = v
    p["dx"] = 1.0 / p["n"]
    if p["ls_radius"] is None:
        p["ls_radius"] = (0.73 if p["dim"] == 2 else 0.867) * p["dx"]
    if p["sample_density"] is None:
        p["sample_density"] = (4.0 / p["dx"]) if p["dim"] == 2 else (8.0 / p["dx"] ** 2)
    g = list(p["gravity"]) + [0.0] * 3
    p["gravity"] = tuple(float(t) for t in g[:3])
    return p


# Four points per cell (3D): the corners of a regular tetrahedron inside the cell, at a
# quarter of the cell from its faces (the face-centred pattern).
TETRA4 = np.array([[0.25, 0.25, 0.25], [0.75, 0.75, 0.25], [0.75, 0.25, 0.75], [0.25, 0.75, 0.75]])


def lattice(n, dim, inside, seed, ppc_axis=2, jitter=0.25, lo=None, hi=None, offsets=None):
    """Jittered sub-cell lattice: ppc_axis^dim points per cell at offsets
    (k + 1/2)/ppc_axis * dx (or at the given per-cell offsets, in cells), each coordinate
    jittered by U[-jitter, jitter]*dx, kept where inside(x) is true.  Cells are visited
    z-major, x fastest; the jitter stream is numpy PCG64(seed), one draw per point and axis
    in visiting order."""
    dx = 1.0 / n
    lo = np.zeros(dim, int) if lo is None else np.asarray(lo, int)
    hi = np.full(dim, n, int) if hi is None else np.asarray(hi, int)
    rng = np.random.Generator(np.random.PCG64(seed))
    axes = [np.arange(lo[a], hi[a]) for a in range(dim)]
    cells = np.stack(np.meshgrid(*axes[::-1], indexing="ij")[::-1], -1).reshape(-1, dim)
    if offsets is None:
        sub = np.stack(np.meshgrid(*([np.arange(ppc_axis)] * dim)[::-1], indexing="ij")[::-1], -1).reshape(-1, dim)
        off = (sub + 0.5) / ppc_axis
    else:
        off = np.asarray(offsets, np.float64).reshape(-1, dim)
    pts = (cells[:, None, :] + off[None, :, :]).reshape(-1, dim) * dx
    pts = pts + rng.uniform(-jitter, jitter, size=pts.shape) * dx
    keep = inside(pts)
    return np.ascontiguousarray(pts[keep])


def particles_from_positions(x, dim, dx, rho=1000.0, ppc=None, T=None, gradT=None):
    N = x.shape[0]
    ppc = (2 ** dim) if ppc is None else ppc
    V0 = np.full(N, dx ** dim / ppc)
    return dict(
        x=np.ascontiguousarray(x, dtype=np.float64),
        v=np.zeros((N, dim)), A=np.zeros((N, dim, dim)), J=np.ones(N),
        V0=V0, m=rho * V0,
        T=np.zeros(N) if T is None else np.asarray(T, np.float64),
        gradT=np.zeros((N, dim)) if gradT is None else np.asarray(gradT, np.float64),
    )


def square2d(seed=1, n=64):
    """2D square droplet: [0.25,0.75]^2 at 2x2 per cell, rho 1000, bulk 1e4, gamma 0.07,
    no gravity, dt 1e-3, Newton tol 1e-8."""
    p = make_params(dim=2, n=n, dt=1e-3, bulk=1e4, g0=0.07, newton_tol=1e-8, seed=seed)
    inside = lambda q: np.all((q >= 0.25) & (q < 0.75), axis=1)
    x = lattice(n, 2, inside, seed)
    return dict(params=p, particles=particles_from_positions(x, 2, p["dx"]), name="square2d", steps=5)


def marangoni3d(seed=2, n=128, radius=0.2):
    """3D droplet, linear temperature in x (300 K at x=0.3 to 350 K at x=0.7),
    gamma(T) = 0.072 - 1.5e-4 (T-300), insulated heat solve (c_p 1, K 0.1)."""
    p = make_params(dim=3, n=n, dt=5e-4, bulk=1e4, g0=0.072, g1=-1.5e-4, gT0=300.0,
                    heat=1, cp=1.0, K=0.1, h=0.0, b=0.0, T_amb=300.0, seed=seed)
    c = np.array([0.5, 0.5, 0.5])
    inside = lambda q: np.sum((q - c) ** 2, axis=1) < radius ** 2
    lo = np.floor((c - radius) * n).astype(int) - 1
    hi = np.ceil((c + radius) * n).astype(int) + 1
    x = lattice(n, 3, inside, seed, lo=lo, hi=hi)
    T = 300.0 + 50.0 * (x[:, 0] - 0.3) / 0.4
    gT = np.zeros_like(x)
    gT[:, 0] = 125.0
    return dict(params=p, particles=particles_from_positions(x, 3, p["dx"], T=T, gradT=gT),
                name="marangoni3d", steps=20)


def contact3d(seed=3, n=192, radius=0.15):
    """3D hemisphere-cap droplet resting on a static slab y in [2dx, 6dx).  Surface
    samples inside the slab's (dilated) box take gamma_SL - gamma_SA, the rest gamma_LA.
    Nodes inside the slab box have zero normal (y) velocity."""
    dx = 1.0 / n
    yb = 6 * dx
    rls = 0.867 * dx
    p = make_params(dim=3, n=n, dt=5e-4, bulk=1e4, gravity=(0.0, -9.8, 0.0),
                    gamma_by_label=1, gamma_label=(0.072, 0.06 - 0.04, 0.0, 0.0),
                    slab=1, slab_lo=(2 * dx, 2 * dx, 2 * dx), slab_hi=(1 - 2 * dx, yb, 1 - 2 * dx),
                    slab_axis=1,
                    label_lo=(2 * dx - rls, 2 * dx - rls, 2 * dx - rls),
                    label_hi=(1 - 2 * dx + rls, yb + rls, 1 - 2 * dx + rls),
                    momentum_fix=0, seed=seed)
    c = np.array([0.5, yb, 0.5])
    inside = lambda q: (np.sum((q - c) ** 2, axis=1) < radius ** 2) & (q[:, 1] >= yb)
    lo = np.floor((c - radius) * n).astype(int) - 1
    hi = np.ceil((c + radius) * n).astype(int) + 1
    lo[1] = int(round(yb * n))
    x = lattice(n, 3, inside, seed, lo=lo, hi=hi)
    return dict(params=p, particles=particles_from_positions(x, 3, dx), name="contact3d", steps=50)


def meltslab3d(seed=4, n=256, ppc_axis=2, lo=0.2, hi=0.8, height=0.2, solid=False, ppc=None):
    """3D wax slab x,z in [lo,hi] (default [0.2,0.8]), y in [2dx, 2dx+height] (default 0.2),
    T0 290 K heated by a 400 K ambient through the Robin term (h 20, b 0, K 0.25, c_p 1),
    mu(T) = 1e3 exp(-0.05 (T-290)), gamma(T) as in marangoni3d, gravity -9.8, slip floor
    (two node layers).  solid=True: the wax starts as a fixed-corotated solid (F = I) that
    melts at T_melt = 300 K (Section 3.5), Lame constants (5e3, 1e4) exp(-0.05 (T - 290)).
    ppc = 4: four particles per cell (TETRA4) instead of ppc_axis^3."""
    dx = 1.0 / n
    extra = dict(T_melt=300.0, muh0=5e3, lamh0=1e4, kh=0.05, Th0=290.0) if solid else {}
    p = make_params(dim=3, n=n, dt=1e-3, bulk=1e4, gravity=(0.0, -9.8, 0.0),
                    mu0=1e3, mu_k=0.05, mu_T0=290.0,
                    g0=0.072, g1=-1.5e-4, gT0=300.0,
                    heat=1, cp=1.0, K=0.25, h=20.0, b=0.0, T_amb=400.0,
                    wall_layers=2, momentum_fix=0, seed=seed, **extra)
    y0, y1 = 2 * dx, 2 * dx + height
    inside = lambda q: (np.all((q[:, [0, 2]] >= lo) & (q[:, [0, 2]] < hi), axis=1)
                        & (q[:, 1] >= y0) & (q[:, 1] < y1))
    clo = np.array([int(lo * n) - 1, 2, int(lo * n) - 1])
    chi = np.array([int(hi * n) + 2, int(y1 * n) + 2, int(hi * n) + 2])
    if ppc == 4:
        x = lattice(n, 3, inside, seed, lo=clo, hi=chi, offsets=TETRA4)
    else:
        x = lattice(n, 3, inside, seed, ppc_axis=ppc_axis, lo=clo, hi=chi)
    T = np.full(x.shape[0], 290.0)
    P = particles_from_positions(x, 3, dx, ppc=4 if ppc == 4 else ppc_axis ** 3, T=T)
    if solid:
        P["F"] = np.tile(np.eye(3), (x.shape[0], 1, 1))
    name = "meltslab3d_solid" if solid else ("meltslab3d_4ppc" if ppc == 4 else "meltslab3d")
    return dict(params=p, particles=P, name=name, steps=20)


def ellipse2d(seed=6, n=64, cfl=0.0):
    """The oscillating ellipse of the paper's conservation example (Section 6.1): zero
    gravity, bulk 4166.67, surface tension k = 0.1, dx = 1/64 (the paper's 1/63 is not a
    multiple of the 8-node tiles), semi-axes 0.2 and 0.12 about the centre, 8 particles per
    cell drawn uniformly in each cell and kept inside the ellipse, density 1000.  Explicit
    stepping; with cfl > 0 the time step is CFL-limited to [1e-6, 1e-4] as in the paper, which
    gives no CFL number: with the pressure-wave speed sqrt(4166.67 / 1000) = 2.04, cfl = 0.01
    puts the step at about 7.7e-5, inside the range."""
    p = make_params(dim=2, n=n, dt=1e-5, bulk=4166.67, g0=0.1, seed=seed, cfl=cfl, dt_min=1e-6, dt_max=1e-4)
    rng = np.random.default_rng(seed)
    lo, hi = n // 4, 3 * n // 4
    cells = np.stack(np.meshgrid(np.arange(lo, hi), np.arange(lo, hi), indexing="xy"), -1).reshape(-1, 2)
    x = (cells[:, None, :] + rng.uniform(0, 1, size=(len(cells), 8, 2))).reshape(-1, 2) / n
    x = x[((x[:, 0] - 0.5) / 0.2) ** 2 + ((x[:, 1] - 0.5) / 0.12) ** 2 < 1]
    return dict(params=p, particles=particles_from_positions(x, 2, p["dx"], ppc=8), name="ellipse2d", steps=120)


def cavity2d(seed=7, n=64, cfl=0.5):
    """The 2D lid-driven Marangoni cavity (Section 6.4): the unit square filled with fluid
    up to height 1 - 4 dx between slip walls (two node layers each side), 2x2 particles per
    cell, temperature linear from 1 at the left wall to 0 at the right (carried by the
    particles, no conduction), k = clamp(1 - T, 0, 1) on the free surface, no gravity,
    viscosity 1e-6, implicit steps with dt <= 1e-3 (CFL 0.5).  The paper's dx = 1/63 is
    not a multiple of the 8-node tiles; n = 64.  Surface samples against the walls (outside
    [2dx, 1-2dx) x [2dx, 1)) carry no surface energy: the paper drives the flow by the free
    surface alone and states no wall energy."""
    dx = 1.0 / n
    p = make_params(dim=2, n=n, dt=1e-3, bulk=1e4, g0=1.0, g1=-1.0, gT0=0.0, gmin=0.0, gmax=1.0,
                    mu0=1e-6, wall_layers=2, momentum_fix=0,
                    gamma_by_label=2, gamma_label=(0.0, 0.0, 0.0, 0.0),
                    label_lo=(2 * dx, 2 * dx, 0.0), label_hi=(1 - 2 * dx, 1.0, 0.0),
                    cfl=cfl, dt_min=1e-6, dt_max=1e-3, seed=seed)
    top = 1 - 4 * dx
    inside = lambda q: (q[:, 0] >= 2 * dx) & (q[:, 0] < 1 - 2 * dx) & (q[:, 1] >= 2 * dx) & (q[:, 1] < top)
    x = lattice(n, 2, inside, seed, lo=np.array([2, 2]), hi=np.array([n - 2, n - 4]))
    x0, x1 = 2 * dx, 1 - 2 * dx
    T = (x1 - x[:, 0]) / (x1 - x0)
    gT = np.zeros_like(x)
    gT[:, 0] = -1.0 / (x1 - x0)
    return dict(params=p, particles=particles_from_positions(x, 2, dx, T=T, gradT=gT), name="cavity2d", steps=500)


def _ramp_plane(theta_deg, o):
    t = math.radians(theta_deg)
    return (tuple(o), (-math.sin(t), math.cos(t), 0.0))


def ramp2d(seed=8, n=32, mu=0.2, theta=5.5, radius=0.15, v0=-0.5):
    """2D droplet landing on a ramp (the mechanism of Section 6.3 in 2D): a static
    half-space through (0.5, 0.25) rising at theta degrees toward +x, Coulomb friction mu,
    the droplet (radius 0.15 at 2x2 per cell, gamma 0.072) just above it and moving down
    at v0, gravity, slip domain walls, dt 1e-3."""
    dx = 1.0 / n
    o, nrm = _ramp_plane(theta, (0.5, 0.25, 0.0))
    p = make_params(dim=2, n=n, dt=1e-3, bulk=1e4, g0=0.072, gravity=(0.0, -9.8, 0.0), wall_layers=2,
                    momentum_fix=0, planes=((o, nrm, mu),), seed=seed)
    t = math.radians(theta)
    c = np.array([0.6, 0.25 + (0.6 - 0.5) * math.tan(t) + (radius + 1.5 * dx) / math.cos(t)])
    inside = lambda q: np.sum((q - c) ** 2, axis=1) < radius ** 2
    x = lattice(n, 2, inside, seed)
    P = particles_from_positions(x, 2, dx)
    P["v"][:, 1] = v0
    return dict(params=p, particles=P, name="ramp2d", steps=100)


def ramp3d(seed=9, n=64, mu=0.2, theta=5.5, radius=0.1, v0=-0.5):
    """3D droplet falling on a 5.5 degree ramp with Coulomb friction 0.2 (Section 6.3; one
    drop, gamma_LA 0.072 everywhere: the paper's per-ratio wetting of the ramp would need
    labels along the inclined plane, which the box labels do not give), 8 particles per
    cell, gravity, slip domain walls, dt 1e-3.  The paper's dx = 1/63 becomes 1/64."""
    dx = 1.0 / n
    o, nrm = _ramp_plane(theta, (0.5, 0.25, 0.5))
    p = make_params(dim=3, n=n, dt=1e-3, bulk=1e4, g0=0.072, gravity=(0.0, -9.8, 0.0), wall_layers=2,
                    momentum_fix=0, planes=((o, nrm, mu),), seed=seed)
    t = math.radians(theta)
    c = np.array([0.6, 0.25 + (0.6 - 0.5) * math.tan(t) + (radius + 1.5 * dx) / math.cos(t), 0.5])
    inside = lambda q: np.sum((q - c) ** 2, axis=1) < radius ** 2
    lo = np.floor((c - radius) * n).astype(int) - 1
    hi = np.ceil((c + radius) * n).astype(int) + 1
    x = lattice(n, 3, inside, seed, lo=lo, hi=hi)
    P = particles_from_positions(x, 3, dx)
    P["v"][:, 1] = v0
    return dict(params=p, particles=P, name="ramp3d", steps=100)


def droplet3d(n, seed, gamma0, grad, radius=0.24, dt=5e-4):
    """One serving-stream scene: sphere r=0.24 at the centre, linear temperature
    T = 300 + grad . (x - c), gamma(T) = gamma0 - 1.5e-4 (T - 300)."""
    p = make_params(dim=3, n=n, dt=dt, bulk=1e4, g0=gamma0, g1=-1.5e-4, gT0=300.0,
                    heat=1, cp=1.0, K=0.1, h=0.0, b=0.0, T_amb=300.0, seed=seed)
    c = np.full(3, 0.5)
    inside = lambda q: np.sum((q - c) ** 2, axis=1) < radius ** 2
    lo = np.floor((c - radius) * n).astype(int) - 1
    hi = np.ceil((c + radius) * n).astype(int) + 1
    x = lattice(n, 3, inside, seed, lo=lo, hi=hi)
    grad = np.asarray(grad, np.float64)
    T = 300.0 + (x - c) @ grad
    gT = np.tile(grad, (x.shape[0], 1))
    return dict(params=p, particles=particles_from_positions(x, 3, p["dx"], T=T, gradT=gT),
                name=f"droplet{n}", steps=1)


class ServingInputs:
    """Inputs of a serving stream without rebuilding a lattice per request: one droplet
    lattice per grid size (seed = n), and per request its own parameters (gamma0, sampler
    seed) and linear temperature field.  soa(req) returns the host SoA double arrays
    (x, v, A, J, V0, m shared per size; T, gradT per request)."""

    def __init__(self, radius=0.24):
        self.radius = radius
        self.base = {}

    def _lattice(self, n):
        if n not in self.base:
            S = droplet3d(n, n, 0.05, [0.0, 0.0, 0.0], radius=self.radius)
            P = S["particles"]
            N = len(P["m"])
            self.base[n] = dict(x=np.ascontiguousarray(P["x"].T), v=np.zeros((3, N)), A=np.zeros((9, N)),
                                J=np.ones(N), V0=np.ascontiguousarray(P["V0"]), m=np.ascontiguousarray(P["m"]))
        return self.base[n]

    def params(self, req):
        return make_params(dim=3, n=req["n"], dt=5e-4, bulk=1e4, g0=req["gamma0"], g1=-1.5e-4, gT0=300.0,
                           heat=1, cp=1.0, K=0.1, h=0.0, b=0.0, T_amb=300.0, seed=req["seed"])

    def soa(self, req):
        b = self._lattice(req["n"])
        grad = np.asarray(req["grad"], np.float64)
        T = 300.0 + (b["x"] - 0.5).T @ grad
        gT = np.ascontiguousarray(np.repeat(grad[:, None], b["x"].shape[1], axis=1))
        return dict(b, T=np.ascontiguousarray(T), gradT=gT)


def serving_stream(count=512, rate=200.0, seed=5, sizes=(16, 32, 48, 64, 96)):
    """Request stream: exponential inter-arrival times (mean 1/rate), grid edge uniform
    in sizes, gamma0 ~ U[0.02,0.08], temperature gradient = random direction x U[0,125]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    reqs = []
    for i in range(count):
        n = int(rng.choice(sizes))
        g0 = float(rng.uniform(0.02, 0.08))
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        grad = d * rng.uniform(0.0, 125.0)
        reqs.append(dict(arrival=float(t[i]), n=n, gamma0=g0, grad=grad.tolist(), seed=1000 + i))
    return reqs


def random_scene(dim, n, count, seed, box=(0.3, 0.7), vel=0.5, affine=5.0, temp=True,
                 **param_kw):
    """Small random scene for unit and property tests: count particles uniform in
    box^dim with random v, A, J, T, grad T."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = make_params(dim=dim, n=n, seed=seed, **param_kw)
    x = rng.uniform(box[0], box[1], size=(count, dim))
    P = particles_from_positions(x, dim, p["dx"])
    P["v"] = rng.uniform(-vel, vel, size=(count, dim))
    P["A"] = rng.uniform(-affine, affine, size=(count, dim, dim))
    P["J"] = rng.uniform(0.9, 1.1, size=count)
    P["m"] = P["m"] * rng.uniform(0.5, 1.5, size=count)
    if temp:
        P["T"] = rng.uniform(280.0, 320.0, size=count)
        P["gradT"] = rng.uniform(-50.0, 50.0, size=(count, dim))
    return dict(params=p, particles=P, name=f"random{dim}d", steps=1)


def random_surface(P, count, seed, spread=1.0, dx=None, dim=None):
    """Synthetic surface quadrature points for unit tests of the transfer and energy
    operators: points near randomly chosen particles with random area-weighted normals.
    (The real workloads sample the union-of-spheres level set instead.)"""
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    x = P["x"]
    dim = x.shape[1] if dim is None else dim
    base = x[rng.integers(0, x.shape[0], size=count)]
    s = base + rng.uniform(-spread, spread, size=(count, dim)) * dx
    nrm = rng.normal(size=(count, dim))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    dA = nrm * rng.uniform(0.05, 0.3, size=(count, 1)) * dx ** (dim - 1)
    label = rng.integers(0, 2, size=count).astype(np.int32)
    return dict(s=np.ascontiguousarray(s), dA=np.ascontiguousarray(dA), label=label)


CONFIGS = dict(square2d=square2d, marangoni3d=marangoni3d, contact3d=contact3d,
               meltslab3d=meltslab3d, cavity2d=cavity2d, ramp2d=ramp2d, ramp3d=ramp3d,
               meltslab3d_4ppc=lambda **kw: meltslab3d(ppc=4, **kw))
