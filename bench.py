"""Benchmark of the implicit APIC MPM hot path on one MI355X.

Headline workload: the melting slab at the largest single-GPU size, 256^3 grid on the
unit cube, box 0.6 x 0.2 x 0.6 at 8 particles per cell (9,663,637 particles, ~966k
surface samples per step), T0 290 K heated by a 400 K ambient through the particle Robin
term (h 20, K 0.25), viscosity mu(T) = 1e3 exp(-0.05 (T - 290)), gamma(T) = 0.072 -
1.5e-4 (T - 300), gravity, slip floor, dt 1e-3, implicit Newton-CG momentum solve and
implicit heat CG.  Precision MIXED (FP32 transfers, operators and Krylov vectors; FP64
energies, dot products, norms and momentum sums), with the FP64 GPU path timed over the
same number of steps beside it.

A step is one full pass of the hot path: cell sort, parents / balance points / split,
P2G with the grid set-up, the Newton-CG momentum solve, the heat CG solve, G2P with
merge and advection.  The surface samples are an input of the step: the device sampler
(the host input stage's samples bit for bit) draws them for every step of the trajectory
in an untimed recording pass and they stay in HBM, so the timed pass replays the same
trajectory (bit-identical, the kernels are deterministic) with all inputs resident.  The
rate with each step's device sampling inside the timed region is reported beside
(all_in), and so is the rate a host sampler would give (host_stage).

Also reported: the MIXED-vs-FP64 error of the grid forces and of one step's particle
state on the headline workload; the other workloads (2D square droplet, Marangoni
droplet, contact angle) in a secondary block; the serving stream; the roofline of the
dominant kernel; the oracle on the host cores (one core and all cores).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def clone_state(P):
    return {k: v.clone() for k, v in P.items()}


def free_gpu():
    import gc
    import torch
    gc.collect()
    torch.cuda.empty_cache()


def run_gpu(scene_fn, precision, steps, warmup, want_timing, label, autotune=False):
    """Records warmup + steps steps (each step's surface drawn by the device sampler and
    kept in HBM), then replays them with every input in HBM: the timed pass, and with
    want_timing a second pass with per-launch HIP events for the per-class breakdown.  A
    last pass times the steps all-in, each with its own device sampling.  The host input
    stage is timed once on the first step's positions for comparison."""
    import torch
    from paper_2101_12408_amd import api
    S = scene_fn()
    P0, p = S["particles"], S["params"]
    N = len(P0["m"])
    t0 = time.perf_counter()
    ts = time.perf_counter()
    surf0 = api.sample_surface(P0["x"], p, step=0)
    host_sample_s = time.perf_counter() - ts
    cap_s = int(len(surf0["s"]) * 1.5) + 1024
    scene = api.Scene(p, cap_part=N, cap_surf=cap_s, precision=precision)
    Pd = scene.to_device(P0)
    init = clone_state(Pd)
    torch.cuda.synchronize()
    tu = time.perf_counter()
    scene.to_device(S=surf0)
    torch.cuda.synchronize()
    upload_s = time.perf_counter() - tu
    surfs = []
    tuning = None
    if autotune:
        # the tile kernels' XCD run lengths, timed on the first step's scene (bitwise
        # the same results for every choice)
        S0 = scene.sample_surface(Pd, step=0)
        scene.p2g(Pd, S0)
        tuning = scene.autotune()
        log(f"{label} {precision}: autotune " + ", ".join(f"{k} run {v[0]}" for k, v in tuning.items()))
        del S0
    for k in range(warmup + steps):
        Sd = scene.sample_surface(Pd, step=k)
        surfs.append(Sd)
        scene.step(Pd, Sd)
    log(f"{label} {precision}: recorded {warmup + steps} steps in {time.perf_counter() - t0:.1f} s "
        f"(N={N}, S~{len(surf0['s'])}, host sampling {host_sample_s:.3f} s for one step)")

    def reset_and_warm(sample):
        for k, v in init.items():
            Pd[k].copy_(v)
        for k in range(warmup):
            scene.step(Pd, scene.sample_surface(Pd, step=k) if sample else surfs[k])
        torch.cuda.synchronize()

    def replay(timed_events):
        reset_and_warm(False)
        if timed_events:
            scene.timing(True)
        stats = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(warmup, warmup + steps):
            scene.step(Pd, surfs[k])
            stats.append(scene.stats())
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        timing = None
        if timed_events:
            timing = dict(all=scene.timing_read(), work=scene.timing_read(work=True))
            scene.timing(False)
        return elapsed, stats, timing

    # the timed region carries no profiling events; a second replay of the same steps
    # records per-kernel HIP events for the breakdown and the roofline
    elapsed, stats, _ = replay(False)
    timing, elapsed_ev = None, None
    if want_timing:
        elapsed_ev, _, timing = replay(True)
    # all-in: device sampling and the step, from the same state
    reset_and_warm(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(warmup, warmup + steps):
        scene.step(Pd, scene.sample_surface(Pd, step=k))
    torch.cuda.synchronize()
    elapsed_all = time.perf_counter() - t1
    log(f"{label} {precision}: {1e3 * elapsed / steps:.3f} ms/step"
        + (f", with per-launch events {1e3 * elapsed_ev / steps:.3f}" if want_timing else "")
        + f", all-in with device sampling {1e3 * elapsed_all / steps:.3f}")
    out = dict(N=N, elapsed=elapsed, elapsed_events=elapsed_ev, elapsed_all_in=elapsed_all, stats=stats,
               timing=timing, S=len(surf0["s"]), params=p, host_sample_s=host_sample_s, upload_s=upload_s,
               tuning=tuning)
    del scene, Pd, init, surfs
    free_gpu()
    return out


def per_step(stats, key):
    return round(float(np.mean([s[key] for s in stats])), 2)


def summary(r, steps):
    st = r["stats"]
    return dict(value=round(r["N"] * steps / r["elapsed"], 1), unit="particle-steps/s",
                ms_per_step=round(1e3 * r["elapsed"] / steps, 3), steps=steps, particles=r["N"],
                surface_samples=r["S"], newton_iters_per_step=per_step(st, "newton_iters"),
                cg_iters_per_step=per_step(st, "cg_iters"), heat_iters_per_step=per_step(st, "heat_iters"),
                hessvec_per_s=round(sum(s["hessvecs"] for s in st) / r["elapsed"], 1),
                host_waits_per_step=per_step(st, "host_waits"),
                converged=[int(s["converged"]) for s in st][:3] + (["..."] if len(st) > 3 else []))


def mixed_vs_fp64(scene_fn):
    """MIXED against FP64 on the same inputs (FP64 host state, one set of surface samples):
    the grid forces P grad Phi at v^ = v^n of the FP64 grid, and the particle state after
    one implicit step (v, T, and the updates of x and J), each as the norm-wise relative
    error and the worst element relative to the largest FP64 value."""
    import torch
    from paper_2101_12408_amd import _lib as L
    from paper_2101_12408_amd import api
    S = scene_fn()
    P, p = S["particles"], S["params"]
    surf = api.sample_surface(P["x"], p, step=0)
    N = len(P["m"])
    res, grads, outs, parents = {}, {}, {}, {}
    for prec in ("fp64", "mixed"):
        s = api.Scene(p, cap_part=N, cap_surf=len(surf["s"]) + 1024, precision=prec)
        Pd, Sd = s.to_device(P, surf)
        s.p2g(Pd, Sd)
        parents[prec] = s.view(L.F_PARENT).cpu().numpy().copy()
        if prec == "fp64":
            vref = s.view(L.F_VN).clone()
        g = s.grid_vector()
        s.energy_grad(vref.to(s.dtype), g)
        grads[prec] = g.double().cpu().numpy()
        x0 = Pd["x"].double().clone()
        J0 = Pd["J"].double().clone()
        s.step(Pd, Sd)
        perm = s.view(L.F_PERM).long()
        inv = torch.empty_like(perm)
        inv[perm] = torch.arange(N, device=perm.device)
        outs[prec] = dict(v=Pd["v"].double()[:, inv].cpu().numpy(), T=Pd["T"].double()[inv].cpu().numpy(),
                          dx=(Pd["x"].double()[:, inv] - x0).cpu().numpy(), dJ=(Pd["J"].double()[inv] - J0).cpu().numpy())
        del s, Pd, Sd
        free_gpu()

    def err(a, b):
        return dict(rel=float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)),
                    worst=float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)))

    res["grid_forces"] = err(grads["mixed"], grads["fp64"])
    for k in ("v", "T", "dx", "dJ"):
        res[f"step_{k}"] = err(outs["mixed"][k], outs["fp64"][k])
    log("mixed vs fp64: " + ", ".join(f"{k} {v['rel']:.2e}/{v['worst']:.2e}" for k, v in res.items()))
    out = {k: {kk: float(f"{vv:.3e}") for kk, vv in v.items()} for k, v in res.items()}
    # surface samples whose nearest parent differs once the positions are FP32, and whether
    # the particle with the worst step-v error is a parent of one of them (either side)
    flip = parents["mixed"] != parents["fp64"]
    near = set(parents["mixed"][flip].tolist()) | set(parents["fp64"][flip].tolist())
    dv = np.abs(outs["mixed"]["v"] - outs["fp64"]["v"]).max(axis=0)
    worst_p = int(np.argmax(dv))
    out["parent_flips"] = {"count": int(flip.sum()), "of": int(flip.size), "worst_v_is_flipped_parent": worst_p in near}
    log(f"mixed vs fp64: {int(flip.sum())} of {flip.size} parents differ; worst v at a flipped parent: {worst_p in near}")
    return out


# ---------------------------------------------------------------------------------------
# Algorithmic bytes and flops per launch, per unit of work (3D; R bytes per real: 4 in
# MIXED, 8 in FP64; 4 per int32).  Bytes: each needed particle field read once, each
# output written once, each active node's fields read or written once.  Flops: the
# method's arithmetic per point for the scene's own terms.
#   Hessian-vector product, point kernel: interior x3 + c_J + mu V^n (5 reals), surface
#     s3 dA3 k + cached F9 (16 reals), nodes: w3 read (the merge writes the output);
#     flops J-only ~450 per interior particle, ~1100 with viscosity, ~1500 per surface
#     sample.
#   Energy / gradient, point kernel: interior x3 J V0 mu V^n (6), surface s3 dA3 k (7),
#     nodes v^3; flops as the Hessian plus the energy, ~500 / ~1150 / ~1500.
#   Heat operator, point kernel: interior x3 + K V^n (4), surface s3 + h|dA| (4), nodes T;
#     ~400 per interior particle, ~200 per sample.
#   P2G: x3 v3 A9 m T gradT3 + count (20 reals + int), surface s3 + parent, nodes m mv3
#     W WT E ET written; ~700 per interior particle, ~400 per surface or balance point.
#   G2P: x3 J + count read, v3 A9 T gradT3 x3 J written, surface s3 + parent, nodes v^3 T;
#     ~750 per interior particle, ~300 per surface or balance point.
#   Node merges: read the partials of each node's tiles and the node fields, write one
#     vector; ~10 flops per node.
# N interior particles, S surface samples (each with its balance point), G nodes of the
# active tiles.
# ---------------------------------------------------------------------------------------
def algorithmic(cls, N, S, G, R, visc, dim=3):
    d, d2, I = dim, dim * dim, 4
    fi = 1100 if visc else 450
    if cls == "hess_int":
        return dict(bytes=N * (d + 2) * R + S * (2 * d + 1 + d2) * R + G * d * R, flops=N * fi + S * 1500)
    if cls == "energy_int":
        return dict(bytes=N * (d + 3) * R + S * (2 * d + 1) * R + G * d * R,
                    flops=N * (fi + 50) + S * 1500)
    if cls == "heat_pt":
        return dict(bytes=N * (d + 1) * R + S * (d + 1) * R + G * R, flops=N * 400 + S * 200)
    if cls == "p2g":
        return dict(bytes=N * ((3 * d + d2 + 2) * R + I) + S * (d * R + I) + G * (d + 5) * R,
                    flops=N * 700 + 2 * S * 400)
    if cls == "g2p":
        return dict(bytes=N * ((d + 1) * R + I) + N * (d + d2 + 1 + d + d + 1) * R + S * (d * R + I)
                    + G * (d + 1) * R, flops=N * 750 + 2 * S * 300)
    if cls in ("energy_node", "hess_node"):
        return dict(bytes=G * ((2 * d + 1) * R + 1 + d * R), flops=G * 10)
    if cls == "heat_node":
        return dict(bytes=G * (3 * R + 1), flops=G * 4)
    return None


HBM_PEAK = 8000.0                    # GB/s, MI355X
VALU_PEAK = {4: 157.3, 8: 78.6}      # TFLOP/s, MI355X vector FP32 (packed) / FP64


def roofline_of(cls, tm, N, S, G, R, K, visc, traffic):
    """Roofline of one kernel class from its average launch time over the launches that
    did work (tm: the work totals of the timing read): a CG queued ahead of a Newton
    decision that the device then calls off still launches, and its kernels return at
    once."""
    ms, work = tm[cls]
    avg_s = ms / work * 1e-3
    alg = algorithmic(cls, N, S, G, R, visc)
    gbs = alg["bytes"] / avg_s / 1e9
    tfl = alg["flops"] / avg_s / 1e12
    t_hbm = alg["bytes"] / (HBM_PEAK * 1e9)
    t_alu = alg["flops"] / (VALU_PEAK[R] * 1e12)
    common = dict(kernel=cls, avg_launch_us=round(avg_s * 1e6, 2), launches_per_step=round(work / K, 2),
                  alg_bytes=int(alg["bytes"]), alg_flops=int(alg["flops"]),
                  hbm_frac=round(gbs / HBM_PEAK, 4), valu_frac=round(tfl / VALU_PEAK[R], 4))
    if t_hbm >= t_alu:
        r = dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK, unit="GB/s", frac=round(gbs / HBM_PEAK, 4))
    else:
        r = dict(bound="alu", achieved=round(tfl, 3), peak=VALU_PEAK[R], unit="TFLOP/s",
                 frac=round(tfl / VALU_PEAK[R], 4))
    r["traffic"] = traffic
    r.update(common)
    return r


def secondary_roofline(r, K, precision):
    """The Hessian tile kernel's average launch and its HBM and VALU fractions on a
    secondary workload (the section 8(d) counts of that scene's own terms)."""
    if not r["timing"] or r["params"]["dim"] != 3:      # the counts are the 3D ones
        return None
    st = r["stats"]
    N = r["N"]
    G = int(np.mean([s["n_tiles"] for s in st])) * 64
    S = int(np.mean([s["n_surf"] for s in st]))
    visc = r["params"]["mu0"] > 0 and (r["params"]["term_mask"] & 4)
    tm = r["timing"]["work"]
    if not tm["hess_int"][1]:
        return None
    rf = roofline_of("hess_int", tm, N, S, G, 4 if precision == "mixed" else 8, K, visc, None)
    return {k: rf[k] for k in ("bound", "frac", "avg_launch_us", "hbm_frac", "valu_frac")}


def kernel_sources_digest():
    """Digest of the device code with its comments and blank space left out, so that a
    change of a comment does not mark the measured traffic as taken on other kernels."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("common.h", "kernels.h", "tiles.h"):   # the device code
        with open(os.path.join(ROOT, "paper_2101_12408_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(cls, precision, workload):
    """HBM bytes per launch from the committed PMC summary, if it was taken on the current
    kernel sources and workload (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    e = t.get(f"{workload}:{cls}:{precision}")
    if not e or e.get("sources") != kernel_sources_digest():
        return None
    return e.get("bytes_per_launch")


def copy_calibration(mib=512, reps=5):
    """A plain device copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    a = torch.empty(mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: {reps} copies of {mib} MiB")


def run_serving(count, rate, precision, concurrency, budget_bytes, saturate=False):
    """The serving stream (Poisson arrivals at `rate`, droplets on n in {16,...,96}, one
    implicit step each) through the native serving runtime.  Latency is measured from
    each request's scheduled arrival to its completion (admission, upload, device
    sampling, step, download).  saturate: every request arrives at once, so the rate is
    the runtime's capacity rather than the offered load."""
    import mpm_scenes as sc
    from paper_2101_12408_amd import api
    reqs = sc.serving_stream(count=count, rate=rate, seed=5)
    if saturate:
        reqs = [dict(r, arrival=0.0) for r in reqs]
    si = sc.ServingInputs()
    inputs = [(si.params(r), si.soa(r)) for r in reqs]       # kept alive: the server borrows them
    srv = api.Server(budget_bytes, max_concurrent=concurrency)
    clock = api.Server.clock
    t0 = clock() + 0.05
    for i, (r, (p, soa)) in enumerate(zip(reqs, inputs)):
        wait = t0 + r["arrival"] - clock()
        if wait > 0:
            time.sleep(wait)
        srv.submit(i, p, soa=soa, borrow=True, precision=precision)
    srv.wait(-1.0)
    comps = srv.poll(cap=count + 16)
    info = srv.info()
    srv.close()
    lat = np.array([c["t_done"] - (t0 + reqs[c["id"]]["arrival"]) for c in comps]) * 1e3
    done = max(c["t_done"] for c in comps)
    ps = sum(c["n_part"] * c["steps_done"] for c in comps)
    failed = sum(1 for c in comps if c["status"] != 0)
    log(f"serving {precision} x{concurrency}{' saturated' if saturate else ''}: {count} requests, "
        f"p50 {np.percentile(lat, 50):.1f} ms, "
        f"p99 {np.percentile(lat, 99):.1f} ms, {ps / (done - t0):.3e} particle-steps/s, failed {failed}")
    return dict(requests=count, arrival_rate_per_s=rate, precision=precision, max_concurrent=concurrency,
                budget_gb=round(budget_bytes / 2 ** 30, 2), p50_ms=round(float(np.percentile(lat, 50)), 2),
                p99_ms=round(float(np.percentile(lat, 99)), 2), mean_ms=round(float(lat.mean()), 2),
                particle_steps_per_s=round(ps / (done - t0), 1), makespan_s=round(done - t0, 3),
                peak_running=info["peak_running"], peak_gb=round(info["peak_bytes"] / 2 ** 30, 3), failed=failed)


# ---------------------------------------------------------------------------------------
# CPU baseline: the oracle (plain numpy FP64) on the host cores.  One implicit step of the
# headline workload takes the oracle minutes even on a small part of the slab (its grids
# are dense 256^3 arrays and the viscous system takes ~110 CG iterations per step), so the
# sample is bounded: on a sub-slab of the same 256^3 grid, same density and physics, it
# times P2G with the grid set-up, one energy-and-gradient evaluation, one iteration of the
# Newton-CG, one iteration of the heat CG and G2P, and scales them to one step with the
# per-step counts of the timed GPU run (energy evaluations, CG and heat CG iterations).
# ---------------------------------------------------------------------------------------
CPU_SAMPLE = dict(lo=0.44, hi=0.56, height=0.06)


def _cpu_sample_inproc(seed, n_energy, n_cg, n_heat):
    import mpm_scenes as sc
    from oracle import energy, resample, sampler, solve, transfer
    S = sc.meltslab3d(seed=seed, **CPU_SAMPLE)
    P, p = S["particles"], S["params"]
    surf = sampler.sample_surface(P["x"], p)
    T = {}
    t = time.perf_counter()
    sp = resample.split(P, surf)
    g = transfer.p2g(P, surf, sp, p)
    st = transfer.grid_setup(P, surf, sp, g, p)
    ctx = energy.Context(P, surf, g, st, p)
    heat = solve.Heat(P, surf, g, st, p)
    T["p2g_setup"] = time.perf_counter() - t
    v = ctx.project(ctx.vn.copy())
    t = time.perf_counter()
    ctx.Phi(v)
    gr = ctx.project(ctx.grad_Phi(v))
    T["energy"] = time.perf_counter() - t
    diag = ctx.jacobi_diag()
    t = time.perf_counter()
    solve.pcg(lambda w: ctx.project(ctx.hessvec(v, ctx.project(w))), -gr, diag, 0.0, 1)
    T["cg_iter"] = time.perf_counter() - t
    hd = heat.diag()
    t = time.perf_counter()
    solve.pcg(heat.apply, heat.rhs, hd, 0.0, 1, x0=heat.Tn.copy())
    T["heat_iter"] = time.perf_counter() - t
    t = time.perf_counter()
    transfer.g2p(P, surf, sp, v, st["Tn"], p)
    T["g2p"] = time.perf_counter() - t
    step_s = T["p2g_setup"] + n_energy * T["energy"] + n_cg * T["cg_iter"] + n_heat * T["heat_iter"] + T["g2p"]
    return dict(N=len(P["m"]), S=len(surf["s"]), parts={k: round(x, 3) for k, x in T.items()},
                measured_s=sum(T.values()), step_s=step_s)


def cpu_baseline(n_energy, n_cg, n_heat):
    """The oracle timing: one child process pinned to one BLAS/OpenMP thread, then one
    child per host core (each on its own seeded sub-slab) at the same time."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")

    def launch(seed):
        code = (f"import json, bench; print(json.dumps(bench._cpu_sample_inproc({seed}, {n_energy}, {n_cg}, "
                f"{n_heat})))")
        return subprocess.Popen([sys.executable, "-c", code], cwd=ROOT, env=env, stdout=subprocess.PIPE,
                                stderr=subprocess.PIPE, text=True)

    def collect(pr):
        out, errs = pr.communicate(timeout=900)
        if pr.returncode != 0:
            log(f"cpu baseline child failed: {errs[-400:]}")
            return None
        return json.loads(out.strip().splitlines()[-1])

    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            model = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except Exception:
        pass
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    one = collect(launch(100))
    if one is None:
        return None
    rate1 = one["N"] / one["step_s"]
    log(f"cpu oracle, 1 core: {rate1:.1f} particle-steps/s ({one['measured_s']:.1f} s measured; parts {one['parts']})")
    # all cores: as many samples at once as cores (at most 16), each ~5 GB of host memory
    k = max(1, min(cores, 16))
    t0 = time.perf_counter()
    runs = [collect(p) for p in [launch(100 + j) for j in range(k)]]
    runs = [r for r in runs if r]
    wall = time.perf_counter() - t0
    rate_all = sum(r["N"] / r["step_s"] for r in runs)
    log(f"cpu oracle, {len(runs)} cores: {rate_all:.1f} particle-steps/s (wall {wall:.1f} s)")
    sample = (f"melting slab on the same 256^3 grid, sub-slab x,z in [{CPU_SAMPLE['lo']},{CPU_SAMPLE['hi']}], "
              f"height {CPU_SAMPLE['height']}, 8 ppc ({one['N']} particles, {one['S']} surface samples): P2G with "
              f"the grid set-up, 1 energy evaluation, 1 Newton-CG iteration, 1 heat-CG iteration and G2P timed "
              f"({one['measured_s']:.1f} s), scaled to one step with the GPU run's per-step counts ({n_energy} "
              f"energy evaluations, {n_cg} CG and {n_heat} heat-CG iterations); all cores: {len(runs)} such "
              f"samples at once, one per process")
    return dict(value=round(rate1, 1), unit="particle-steps/s", cores=1, kind="oracle", sample=sample,
                all_cores=dict(value=round(rate_all, 1), cores=len(runs), wall_s=round(wall, 1)),
                cpu_model=model, host_cores=cores, parts_1core=one["parts"])


# ---------------------------------------------------------------------------------------
# Summaries of rocprofv3 output (host only): the kernel-trace table and the PMC traffic
# per launch that profiles/ holds.
# ---------------------------------------------------------------------------------------
KERNEL_CLASS_OF = {}
for _r in ("float", "double"):
    for _var in ("0", "1", "2"):       # the fluid, solid-phase and J-term-only instantiations
        KERNEL_CLASS_OF[f"k_tile_stress<3, {_r}, 1, {_var}>"] = "hess_int"
        KERNEL_CLASS_OF[f"k_tile_stress<3, {_r}, 0, {_var}>"] = "energy_int"
    for _sol in ("false", "true"):
        KERNEL_CLASS_OF[f"k_tile_g2p<3, {_r}, {_sol}>"] = "g2p"
    KERNEL_CLASS_OF[f"k_tile_heat<3, {_r}>"] = "heat_pt"
    KERNEL_CLASS_OF[f"k_tile_p2g<3, {_r}>"] = "p2g"
    KERNEL_CLASS_OF[f"k_merge_heat<3, {_r}>"] = "heat_node"


def _short(name):
    n = name.split("(")[0]
    for pre in ("void ", "mpm::"):
        n = n.replace(pre, "")
    return n


def _work_launches(vals):
    """Launches that did work: a CG called off on the device still launches its kernels,
    which return at once; they are left out (below a tenth of the 95th percentile)."""
    v = np.asarray(vals, np.float64)
    return v[v >= 0.1 * np.percentile(v, 95)] if len(v) else v


def summarize_ktrace(d):
    import csv
    import glob
    path = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)[0]
    dur = {}
    for r in csv.DictReader(open(path)):
        dur.setdefault(_short(r["Kernel_Name"]), []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    total = sum(sum(v) for v in dur.values())
    lines = [f"# {'kernel':58s} {'calls':>7s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s} {'work_n':>7s} {'work_us':>9s}"]
    for k, v in sorted(dur.items(), key=lambda kv: -sum(kv[1]))[:30]:
        w = _work_launches(v)
        lines.append(f"  {k[:58]:58s} {len(v):7d} {np.mean(v):10.2f} {sum(v) * 1e-3:10.3f} {100 * sum(v) / total:6.2f} "
                     f"{len(w):7d} {np.mean(w):9.2f}")
    return "\n".join(lines)


def summarize_pmc(fetch_dir, write_dir, workload, precision):
    """Per-launch HBM bytes of the tile kernels from a FETCH_SIZE pass and a WRITE_SIZE pass
    (KiB per dispatch), each scaled by what the counter reads for the 512 MiB device copy
    of --copy-calibration in the same run; written to profiles/traffic.json."""
    import csv
    import glob

    def load(d, counter):
        path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        out = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                out.setdefault(_short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]) * 1024.0)
        return out

    fetch, write = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    copy = 512 * 2 ** 20

    def factor(tab):
        vals = [max(v) for k, v in tab.items() if "copyBuffer" in k or "copy" in k.lower()]
        big = max(vals) if vals else 0.0
        return copy / big if big > 0.25 * copy else 1.0

    ff, fw = factor(fetch), factor(write)
    path = os.path.join(ROOT, "profiles", "traffic.json")
    table = json.load(open(path)) if os.path.exists(path) else {}
    lines = [f"# copy kernel: factors fetch x{ff:.3f}, write x{fw:.3f}",
             f"# {'kernel':40s} {'n':>5s} {'fetch_MB':>10s} {'write_MB':>10s} {'total_MB':>10s}"]
    for k in sorted(fetch, key=lambda k: -sum(fetch[k])):
        if k not in KERNEL_CLASS_OF:
            continue
        fv = _work_launches(fetch[k])
        wv = _work_launches(write.get(k, [0.0]))
        fb, wb = float(np.mean(fv)) * ff, float(np.mean(wv)) * fw
        lines.append(f"  {k:40s} {len(fv):5d} {fb / 1e6:10.2f} {wb / 1e6:10.2f} {(fb + wb) / 1e6:10.2f}")
        table[f"{workload}:{KERNEL_CLASS_OF[k]}:{precision}"] = dict(
            kernel=k, bytes_per_launch=int(fb + wb), fetch_bytes=int(fb), write_bytes=int(wb),
            fetch_factor=round(ff, 4), write_factor=round(fw, 4), sources=kernel_sources_digest())
    with open(path, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--workload", default="meltslab3d", choices=["meltslab3d", "marangoni3d", "contact3d"],
                    help="headline workload (default: the 256^3 melting slab)")
    ap.add_argument("--fp64-steps", type=int, default=-1,
                    help="steps of the FP64 GPU comparison run (-1: as --steps; 0: skip)")
    ap.add_argument("--no-errors", action="store_true", help="skip the MIXED-vs-FP64 error report")
    ap.add_argument("--no-secondary", action="store_true", help="skip the other workloads")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the built-in tile run-length rule")
    ap.add_argument("--serving-requests", type=int, default=512,
                    help="requests of the serving stream (0: skip the serving measurement)")
    ap.add_argument("--serving-concurrency", type=int, default=8)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 512 MiB device copy (PMC traffic calibration)")
    ap.add_argument("--summarize-ktrace", metavar="DIR", help="print the kernel table of a rocprofv3 "
                    "--kernel-trace output directory and exit (no GPU)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="update profiles/traffic.json from a FETCH_SIZE and a WRITE_SIZE rocprofv3 --pmc "
                    "output directory of the workload and precision given, print the table and exit (no GPU)")
    args = ap.parse_args()
    if args.summarize_ktrace:
        print(summarize_ktrace(args.summarize_ktrace))
        return
    if args.summarize_pmc:
        print(summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.workload, args.precision))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    import mpm_scenes as sc
    scene_fn = sc.CONFIGS[args.workload]
    if args.copy_calibration:
        copy_calibration()
    K = args.steps
    main_run = run_gpu(scene_fn, args.precision, K, args.warmup, not args.no_timing, args.workload,
                       autotune=not args.no_autotune)
    N = main_run["N"]
    value = N * K / main_run["elapsed"]
    st = main_run["stats"]
    hv = sum(s["hessvecs"] for s in st)
    G = int(np.mean([s["n_tiles"] for s in st])) * 64
    S = int(np.mean([s["n_surf"] for s in st]))
    visc = main_run["params"]["mu0"] > 0 and (main_run["params"]["term_mask"] & 4)
    out_extra = {}
    roofline = None
    R = 4 if args.precision == "mixed" else 8
    if main_run["timing"]:
        tma, tm = main_run["timing"]["all"], main_run["timing"]["work"]
        total = sum(v[0] for v in tma.values())
        out_extra["kernel_ms_per_step"] = {k: round(v[0] / K, 4) for k, v in tma.items() if v[1]}
        cand = [k for k in tm if tm[k][1] and algorithmic(k, N, S, G, R, visc)]
        dom = max(cand, key=lambda k: tma[k][0])
        roofline = roofline_of(dom, tm, N, S, G, R, K, visc, measured_traffic(dom, args.precision, args.workload))
        out_extra["kernel_rooflines"] = {k: {kk: roofline_of(k, tm, N, S, G, R, K, visc, None)[kk]
                                             for kk in ("avg_launch_us", "hbm_frac", "valu_frac")} for k in cand}
        # summed kernel time of both streams per step over the event-free step time (above 1
        # where the heat solve's stream overlaps the momentum solve's)
        out_extra["kernel_sum_over_step"] = round(total / (main_run["elapsed"] * 1e3), 3)
        out_extra["ms_per_step_with_events"] = round(1e3 * main_run["elapsed_events"] / K, 3)
    # with each step's device sampling timed; and, for comparison, the host input stage and
    # the upload of its samples added to the step
    all_in = N * K / main_run["elapsed_all_in"]
    host_stage = N / (main_run["elapsed"] / K + main_run["host_sample_s"] + main_run["upload_s"])
    fp64 = None
    k64 = K if args.fp64_steps < 0 else args.fp64_steps
    if k64 > 0 and args.precision != "fp64":
        r64 = run_gpu(scene_fn, "fp64", k64, args.warmup, False, args.workload)
        fp64 = summary(r64, k64)
        fp64["speedup_mixed_over_fp64"] = round(value / fp64["value"], 3)
    errors = None
    if not args.no_errors and args.precision != "fp64":
        errors = mixed_vs_fp64(scene_fn)
    secondary = None
    if not args.no_secondary:
        secondary = {}
        plan = [("square2d", ["fp64"], 5), ("marangoni3d", ["mixed", "fp64"], 20),
                ("contact3d", ["mixed", "fp64"], 50), ("meltslab3d_4ppc", ["mixed", "fp64"], 20)]
        for name, precs, steps in plan:
            if name == args.workload:
                continue
            secondary[name] = {}
            for prec in precs:
                r = run_gpu(sc.CONFIGS[name], prec, steps, 2, True, name)
                secondary[name][prec] = summary(r, steps)
                secondary[name][prec]["hess_int"] = secondary_roofline(r, steps, prec)
            if len(precs) == 2:
                secondary[name]["speedup_mixed_over_fp64"] = round(
                    secondary[name]["mixed"]["value"] / secondary[name]["fp64"]["value"], 3)
    serving = None
    if args.serving_requests > 0:
        free, _ = torch.cuda.mem_get_info()
        budget = int(min(0.8 * free, 64 * 2 ** 30))
        mixed = run_serving(args.serving_requests, 200.0, "mixed", args.serving_concurrency, budget)
        base = run_serving(args.serving_requests, 200.0, "fp64", 1, budget)
        # capacity: the same requests all at once
        mixed_sat = run_serving(args.serving_requests, 200.0, "mixed", args.serving_concurrency, budget, saturate=True)
        base_sat = run_serving(args.serving_requests, 200.0, "fp64", 1, budget, saturate=True)
        serving = dict(batched=mixed, one_at_a_time_fp64=base,
                       p99_speedup=round(base["p99_ms"] / mixed["p99_ms"], 3),
                       saturated=dict(batched=mixed_sat, one_at_a_time_fp64=base_sat,
                                      throughput_speedup=round(mixed_sat["particle_steps_per_s"]
                                                               / base_sat["particle_steps_per_s"], 3)))
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(max(1, round(np.mean([s["energy_evals"] for s in st]))),
                           max(1, round(np.mean([s["cg_iters"] for s in st]))),
                           max(1, round(np.mean([s["heat_iters"] for s in st]))))
    p = main_run["params"]
    wl = {"meltslab3d": f"meltslab3d: 256^3 grid, slab 0.6x0.2x0.6 at 8 ppc, {N} particles, ~{S} surface samples, "
                        f"mu(T)=1e3 exp(-0.05(T-290)), Robin heating h=20 to 400 K, gravity, slip floor, dt 1e-3, "
                        f"implicit Newton-CG + heat CG",
          "marangoni3d": f"marangoni3d: 128^3 grid, sphere r=0.2 at 8 ppc, {N} particles, ~{S} surface samples, "
                         f"dt 5e-4, implicit Newton-CG + heat CG",
          "contact3d": f"contact3d: 192^3 grid, cap r=0.15 on a slab at 8 ppc, {N} particles, ~{S} surface samples, "
                       f"dt 5e-4, implicit Newton-CG"}[args.workload]
    line = {
        "metric": "implicit MPM particle-steps/s",
        "value": round(value, 1),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * main_run["elapsed"] / K, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": wl, "precision": args.precision, "global_batch": N, "dt": p["dt"], "n": p["n"]},
        "hessvec_per_s": round(hv / main_run["elapsed"], 1),
        "newton_iters_per_step": per_step(st, "newton_iters"),
        "cg_iters_per_step": per_step(st, "cg_iters"),
        "heat_iters_per_step": per_step(st, "heat_iters"),
        "host_waits_per_step": per_step(st, "host_waits"),
        "all_in": dict(value=round(all_in, 1), unit="particle-steps/s",
                       ms_per_step=round(1e3 * main_run["elapsed_all_in"] / K, 3),
                       sampling_ms_per_step=round(1e3 * (main_run["elapsed_all_in"] - main_run["elapsed"]) / K, 3),
                       host_stage=dict(value=round(host_stage, 1), host_sampling_s_per_step=round(
                           main_run["host_sample_s"], 4), upload_s_per_step=round(main_run["upload_s"], 4))),
        "autotune": main_run["tuning"],
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp64_gpu": fp64,
        "mixed_vs_fp64_error": errors,
        "secondary": secondary,
        "serving": serving,
    }
    line.update(out_extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
