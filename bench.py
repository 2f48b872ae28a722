"""Benchmark of the implicit APIC MPM hot path on one MI355X.

Workload: the 3D Marangoni droplet (128^3 grid on the unit cube, sphere r = 0.2 at 8
particles per cell, ~562k particles, linear temperature 300-350 K, gamma(T) =
0.072 - 1.5e-4 (T - 300), bulk 1e4, dt 5e-4, implicit heat solve), FP32 transfers and
Hessian-vector products with FP64 reductions.

A step is one full pass of the hot path: cell sort, parents / balance points / split,
P2G with the grid set-up, the Newton-CG momentum solve, the heat CG solve, G2P with
merge and advection.  The surface samples are an input of the step (the host sampler
is the input stage); they are drawn for every step of the trajectory in an untimed
recording pass and kept in HBM, so the timed pass replays the same trajectory
(bit-identical, the kernels are deterministic) with all inputs resident.

Prints one JSON line (metric, value, roofline of the dominant kernel, cpu_baseline).
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


def run_gpu(scene_fn, precision, steps, warmup, want_timing):
    import torch
    from paper_2101_12408_amd import api
    S = scene_fn()
    P0, p = S["particles"], S["params"]
    N = len(P0["m"])
    t0 = time.perf_counter()
    surf0 = api.sample_surface(P0["x"], p, step=0)
    cap_s = int(len(surf0["s"]) * 1.5) + 1024
    scene = api.Scene(p, cap_part=N, cap_surf=cap_s, precision=precision)
    Pd = scene.to_device(P0)
    init = clone_state(Pd)
    # recording pass (untimed): warmup + steps, surface samples of every step kept in HBM
    surfs = []
    for k in range(warmup + steps):
        xh = Pd["x"].double().cpu().numpy().T.copy()
        surf = surf0 if k == 0 else api.sample_surface(xh, p, step=k)
        Sd = scene.to_device(S=surf)
        surfs.append(Sd)
        scene.step(Pd, Sd)
    log(f"{precision}: recorded {warmup + steps} steps in {time.perf_counter() - t0:.1f} s "
        f"(N={N}, S~{len(surf0['s'])})")
    def replay(timed_events):
        for k, v in init.items():
            Pd[k].copy_(v)
        for k in range(warmup):
            scene.step(Pd, surfs[k])
        torch.cuda.synchronize()
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
            timing = scene.timing_read()
            scene.timing(False)
        return elapsed, stats, timing

    # the timed region carries no profiling events; a second replay of the same steps
    # records per-kernel HIP events for the breakdown and the roofline
    elapsed, stats, _ = replay(False)
    timing, elapsed_ev = None, None
    if want_timing:
        elapsed_ev, _, timing = replay(True)
        log(f"{precision}: {1e3 * elapsed / steps:.3f} ms/step, with per-launch events {1e3 * elapsed_ev / steps:.3f}")
    return dict(N=N, elapsed=elapsed, elapsed_events=elapsed_ev, stats=stats, timing=timing, S=len(surf0["s"]),
                params=p)


def cpu_baseline():
    """Runs the oracle timing in a child process pinned to one BLAS/OpenMP thread, so the
    reported core count is the number of threads actually used."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")
    code = "import json, bench; print(json.dumps(bench._cpu_baseline_inproc()))"
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    if r.returncode != 0:
        log(f"cpu baseline failed: {r.stderr[-500:]}")
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def _cpu_baseline_inproc():
    """The oracle, timed on the host on a bounded sample: one full implicit step of the
    same Marangoni scene at the same grid (128^3), particle density and parameters, with
    a droplet of radius 0.1 instead of 0.2 (1/8 of the particles)."""
    import mpm_scenes as sc
    from oracle import sampler, step as ostep
    S = sc.marangoni3d(radius=0.1)
    P, p = S["particles"], S["params"]
    surf = sampler.sample_surface(P["x"], p)
    t0 = time.perf_counter()
    _, info = ostep.step(P, p, surf)
    dt = time.perf_counter() - t0
    n = len(P["m"])
    return dict(value=n / dt, unit="particle-steps/s", cores=1, kind="oracle",
                sample=f"one implicit step of marangoni3d at 128^3 with droplet radius 0.1 "
                       f"({n} particles, {len(surf['s'])} surface samples; newton {info['newton']}, "
                       f"cg {info['cg']}, heat cg {info.get('heat_cg')}): {dt:.1f} s single-threaded numpy")


# Algorithmic bytes and flops per launch of each timed kernel class.  Bytes: the minimum
# the method moves (each needed particle field read once, each output written once, each
# active node's fields read or written once), R bytes per real (4 in MIXED, 8 in FP64), 4
# per int32.  Flops: the method's arithmetic in direct tensor-product form over the 3^d
# stencil (3D counts): per point the 1D weight tables and the 27 node weights and
# gradients (252), then per node what the kernel accumulates, e.g. the gradient gather
# sum_i u_i (x) grad N_i (9 FMA = 18 flops) and the stress scatter S grad N_i (18 flops).
#   energy / Hessian, interior: 252 + 486 + ~15 + 486 = ~1240; surface: ~1350 / ~1420
#   heat operator: interior 252 + 162 + 162 = ~580; surface (value only) ~360
#   P2G: interior ~62 per node (~1930); surface and balance points ~42 per node (~1390)
#   G2P: interior ~38 per node (~1280); each surface and balance member ~24 per node (~900)
# N interior particles, S surface samples (each with its balance point), G nodes of the
# active tiles.
def algorithmic(cls, N, S, G, R, dim=3):
    d, d2, I = dim, dim * dim, 4
    if cls == "p2g":           # read x v A m T gradT + group count; s + parent; write m mv W WT E ET
        return dict(bytes=N * ((3 * d + d2 + 2) * R + I) + S * (d * R + I) + G * (d + 5) * R,
                    flops=N * 1930 + 2 * S * 1390)
    if cls == "energy_int":    # read x J V0 muV, s dA k, v^ at the nodes
        return dict(bytes=N * (d + 3) * R + S * (2 * d + 1) * R + G * d * R, flops=N * 1240 + S * 1350)
    if cls == "hess_int":      # read x cJ muV, s dA k + cached F (d^2), w at the nodes
        return dict(bytes=N * (d + 2) * R + S * (2 * d + 1 + d2) * R + G * d * R, flops=N * 1240 + S * 1420)
    if cls in ("energy_node", "hess_node"):   # read w/v^, v^n, m, flags; write out
        return dict(bytes=G * ((2 * d + 1) * R + 1 + d * R), flops=G * 8 * d)
    if cls == "heat_pt":       # read x KV, s h|dA|, T at the nodes
        return dict(bytes=N * (d + 1) * R + S * (d + 1) * R + G * R, flops=N * 580 + S * 360)
    if cls == "heat_node":
        return dict(bytes=G * (3 * R + 1), flops=G * 4)
    if cls == "g2p":           # read x J count, s + parent, v^ T^; write v A T gradT x J
        return dict(bytes=N * ((d + 1) * R + I) + N * (d + d2 + 1 + d + d + 1) * R + S * (d * R + I) + G * (d + 1) * R,
                    flops=N * 1280 + 2 * S * 900)
    return None


HBM_PEAK = 8000.0      # GB/s
VALU_PEAK = {4: 157.3, 8: 78.6}   # TFLOP/s, vector FP32 / FP64


def roofline_of(cls, tm, N, S, G, R, K, traffic, hessvecs=None):
    """Roofline of one kernel class.  The Hessian classes are averaged over the operator
    applications that did work (hessvecs): a CG queued ahead of a Newton decision that
    the device then calls off still launches, and its kernels return at once."""
    ms, launches = tm[cls]
    work = hessvecs if (hessvecs and cls in ("hess_int", "hess_node")) else launches
    avg_s = ms / work * 1e-3
    alg = algorithmic(cls, N, S, G, R)
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


def kernel_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in ("common.h", "kernels.h", "tiles.h"):   # the device code
        with open(os.path.join(ROOT, "paper_2101_12408_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(cls, precision):
    """HBM bytes per launch from the committed PMC summary, if it was taken on the current
    kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    e = t.get(f"{cls}:{precision}")
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


def run_serving(count, rate, precision, concurrency, budget_bytes):
    """The serving stream (Poisson arrivals at `rate`, droplets on n in {16,...,96}, one
    implicit step each) through the native serving runtime.  Latency is measured from
    each request's scheduled arrival to its completion (host sampling, admission,
    upload, step, download)."""
    import mpm_scenes as sc
    from paper_2101_12408_amd import api
    reqs = sc.serving_stream(count=count, rate=rate, seed=5)
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
    log(f"serving {precision} x{concurrency}: {count} requests, p50 {np.percentile(lat, 50):.1f} ms, "
        f"p99 {np.percentile(lat, 99):.1f} ms, {ps / (done - t0):.3e} particle-steps/s, failed {failed}")
    return dict(requests=count, arrival_rate_per_s=rate, precision=precision, max_concurrent=concurrency,
                budget_gb=round(budget_bytes / 2 ** 30, 2), p50_ms=round(float(np.percentile(lat, 50)), 2),
                p99_ms=round(float(np.percentile(lat, 99)), 2), mean_ms=round(float(lat.mean()), 2),
                particle_steps_per_s=round(ps / (done - t0), 1), makespan_s=round(done - t0, 3),
                peak_running=info["peak_running"], peak_gb=round(info["peak_bytes"] / 2 ** 30, 3), failed=failed)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--fp64-steps", type=int, default=3, help="steps of the FP64 GPU comparison run (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=512,
                    help="requests of the serving stream (0: skip the serving measurement)")
    ap.add_argument("--serving-concurrency", type=int, default=8)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 512 MiB device copy (PMC traffic calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    import mpm_scenes as sc
    scene_fn = sc.marangoni3d
    if args.copy_calibration:
        copy_calibration()
    main_run = run_gpu(scene_fn, args.precision, args.steps, args.warmup, not args.no_timing)
    N, K = main_run["N"], args.steps
    value = N * K / main_run["elapsed"]
    ms_per_step = 1e3 * main_run["elapsed"] / K
    st = main_run["stats"]
    hv = sum(s["hessvecs"] for s in st)
    G = int(np.mean([s["n_tiles"] for s in st])) * 64
    S = int(np.mean([s["n_surf"] for s in st]))
    out_extra = {}
    roofline = None
    R = 4 if args.precision == "mixed" else 8
    if main_run["timing"]:
        tm = main_run["timing"]
        total = sum(v[0] for v in tm.values())
        out_extra["kernel_ms_per_step"] = {k: round(v[0] / K, 4) for k, v in tm.items() if v[1]}
        cand = [k for k in tm if tm[k][1] and algorithmic(k, N, S, G, R)]
        dom = max(cand, key=lambda k: tm[k][0])
        roofline = roofline_of(dom, tm, N, S, G, R, K, measured_traffic(dom, args.precision), hv)
        out_extra["kernel_rooflines"] = {k: {kk: roofline_of(k, tm, N, S, G, R, K, None, hv)[kk]
                                             for kk in ("avg_launch_us", "hbm_frac", "valu_frac")} for k in cand}
        # summed kernel time of both streams per step over the event-free step time (above 1
        # where the heat solve's stream overlaps the momentum solve's)
        out_extra["kernel_sum_over_step"] = round(total / (main_run["elapsed"] * 1e3), 3)
        out_extra["ms_per_step_with_events"] = round(1e3 * main_run["elapsed_events"] / K, 3)
    fp64 = None
    if args.fp64_steps > 0 and args.precision != "fp64":
        r64 = run_gpu(scene_fn, "fp64", args.fp64_steps, 1, False)
        v64 = r64["N"] * args.fp64_steps / r64["elapsed"]
        fp64 = dict(value=round(v64, 1), unit="particle-steps/s", steps=args.fp64_steps,
                    speedup_mixed_over_fp64=round(value / v64, 3))
    serving = None
    if args.serving_requests > 0:
        free, _ = torch.cuda.mem_get_info()
        budget = int(min(0.8 * free, 64 * 2 ** 30))
        mixed = run_serving(args.serving_requests, 200.0, "mixed", args.serving_concurrency, budget)
        base = run_serving(args.serving_requests, 200.0, "fp64", 1, budget)
        serving = dict(batched=mixed, one_at_a_time_fp64=base,
                       throughput_speedup=round(mixed["particle_steps_per_s"] / base["particle_steps_per_s"], 3),
                       p99_speedup=round(base["p99_ms"] / mixed["p99_ms"], 3))
    cpu = None if args.no_cpu_baseline else cpu_baseline()
    if cpu:
        cpu["value"] = round(cpu["value"], 1)
    line = {
        "metric": "implicit MPM particle-steps/s",
        "value": round(value, 1),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "marangoni3d: 128^3 grid, sphere r=0.2 at 8 ppc, "
                               f"{N} particles, ~{S} surface samples, dt 5e-4, implicit Newton-CG + heat CG",
                   "precision": args.precision, "global_batch": N},
        "hessvec_per_s": round(hv / main_run["elapsed"], 1),
        "newton_iters_per_step": round(np.mean([s["newton_iters"] for s in st]), 2),
        "cg_iters_per_step": round(np.mean([s["cg_iters"] for s in st]), 2),
        "heat_iters_per_step": round(np.mean([s["heat_iters"] for s in st]), 2),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp64_gpu": fp64,
        "serving": serving,
    }
    line.update(out_extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
