"""Benchmark: one time step of the ternary wetting LBM update on one MI355X.

Headline workload (the lubricated sessile drop): D3Q27, 256^3 nodes, walls at
z = 0 and 255, a liquid-2 sphere of radius 48 resting on an 8-node liquid-3
film over the bottom wall, gas above, density ratio 1000, gamma12 = gamma13 =
0.02, gamma23 = 0.01, interface width 4, tau = 1, geometric-interpolation
walls at 90 degrees; FP32 arithmetic and storage.  Inputs are synthetic
(seeded geometry) and resident in HBM before the timed region.

Prints one JSON line: MLUPS over fluid nodes, the roofline of the dominant
kernel from HIP events recorded by the kernels' own dispatch packets on the
library's stream, the step's fraction of the algorithmic HBM roofline, and
the CPU oracle timed on the host on a bounded sample of the same workload;
beside them the FP16-storage and FP64 forms of the same grid, the two D2Q9
channel workloads, and the serving comparison.
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS and % HBM roofline per step; serving p50/p99 time-to-result vs plain"
HBM_PEAK_GBS = 8000.0
N3 = (256, 256, 256)
GAMMA3 = (0.02, 0.02, 0.01)
R_DROP, FILM = 48, 8
SAMPLE_EVERY = 10   # HIP events on the launches of every 10th timed step
KERNEL_SOURCE = os.path.join(ROOT, "paper_1904_06881_amd", "csrc", "lbm3_kernels.hip")
PMC_SUMMARY = os.path.join(ROOT, "profiles", "d3q27_256cube_counters.md")


def params3(L, precision, n=N3):
    return L.make_params(L.D3Q27, n, gamma=GAMMA3, width=4.0, tau_f=1.0, tau_g=1.0,
                         wetting=L.WET_GEOM_INTERP, theta_deg=90.0, precision=precision)


def fields3(I, n=N3):
    s = n[0] / 256.0
    return I.lubricated_drop_3d(*n, R_DROP * s, film=max(2, int(round(FILM * s))))


def kernel_bytes(Q, s, sf, fp16, g_read, implicit_g):
    """Algorithmic HBM bytes per fluid node of each kernel of the two-kernel
    3D step (s: population bytes, sf: field bytes).  With stored g:
      moments  read both population sets, write rho, phi (FP16 storage: and
               read the previous fields the offsets are decoded with);
      stencil  read rho, phi, write F (3) and mu_phi;
      collide  read f (and g unless tau_g = 1), rho, phi, F, mu_phi (FP16:
               the previous fields), write both population sets.
    With implicit g (tau_g = 1: the collision stores the five values (a, phi,
    v) that fix g^eq, in the compute type, instead of the 27 g):
      moments  read f and the five values (each node's once), write rho, phi
               (FP16 storage: and read the density f was encoded with);
      collide  read f, rho, phi, F, mu_phi, write f and the five values
               (FP16: and the density f was encoded with).
    step_alg: the step's algorithmic minimum for stored populations, 4 Q s +
    4 sf (read and write both population sets once, write and read rho, phi
    once); step_path: the same minimum for the path that runs (implicit g:
    2 Q s + 14 sf, the five values written and read once in place of g; FP16
    storage: + 2 sf for the decoding densities)."""
    dec = 2 * sf if fp16 else 0
    std = 4 * Q * s + 4 * sf
    if implicit_g:
        d1 = sf if fp16 else 0
        return {"moments": Q * s + 5 * sf + 2 * sf + d1, "stencil": 6 * sf,
                "collide": 2 * Q * s + 6 * sf + 5 * sf + d1, "step_alg": std,
                "step_path": 2 * Q * s + 14 * sf + 2 * d1}
    return {"moments": 2 * Q * s + 2 * sf + dec,
            "stencil": 6 * sf,
            "collide": (2 if g_read else 1) * Q * s + 2 * Q * s + 6 * sf + dec,
            "step_alg": std, "step_path": std}


def _summary_kv(path):
    kv = {}
    try:
        text = open(path).read()
    except OSError:
        return kv
    for line in text.splitlines():
        if ":" in line and not line.startswith((" ", "|", "#", "`")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    return kv


def measured_traffic(kernel, precision):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE per dispatch, scaled by what the same
    counters read for a plain device copy), or None when the kernel source
    has changed since the counters were taken."""
    kv = _summary_kv(PMC_SUMMARY)
    try:
        src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    if kv.get("kernel_source_sha256") != src:
        return None
    key = "%s_%s" % (kernel, precision)
    try:
        return 1024.0 * (float(kv[key + "_fetch_kib"]) * float(kv["fetch_factor"]) +
                         float(kv[key + "_write_kib"]) * float(kv["write_factor"]))
    except (KeyError, ValueError):
        return None


def run3(L, I, precision, steps, warmup, n=N3, init=None):
    import torch
    p = params3(L, precision, n)
    sim = L.Sim(p, device="cuda:0")
    sim.init(*(init if init is not None else fields3(I, n)))
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prof = sim.step_profiled(steps, SAMPLE_EVERY)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    obs = sim.observe()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return wall, prof, obs


# Other workloads, timed the same way: the two D2Q9 channels.
#   capillary channel 2048 x 64: liquid-2 slug x < 256, liquid-3 films of 3
#     rows, theta 60 deg (state 21 MB: resident in the 256 MB Infinity Cache,
#     so no HBM fraction is quoted for it);
#   drop train 4096 x 256: 16 alternating drops r = 40 spaced 200 (PCG64
#     seed 0 jitter), theta (45, 120, 90) deg.
def other_grids(L, I):
    import torch
    out = {}
    cases = (
        ("d2q9_2048x64_capillary_fp32", (2048, 64), 60.0, lambda: I.capillary_2d(2048, 64, 256, film=3), 2000, 200,
         False),
        ("d2q9_4096x256_drop_train_fp32", (4096, 256), (45.0, 120.0, 90.0), lambda: I.drop_train_2d(4096, 256),
         400, 50, True),
    )
    for name, n, th, mk, steps, warm, hbm in cases:
        p = L.make_params(L.D2Q9, n, gamma=(0.01, 0.01, 0.01), width=4.0, theta_deg=th, precision=L.FP32)
        s = L.Sim(p, device="cuda:0")
        s.init(*mk())
        s.step(warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pr = s.step_profiled(steps, SAMPLE_EVERY)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        o = s.observe()
        s.close()
        del s
        torch.cuda.empty_cache()
        fluid = n[0] * (n[1] - 2)
        rec = {"MLUPS": fluid * steps / wall / 1e6, "ms_per_step": 1e3 * wall / steps,
               "moments_ms": pr["moments"], "fused_ms": pr["fused"], "steps": steps, "n_bad": o["n_bad"]}
        if hbm:
            alg = 4 * 9 * 4 + 4 * 4
            rec["step_frac_alg"] = fluid * steps / wall * alg / (HBM_PEAK_GBS * 1e9)
        out[name] = rec
    return out


# Serving: 48 requests drawn from the configuration-5 distribution (seed
# 2024: 70% D2Q9 squares 64..1024, 30% D3Q27 cubes 64..192, contact angle
# 30..150 deg, tensions 0.005..0.03, FP32 or FP16-offset storage) with the
# configured step counts (5k..20k) divided by 20, served twice: as a burst
# (all arriving at once: the throughput ratio is the capacity ratio), then
# as a Poisson stream (seeded) at 0.8 times the sequential capacity that the
# burst measured.  A burst of 48 small D2Q9 grids (64^2..256^2) is timed
# beside it.
SERVE_N, SERVE_STEPS, SERVE_QUANTUM, SERVE_LOAD = 48, (250, 1000), 50, 0.8
SERVE_DIV = 20   # the configured 5k..20k steps per request, divided
SERVE_POOL = 24 << 30


def serving_requests(L, I, small2d=False):
    if small2d:
        reqs = I.serving_requests(SERVE_N, seed=2025, frac_2d=1.0, grid2=(64, 256), steps=SERVE_STEPS)
    else:
        reqs = I.serving_requests(SERVE_N, seed=2024, steps=SERVE_STEPS)
    for q in reqs:
        lat = L.D2Q9 if q["lattice"] == "D2Q9" else L.D3Q27
        prec = L.FP32 if q["precision"] == "fp32" else L.FP16S
        q["params"] = L.make_params(lat, q["n"], gamma=q["gamma"], theta_deg=q["theta"], precision=prec)
        q["fields"] = I.request_fields(q)
        q["updates"] = float(np.prod(q["n"])) * q["nsteps"]
        q["arrival"] = 0.0
    return reqs


def _pct(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else None


def run_serving(L, reqs):
    """Continuous batching: submit each request at its arrival time, run
    rounds of SERVE_QUANTUM batched steps, collect results.  Time to result
    is completion minus scheduled arrival."""
    srv = L.Server(SERVE_POOL, max_resident=64, max_skips=4)
    t0 = srv.clock()
    done, i, n = {}, 0, len(reqs)
    while len(done) < n:
        now = srv.clock() - t0
        while i < n and reqs[i]["arrival"] <= now:
            q = reqs[i]
            srv.submit(q["params"], *q["fields"], q["nsteps"], tag=q["tag"])
            i += 1
        nr, nq = srv.run(SERVE_QUANTUM)
        for r in srv.poll():
            done[r["tag"]] = r
            if len(done) % 64 == 0:
                print("serving: %d/%d batched requests done" % (len(done), n), file=sys.stderr, flush=True)
        if nr == 0 and nq == 0 and i < n and len(done) == i:
            time.sleep(max(0.0, reqs[i]["arrival"] - (srv.clock() - t0)))
    makespan = max(r["t_done"] for r in done.values()) - t0
    srv.close()
    lat = [done[q["tag"]]["t_done"] - t0 - q["arrival"] for q in reqs]
    ok = sum(1 for r in done.values() if r["status"] == 0)
    return lat, makespan, ok


def run_plain(L, reqs):
    """The same stream solved one request at a time (first come first
    served), each alone on the GPU with lbm3_step."""
    import torch
    t0 = time.perf_counter()
    lat, ok = [], 0
    for q in reqs:
        now = time.perf_counter() - t0
        if q["arrival"] > now:
            time.sleep(q["arrival"] - now)
        s = L.Sim(q["params"])
        s.init(*q["fields"])
        s.step(q["nsteps"])
        o = s.observe()
        s.close()
        del s
        ok += o["status"] == 0
        lat.append(time.perf_counter() - t0 - q["arrival"])
        if len(lat) % 64 == 0:
            print("serving: %d/%d requests done one at a time" % (len(lat), len(reqs)), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return lat, time.perf_counter() - t0, ok


def _compare(L, reqs):
    total = sum(q["updates"] for q in reqs)
    lat_s, span_s, ok_s = run_serving(L, reqs)
    print("serving: %d requests batched in %.1f s" % (len(reqs), span_s), file=sys.stderr, flush=True)
    lat_p, span_p, ok_p = run_plain(L, reqs)
    print("serving: %d requests one at a time in %.1f s" % (len(reqs), span_p), file=sys.stderr, flush=True)
    return {
        "node_updates": total,
        "batched": {"MLUPS": total / span_s / 1e6, "makespan_s": span_s, "p50_s": _pct(lat_s, 50),
                    "p99_s": _pct(lat_s, 99), "ok": ok_s, "quantum": SERVE_QUANTUM, "pool_bytes": SERVE_POOL},
        "plain": {"MLUPS": total / span_p / 1e6, "makespan_s": span_p, "p50_s": _pct(lat_p, 50),
                  "p99_s": _pct(lat_p, 99), "ok": ok_p},
        "throughput_ratio": span_p / span_s,
    }


def serving_leg(L, I):
    reqs = serving_requests(L, I)
    burst = _compare(L, reqs)
    # sequential capacity (requests per second) from the burst's one-at-a-time run
    cap = len(reqs) / burst["plain"]["makespan_s"]
    rate = SERVE_LOAD * cap
    rng = np.random.Generator(np.random.PCG64(2026))
    t = np.cumsum(rng.exponential(1.0 / rate, len(reqs)))
    for q, a in zip(reqs, t):
        q["arrival"] = float(a)
    stream = _compare(L, reqs)
    desc = ("%d requests of the configuration-5 distribution (seed 2024): 70%% D2Q9 64^2..1024^2, 30%% D3Q27 "
            "64^3..192^3, sessile drops theta 30..150 deg, gamma 0.005..0.03, FP32 / FP16-offset storage, "
            "%d..%d steps (the configured 5k..20k / %d)" % (SERVE_N, SERVE_STEPS[0], SERVE_STEPS[1], SERVE_DIV))
    burst["workload"] = desc + ", all arriving together"
    stream["workload"] = desc + (", Poisson arrivals (seed 2026) at %.2f/s = %.1f x the sequential capacity "
                                 "measured on the burst" % (rate, SERVE_LOAD))
    small = _compare(L, serving_requests(L, I, small2d=True))
    small["workload"] = "burst of %d D2Q9 requests 64^2..256^2 (seed 2025), otherwise as above" % SERVE_N
    return {"stream": stream, "burst": burst, "burst_small_2d": small}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline():
    """The FP64 CPU oracle on the host: all threads on 2 steps of the full
    256^3 workload, and one thread on 1 step of a 96^3 grid of the same
    recipe (sphere and film scaled), each after its own initialisation."""
    from oracle import oracle as O
    from paper_1904_06881_amd import inputs as I
    from paper_1904_06881_amd import lbm3 as L

    def time_oracle(n, steps):
        d = L.lbm3_resolve(params3(L, L.FP64, n))
        eos = {k: getattr(d, k) for k in ("a", "b", "T", "C", "psi0", "rho_l", "rho_g")}
        po = O.make_params(3, n, lam=list(d.lam), kap=list(d.kap), theta_deg=90.0, eos=eos,
                           rho_l=d.rho_l, rho_g=d.rho_g)
        sim = O.Sim(po)
        sim.init(*fields3(I, n))
        t0 = time.perf_counter()
        sim.step(steps)
        dt = time.perf_counter() - t0
        del sim
        fluid = n[0] * n[1] * (n[2] - 2)
        return fluid * steps / dt / 1e6, dt

    threads = O.get_threads()
    v_all, dt_all = time_oracle(N3, 2)
    O.set_threads(1)
    n1 = (96, 96, 96)
    v_one, dt_one = time_oracle(n1, 1)
    O.set_threads(threads)
    return {"value": v_all, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "2 steps of the 256^3 FP64 workload after initialisation (%.1f s)" % dt_all,
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "one_core": {"value": v_one, "unit": "MLUPS", "cores": 1,
                         "sample": "1 step of a 96^3 grid of the same recipe (sphere r 18, film 3; %.1f s)"
                                   % dt_one}}


def main():
    global SERVE_N, SERVE_STEPS, SERVE_DIV
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-variants", action="store_true", help="skip the FP16-storage and FP64 forms")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving comparison")
    ap.add_argument("--no-other", action="store_true", help="skip the D2Q9 channel workloads")
    ap.add_argument("--precision", default="fp32", choices=("fp32", "fp16s", "fp64"),
                    help="storage of the timed run (the headline is fp32)")
    ap.add_argument("--serve-requests", type=int, default=SERVE_N,
                    help="requests of the serving comparison (the configuration asks 512)")
    ap.add_argument("--serve-step-div", type=int, default=20,
                    help="divide the configured 5k..20k steps per request by this (1: the full counts)")
    ap.add_argument("--serve-profile", action="store_true",
                    help="only run the serving burst (batched, then plain) and print the phase clocks; for a "
                         "kernel trace of the two")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 256 MiB device copy (HBM counter calibration) and exit")
    ap.add_argument("--scale-grid", type=int, default=0, metavar="N",
                    help="only run the 256^3 workload's recipe scaled to N^3 (FP32; sphere and film scaled) and "
                         "print its step rate, kernel times, workspace and mass drift, then exit")
    ap.add_argument("--hbm-rate", action="store_true",
                    help="only time torch's own 2 GiB device copy and fill (an attainable HBM rate to set the "
                         "kernels' rates beside) and exit")
    args = ap.parse_args()
    SERVE_N = args.serve_requests
    SERVE_DIV = args.serve_step_div
    SERVE_STEPS = (5000 // args.serve_step_div, 20000 // args.serve_step_div)
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs each simulation on a single device "
              "(--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1904_06881_amd import inputs as I
    from paper_1904_06881_amd import lbm3 as L
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.serve_profile:
        reqs = serving_requests(L, I)
        torch.cuda.synchronize()
        t0 = time.monotonic_ns()
        _, span_b, ok_b = run_serving(L, reqs)
        t1 = time.monotonic_ns()
        _, span_p, ok_p = run_plain(L, reqs)
        t2 = time.monotonic_ns()
        print(json.dumps({"serve_profile": True, "monotonic_ns": [t0, t1, t2], "makespan_batched_s": span_b,
                          "makespan_plain_s": span_p, "ok": [ok_b, ok_p]}), flush=True)
        return
    if args.copy_calib:
        x = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4}), flush=True)
        return

    if args.hbm_rate:
        x = torch.ones(1 << 29, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        nb = x.numel() * 4

        def timed(fn, reps=20):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps / 1e3

        tc = timed(lambda: y.copy_(x))
        tf = timed(lambda: y.fill_(2.0))
        print(json.dumps({"bytes": nb, "copy_ms": tc * 1e3, "copy_TBs": 2 * nb / tc / 1e12,
                          "fill_ms": tf * 1e3, "fill_TBs": nb / tf / 1e12}), flush=True)
        return

    if args.scale_grid:
        n = (args.scale_grid,) * 3
        fl = n[0] * n[1] * (n[2] - 2)
        p = params3(L, L.FP32, n)
        sim = L.Sim(p, device="cuda:0")
        sim.init(*fields3(I, n))
        o0 = sim.observe()
        sim.step(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prof = sim.step_profiled(args.steps, SAMPLE_EVERY)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        o = sim.observe()
        print(json.dumps({"grid": list(n), "fluid_nodes": fl, "precision": "fp32", "steps": args.steps,
                          "warmup": args.warmup, "MLUPS": fl * args.steps / wall / 1e6,
                          "ms_per_step": 1e3 * wall / args.steps,
                          "kernel_ms_per_launch": {k: prof[k] for k in ("moments", "stencil", "collide", "ghost")},
                          "workspace_bytes": L.lbm3_footprint(p), "n_bad": o["n_bad"], "status": o["status"],
                          "mass_drift": [abs(o["mass"][k] - o0["mass"][k]) / max(abs(o0["mass"][k]), 1e-300)
                                         for k in range(3)]}), flush=True)
        return

    precs = {"fp32": (L.FP32, 4, 4, False), "fp16s": (L.FP16S, 2, 4, True), "fp64": (L.FP64, 8, 8, False)}
    P, s, sf, fp16 = precs[args.precision]
    fluid = N3[0] * N3[1] * (N3[2] - 2)
    init = fields3(I)
    wall, prof, obs = run3(L, I, P, args.steps, args.warmup, init=init)
    ms_step = 1e3 * wall / args.steps
    mlups = fluid * args.steps / wall / 1e6

    kb = kernel_bytes(27, s, sf, fp16, g_read=False, implicit_g=True)
    kern = {"moments": prof["moments"], "stencil": prof["stencil"], "collide": prof["collide"],
            "ghost": prof["ghost"]}
    dom = max(("moments", "stencil", "collide"), key=lambda k: kern[k])
    per_launch = kb[dom] * fluid
    achieved = per_launch / (kern[dom] * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": "k_" + dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom, args.precision),
            "bytes_per_node": kb[dom], "bytes_per_launch": per_launch, "avg_launch_ms": kern[dom],
            "launches_timed": prof["sampled"]}
    step_frac = mlups * 1e6 * kb["step_path"] / (HBM_PEAK_GBS * 1e9)

    variants = {}
    if not args.no_variants:
        for name in ("fp16s", "fp64"):
            if name == args.precision:
                continue
            Pv, sv, sfv, f16v = precs[name]
            n = 50 if name == "fp16s" else 20
            w, pr, o = run3(L, I, Pv, n, 5, init=init)
            kv = kernel_bytes(27, sv, sfv, f16v, g_read=False, implicit_g=True)
            mv = fluid * n / w / 1e6
            variants[name] = {"MLUPS": mv, "ms_per_step": 1e3 * w / n, "moments_ms": pr["moments"],
                              "stencil_ms": pr["stencil"], "collide_ms": pr["collide"],
                              "step_frac_path": mv * 1e6 * kv["step_path"] / (HBM_PEAK_GBS * 1e9),
                              "bytes_per_node_path": kv["step_path"], "n_bad": o["n_bad"]}

    line = {
        "metric": METRIC, "value": mlups, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp32": "f32", "fp16s": "f32", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "D3Q27 lubricated sessile drop 256^3: liquid-2 sphere r 48 on an 8-node liquid-3 "
                               "film, gas above, density ratio 1000, gamma 0.02/0.02/0.01, width 4, tau 1, "
                               "geometric interpolation 90 deg walls at z = 0, 255; %s storage" % args.precision,
                   "grid": list(N3), "fluid_nodes": fluid, "precision": args.precision,
                   "kernels_per_step": 4},
        "roofline": roof,
        "step_roofline": {"bytes_per_node_path": kb["step_path"], "achieved": mlups * kb["step_path"] / 1e3,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": step_frac,
                          "bytes_per_node_stored_g": kb["step_alg"],
                          "equivalent_stored_g_GBs": mlups * kb["step_alg"] / 1e3},
        "kernel_ms_per_launch": kern,
        "kernel_bytes_per_node": kb,
        "n_bad": obs["n_bad"],
        "alpha_kinds": {"newton": obs["n_newton"], "small_deviation": obs["n_shortcut"],
                        "fallback": obs["n_fallback"]},
        "variants": variants,
    }
    if not args.no_other:
        line["other_grids"] = other_grids(L, I)
    if not args.no_serving:
        line["serving"] = serving_leg(L, I)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
