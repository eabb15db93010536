"""Benchmark: one time step of the ternary wetting LBM update on one MI355X.

Workload (the capillary-filling channel): D2Q9, 2048 x 64 nodes, walls at
y = 0 and 63, liquid-2 slug on x < 256 displacing gas, liquid-3 films of 3
rows on both walls, gamma_ij = 0.01, interface width 4, tau = 1, density
ratio 1000, geometric-interpolation wetting at 60 degrees; FP32 arithmetic
and storage (FP64 and FP16-offset storage timed beside it).  Inputs are
synthetic (seeded geometry) and resident in HBM before the timed region.

Prints one JSON line: MLUPS over fluid nodes, the roofline of the dominant
kernel from HIP events on the library's stream, and the CPU oracle's MLUPS on
a bounded sample of the same workload; beside them the HBM fractions of the
256^3 D3Q27 and 4096 x 256 D2Q9 grids, and the serving comparison.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS and % HBM roofline per step; serving p50/p99 time-to-result vs plain"
HBM_PEAK_GBS = 8000.0
NX, NY = 2048, 64
X_FRONT, FILM, THETA = 256, 3, 60.0


def workload_params(L, precision):
    return L.make_params(L.D2Q9, (NX, NY), gamma=(0.01, 0.01, 0.01), width=4.0, tau_f=1.0, tau_g=1.0,
                         wetting=L.WET_GEOM_INTERP, theta_deg=THETA, precision=precision)


SAMPLE_EVERY = 25  # events around the launches of every 25th step
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_fused_d2q9_2048x64.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1904_06881_amd", "csrc", "lbm3_kernels.hip")


def measured_traffic(summary=PMC_SUMMARY, prefix="traffic"):
    """HBM bytes per launch (per fused pass in the 3D two-kernel step) from a
    committed rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE per
    dispatch, scaled by the copy calibration), or None when the kernel
    source has changed since the counters were taken."""
    import hashlib
    try:
        text = open(summary).read()
        src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    kv = {}
    for line in text.splitlines():
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != src:
        return None
    try:
        return 1024.0 * (float(kv[prefix + "_fetch_kib_per_dispatch"]) * float(kv["fetch_factor"]) +
                         float(kv[prefix + "_write_kib_per_dispatch"]) * float(kv["write_factor"]))
    except (KeyError, ValueError):
        return None


def bytes_per_node(Q, s, sf, fp16, two_kernel=False):
    """Algorithmic HBM bytes per fluid-node update.  Fused kernel: read and
    write both population sets (4 Q s) and read rho, phi (2 s_f), plus the
    previous step's rho, phi for FP16 decoding.  The 3D two-kernel step
    (stencil pass + collide) adds a second read of rho, phi and the write and
    read of F, mu_phi (4 values in FP32).  Moments kernel: read both sets
    (2 Q s), write rho, phi (2 s_f) (+ decode fields for FP16).  The wall
    ghost layers are left out."""
    extra = 2 * sf if fp16 else 0
    fused = 4 * Q * s + 2 * sf + extra + ((2 * sf + 2 * 4 * 4) if two_kernel else 0)
    moments = 2 * Q * s + 2 * sf + extra
    alg = 4 * Q * s + 4 * sf  # one read + one write of everything a step must touch
    return fused, moments, alg


def run_gpu(L, I, precision, steps, warmup):
    import torch
    p = workload_params(L, precision)
    sim = L.Sim(p, device="cuda:0")
    rho0, phi0 = I.capillary_2d(NX, NY, X_FRONT, film=FILM)
    sim.init(rho0, phi0)
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prof = sim.step_profiled(steps, SAMPLE_EVERY)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    obs = sim.observe()
    sim.close()
    return wall, prof, obs


# Large grids: the other two stencil workloads at full size, timed with the
# same sampled events (fused-launch HBM fraction at algorithmic bytes).
#   D3Q27 lubricated sessile drop, 256^3, sphere r = 48 on an 8-node film,
#   gamma (0.02, 0.02, 0.01), 90 deg walls: FP32 and FP16-offset storage;
#   D2Q9 drop train, 4096 x 256, 16 alternating drops r = 40 spaced 200,
#   theta (45, 120, 90) deg: FP32.
LARGE = (
    ("d3q27_256cube_fp32", "D3Q27", (256, 256, 256), "fp32", 20, 5),
    ("d3q27_256cube_fp16s", "D3Q27", (256, 256, 256), "fp16s", 20, 5),
    ("d2q9_4096x256_fp32", "D2Q9", (4096, 256), "fp32", 400, 100),
)
# counter summaries of the same runs: (file, key prefix) per grid
LARGE_PMC = {
    "d3q27_256cube_fp32": (os.path.join(ROOT, "profiles", "k_collide_d3q27_256cube.md"), "traffic_fp32"),
    "d3q27_256cube_fp16s": (os.path.join(ROOT, "profiles", "k_collide_d3q27_256cube.md"), "traffic_fp16s"),
    "d2q9_4096x256_fp32": (os.path.join(ROOT, "profiles", "k_fused_d2q9_4096x256.md"), "traffic"),
}


def large_grids(L, I):
    import torch
    out = {}
    init3 = None
    for name, lat, n, prec, steps, warm in LARGE:
        P = {"fp32": L.FP32, "fp16s": L.FP16S}[prec]
        if lat == "D3Q27":
            p = L.make_params(L.D3Q27, n, gamma=(0.02, 0.02, 0.01), width=4.0, theta_deg=90.0, precision=P)
            if init3 is None:
                init3 = I.lubricated_drop_3d(*n, 48, film=8)
            init, Q, fluid = init3, 27, n[0] * n[1] * (n[2] - 2)
        else:
            p = L.make_params(L.D2Q9, n, gamma=(0.01, 0.01, 0.01), width=4.0, theta_deg=(45.0, 120.0, 90.0),
                              precision=P)
            init, Q, fluid = I.drop_train_2d(*n), 9, n[0] * (n[1] - 2)
        s = L.Sim(p, device="cuda:0")
        s.init(*init)
        s.step(warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pr = s.step_profiled(steps, 5)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        o = s.observe()
        s.close()
        del s
        torch.cuda.empty_cache()
        fb, mb, ab = bytes_per_node(Q, 2 if prec == "fp16s" else 4, 4, prec == "fp16s", two_kernel=Q == 27)
        fgbs = fb * fluid / (pr["fused"] * 1e-3) / 1e9
        mgbs = mb * fluid / (pr["moments"] * 1e-3) / 1e9
        out[name] = {"MLUPS": fluid * steps / wall / 1e6, "ms_per_step": 1e3 * wall / steps,
                     "fused_ms": pr["fused"], "fused_GBs": fgbs, "fused_frac": fgbs / HBM_PEAK_GBS,
                     "moments_ms": pr["moments"], "moments_GBs": mgbs, "moments_frac": mgbs / HBM_PEAK_GBS,
                     "bytes_per_node": {"fused": fb, "moments": mb, "step_min": ab},
                     "step_frac": fluid * steps / wall * ab / (HBM_PEAK_GBS * 1e9),
                     "fused_traffic": measured_traffic(*LARGE_PMC[name]),
                     "n_bad": o["n_bad"]}
    return out


# Serving sample: 48 requests of the serving stream (Poisson arrivals at 16
# per second; 70% D2Q9 squares 64..1024, 30% D3Q27 cubes 64..192; contact
# angle 30..150 deg; tensions 0.005..0.03; FP32 or FP16-offset storage) with
# the step counts of the full stream (5k..20k) divided by 20.
SERVE_N, SERVE_RATE, SERVE_STEPS, SERVE_QUANTUM = 48, 16.0, (250, 1000), 50
SERVE_POOL = 24 << 30


def serving_requests(L, I, burst=False):
    if burst:
        # burst: small D2Q9 requests (64^2..256^2) all arriving at once
        reqs = I.serving_requests(SERVE_N, seed=2025, rate=SERVE_RATE, frac_2d=1.0, grid2=(64, 256),
                                  steps=SERVE_STEPS)
        for q in reqs:
            q["arrival"] = 0.0
    else:
        reqs = I.serving_requests(SERVE_N, seed=2024, rate=SERVE_RATE, steps=SERVE_STEPS)
    for q in reqs:
        lat = L.D2Q9 if q["lattice"] == "D2Q9" else L.D3Q27
        prec = L.FP32 if q["precision"] == "fp32" else L.FP16S
        q["params"] = L.make_params(lat, q["n"], gamma=q["gamma"], theta_deg=q["theta"], precision=prec)
        q["fields"] = I.request_fields(q)
        q["updates"] = float(np.prod(q["n"])) * q["nsteps"]
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
    torch.cuda.synchronize()
    return lat, time.perf_counter() - t0, ok


def _compare(L, reqs):
    total = sum(q["updates"] for q in reqs)
    lat_s, span_s, ok_s = run_serving(L, reqs)
    lat_p, span_p, ok_p = run_plain(L, reqs)
    return {
        "node_updates": total,
        "batched": {"MLUPS": total / span_s / 1e6, "makespan_s": span_s, "p50_s": _pct(lat_s, 50),
                    "p99_s": _pct(lat_s, 99), "ok": ok_s, "quantum": SERVE_QUANTUM, "pool_bytes": SERVE_POOL},
        "plain": {"MLUPS": total / span_p / 1e6, "makespan_s": span_p, "p50_s": _pct(lat_p, 50),
                  "p99_s": _pct(lat_p, 99), "ok": ok_p},
        "throughput_ratio": span_p / span_s,
    }


def serving_leg(L, I):
    out = _compare(L, serving_requests(L, I))
    out["workload"] = ("%d requests of the serving stream (seed 2024): Poisson arrivals %.0f/s, 70%% D2Q9 "
                       "64^2..1024^2, 30%% D3Q27 64^3..192^3, sessile drops theta 30..150 deg, gamma 0.005..0.03, "
                       "FP32 / FP16-offset storage, %d..%d steps (full stream / 20)"
                       % (SERVE_N, SERVE_RATE, SERVE_STEPS[0], SERVE_STEPS[1]))
    burst = _compare(L, serving_requests(L, I, burst=True))
    burst["workload"] = ("burst: %d D2Q9 requests 64^2..256^2 (seed 2025) arriving together, otherwise as the "
                         "stream" % SERVE_N)
    out["burst"] = burst
    return out


def cpu_baseline(target_s=12.0):
    import numpy as np
    from oracle import oracle as O
    from paper_1904_06881_amd import inputs as I
    from paper_1904_06881_amd import lbm3 as L
    d = L.lbm3_resolve(workload_params(L, L.FP64))
    eos = {k: getattr(d, k) for k in ("a", "b", "T", "C", "psi0", "rho_l", "rho_g")}
    po = O.make_params(2, (NX, NY), lam=list(d.lam), kap=list(d.kap), theta_deg=THETA, eos=eos,
                       rho_l=d.rho_l, rho_g=d.rho_g)
    sim = O.Sim(po)
    rho0, phi0 = I.capillary_2d(NX, NY, X_FRONT, film=FILM)
    sim.init(rho0, phi0)
    t0 = time.perf_counter()
    sim.step(5)
    t5 = time.perf_counter() - t0
    n = max(10, int(target_s / max(t5 / 5, 1e-6)))
    t0 = time.perf_counter()
    sim.step(n)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    fluid = NX * (NY - 2)
    return {"value": fluid * n / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "%d steps of the same 2048x64 FP64 workload after 5 warm-up steps (%.1f s)" % (n, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-variants", action="store_true", help="skip the FP64 / FP16-storage runs")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving comparison")
    ap.add_argument("--no-large", action="store_true", help="skip the 256^3 and 4096x256 grids")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 256 MiB device copy (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the build runs a single simulation per device "
              "(--gpus %d not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1904_06881_amd import inputs as I
    from paper_1904_06881_amd import lbm3 as L
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calib:
        x = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4}), flush=True)
        return

    fluid = NX * (NY - 2)
    wall, prof, obs = run_gpu(L, I, L.FP32, args.steps, args.warmup)
    ms_step = 1e3 * wall / args.steps
    mlups = fluid * args.steps / wall / 1e6

    fused_b, mom_b, alg_b = bytes_per_node(9, 4, 4, False)
    kern = {k: prof[k] for k in ("moments", "fused")}  # mean ms per launch
    dom = max(kern, key=kern.get)
    per_launch_bytes = {"fused": fused_b * fluid, "moments": mom_b * fluid}[dom]
    achieved = per_launch_bytes / (kern[dom] * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": "k_" + dom,
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic() if dom == "fused" else None, "bytes_per_launch": per_launch_bytes, "avg_launch_ms": kern[dom],
            "launches_timed": prof["sampled"]}

    variants = {}
    for name, prec, b in () if args.no_variants else (("f64", L.FP64, bytes_per_node(9, 8, 8, False)),
                                                      ("f16s", L.FP16S, bytes_per_node(9, 2, 4, True))):
        n = max(200, args.steps // 4)
        w, pr, o = run_gpu(L, I, prec, n, min(args.warmup, 200))
        variants[name] = {"MLUPS": fluid * n / w / 1e6, "fused_ms": pr["fused"],
                          "fused_GBs": b[0] * fluid / (pr["fused"] * 1e-3) / 1e9,
                          "n_bad": o["n_bad"], "alpha_fallback": o["n_fallback"]}

    line = {
        "metric": METRIC, "value": mlups, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "D2Q9 capillary filling 2048x64, liquid-2 slug x<256, liquid-3 films "
                               "3 rows, density ratio 1000, gamma 0.01, width 4, tau 1, geometric "
                               "interpolation 60 deg, FP32 storage",
                   "grid": [NX, NY], "fluid_nodes": fluid, "precision": "fp32", "stream_launches_per_step": 2},
        "hbm_frac_of_step": mlups * 1e6 * alg_b / (HBM_PEAK_GBS * 1e9),
        "bytes_per_node_alg": alg_b,
        "kernel_ms_per_launch": kern,
        "n_bad": obs["n_bad"],
        "alpha_kinds": {"newton": obs["n_newton"], "small_deviation": obs["n_shortcut"],
                        "fallback": obs["n_fallback"]},
        "variants": variants,
        "roofline": roof,
    }
    if not args.no_large:
        line["large_grids"] = large_grids(L, I)
    if not args.no_serving:
        line["serving"] = serving_leg(L, I)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
