"""Benchmark: one time step of the ternary wetting LBM update on one MI355X.

Workload (the capillary-filling channel): D2Q9, 2048 x 64 nodes, walls at
y = 0 and 63, liquid-2 slug on x < 256 displacing gas, liquid-3 films of 3
rows on both walls, gamma_ij = 0.01, interface width 4, tau = 1, density
ratio 1000, geometric-interpolation wetting at 60 degrees; FP32 arithmetic
and storage (FP64 and FP16-offset storage timed beside it).  Inputs are
synthetic (seeded geometry) and resident in HBM before the timed region.

Prints one JSON line: MLUPS over fluid nodes, the roofline of the dominant
kernel from HIP events on the library's stream, and the CPU oracle's MLUPS on
a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS and % HBM roofline per step; serving p50/p99 time-to-result vs plain"
HBM_PEAK_GBS = 8000.0
NX, NY = 2048, 64
X_FRONT, FILM, THETA = 256, 3, 60.0


def workload_params(L, precision):
    return L.make_params(L.D2Q9, (NX, NY), gamma=(0.01, 0.01, 0.01), width=4.0, tau_f=1.0, tau_g=1.0,
                         wetting=L.WET_GEOM_INTERP, theta_deg=THETA, precision=precision)


def bytes_per_node(Q, s, sf, fp16):
    """Algorithmic HBM bytes per fluid-node update.  Fused kernel: read and
    write both population sets (4 Q s) and read rho, phi (2 s_f), plus the
    previous step's rho, phi for FP16 decoding.  Moments kernel: read both
    sets (2 Q s), write rho, phi (2 s_f) (+ decode fields for FP16)."""
    extra = 2 * sf if fp16 else 0
    fused = 4 * Q * s + 2 * sf + extra
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
    prof = sim.step_profiled(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    obs = sim.observe()
    sim.close()
    return wall, prof, obs


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
    ap.add_argument("--no-cpu", action="store_true")
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

    fluid = NX * (NY - 2)
    wall, prof, obs = run_gpu(L, I, L.FP32, args.steps, args.warmup)
    ms_step = 1e3 * wall / args.steps
    mlups = fluid * args.steps / wall / 1e6

    fused_b, mom_b, alg_b = bytes_per_node(9, 4, 4, False)
    kern = {k: prof[k] / args.steps for k in ("moments", "ghost", "fused")}
    dom = max(kern, key=kern.get)
    per_launch_bytes = {"fused": fused_b * fluid, "moments": mom_b * fluid,
                        "ghost": 2 * NX * (4 * 4 + 2 * 4)}[dom]
    achieved = per_launch_bytes / (kern[dom] * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": "k_fused" if dom == "fused" else "k_" + dom,
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": None, "bytes_per_launch": per_launch_bytes, "avg_launch_ms": kern[dom]}

    variants = {}
    for name, prec, b in (("f64", L.FP64, bytes_per_node(9, 8, 8, False)),
                          ("f16s", L.FP16S, bytes_per_node(9, 2, 4, True))):
        n = max(200, args.steps // 4)
        w, pr, o = run_gpu(L, I, prec, n, min(args.warmup, 200))
        variants[name] = {"MLUPS": fluid * n / w / 1e6, "fused_ms": pr["fused"] / n,
                          "fused_GBs": b[0] * fluid / (pr["fused"] / n * 1e-3) / 1e9,
                          "n_bad": o["n_bad"], "alpha_fallback": o["n_fallback"]}

    line = {
        "metric": METRIC, "value": mlups, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "D2Q9 capillary filling 2048x64, liquid-2 slug x<256, liquid-3 films "
                               "3 rows, density ratio 1000, gamma 0.01, width 4, tau 1, geometric "
                               "interpolation 60 deg, FP32 storage",
                   "grid": [NX, NY], "fluid_nodes": fluid, "precision": "fp32", "stream_launches_per_step": 3},
        "hbm_frac_of_step": mlups * 1e6 * alg_b / (HBM_PEAK_GBS * 1e9),
        "bytes_per_node_alg": alg_b,
        "kernel_ms_per_step": kern,
        "n_bad": obs["n_bad"],
        "alpha_kinds": {"newton": obs["n_newton"], "small_deviation": obs["n_shortcut"],
                        "fallback": obs["n_fallback"]},
        "variants": variants,
        "roofline": roof,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
