"""Batched stepping and the continuous-batching server on the GPU.

A simulation's result must not depend on what runs beside it: every case
compares the batched or served run with the same simulation stepped alone by
lbm3_step, bit for bit (the batched kernels run the same per-node arithmetic).
"""
import sys

import numpy as np
import pytest

from paper_1904_06881_amd import inputs as I
from paper_1904_06881_amd import lbm3 as L

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


G = (0.01, 0.012, 0.009)


def mixed_cases():
    """Seven simulations over every batch class: 2D 62-node tiles in three
    precisions, a periodic 2D box, 3D in FP32, FP64 and FP16 storage
    (ghost-layer launch, implicit g)."""
    return [
        (L.make_params(L.D2Q9, (96, 48), gamma=G, theta_deg=60.0, precision=L.FP64),
         I.sessile_drop_2d(96, 48, 16)),
        (L.make_params(L.D2Q9, (130, 40), gamma=G, theta_deg=120.0, precision=L.FP32,
                       wetting=L.WET_GEOM_EXTRAP), I.sessile_drop_2d(130, 40, 14, xc=40.0)),
        (L.make_params(L.D2Q9, (64, 64), gamma=G, theta_deg=(45.0, 100.0, 80.0), precision=L.FP16S),
         I.capillary_2d(64, 64, 20, film=3)),
        (L.make_params(L.D2Q9, (70, 36), gamma=G, walls=False, precision=L.FP32),
         I.random_fields((36, 70), seed=3)),
        (L.make_params(L.D3Q27, (40, 24, 20), gamma=G, theta_deg=70.0, precision=L.FP32),
         I.sessile_drop_3d(40, 24, 20, 8)),
        (L.make_params(L.D3Q27, (24, 24, 16), gamma=G, theta_deg=110.0, precision=L.FP64),
         I.sessile_drop_3d(24, 24, 16, 6)),
        (L.make_params(L.D3Q27, (28, 20, 14), gamma=G, theta_deg=100.0, precision=L.FP16S),
         I.sessile_drop_3d(28, 20, 14, 6)),
    ]


def alone(p, init, nsteps, counts=None):
    s = L.Sim(p)
    s.init(*init)
    s.step(nsteps)
    out = s.fields() + s.pops()
    if counts is not None:
        o = s.observe()
        counts.extend(o[k] for k in ("n_newton", "n_shortcut", "n_fallback", "n_fast"))
    s.close()
    return out


def test_batched_steps_equal_steps_alone():
    cases = mixed_cases()
    sims = []
    for k, (p, init) in enumerate(cases):
        say("batch member", k, tuple(p.n), "precision", p.precision)
        s = L.Sim(p)
        s.init(*init)
        sims.append(s)
    # odd step counts over two calls exercise the buffer parities
    ws1 = L.step_batch(sims, 13)
    ws2 = L.step_batch(sims, 18)
    import torch
    torch.cuda.synchronize()
    del ws1, ws2
    for k, (p, init) in enumerate(cases):
        say("compare", k)
        cref = []
        ref = alone(p, init, 31, cref)
        got = sims[k].fields() + sims[k].pops()
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), k
        o = sims[k].observe()
        assert o["step"] == 31
        # the entropic-alpha statistics, counted in the batched kernels'
        # own slots, equal those of the run alone
        assert [o[q] for q in ("n_newton", "n_shortcut", "n_fallback", "n_fast")] == cref, k
        sims[k].close()


def test_server_results_equal_runs_alone_and_fit_the_pool():
    """Requests arrive while others run; the pool admits about three at a
    time; every result equals its run alone, and the simulations resident at
    any moment fit in the pool."""
    cases = mixed_cases()
    steps = [23, 40, 17, 31, 12, 9, 14]
    need = [L.server_request_bytes(p) for p, _ in cases]
    pool = int(sum(sorted(need)[-3:]) + 2 * (1 << 20) + max(1 << 20, sum(need) // 256))
    srv = L.Server(pool, max_resident=8, max_skips=2)
    say("pool bytes", pool, "request bytes", need)
    for k in range(3):
        srv.submit(cases[k][0], *cases[k][1], steps[k], tag=k, keep_fields=True)
    bad = L.make_params(L.D2Q9, (32, 32), gamma=(0.001, 0.05, 0.001))  # no calibration exists
    srv.submit(bad, *I.sessile_drop_2d(32, 32, 8), 10, tag=99)
    srv.run(5)
    srv.run(5)
    for k in range(3, len(cases)):
        srv.submit(cases[k][0], *cases[k][1], steps[k], tag=k, keep_fields=True)
    results = {}
    for _ in range(200):
        nr, nq = srv.run(7)
        for r in srv.poll():
            results[r["tag"]] = r
        if nr == 0 and nq == 0 and len(results) == len(cases) + 1:
            break
    for r in srv.poll():
        results[r["tag"]] = r
    assert results[99]["status"] == -6  # LBM3_ECALIB, from the calibration on a worker thread
    fields = {}
    for k in range(len(cases)):
        r = results[k]
        assert r["status"] == 0 and r["has_fields"], r
        assert r["steps"] == steps[k]
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
        fields[k] = srv.fields(k)
    # resident bytes at every admission stay within the pool
    ok = [results[k] for k in range(len(cases))]
    for a in ok:
        held = sum(b["bytes"] for b in ok if b["t_admit"] <= a["t_admit"] < b["t_done"])
        assert held <= pool
    srv.close()
    for k, (p, init) in enumerate(cases):
        say("server vs alone", k)
        ref = alone(p, init, steps[k])
        assert np.array_equal(ref[0], fields[k][0]), k
        assert np.array_equal(ref[1], fields[k][1]), k


def test_server_stream_of_requests_completes():
    """A seeded stream from the serving workload at reduced sizes: all finish
    with finite fields and their requested step counts."""
    reqs = I.serving_requests(12, seed=5, grid2=(48, 160), grid3=(24, 40), steps=(20, 60))
    srv = L.Server(1 << 30, max_resident=16, max_skips=4)
    for q in reqs:
        lat = L.D2Q9 if q["lattice"] == "D2Q9" else L.D3Q27
        prec = L.FP32 if q["precision"] == "fp32" else L.FP16S
        p = L.make_params(lat, q["n"], gamma=q["gamma"], theta_deg=q["theta"], precision=prec)
        srv.submit(p, *I.request_fields(q), q["nsteps"], tag=q["tag"])
    done = {}
    for _ in range(100):
        nr, nq = srv.run(16)
        for r in srv.poll():
            done[r["tag"]] = r
        if nr == 0 and nq == 0 and len(done) == len(reqs):
            break
    srv.close()
    assert len(done) == len(reqs)
    for q in reqs:
        r = done[q["tag"]]
        say("request", q["tag"], q["lattice"], q["n"], "status", r["status"])
        assert r["status"] == 0 and r["steps"] == q["nsteps"] and r["obs"]["n_bad"] == 0
