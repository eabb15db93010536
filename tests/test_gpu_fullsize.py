"""Parity at the benchmarked sizes, in the launch configuration bench.py
times: the lubricated drop at 256^3 (D3Q27, the two-kernel step with
implicit g, 16.6 M fluid nodes) and the 4096 x 256 drop train (D2Q9, the
254-node fused tiles), every fluid node of the GPU run against the FP64 CPU
oracle run on the same seeded input.  The oracle needs about 18 GB of host
memory and 5 s per 256^3 step on 16 threads, so the 3D case runs 2 steps.
The drop train's contact lines amplify rounding differences of any origin
(one e-fold in about 5 steps from step 50 on, saturating near 1e-5): FP64
runs of the GPU and the oracle, which differ only in summation order, agree
to 1e-15 for 50 steps, to 1e-10 at step 100 and to 1e-5 after 2000, so the
drop train is compared to rounding over 50 steps, and over 2000 steps the
divergence is checked to stay bounded.  Tolerances on max-abs C_k: FP64
1e-12, FP32 1e-5 (the FP32 rounding of the initial fields alone is 1e-7)."""
import pytest

from _common import conc_err, oracle_params_from, say
from oracle import oracle as O
from paper_1904_06881_amd import inputs as I
from paper_1904_06881_amd import lbm3 as L

pytestmark = pytest.mark.gpu


def _gpu(p, init, steps):
    s = L.Sim(p)
    s.init(*init)
    s.step(steps)
    o = s.observe()
    assert o["status"] == 0 and o["n_bad"] == 0
    return s


def _oracle(p, derived, init, steps):
    o = O.Sim(oracle_params_from(p, derived))
    o.init(*init)
    o.step(steps)
    return o


def test_cfg3_full_size_2_steps_matches_oracle():
    """Config 3 at 256^3 as bench.py runs it (liquid-2 sphere r 48 on an
    8-node liquid-3 film, gamma 0.02/0.02/0.01, width 4, tau 1, geometric
    interpolation at 90 degrees), FP64 and FP32, 2 steps, all nodes."""
    n = (256, 256, 256)
    init = I.lubricated_drop_3d(*n, 48, film=8)
    mk = lambda prec: L.make_params(L.D3Q27, n, gamma=(0.02, 0.02, 0.01), width=4.0, tau_f=1.0, tau_g=1.0,
                                    wetting=L.WET_GEOM_INTERP, theta_deg=90.0, precision=prec)
    say("cfg3 256^3 fp64")
    s64 = _gpu(mk(L.FP64), init, 2)
    say("cfg3 256^3 oracle")
    ora = _oracle(mk(L.FP64), s64.derived, init, 2)
    e64 = conc_err(s64, ora)
    del s64
    say("cfg3 256^3 fp32")
    s32 = _gpu(mk(L.FP32), init, 2)
    e32 = conc_err(s32, ora)
    say("cfg3 256^3 after 2 steps: fp64", e64, "fp32", e32)
    assert e64 <= 1e-12
    assert e32 <= 1e-5


def test_cfg4_full_size_50_steps_matches_oracle():
    """Config 4 at full size as bench.py runs it (4096 x 256, 16 alternating
    drops r 40 spaced 200 with seeded jitter, walls theta21 45 / theta31 120 /
    theta23 90 degrees), FP64 and FP32, 50 steps, all nodes (measured 4e-15
    and 1e-6)."""
    n = (4096, 256)
    init = I.drop_train_2d(4096, 256)
    mk = lambda prec: L.make_params(L.D2Q9, n, gamma=(0.01, 0.01, 0.01), width=4.0, theta_deg=(45.0, 120.0, 90.0),
                                    precision=prec)
    s64 = _gpu(mk(L.FP64), init, 50)
    ora = _oracle(mk(L.FP64), s64.derived, init, 50)
    e64 = conc_err(s64, ora)
    s32 = _gpu(mk(L.FP32), init, 50)
    e32 = conc_err(s32, ora)
    say("cfg4 4096x256 after 50 steps: fp64", e64, "fp32", e32)
    assert e64 <= 1e-12
    assert e32 <= 1e-5


def test_cfg4_rounding_amplification_is_bounded():
    """The drop train's sensitivity, measured on the first five drops (1024 x
    256, FP64, 2000 steps): the GPU and the oracle agree to rounding for 50
    steps; then the difference grows at first-layer contact-line nodes but
    stays bounded (measured 3.5e-5 at step 1000, 1.4e-5 at step 2000), and the
    alpha-kind counts, a discrete decision at every node and step, agree to
    0.1 % (or 10 node-steps)."""
    init = I.drop_train_2d(1024, 256, n_drops=5, r=40, spacing=200, first=100, jitter=10, seed=0)
    p = L.make_params(L.D2Q9, (1024, 256), gamma=(0.01, 0.01, 0.01), width=4.0, theta_deg=(45.0, 120.0, 90.0),
                      precision=L.FP64)
    s = L.Sim(p)
    s.init(*init)
    o = O.Sim(oracle_params_from(p, s.derived))
    o.init(*init)
    done = 0
    for t, bound in ((50, 1e-12), (1000, 1e-4), (2000, 1e-4)):
        s.step(t - done)
        o.step(t - done)
        done = t
        err = conc_err(s, o)
        og, oo = s.observe(), o.observe()
        say("cfg4 crop fp64 step", t, "err", err, "newton", og["n_newton"], oo["n_newton"])
        assert og["status"] == 0 and og["n_bad"] == 0
        assert err <= bound
        for k in ("n_newton", "n_shortcut", "n_fallback"):
            assert abs(og[k] - oo[k]) <= max(1e-3 * oo[k], 10)


def test_large_grid_512_cube_properties():
    """The config-3 recipe scaled to 512^3 (134 M nodes, a 51.5 GB workspace:
    each population set spans 14.5 GB, addressed from 64-bit array bases with
    32-bit offsets inside each array), FP32, 10 steps: no bad node, no
    instability, component masses conserved to FP32 summation accuracy."""
    n = (512, 512, 512)
    p = L.make_params(L.D3Q27, n, gamma=(0.02, 0.02, 0.01), width=4.0, tau_f=1.0, tau_g=1.0,
                      wetting=L.WET_GEOM_INTERP, theta_deg=90.0, precision=L.FP32)
    assert L.lbm3_footprint(p) > 50e9
    say("512^3 fp32")
    s = L.Sim(p)
    s.init(*I.lubricated_drop_3d(*n, 96, film=16))
    o0 = s.observe()
    s.step(10)
    o = s.observe()
    say("512^3 masses", o0["mass"], o["mass"])
    assert o["status"] == 0 and o["n_bad"] == 0
    for k in range(3):
        assert abs(o["mass"][k] - o0["mass"][k]) <= 1e-6 * abs(o0["mass"][k])


def test_library_call_before_torch_in_a_fresh_process():
    """Load order: a process whose first call into the library (here
    lbm3_footprint) comes before anything imports torch must still step on
    the GPU (torch ships its own HIP and HSA runtimes; the binding imports
    torch before it opens the library, so the library binds to those)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import numpy as np\n"
            "from paper_1904_06881_amd import lbm3 as L, inputs as I\n"
            "p = L.make_params(L.D2Q9, (64, 32), gamma=(0.01, 0.01, 0.01), width=4.0, theta_deg=60.0,"
            " precision=L.FP32)\n"
            "assert L.lbm3_footprint(p) > 0\n"
            "s = L.Sim(p)\n"
            "s.init(*I.sessile_drop_2d(64, 32, 10, xc=32))\n"
            "s.step(5)\n"
            "print('status', s.observe()['status'])\n")
    say("fresh process: library before torch")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=240)
    say("fresh process rc", r.returncode, r.stdout.strip()[-200:], r.stderr.strip()[-400:])
    assert r.returncode == 0 and "status 0" in r.stdout
