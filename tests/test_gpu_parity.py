"""GPU (HIP, gfx950) parity against the FP64 CPU oracle through the C ABI.

Same seeded inputs, same parameters (the library's resolved constants are
handed to the oracle as numbers).  Tolerances: FP64 max-abs C_k <= 1e-12 after
one step and <= 1e-9 after 2000 (config 1); FP32 <= 1e-4 and FP16 storage
<= 2e-3 after 2000 steps; streaming bit-exact.
"""
import numpy as np
import pytest

from _common import conc, conc_err, oracle_params_from, run_both, say
from oracle import oracle as O
from paper_1904_06881_amd import inputs as I
from paper_1904_06881_amd import lbm3 as L

pytestmark = pytest.mark.gpu


def cfg1_params(precision=L.FP64, **kw):
    base = dict(gamma=(0.01, 0.01, 0.01), width=4.0, theta_deg=60.0, wetting=L.WET_GEOM_INTERP,
                precision=precision)
    base.update(kw)
    return L.make_params(L.D2Q9, (128, 64), **base)


# ------------------------------------------------------------ streaming ---
@pytest.mark.parametrize("lattice,n,walls", [(L.D2Q9, (13, 9), True), (L.D2Q9, (12, 10), False),
                                             (L.D3Q27, (9, 7, 6), True)])
def test_streaming_bit_exact(lattice, n, walls):
    """Collisions off: the step is streaming plus halfway bounce-back, a
    permutation; f is bit-identical to the oracle, g (whose initial value
    involves the stencil sums) equal to rounding."""
    D = 2 if lattice == L.D2Q9 else 3
    shape = (n[1], n[0]) if D == 2 else (n[2], n[1], n[0])
    rho0, phi0 = I.random_fields(shape, seed=3)
    p = L.make_params(lattice, n, walls=walls, lam=(0.07, 0.03, 0.03), kap=(0.03, 0.03, 0.03),
                      flags=L.NO_COLLIDE, theta_deg=90.0)
    sim, ora = run_both(p, rho0, phi0, 5)
    fg, gg = sim.pops()
    fo, go = ora.pops()
    sl = (slice(None), slice(1, -1)) if walls else (slice(None),)
    assert np.array_equal(fg[sl], fo[sl])
    assert np.abs(gg[sl] - go[sl]).max() < 1e-14


# ------------------------------------------------------ FP64 parity -------
def test_fp64_one_step_cfg1():
    rho0, phi0 = I.sessile_drop_2d(128, 64, 20, xc=64)
    sim, ora = run_both(cfg1_params(), rho0, phi0, 1)
    assert conc_err(sim, ora) <= 1e-12
    fg, gg = sim.pops()
    fo, go = ora.pops()
    assert np.abs(fg[:, 1:-1] - fo[:, 1:-1]).max() < 1e-13
    assert np.abs(gg[:, 1:-1] - go[:, 1:-1]).max() < 1e-13


def test_fp64_2000_steps_cfg1():
    """P1: config 1 (128x64, semicircular drop r = 20, gamma = 0.01, W = 4,
    geometric interpolation at 60 degrees), 2000 steps."""
    rho0, phi0 = I.sessile_drop_2d(128, 64, 20, xc=64)
    sim, ora = run_both(cfg1_params(), rho0, phi0, 2000, gpu_chunks=[1000, 1000])
    err = conc_err(sim, ora)
    say("cfg1 fp64 2000 steps max-abs C_k", err)
    assert err <= 1e-9
    og, oo = sim.observe(), ora.observe()
    for k in range(3):
        assert abs(og["mass"][k] - oo["mass"][k]) < 1e-9
    # entropic alpha statistics: same kinds, up to rare rounding-level flips
    for key in ("n_newton", "n_shortcut", "n_fallback", "n_fast"):
        assert abs(og[key] - oo[key]) <= max(2, 1e-5 * oo[key]), (key, og[key], oo[key])


@pytest.mark.parametrize("case", ["force", "extrap", "periodic", "ragged", "asym_random", "high_wall",
                                  "steep_random", "detect_ratio"])
def test_fp64_variants(case):
    """FP64 parity over 40 steps on the other code paths: force method with
    wall forces, geometric extrapolation, fully periodic, a ragged grid, three
    components with kappa2 != kappa3 on random fields, angles that differ per
    wall and interface, steep angles whose interpolation points lie beyond
    the LDS halo (read from the fields in memory), and a liquid-liquid
    drop with the detection threshold raised to 0.1."""
    steps = 40
    if case == "force":
        rho0, phi0 = I.sessile_drop_2d(64, 40, 12, xc=32)
        p = L.make_params(L.D2Q9, (64, 40), gamma=(0.01, 0.01, 0.01), width=4.0, wetting=L.WET_FORCE,
                          kw=((0.004, 0.002), (-0.003, 0.001)))
    elif case == "extrap":
        rho0, phi0 = I.sessile_drop_2d(64, 40, 12, xc=32)
        p = L.make_params(L.D2Q9, (64, 40), gamma=(0.01, 0.01, 0.01), width=4.0,
                          wetting=L.WET_GEOM_EXTRAP, theta_deg=70.0)
    elif case == "periodic":
        rho0, phi0 = I.bubble_2d(48, 40, 10, inside=(1, 0), outside=(0, 0))
        p = L.make_params(L.D2Q9, (48, 40), walls=False, gamma=(0.01, 0.01, 0.01), width=4.0)
    elif case == "ragged":
        rho0, phi0 = I.sessile_drop_2d(77, 23, 8, xc=30)
        p = L.make_params(L.D2Q9, (77, 23), gamma=(0.01, 0.01, 0.01), width=4.0, theta_deg=110.0)
    elif case == "steep_random":
        # contact angles with |cot| up to 2.9: interpolation points up to
        # three nodes along the wall, beyond the tile's LDS halo at its edges
        rho0, phi0 = I.random_fields((30, 70), seed=23)
        p = L.make_params(L.D2Q9, (70, 30), gamma=(0.01, 0.01, 0.01), width=4.0,
                          theta_deg=[[20, 160, 25], [155, 22, 158]])
    elif case == "detect_ratio":
        x, y = np.mgrid[0:40, 0:80][1].astype(float), np.mgrid[0:40, 0:80][0].astype(float)
        sh = I.profile(14.0 - np.sqrt((x - 40.0) ** 2 + (y - 0.5) ** 2), 4.0)
        rho0, phi0 = I.fields_from_conc(sh, 1.0 - sh)
        p = L.make_params(L.D2Q9, (80, 40), gamma=(0.01, 0.01, 0.01), width=4.0, theta_deg=(90.0, 90.0, 120.0),
                          detect_ratio=0.1)
    elif case == "asym_random":
        rho0, phi0 = I.random_fields((30, 50), seed=11)
        p = L.make_params(L.D2Q9, (50, 30), lam=(0.07, 0.04, 0.02), kap=(0.03, 0.05, 0.012),
                          theta_deg=[[50, 70, 100], [120, 80, 60]])
    else:
        rho0, phi0 = I.drop_train_2d(96, 40, n_drops=2, r=10, spacing=48, first=24, jitter=3, seed=5)
        p = L.make_params(L.D2Q9, (96, 40), gamma=(0.02, 0.015, 0.01), width=4.0,
                          theta_deg=[[45, 120, 90], [135, 60, 30]])
    sim, ora = run_both(p, rho0, phi0, steps)
    err = conc_err(sim, ora, walls=bool(p.walls))
    say(case, "max-abs C_k", err)
    assert err <= 1e-11


@pytest.mark.parametrize("wetting", [L.WET_GEOM_INTERP, L.WET_FORCE])
def test_fp64_d3q27(wetting):
    """D3Q27 sessile drop with 3D geometric interpolation (or the force
    method) on a ragged 3D grid."""
    nx, ny, nz = 37, 22, 18
    rho0, phi0 = I.sessile_drop_3d(nx, ny, nz, 7, center=(18.3, 10.7))
    p = L.make_params(L.D3Q27, (nx, ny, nz), gamma=(0.01, 0.01, 0.01), width=4.0, wetting=wetting,
                      theta_deg=65.0, kw=((0.003, 0.001), (0.0, 0.0)))
    sim, ora = run_both(p, rho0, phi0, 10)
    err = conc_err(sim, ora)
    say("d3q27", wetting, "max-abs C_k", err)
    assert err <= 1e-11


@pytest.mark.parametrize("prec,tol", [(L.FP64, 1e-13), (L.FP32, 2e-5), (L.FP16S, 2e-3)])
@pytest.mark.parametrize("wetting", [L.WET_GEOM_INTERP, L.WET_FORCE, "periodic"])
def test_two_kernel_3d_step_matches_fused(prec, tol, wetting):
    """D3Q27: the default step (stencil pass, then one thread per node for
    collision and streaming) against the one-kernel fused step
    (LBM3_FUSED_3D) on a ragged grid, 30 steps: the same arithmetic in
    another kernel shape; with walls (both schemes) and fully periodic
    (smooth random fields).  In FP64 the two-kernel result is also compared
    with the oracle (max-abs C_k <= 1e-11).  The stencil pass factors the
    isotropic stencils along the axes and the compiler may fuse different
    products into FMAs, so the two kernels agree to the growth of a few
    roundings per step over 30 steps, not bit for bit: in FP32 2e-5, about
    40 units in the last place of the largest field value (|phi| up to
    chi = 5; measured 1.0e-5)."""
    nx, ny, nz = 37, 22, 18
    walls = wetting != "periodic"
    if walls:
        rho0, phi0 = I.sessile_drop_3d(nx, ny, nz, 7, center=(18.3, 10.7))
    else:
        rho0, phi0 = I.random_fields((nz, ny, nx), seed=11)
    out = []
    for fl in (0, L.FUSED_3D):
        p = L.make_params(L.D3Q27, (nx, ny, nz), gamma=(0.01, 0.012, 0.009), width=4.0,
                          wetting=wetting if walls else L.WET_GEOM_INTERP, walls=walls,
                          theta_deg=65.0, kw=((0.003, 0.001), (0.0, 0.0)), precision=prec, flags=fl)
        say("two-kernel vs fused", "prec", prec, "wet", wetting, "flags", fl)
        s = L.Sim(p)
        s.init(rho0, phi0)
        s.step(30)
        out.append((s.fields(), s.pops(), s.observe()))
        if fl == 0 and prec == L.FP64:
            ora = O.Sim(oracle_params_from(p, s.derived))
            ora.init(rho0, phi0)
            ora.step(30)
            err = conc_err(s, ora, walls=walls)
            say("two-kernel vs oracle", err)
            assert err <= 1e-11
        s.close()
    (f2, p2, o2), (f1, p1, o1) = out
    d = max(float(np.abs(a - b).max()) for a, b in zip(f2, f1))
    sl = (slice(None), slice(1, -1)) if walls else (slice(None),)
    dp = max(float(np.abs(a[sl] - b[sl]).max()) for a, b in zip(p2, p1))
    say("max |fields| diff", d, "max |pops| diff", dp)
    assert d <= tol and dp <= tol
    assert o2["n_bad"] == 0 and o1["n_bad"] == 0


def test_force_kw0_equals_geometric90_gpu():
    """Neutral wetting: force method without wall force and geometric
    interpolation at 90 degrees are the same ghost copy, bit for bit."""
    rho0, phi0 = I.sessile_drop_2d(64, 32, 12, xc=32)
    out = []
    for wet in (L.WET_FORCE, L.WET_GEOM_INTERP):
        p = L.make_params(L.D2Q9, (64, 32), gamma=(0.01, 0.01, 0.01), width=4.0, wetting=wet,
                          theta_deg=90.0)
        say("neutral", wet)
        s = L.Sim(p)
        s.init(rho0, phi0)
        s.step(30)
        out.append(s.pops())
    fl = (slice(None), slice(1, -1))
    assert np.array_equal(out[0][0][fl], out[1][0][fl]) and np.array_equal(out[0][1][fl], out[1][1][fl])


# ------------------------------------------------------ precision forms ---
@pytest.mark.parametrize("prec,tol", [(L.FP32, 1e-4), (L.FP16S, 2e-3)])
def test_reduced_precision_2000_steps_cfg1(prec, tol):
    """P2: FP32 arithmetic (FP32 or FP16-offset population storage) against
    the FP64 oracle after 2000 steps of config 1, at the stated tolerances
    (max-abs C_k <= 1e-4 FP32, <= 2e-3 FP16 storage; contact angle within 1
    degree).  Measured: FP32 5.7e-5, FP16 storage 3.4e-4, largest at the
    contact line in the first fluid layer."""
    rho0, phi0 = I.sessile_drop_2d(128, 64, 20, xc=64)
    sim, ora = run_both(cfg1_params(precision=prec), rho0, phi0, 2000)
    err = conc_err(sim, ora)
    say("cfg1 prec", prec, "max-abs C_k", err)
    assert err <= tol
    # P2: the contact angle of the reduced-precision run within 1 degree of
    # the oracle's (same circle fit on both, C2 = 1/2 contour, 2W excluded)
    d = sim.derived
    rg, pg = sim.fields()
    ro, po = ora.fields()
    ag = O.contact_angle_2d(conc(rg, pg, d.rho_l, d.rho_g)[1], exclude=8.0)[0]
    ao = O.contact_angle_2d(conc(ro, po, d.rho_l, d.rho_g)[1], exclude=8.0)[0]
    say("cfg1 prec", prec, "contact angle", ag, "oracle", ao)
    assert abs(ag - ao) < 1.0


def test_mass_conservation_gpu_fp64():
    """Collision and bounce-back conserve sum rho and sum phi, hence the
    component masses (affine in both): relative drift <= 1e-12 over 2000 steps
    (the rounding of the update itself drifts ~1e-13)."""
    rho0, phi0 = I.sessile_drop_2d(128, 64, 20, xc=64)
    p = cfg1_params()
    say("mass fp64")
    s = L.Sim(p)
    s.init(rho0, phi0)
    o0 = s.observe()
    s.step(2000)
    o = s.observe()
    d = s.derived
    assert abs(o["rho_sum"] - o0["rho_sum"]) <= 1e-12 * o0["rho_sum"]
    assert abs(o["phi_sum"] - o0["phi_sum"]) <= 1e-12 * abs(o0["phi_sum"])
    scale = o0["rho_sum"] / (d.rho_l - d.rho_g) + abs(o0["phi_sum"]) / 5.0
    for k in range(3):
        assert abs(o["mass"][k] - o0["mass"][k]) <= 1e-12 * max(abs(o0["mass"][k]), scale)
    assert o["n_bad"] == 0


def test_contact_angle_fit_matches_numpy():
    """The FP64 on-device contour + circle fit equals the oracle-side numpy fit
    of the same field."""
    rho0, phi0 = I.cap_drop_2d(160, 80, 30, 70.0, xc=80.3)
    p = cfg1_params()
    p.n[0], p.n[1] = 160, 80
    say("contact angle")
    s = L.Sim(p)
    s.init(rho0, phi0)
    out = s.contact_angle(comp=2, wall=0, exclude=8.0)
    r, ph = s.fields()
    d = s.derived
    C2 = conc(r, ph, d.rho_l, d.rho_g)[1]
    th, (xc, yc, R) = O.contact_angle_2d(C2[1:-1], wall_y=-0.5, exclude=8.0)
    assert abs(out[0] - th) < 1e-8
    assert abs(out[4] - R) < 1e-8
    assert abs(out[0] - 70.0) < 0.5


# ------------------------------------------------------ full-size configs -
def test_cfg2_full_size_fp32_and_fp64():
    """Config 2 at its full size (2048 x 64 capillary channel, liquid-2 slug
    x < 256, liquid-3 films of 3 rows, 60 degrees), in the launch
    configuration the benchmark times: 30 steps, FP64 to 1e-11 and FP32 to
    1e-4 against the oracle."""
    rho0, phi0 = I.capillary_2d(2048, 64, 256, film=3)
    for prec, tol in ((L.FP64, 1e-11), (L.FP32, 1e-4)):
        p = L.make_params(L.D2Q9, (2048, 64), gamma=(0.01, 0.01, 0.01), width=4.0, theta_deg=60.0,
                          precision=prec)
        sim, ora = run_both(p, rho0, phi0, 30)
        err = conc_err(sim, ora)
        say("cfg2 prec", prec, "err", err)
        assert err <= tol


def test_cfg3_analogue_64cube():
    """Config 3 at 64^3 (lubricated sessile drop on a liquid-3 film, gamma12 =
    gamma13 = 0.02, gamma23 = 0.01): FP32 and FP16-offset storage against the
    oracle after 20 steps."""
    n = 64
    rho0, phi0 = I.lubricated_drop_3d(n, n, n, 12, film=2)
    for prec, tol in ((L.FP32, 1e-5), (L.FP16S, 5e-4)):
        p = L.make_params(L.D3Q27, (n, n, n), gamma=(0.02, 0.02, 0.01), width=4.0, theta_deg=90.0,
                          precision=prec)
        sim, ora = run_both(p, rho0, phi0, 20)
        err = conc_err(sim, ora)
        say("cfg3@64 prec", prec, "err", err)
        assert err <= tol


def test_cfg4_full_size_fp32_one_step():
    """Config 4 at full size (4096 x 256 train of 16 alternating drops, walls
    at 45 / 120 degrees): one FP32 step against the oracle."""
    rho0, phi0 = I.drop_train_2d(4096, 256, n_drops=16, r=40, spacing=200, first=100, jitter=10, seed=0)
    p = L.make_params(L.D2Q9, (4096, 256), gamma=(0.01, 0.01, 0.01), width=4.0,
                      theta_deg=[45.0, 120.0, 90.0], precision=L.FP32)
    sim, ora = run_both(p, rho0, phi0, 1)
    err = conc_err(sim, ora)
    say("cfg4 err", err)
    assert err <= 1e-5


def test_fp64_small_tiles_multi_plane_chunks():
    """A small-tile 2D grid large enough for multi-plane chunks (1024 x 600:
    17 x 598 tile planes, two planes per block, the six planes next to each
    wall one per block) with drops on both walls: FP64 after 12 steps
    against the oracle."""
    nx, ny = 1024, 600
    r1, p1 = I.sessile_drop_2d(nx, ny, 60, xc=300.0)
    # a second drop hanging from the top wall (mirrored rows)
    r2, p2 = I.sessile_drop_2d(nx, ny, 45, xc=700.0, comp=3)
    rho0 = np.where(np.abs(r1 - r1[0, 0]) > 1e-12, r1, r2[::-1])
    phi0 = np.where(np.abs(r1 - r1[0, 0]) > 1e-12, p1, p2[::-1])
    p = L.make_params(L.D2Q9, (nx, ny), gamma=(0.01, 0.012, 0.009), width=4.0,
                      theta_deg=[[60.0, 60.0, 60.0], [120.0, 120.0, 120.0]], precision=L.FP64)
    sim, ora = run_both(p, rho0, phi0, 12)
    err = conc_err(sim, ora)
    say("1024x600 fp64 err", err)
    assert err <= 1e-11


def test_cfg3_full_size_properties():
    """Config 3 at full size (256^3, FP32 and FP16 storage): 20 steps stay
    finite, conserve the component masses to FP32 summation accuracy."""
    n = 256
    rho0, phi0 = I.lubricated_drop_3d(n, n, n, 48, film=8)
    for prec, tol in ((L.FP32, 1e-5), (L.FP16S, 2e-3)):
        p = L.make_params(L.D3Q27, (n, n, n), gamma=(0.02, 0.02, 0.01), width=4.0, theta_deg=90.0,
                          precision=prec)
        say("cfg3 full size prec", prec)
        s = L.Sim(p)
        s.init(rho0, phi0)
        o0 = s.observe()
        s.step(20)
        o = s.observe()
        assert o["n_bad"] == 0
        nF = n * n * (n - 2)
        for k in range(3):
            assert abs(o["mass"][k] - o0["mass"][k]) <= tol * max(abs(o0["mass"][k]), 1e-3 * nF)
        del s


@pytest.mark.parametrize("D", [2, 3])
@pytest.mark.parametrize("lam", [2.0, 2.5])
def test_too_fast_count_matches_oracle(D, lam):
    """|u + du| >= 1 collisions (the observables' n_fast, and LBM3_EUNSTABLE
    from observe) counted as the oracle counts them: a sharp flat liquid-gas
    interface, 1 and 3 steps, FP64; in 3D through the two-kernel step (a
    quasi-2D slab, 4 planes)."""
    nx, ny = 32, 16
    rho0, phi0 = I.flat_interface_2d(nx, ny, left=(0, 0), right=(1, 0), W=2.0)
    n = (nx, ny) if D == 2 else (nx, ny, 4)
    if D == 3:
        rho0, phi0 = np.repeat(rho0[None], 4, axis=0), np.repeat(phi0[None], 4, axis=0)
    p = L.make_params(L.D2Q9 if D == 2 else L.D3Q27, n, walls=False, rho_l=1.0, rho_g=1e-3,
                      lam=(lam, lam, lam), kap=(0.03, 0.03, 0.03), precision=L.FP64)
    s = L.Sim(p)
    s.init(rho0, phi0)
    ora = O.Sim(oracle_params_from(p, s.derived))
    ora.init(rho0, phi0)
    for k in (1, 2):
        s.step(k)
        ora.step(k)
        g, o = s.observe(), ora.observe()
        say("too fast", D, lam, "gpu", g["n_fast"], "oracle", o["n_fast"], "status", g["status"])
        assert g["n_fast"] == o["n_fast"] and g["n_bad"] == o["n_bad"]
        if g["n_bad"] == 0:
            assert (g["status"] == -3) == (g["n_fast"] > 0)
    s.close()
