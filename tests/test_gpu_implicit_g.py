"""The implicit-g step of D3Q27 at tau_g = 1 (FP32, FP64): the collision
keeps the five values (a, phi, v) that fix g^eq at each node (Eqs. 33-35:
at tau_g = 1 the post-collision g is g^eq) instead of pushing 27 g
populations, and the next moments pass rebuilds the g that streaming and
bounce-back deliver from them.  It evaluates the same expressions on the same
inputs in the same order, so every field, population and observable must be
bit-identical to the stored-g step (LBM3_STORED_G), on walled grids (both
wetting schemes, distinct angles per wall and interface), fully periodic
grids, tiles that overhang the grid, grids narrower than a tile, a single
fluid plane, and across every switch between the two forms of g: exports and
observables (which write g out), batched steps (which rebuild it per
simulation) and single steps."""
import sys

import numpy as np
import pytest

from _common import conc
from paper_1904_06881_amd import inputs as I
from paper_1904_06881_amd import lbm3 as L

pytestmark = pytest.mark.gpu
G = (0.01, 0.012, 0.009)
ANG = [[50.0, 70.0, 100.0], [120.0, 80.0, 60.0]]


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def case(kind, prec, flags=0):
    if kind == "walled":
        n = (37, 22, 18)
        p = L.make_params(L.D3Q27, n, gamma=G, theta_deg=ANG, precision=prec, flags=flags)
        return p, I.sessile_drop_3d(*n, 7, center=(18.3, 10.7))
    if kind == "extrap":
        n = (70, 9, 12)
        p = L.make_params(L.D3Q27, n, gamma=G, theta_deg=ANG, wetting=L.WET_GEOM_EXTRAP, precision=prec,
                          flags=flags)
        return p, I.sessile_drop_3d(*n, 5, center=(30.0, 4.5))
    if kind == "force":
        n = (33, 17, 14)
        p = L.make_params(L.D3Q27, n, gamma=G, wetting=L.WET_FORCE, kw=((0.003, 0.001), (0.0, -0.002)),
                          precision=prec, flags=flags)
        return p, I.sessile_drop_3d(*n, 6)
    if kind == "periodic":
        n = (20, 13, 11)
        p = L.make_params(L.D3Q27, n, gamma=G, walls=False, precision=prec, flags=flags)
        return p, I.random_fields((n[2], n[1], n[0]), seed=5)
    if kind == "tiny":
        n = (5, 3, 4)
        p = L.make_params(L.D3Q27, n, gamma=G, walls=False, precision=prec, flags=flags)
        return p, I.random_fields((n[2], n[1], n[0]), seed=6)
    if kind == "one_plane":
        n = (24, 10, 3)
        p = L.make_params(L.D3Q27, n, gamma=G, theta_deg=ANG, precision=prec, flags=flags)
        return p, I.random_fields((n[2], n[1], n[0]), seed=7)
    raise ValueError(kind)


def run(kind, prec, flags, plan):
    """plan: list of ("step", k), ("batch", k), ("pops",), ("obs",), ("angle",)."""
    p, init = case(kind, prec, flags)
    s = L.Sim(p)
    s.init(*init)
    other = L.Sim(case("periodic", L.FP32)[0])
    other.init(*case("periodic", L.FP32)[1])
    out = []
    for item in plan:
        if item[0] == "step":
            s.step(item[1])
        elif item[0] == "batch":
            keep = L.step_batch([other, s], item[1])
            del keep
        elif item[0] == "pops":
            out.extend(s.pops())
        elif item[0] == "obs":
            o = s.observe()
            out.append(np.array([o[k] for k in ("n_bad", "n_newton", "n_shortcut", "n_fallback")]))
        elif item[0] == "angle":
            out.append(np.asarray(s.contact_angle(2, 0, 4.0), dtype=np.float64))
    out.extend(s.fields())
    out.extend(s.pops())
    s.close()
    other.close()
    return out


PLAN = [("step", 7), ("obs",), ("step", 3)]
MIXED = [("step", 4), ("batch", 3), ("step", 2), ("pops",), ("step", 1), ("batch", 2), ("obs",), ("batch", 1),
         ("step", 3)]


@pytest.mark.parametrize("prec", [L.FP32, L.FP64])
@pytest.mark.parametrize("kind", ["walled", "extrap", "force", "periodic", "tiny", "one_plane"])
def test_implicit_g_bit_identical_to_stored_g(kind, prec):
    say("implicit vs stored g", kind, prec)
    a = run(kind, prec, 0, PLAN)
    b = run(kind, prec, L.STORED_G, PLAN)
    for k, (x, y) in enumerate(zip(a, b)):
        assert np.array_equal(x, y), (kind, prec, k, float(np.nanmax(np.abs(x - y))))
    assert np.isfinite(a[-1]).all()


@pytest.mark.parametrize("prec", [L.FP32, L.FP64])
@pytest.mark.parametrize("kind", ["walled", "periodic"])
def test_implicit_g_across_batched_steps_and_exports(kind, prec):
    say("implicit g, mixed single / batched steps and exports", kind, prec)
    a = run(kind, prec, 0, MIXED)
    b = run(kind, prec, L.STORED_G, MIXED)
    c = run(kind, prec, 0, [("step", 16)])
    for k, (x, y) in enumerate(zip(a, b)):
        assert np.array_equal(x, y), (kind, prec, k)
    # the mixed sequence is 16 steps in all: its final state equals 16 single steps
    for x, y in zip(a[-4:], c[-4:]):
        assert np.array_equal(x, y)


def test_implicit_g_angle_and_footprint():
    p, init = case("walled", L.FP32)
    ps, _ = case("walled", L.FP32, L.STORED_G)
    n = 37 * 22 * 18
    # one g set (both parities share it) plus five FP32 values per node,
    # against two g sets: 27 * 4 - 5 * 4 bytes per node less, to alignment
    saved = L.lbm3_footprint(ps) - L.lbm3_footprint(p)
    assert abs(saved - (27 - 5) * 4 * n) <= 512, saved
    a = run("walled", L.FP32, 0, [("step", 20), ("angle",)])
    b = run("walled", L.FP32, L.STORED_G, [("step", 20), ("angle",)])
    assert np.array_equal(a[0], b[0]) and np.isfinite(a[0]).all()


@pytest.mark.parametrize("kind", ["walled", "periodic"])
def test_implicit_g_fp16_storage(kind):
    """FP16 population storage with implicit g: f stored as FP16 offsets, g
    rebuilt from the five FP32 values (so never rounded to FP16).  Against
    the stored-g FP16 form and the FP64 run after 60 steps: both FP16 forms
    within the FP16-storage bound (2e-3 max-abs C_k) of FP64, and the
    implicit one no farther from it than the stored one plus 1e-4."""
    p64, init = case(kind, L.FP64)
    runs = {}
    for name, prec, flags in (("fp64", L.FP64, 0), ("imp", L.FP16S, 0), ("stored", L.FP16S, L.STORED_G)):
        p, _ = case(kind, prec, flags)
        s = L.Sim(p)
        s.init(*init)
        s.step(60)
        d = s.derived
        runs[name] = conc(*s.fields(), d.rho_l, d.rho_g)
        assert s.observe()["n_bad"] == 0
        s.close()
    e_imp = float(np.abs(runs["imp"] - runs["fp64"]).max())
    e_sto = float(np.abs(runs["stored"] - runs["fp64"]).max())
    say("fp16 storage", kind, "implicit g", e_imp, "stored g", e_sto)
    assert e_imp <= 2e-3 and e_sto <= 2e-3
    assert e_imp <= e_sto + 1e-4


def test_reinit_after_implicit_steps():
    """Initialising a handle again after implicit-g steps starts from the
    stored g of the new initial state (the same run as a fresh handle)."""
    p, init = case("walled", L.FP32)
    s = L.Sim(p)
    s.init(*init)
    s.step(9)
    s.init(*init)
    s.step(5)
    a = s.fields() + s.pops()
    s.close()
    t = L.Sim(p)
    t.init(*init)
    t.step(5)
    b = t.fields() + t.pops()
    t.close()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
