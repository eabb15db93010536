"""Self-propelled bi-slug (Sec. V) on the GPU path, FP64.

A train of two liquid slugs (liquid 2 then liquid 3, equal lengths) fills
the height H = 39 of a channel that is periodic along x, with gas on both
sides.  Unequal wall tensions drive it: the capillary force is 2 Delta gamma
with Delta gamma = gamma_23 cos theta_23 - gamma_13 cos theta_31 +
gamma_12 cos theta_21 (Eqs. for the capillary force and drive), the
viscous friction of a Poiseuille profile is 12 rho_l nu L xdot / H, and the
centre of mass follows x(t) = x0 + tau v (exp(-t/tau) + t/tau - 1) with
v = H Delta gamma / (6 rho_l nu L) and tau = H^2 / (12 nu) (Sec. V).

Here the drive comes from the liquid-liquid contact lines (theta_23 = 60
degrees, theta_21 = theta_31 = 90 degrees, geometric interpolation), whose
angles this build reproduces; the liquid-gas menisci stay flat.  The centre
of mass of the two liquids is sampled every 400 steps and fitted with the
closed form, v and tau free.

Expected failure, kept to track it: the train moves at about a quarter of
the closed-form velocity (v 2.0e-4 against 8.1e-4 l.u. per step, relaxation
time 3700 against 760 steps).  The steady velocities of this train and of
one five times longer (1.8e-4 and 9.0e-5 against 8.1e-4 and 1.6e-4) both fit
2 Delta gamma = v (12 rho_l nu L / H + zeta) with zeta of about 45 and 50:
a friction independent of the length, i.e. dissipation at the four contact
lines, which the closed form leaves out; it fades only for trains much
longer than H.
"""
import sys

import numpy as np
import pytest
from scipy.optimize import curve_fit

from oracle import oracle as O
from paper_1904_06881_amd import inputs as I
from paper_1904_06881_amd import lbm3 as L

pytestmark = pytest.mark.gpu

H = 39
NX, NY = 640, H + 2           # two wall (ghost) rows
L1 = 120                      # each slug; 200 l.u. of gas on each side
X0 = 200
G = (0.01, 0.01, 0.01)


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def bislug_fields():
    x = np.arange(NX, dtype=float)[None, :].repeat(NY, 0)
    d2 = np.minimum(x - X0, X0 + L1 - x)
    d3 = np.minimum(x - (X0 + L1), X0 + 2 * L1 - x)
    C2 = I.profile(d2, 4.0)
    C3 = I.profile(d3, 4.0)
    return I.fields_from_conc(C2, C3)


@pytest.mark.xfail(reason="v is 0.25 of the closed form: the contact lines add a friction of about "
                          "45 that the closed form (bulk dissipation only) leaves out", strict=False)
def test_bislug_centre_of_mass_follows_the_closed_form():
    p = L.make_params(L.D2Q9, (NX, NY), gamma=G, width=4.0, wetting=L.WET_GEOM_INTERP,
                      theta_deg=(90.0, 90.0, 60.0), precision=L.FP64)
    s = L.Sim(p)
    s.init(*bislug_fields())
    d = s.derived
    eos = {k: getattr(d, k) for k in ("a", "b", "T", "C", "psi0", "rho_l", "rho_g")}
    po = O.make_params(2, (NX, NY), lam=list(d.lam), kap=list(d.kap), eos=eos, rho_l=d.rho_l,
                       rho_g=d.rho_g, theta_deg=(90.0, 90.0, 60.0))
    x = np.arange(NX, dtype=float)[None, :]
    ts, xs = [], []
    every, n = 400, 40
    for k in range(n + 1):
        if k:
            s.step(every)
        r, ph = s.fields()
        _, C2, C3 = O.concentrations(po, r, ph)
        w = (C2 + C3)[1:-1]
        ts.append(k * every)
        xs.append(float((w * x).sum() / w.sum()))
    obs = s.observe()
    s.close()
    assert obs["n_bad"] == 0
    ts, xs = np.array(ts, float), np.array(xs)
    nu = (p.tau_f - 0.5) / 3.0
    L_len = 2 * L1
    dgam = G[2] * np.cos(np.radians(60.0)) - G[1] * np.cos(np.radians(90.0)) + \
        G[0] * np.cos(np.radians(90.0))
    v_pred = H * dgam / (6.0 * d.rho_l * nu * L_len)
    tau_pred = H * H / (12.0 * nu)

    def model(t, v, tau):
        return xs[0] + tau * v * (np.exp(-t / tau) + t / tau - 1.0)

    (v_fit, tau_fit), _ = curve_fit(model, ts, xs, p0=(np.sign(xs[-1] - xs[0]) * v_pred, tau_pred))
    say("displacement %.3f l.u. in %d steps" % (xs[-1] - xs[0], ts[-1]))
    say("v fit %.4e  closed form %.4e  (ratio %.3f)" % (v_fit, v_pred, abs(v_fit) / v_pred))
    say("tau fit %.1f  closed form %.1f" % (tau_fit, tau_pred))
    assert abs(abs(v_fit) / v_pred - 1.0) < 0.25
    assert abs(tau_fit / tau_pred - 1.0) < 0.5
