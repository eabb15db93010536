"""Self-propelled bi-slug (Sec. VI A) on the GPU path, FP64, in the paper's
geometry: a channel of height H = 39 between walls, periodic along x,
holding a train of two liquid slugs of equal length (liquid 2, then liquid
3; L = L1 + L2) with 200 lattice units of gas on each side, and the same
contact angle theta = theta21 = theta31 = theta23 on every interface
(geometric interpolation).  With gamma12 = gamma13 the surface tension
unbalance of Eq. 54 is Delta gamma = gamma23 cos theta, the
drive 2 Delta gamma; a Poiseuille slug of viscosity nu then moves at
v_inf = H Delta gamma / (6 rho_l nu L) after a relaxation time
tau = H^2 / (12 nu) (Eqs. 60-62).

The paper finds the closed form in the limit of long trains and, for
finite trains, explains the extra dissipation by the dynamic contact
angles: with Delta gamma evaluated from the angles measured by circle fits
on the moving train, the closed form matches the measured speeds.  These
tests check, at L = 1500:
  * GPU parity with the oracle over the first 2000 steps (FP64, 1e-9);
  * the measured steady speed against the closed form with the measured
    dynamic angles (the paper's corrected model);
  * the closed form with the static angles, and the relaxation time, as
    the long-train limit (kept as an expected failure where measured off).
"""
import math

import numpy as np
import pytest
from scipy.optimize import curve_fit

from _common import conc, conc_err, oracle_params_from, say
from oracle import oracle as O
from paper_1904_06881_amd import inputs as I
from paper_1904_06881_amd import lbm3 as L

pytestmark = pytest.mark.gpu

H = 39
NY = H + 2                    # two wall (ghost) rows
GAS = 200
G = (0.01, 0.01, 0.01)
W = 4.0
Y_WALL = 0.5                  # bottom wall plane (full-grid coordinates)


def geometry(Ltot):
    L1 = Ltot // 2
    nx = Ltot + 2 * GAS
    return L1, nx


def bislug_fields(Ltot):
    L1, nx = geometry(Ltot)
    x = np.arange(nx, dtype=float)[None, :].repeat(NY, 0)
    d2 = np.minimum(x - GAS, GAS + L1 - x)
    d3 = np.minimum(x - (GAS + L1), GAS + 2 * L1 - x)
    return I.fields_from_conc(I.profile(d2, W), I.profile(d3, W))


def params(Ltot, theta, prec=L.FP64):
    _, nx = geometry(Ltot)
    return L.make_params(L.D2Q9, (nx, NY), gamma=G, width=W, wetting=L.WET_GEOM_INTERP,
                         theta_deg=theta, precision=prec)


def wall_angle(xs, ys, side):
    """Contact angle at the bottom wall of a channel-spanning interface, from
    the Kasa circle through its points: measured in the phase lying on
    `side` (+1: larger x) of the interface, between the wall (pointing into
    that phase) and the interface tangent pointing into the channel."""
    xc, yc, R = O.kasa_fit(xs, ys)
    dy = Y_WALL - yc
    xi = xc + math.copysign(math.sqrt(max(R * R - dy * dy, 0.0)), np.mean(xs) - xc)
    nx_, ny_ = (xi - xc) / R, dy / R
    tx, ty = -ny_, nx_
    if ty < 0:
        tx, ty = -tx, -ty
    return math.degrees(math.acos(max(-1.0, min(1.0, side * tx))))


def dynamic_angles(rho, phi, d, x_front):
    """theta21, theta23, theta31 of the train from circle fits to the C1 = 1/2
    (menisci) and C2 = 1/2 (liquid-liquid) contours in windows around each
    interface, points within 6 of the walls left out."""
    C1, C2, C3 = conc(rho, phi, d.rho_l, d.rho_g)
    out = {}
    for name, field, xwin, side in (("21", C1, x_front[0], +1), ("23", C2, x_front[1], -1),
                                    ("31", C1, x_front[2], -1)):
        xs, ys = O.contour_points_2d(field[1:-1], y_offset=1.0)
        keep = (np.abs(xs - xwin) < 30) & (ys > Y_WALL + 6) & (ys < Y_WALL + H - 6)
        out[name] = wall_angle(xs[keep], ys[keep], side)
    return out


def centre_and_fronts(rho, phi, d):
    C1, C2, C3 = conc(rho, phi, d.rho_l, d.rho_g)
    x = np.arange(rho.shape[1], dtype=float)[None, :]
    w = (C2 + C3)[1:-1]
    xm = float((w * x).sum() / w.sum())
    mid = H // 2 + 1
    liq = C2[mid] + C3[mid]
    idx = np.where(liq > 0.5)[0]
    left, right = float(idx.min()), float(idx.max())
    # liquid-liquid interface: C2 - C3 changes sign along the centre row
    s = np.where(np.diff(np.sign(C2[mid] - C3[mid])) != 0)[0]
    s = s[(s > left) & (s < right)]
    return xm, (left, float(s[0]) if len(s) else 0.5 * (left + right), right)


def test_bislug_oracle_parity_2000_steps():
    """The paper's geometry (H = 39, L = 1500, theta = 60 degrees): GPU FP64
    against the oracle after 2000 steps, max-abs C_k <= 1e-9."""
    p = params(1500, 60.0)
    init = bislug_fields(1500)
    s = L.Sim(p)
    s.init(*init)
    say("bislug parity", list(p.n))
    s.step(2000)
    ora = O.Sim(oracle_params_from(p, s.derived))
    ora.init(*init)
    ora.step(2000)
    err = conc_err(s, ora)
    say("bislug 2000 steps max-abs C_k", err)
    s.close()
    assert err <= 1e-9


def run_train(Ltot, theta, steps, every):
    p = params(Ltot, theta)
    s = L.Sim(p)
    s.init(*bislug_fields(Ltot))
    d = s.derived
    ts, xs = [], []
    for k in range(steps // every + 1):
        if k:
            s.step(every)
        r, ph = s.fields()
        xs.append(centre_and_fronts(r, ph, d)[0])
        ts.append(k * every)
    r, ph = s.fields()
    obs = s.observe()
    s.close()
    assert obs["n_bad"] == 0
    return np.array(ts, float), np.array(xs), r, ph, d


def steady(ts, xs, tail=0.4):
    m = ts >= ts[-1] * (1 - tail)
    return float(np.polyfit(ts[m], xs[m], 1)[0])


NU = (1.0 - 0.5) / 3.0  # tau_f = 1


@pytest.mark.parametrize("theta", [50.0, 70.0])
def test_bislug_speed_follows_the_dynamic_angle_model(theta):
    """L = 1500, 24000 steps: the steady speed of the centre of mass (fitted
    over the last 40 % of the run) against H Delta gamma_dyn / (6 rho_l nu L)
    with Delta gamma_dyn from the dynamic angles measured by circle fits on
    the moving train (the corrected model of Sec. VI A).  Measured: speed /
    model 0.86 (50 degrees) and 0.85 (70 degrees), against 0.40 and 0.46
    for the static-angle closed form; the liquid-liquid contact angle moves
    most (50 -> 73 and 70 -> 80 degrees), the menisci by under 1 degree.
    Asserted: within 20 % of the dynamic-angle model, and at least twice as
    close to it as to the static closed form."""
    ts, xs, r, ph, d = run_train(1500, theta, 24000, 400)
    v = steady(ts, xs)
    xm, fronts = centre_and_fronts(r, ph, d)
    ang = dynamic_angles(r, ph, d, fronts)
    c = {k: math.cos(math.radians(a)) for k, a in ang.items()}
    dg_dyn = G[2] * c["23"] - G[1] * c["31"] + G[0] * c["21"]
    v_dyn = H * dg_dyn / (6.0 * d.rho_l * NU * 1500)
    v_static = H * G[2] * math.cos(math.radians(theta)) / (6.0 * d.rho_l * NU * 1500)
    say("theta", theta, "steady v %.4e" % v, "dynamic angles", ang, "model %.4e" % v_dyn,
        "static closed form %.4e" % v_static)
    assert v > 0
    assert abs(v / v_dyn - 1.0) < 0.20
    assert abs(v / v_dyn - 1.0) < 0.5 * abs(v / v_static - 1.0)


@pytest.mark.xfail(reason="finite trains dissipate at the contact lines as well: the speed at L = 1500 "
                          "is below the static-angle closed form, which holds only for L >> H", strict=False)
def test_bislug_closed_form_static_angles():
    """The closed form with the static angles (theta = 60 degrees, L = 1500):
    centre-of-mass trajectory fitted with Eq. 62 after the
    first 1000 steps, v within 10 % of v_inf and tau within 50 % of
    H^2 / (12 nu)."""
    ts, xs, r, ph, d = run_train(1500, 60.0, 24000, 200)
    v_pred = H * G[2] * math.cos(math.radians(60.0)) / (6.0 * d.rho_l * NU * 1500)
    tau_pred = H * H / (12.0 * NU)
    m = ts >= 1000

    def model(t, x0, v, tau):
        return x0 + tau * v * (np.exp(-t / tau) + t / tau - 1.0)

    (x0, v_fit, tau_fit), _ = curve_fit(model, ts[m], xs[m], p0=(xs[0], v_pred, tau_pred))
    say("static closed form: v fit %.4e pred %.4e  tau fit %.1f pred %.1f" % (v_fit, v_pred, tau_fit, tau_pred))
    assert abs(v_fit / v_pred - 1.0) < 0.10
    assert abs(tau_fit / tau_pred - 1.0) < 0.5
