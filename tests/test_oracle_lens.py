"""A liquid-2 lens floating on a liquid-3 layer in gas, on the oracle (the
three-phase contact whose Neumann angles Eqs. 40-42 give from the tensions,
Sec. III).  Table 1's set 3 at the paper's Carnahan-Starling constants
(lambda = kappa = (0.01, 1.5, 1.5), density ratio 1000): R = 20 drop on the
upper edge of a 70-row layer in a 160 x 160 periodic box, FP64, 10000 steps
(the lens oscillates by a few degrees up to about 8000).  The angles come from circle fits to the
C2 = 1/2 arcs above and below the layer's C3 = 1/2 line
(oracle.lens_angles_2d, itself pinned on drawn lenses of known angles).

* The lens is a mirror image: its two contact points agree within 0.5
  degrees, and theta2 = theta3 within 2 degrees (gamma12 = gamma13 in set
  3, so the Neumann triangle is isosceles; the difference is a size effect:
  4.5 degrees at R = 14, 1.0-1.5 at R = 20, 0.2-0.4 at R = 32).
* The angles sum to 360 degrees.
* Against the Neumann angles of Table 1's printed tensions (86.5 / 136.7 /
  136.7 degrees): expected failure.  The lens settles at 104.4 / 128.4 /
  127.2 degrees (also with R = 32 in a 256 x 256 box: 104.4 / 128.0 /
  127.6), which by the law of sines corresponds to liquid-gas tensions
  about 0.39 against gamma23 = 0.48, 12 % above what the bubble test gives
  on the same model (0.349) and 17 % above the printed 0.333: the excess
  liquid-gas tension of the link-pressure ideal force is larger at the
  contact line than on a curved interface."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1904_06881_amd import inputs as I

NX = NY = 160
R = 20.0


def drawn_lens(t1, t2, a=30.0, n=200, yf=110.0, y0=30.0, W=4.0):
    """Concentration fields of a lens with contact angles t1 (gas), t2
    (liquid 2) at half-width a: two circular arcs through the contact points
    with the given tangents, the layer's edge at yf."""
    y, x = np.mgrid[0:n, 0:n].astype(float)
    X, Y = x - n / 2.0, y - yf
    ca = a / math.tan(math.radians(t1))
    cb = a / math.tan(math.radians(t1 + t2))
    d = np.where(Y >= 0, math.hypot(a, ca) - np.hypot(X, Y - ca), math.hypot(a, cb) - np.hypot(X, Y - cb))
    C2 = I.profile(d, W)
    C3 = I.profile(np.minimum(y - y0, yf - y), W) * (1 - C2)
    return C2, C3


@pytest.mark.parametrize("t1,t2", [(86.5, 136.7), (104.4, 128.4), (151.0, 104.5), (120.0, 100.0)])
def test_lens_angle_measurement_on_drawn_lenses(t1, t2):
    C2, C3 = drawn_lens(t1, t2)
    m, per, yf = O.lens_angles_2d(C2, C3, 100.0)
    assert abs(yf - 110.0) < 0.05
    for got, want in zip(m, (t1, t2, 360.0 - t1 - t2)):
        assert abs(got - want) < 0.1, (m, t1, t2)


_lens = {}


def set3_lens():
    if not _lens:
        eos = O.coexistence(1000.0, 9.227761)
        po = O.make_params(2, (NX, NY), lam=(0.01, 1.5, 1.5), kap=(0.01, 1.5, 1.5), eos=eos,
                           rho_l=eos["rho_l"], rho_g=eos["rho_g"], walls=False)
        s = O.Sim(po)
        s.init(*I.lens_2d(NX, NY, R, band=(20.0, 90.0), rho_l=eos["rho_l"], rho_g=eos["rho_g"]))
        s.step(10000)
        r, ph = s.fields()
        assert np.isfinite(r).all()
        C1, C2, C3 = O.concentrations(po, r, ph)
        _lens["m"], _lens["per"], _ = O.lens_angles_2d(C2, C3, NX / 2.0)
    return _lens["m"], _lens["per"]


def test_lens_is_symmetric_and_closes():
    m, per = set3_lens()
    assert abs(sum(m) - 360.0) < 1e-6
    for k in range(3):
        assert abs(per[0][k] - per[1][k]) < 0.5, per
    assert abs(m[1] - m[2]) < 2.0, m


@pytest.mark.xfail(reason="the lens settles at 104.4 / 128.4 / 127.2 degrees: the liquid-gas tensions at the "
                          "contact line are about 17 % above Table 1's", strict=False)
def test_lens_matches_neumann_angles_of_table1():
    m, _ = set3_lens()
    want = O.neumann_angles(0.333, 0.333, 0.485)
    for got, w in zip(m, want):
        assert abs(got - w) < 2.0, (m, want)
