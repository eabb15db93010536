"""Surface-tension scan as a batched workload (GPU, FP64).

Many small bubble simulations (periodic boxes, Laplace tests) with different
tensions and radii advance together through lbm3_step_batch: one launch per
kernel class serves them all.  Each bubble's pressure jump times its fitted
radius measures the tension the model produces (Laplace law), to be compared
with the tension the parameters were calibrated for.

Liquid-liquid (2-3) drops: Delta P R equals the closed form
gamma_23 = alpha (lambda_2 + lambda_3) / 6 (Eq. 38) within 5 % over a factor
of 2.7 in gamma_23 and for two radii.  Liquid-gas drops carry the excess
tension of the ideal-force discretisation (an expected failure, the same one
as the Laplace pin of the physics tests).
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1904_06881_amd import inputs as I
from paper_1904_06881_amd import lbm3 as L

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def scan(kind, g_list, radii, steps):
    """Step one bubble per (gamma, R) in a single batch; returns rows of
    (gamma, R, Delta P R, closed-form gamma, gas density)."""
    sims, meta = [], []
    for gam in g_list:
        # the scanned pair's tension is gam, the other two 0.01
        G = (0.01, 0.01, gam) if kind == "LL" else (gam, 0.01, 0.01)
        for R in radii:
            nb = 4 * R + 32
            p = L.make_params(L.D2Q9, (nb, nb), gamma=G, width=4.0, walls=False, precision=L.FP64)
            s = L.Sim(p)
            outside = (0, 1) if kind == "LL" else (0, 0)
            s.init(*I.bubble_2d(nb, nb, R, inside=(1, 0), outside=outside))
            sims.append(s)
            meta.append((gam, R, nb))
    say(kind, "batch of", len(sims), "bubbles,", steps, "steps")
    ws = L.step_batch(sims, steps)
    import torch
    torch.cuda.synchronize()
    del ws
    rows = []
    for s, (gam, R, nb) in zip(sims, meta):
        r, ph = s.fields()
        d = s.derived
        eos = {k: getattr(d, k) for k in ("a", "b", "T", "C", "psi0", "rho_l", "rho_g")}
        po = O.make_params(2, (nb, nb), lam=list(d.lam), kap=list(d.kap), eos=eos, rho_l=d.rho_l,
                           rho_g=d.rho_g, walls=False)
        bulk = lambda rr, pp: O.local_thermo(po, rr, pp, [0, 0], [0, 0], 0.0, 0.0)[2][0, 0]
        c = nb // 2
        dP = bulk(r[c, c], ph[c, c]) - bulk(r[2, 2], ph[2, 2])
        C1, C2, C3 = O.concentrations(po, r, ph)
        xs, ys = O.contour_points_2d(C2)
        Rf = O.kasa_fit(np.asarray(xs), np.asarray(ys))[2]
        closed = (d.lam[1] + d.lam[2]) / 6.0 if kind == "LL" else gam
        rows.append((gam, R, dP * Rf, closed, r[2, 2]))
        assert s.observe()["n_bad"] == 0
        s.close()
    for row in rows:
        say(kind, "gamma %.4f R %d  dP*R %.5f  closed %.5f  outer density %.4g" % row)
    return rows


def test_tension_scan_liquid_liquid():
    rows = scan("LL", (0.006, 0.01, 0.016), (16, 24), 16000)
    for gam, R, dPR, closed, _ in rows:
        assert abs(dPR - closed) < 0.05 * closed, (gam, R, dPR, closed)
    # the same tension at both radii
    for k in range(0, len(rows), 2):
        assert abs(rows[k][2] - rows[k + 1][2]) < 0.03 * rows[k][3]


@pytest.mark.xfail(reason="liquid-gas interfaces carry an excess tension with the link-pressure ideal "
                          "force (dP R about 1.7x gamma_12)", strict=False)
def test_tension_scan_liquid_gas():
    rows = scan("LG", (0.006, 0.012), (16,), 16000)
    for gam, R, dPR, closed, _ in rows:
        assert abs(dPR - closed) < 0.05 * closed, (gam, R, dPR, closed)
