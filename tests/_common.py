"""Shared set-ups for the GPU parity tests: the same seeded inputs and the
same parameters go to the HIP library and to the CPU oracle."""
import sys

import numpy as np

from oracle import oracle as O
from paper_1904_06881_amd import inputs as I


def oracle_params_from(p, d):
    """Oracle parameters equal to a library lbm3_params p with its derived
    constants d (lambda, kappa and the EOS constants from lbm3_resolve are
    handed over as plain numbers)."""
    D = 2 if p.lattice == 9 else 3
    eos = {"a": d.a, "b": d.b, "T": d.T, "C": d.C, "psi0": d.psi0, "rho_l": d.rho_l,
           "rho_g": d.rho_g}
    n = (p.n[0], p.n[1]) if D == 2 else (p.n[0], p.n[1], p.n[2])
    th = [[p.theta_deg[w][k] for k in range(3)] for w in range(2)]
    kw = [[p.kw[w][k] for k in range(2)] for w in range(2)]
    return O.make_params(D, n, rho_l=d.rho_l, rho_g=d.rho_g, lam=list(d.lam), kap=list(d.kap),
                         chi=p.chi, tau_f=p.tau_f, tau_g=p.tau_g, Gamma=p.Gamma, walls=bool(p.walls),
                         wetting=p.wetting, theta_deg=th, kw=kw,
                         alpha_eps=p.alpha_eps or 1e-3,
                         alpha_tol=p.alpha_tol or (1e-10 if p.precision == 0 else 1e-5),
                         alpha_maxit=p.alpha_maxit or 20,
                         no_collide=bool(p.flags & 1), force_alpha2=bool(p.flags & 2), eos=eos,
                         detect_ratio=p.detect_ratio)


def conc(rho, phi, rho_l, rho_g, chi=5.0):
    C1 = (rho - rho_l) / (rho_g - rho_l)
    C2 = 0.5 * (1 + phi / chi - C1)
    C3 = 0.5 * (1 - phi / chi - C1)
    return np.stack([C1, C2, C3])


def fluid(arr, walls, D):
    """Fluid part of a field array (strip the ghost layers of the wall axis)."""
    if not walls:
        return arr
    return arr[1:-1] if D == 2 else arr[1:-1]


def say(*a):
    """Name the GPU case before it runs (flushed, so a failing run shows it)."""
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def run_both(p, rho0, phi0, steps, gpu_chunks=None, oracle=True):
    """The library (through the C ABI) and the oracle from the same fields and
    parameters, `steps` steps each; returns (sim, oracle sim or None)."""
    from paper_1904_06881_amd import lbm3 as L
    say("run", "lattice", p.lattice, "n", list(p.n), "prec", p.precision, "wet", p.wetting,
        "walls", p.walls, "steps", steps)
    sim = L.Sim(p)
    sim.init(rho0, phi0)
    if gpu_chunks:
        for c in gpu_chunks:
            sim.step(c)
    else:
        sim.step(steps)
    ora = None
    if oracle:
        ora = O.Sim(oracle_params_from(p, sim.derived))
        ora.init(rho0, phi0)
        ora.step(steps)
    return sim, ora


def conc_err(sim, ora, walls=True):
    """Max-abs difference of C1, C2, C3 over the fluid nodes."""
    d = sim.derived
    rg, pg = sim.fields()
    ro, po = ora.fields()
    sl = (slice(None), slice(1, -1)) if walls else (slice(None),)
    cg = conc(rg, pg, d.rho_l, d.rho_g)[sl]
    co = conc(ro, po, d.rho_l, d.rho_g)[sl]
    assert np.all(np.isfinite(cg))
    return float(np.abs(cg - co).max())
