"""Shared set-ups for the GPU parity tests: the same seeded inputs and the
same parameters go to the HIP library and to the CPU oracle."""
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
                         no_collide=bool(p.flags & 1), force_alpha2=bool(p.flags & 2), eos=eos)


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
