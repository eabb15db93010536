"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU baseline leg import
this module.  It never loads the GPU library and the GPU library never loads
it.  Paper: Bala et al., "Wetting boundaries for ternary high density ratio
lattice Boltzmann method" (arXiv:1904.06881).
"""
import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm3_oracle.so")

FORCE, GEOM_INTERP, GEOM_EXTRAP = 0, 1, 2

# Reference Carnahan-Starling constants of the paper (Sec. II A): a, b, R = 1.
A0, B0 = 0.037, 0.2


class OrParams(C.Structure):
    _fields_ = [
        ("D", C.c_int), ("n", C.c_int * 3), ("walls", C.c_int),
        ("a", C.c_double), ("b", C.c_double), ("T", C.c_double),
        ("C", C.c_double), ("psi0", C.c_double), ("rho_l", C.c_double),
        ("rho_g", C.c_double),
        ("lam", C.c_double * 3), ("kap", C.c_double * 3),
        ("chi", C.c_double), ("beta", C.c_double), ("tau_g", C.c_double),
        ("Gamma", C.c_double),
        ("wetting", C.c_int), ("theta_deg", (C.c_double * 3) * 2),
        ("kw", (C.c_double * 2) * 2),
        ("alpha_eps", C.c_double), ("alpha_tol", C.c_double),
        ("alpha_maxit", C.c_int),
        ("no_collide", C.c_int), ("force_alpha2", C.c_int), ("detect_ratio", C.c_double),
        ("wall_par", C.c_int),
    ]


class OrObs(C.Structure):
    _fields_ = [
        ("mass", C.c_double * 3), ("rho_sum", C.c_double), ("phi_sum", C.c_double),
        ("mom", C.c_double * 3), ("kinetic", C.c_double), ("umax", C.c_double),
        ("n_bad", C.c_int64), ("n_newton", C.c_int64), ("n_shortcut", C.c_int64),
        ("n_fallback", C.c_int64), ("step", C.c_int64), ("n_fast", C.c_int64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.or_psi.restype = C.c_double
        L.or_psi.argtypes = [C.c_double] * 5
        L.or_dpsi.restype = C.c_double
        L.or_dpsi.argtypes = [C.c_double] * 5
        L.or_critical_T.restype = C.c_double
        L.or_critical_T.argtypes = [C.c_double, C.c_double]
        L.or_coexistence.restype = C.c_int
        L.or_coexistence.argtypes = [C.c_double] * 4 + [dp] * 7
        L.or_lattice.restype = C.c_int
        L.or_lattice.argtypes = [C.c_int, C.POINTER(C.c_int), dp]
        L.or_feq.argtypes = [C.c_int, C.c_double, dp, dp]
        L.or_geq.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, dp, dp]
        L.or_alpha.restype = C.c_int
        L.or_alpha.argtypes = [C.c_int, dp, dp, dp, C.c_double, C.c_double, C.c_int, dp]
        L.or_local_thermo.argtypes = [C.POINTER(OrParams), C.c_double, C.c_double,
                                      dp, dp, C.c_double, C.c_double, dp, dp, dp]
        L.or_interp2d.restype = C.c_double
        L.or_interp2d.argtypes = [dp, C.c_int, C.c_int, C.c_double]
        L.or_interp3d.restype = C.c_double
        L.or_interp3d.argtypes = [dp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double]
        L.or_create.restype = C.c_void_p
        L.or_create.argtypes = [C.POINTER(OrParams)]
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_init.restype = C.c_int
        L.or_init.argtypes = [C.c_void_p, dp, dp]
        L.or_set_pops.restype = C.c_int
        L.or_set_pops.argtypes = [C.c_void_p, dp, dp]
        L.or_step.restype = C.c_int
        L.or_step.argtypes = [C.c_void_p, C.c_int64]
        L.or_get.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.or_get_field.argtypes = [C.c_void_p, C.c_int, dp]
        L.or_observe.argtypes = [C.c_void_p, C.POINTER(OrObs)]
        L.or_Q.restype = C.c_int
        L.or_Q.argtypes = [C.c_void_p]
        L.or_N.restype = C.c_int64
        L.or_N.argtypes = [C.c_void_p]
        L.or_set_threads.argtypes = [C.c_int]
        L.or_get_threads.restype = C.c_int
        L.or_flat_tension.restype = C.c_double
        L.or_flat_tension.argtypes = [C.POINTER(OrParams), C.c_int, C.c_int, dp, dp, dp]
        _lib = L
    return _lib


def set_threads(n):
    """OpenMP threads of the oracle's passes (timing only)."""
    lib().or_set_threads(int(n))


def get_threads():
    return lib().or_get_threads()


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- lattice --
def lattice(D):
    c = (C.c_int * 81)()
    w = np.zeros(27)
    Q = lib().or_lattice(D, c, _dp(w))
    cv = np.array(c[: 3 * Q], dtype=np.int64).reshape(Q, 3)[:, :D]
    return cv, w[:Q].copy()


def feq(D, rho, u):
    out = np.zeros(27)
    uu = np.zeros(3)
    uu[:D] = u
    lib().or_feq(D, rho, _dp(uu), _dp(out))
    return out[: 9 if D == 2 else 27]


def geq(D, phi, mu_phi, Gamma, v):
    out = np.zeros(27)
    vv = np.zeros(3)
    vv[:D] = v
    lib().or_geq(D, phi, mu_phi, Gamma, _dp(vv), _dp(out))
    return out[: 9 if D == 2 else 27]


def alpha(fp, delta, eps=1e-3, tol=1e-10, maxit=20):
    fp = _f64(fp)
    delta = _f64(delta)
    Q = fp.size
    w = np.zeros(Q)
    a = C.c_double(0.0)
    kind = lib().or_alpha(Q, _dp(w), _dp(fp), _dp(delta), eps, tol, maxit, C.byref(a))
    return a.value, kind


# ---------------------------------------------------------- thermodynamics --
def psi(rho, a, b, T, Cc):
    return lib().or_psi(rho, a, b, T, Cc)


def dpsi(rho, a, b, T, Cc):
    return lib().or_dpsi(rho, a, b, T, Cc)


def critical_T(a, b):
    return lib().or_critical_T(a, b)


def coexistence(ratio, rho_l, a0=A0, b0=B0):
    out = [C.c_double() for _ in range(7)]
    rc = lib().or_coexistence(a0, b0, ratio, rho_l, *[C.byref(o) for o in out])
    if rc != 0:
        raise ValueError("no coexistence for ratio %g (code %d)" % (ratio, rc))
    keys = ["a", "b", "T", "C", "psi0", "rho_l", "rho_g"]
    return {k: o.value for k, o in zip(keys, out)}


# ------------------------------------------------------------- parameters --
def make_params(D, n, *, rho_l=1.0, rho_g=1e-3, lam=(0.0625, 0.03, 0.03),
                kap=(0.03, 0.03, 0.03), chi=5.0, tau_f=1.0, tau_g=1.0, Gamma=1.0,
                walls=True, wetting=GEOM_INTERP, theta_deg=90.0, kw=((0, 0), (0, 0)),
                alpha_eps=1e-3, alpha_tol=1e-10, alpha_maxit=20, no_collide=False,
                force_alpha2=False, eos=None, wall_par=0, detect_ratio=0.0):
    """Oracle parameters.  beta = 1/(2 tau_f) (nu = (1/beta - 1)/6, Sec. II C).
    theta_deg: scalar, (theta21, theta31, theta23) or a 2x3 per-wall table."""
    p = OrParams()
    p.D = D
    nn = list(n) + [1] * (3 - len(n))
    for k in range(3):
        p.n[k] = nn[k]
    p.walls = 1 if walls else 0
    if eos is None:
        eos = coexistence(rho_l / rho_g, rho_l)
    p.a, p.b, p.T, p.C, p.psi0 = eos["a"], eos["b"], eos["T"], eos["C"], eos["psi0"]
    p.rho_l, p.rho_g = eos["rho_l"], eos["rho_g"]
    for k in range(3):
        p.lam[k] = lam[k]
        p.kap[k] = kap[k]
    p.chi, p.beta, p.tau_g, p.Gamma = chi, 1.0 / (2.0 * tau_f), tau_g, Gamma
    p.wetting = wetting
    th = np.broadcast_to(np.asarray(theta_deg, dtype=np.float64), (2, 3)) \
        if np.ndim(theta_deg) < 2 else np.asarray(theta_deg, dtype=np.float64)
    if np.ndim(theta_deg) == 1:
        th = np.stack([np.asarray(theta_deg, float)] * 2)
    for wl in range(2):
        for k in range(3):
            p.theta_deg[wl][k] = float(th[wl][k])
        for k in range(2):
            p.kw[wl][k] = float(kw[wl][k])
    p.alpha_eps, p.alpha_tol, p.alpha_maxit = alpha_eps, alpha_tol, alpha_maxit
    p.no_collide = int(no_collide)
    p.force_alpha2 = int(force_alpha2)
    p.wall_par = int(wall_par)
    p.detect_ratio = detect_ratio
    return p


def local_thermo(p, rho, phi, grad_rho, grad_phi, lap_rho, lap_phi):
    G = np.zeros(3)
    H = np.zeros(3)
    G[: len(grad_rho)] = grad_rho
    H[: len(grad_phi)] = grad_phi
    mr, mp = C.c_double(), C.c_double()
    P = np.zeros(9)
    lib().or_local_thermo(C.byref(p), rho, phi, _dp(G), _dp(H), lap_rho, lap_phi,
                          C.byref(mr), C.byref(mp), _dp(P))
    return mr.value, mp.value, P.reshape(3, 3)


def interp2d(q, i, l):
    q = _f64(q)
    return lib().or_interp2d(_dp(q), q.size, i, l)


def interp3d(q, i, j, lx, ly):
    """q indexed q[j, i] (x fastest)."""
    q = _f64(q)
    ny, nx = q.shape
    return lib().or_interp3d(_dp(q), nx, ny, i, j, lx, ly)


def flat_tension(p, pair, n=128, return_profile=False):
    w = C.c_double()
    r = np.zeros(n)
    ph = np.zeros(n)
    g = lib().or_flat_tension(C.byref(p), pair, n, C.byref(w), _dp(r), _dp(ph))
    if return_profile:
        return g, w.value, r, ph
    return g, w.value


# ------------------------------------------------------------- simulation --
FIELDS = {"mu_rho": 0, "mu_phi": 1, "Fx": 2, "Fy": 3, "Fz": 4, "grad_rho_x": 5,
          "grad_rho_y": 6, "grad_rho_z": 7, "grad_phi_x": 8, "grad_phi_y": 9,
          "grad_phi_z": 10, "lap_rho": 11, "lap_phi": 12, "alpha": 13}


class Sim:
    """One oracle simulation.  Arrays are shaped (nz, ny, nx) or (ny, nx)."""

    def __init__(self, p):
        self.p = p
        self.D = p.D
        self.shape = (p.n[1], p.n[0]) if p.D == 2 else (p.n[2], p.n[1], p.n[0])
        self.h = lib().or_create(C.byref(p))
        if not self.h:
            raise ValueError("oracle create failed")
        self.Q = lib().or_Q(self.h)
        self.N = lib().or_N(self.h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().or_destroy(h)
            self.h = None

    def init(self, rho0, phi0):
        r = _f64(rho0).reshape(-1)
        ph = _f64(phi0).reshape(-1)
        assert r.size == self.N and ph.size == self.N
        lib().or_init(self.h, _dp(r), _dp(ph))

    def set_pops(self, f, g):
        f = _f64(f).reshape(-1)
        g = _f64(g).reshape(-1)
        lib().or_set_pops(self.h, _dp(f), _dp(g))

    def step(self, n=1):
        lib().or_step(self.h, int(n))

    def fields(self):
        r = np.zeros(self.N)
        ph = np.zeros(self.N)
        lib().or_get(self.h, _dp(r), _dp(ph), None, None)
        return r.reshape(self.shape), ph.reshape(self.shape)

    def pops(self):
        f = np.zeros(self.Q * self.N)
        g = np.zeros(self.Q * self.N)
        lib().or_get(self.h, None, None, _dp(f), _dp(g))
        return f.reshape((self.Q,) + self.shape), g.reshape((self.Q,) + self.shape)

    def field(self, name):
        out = np.zeros(self.N)
        lib().or_get_field(self.h, FIELDS[name], _dp(out))
        return out.reshape(self.shape)

    def observe(self):
        o = OrObs()
        lib().or_observe(self.h, C.byref(o))
        return {"mass": list(o.mass), "rho_sum": o.rho_sum, "phi_sum": o.phi_sum,
                "mom": list(o.mom), "kinetic": o.kinetic, "umax": o.umax,
                "n_bad": o.n_bad, "n_newton": o.n_newton, "n_shortcut": o.n_shortcut,
                "n_fallback": o.n_fallback, "step": o.step, "n_fast": o.n_fast}

    def concentrations(self):
        r, ph = self.fields()
        return concentrations(self.p, r, ph)


def concentrations(p, rho, phi):
    """C1, C2, C3 from rho and phi (Eqs. 5-7)."""
    C1 = (rho - p.rho_l) / (p.rho_g - p.rho_l)
    C2 = 0.5 * (1.0 + phi / p.chi - C1)
    C3 = 0.5 * (1.0 - phi / p.chi - C1)
    return C1, C2, C3


# --------------------------------------------------------------- analysis --
def neumann_angles(g12, g13, g23):
    """Neumann angles theta1..theta3 in degrees from the three tensions
    (Eqs. 40-42)."""
    t1 = math.degrees(math.acos((g23 ** 2 - g12 ** 2 - g13 ** 2) / (2 * g12 * g13)))
    t2 = math.degrees(math.acos((g13 ** 2 - g12 ** 2 - g23 ** 2) / (2 * g12 * g23)))
    t3 = math.degrees(math.acos((g12 ** 2 - g13 ** 2 - g23 ** 2) / (2 * g13 * g23)))
    return t1, t2, t3


def contour_points_2d(c, level=0.5, y_offset=0.0):
    """Points where the field c (ny, nx) crosses `level`, by linear
    interpolation along grid lines.  Returns (x, y) arrays in lattice units."""
    ny, nx = c.shape
    xs, ys = [], []
    for y in range(ny):
        row = c[y]
        for x in range(nx - 1):
            a, b = row[x] - level, row[x + 1] - level
            if a == 0.0:
                xs.append(float(x)); ys.append(float(y))
            elif a * b < 0.0:
                xs.append(x + a / (a - b)); ys.append(float(y))
    for x in range(nx):
        col = c[:, x]
        for y in range(ny - 1):
            a, b = col[y] - level, col[y + 1] - level
            if a * b < 0.0:
                xs.append(float(x)); ys.append(y + a / (a - b))
    return np.array(xs), np.array(ys) + y_offset


def lens_angles_2d(C2, C3, xc, W=4.0):
    """Neumann angles (theta1, theta2, theta3) in degrees of a liquid-2 lens
    floating on the upper edge of a liquid-3 layer in gas (Sec. III, the
    three-phase contact whose angles Eqs. 40-42 give from the tensions).
    The flat 3-gas interface height is the median of the C3 = 1/2 points of
    the layer's upper edge (the upper of its two edges) more than 3 W beside
    the lens; the C2 = 1/2 points
    more than W above it and below it get one circle each; the two circles
    cross at the contact points, where the rays along the upper arc, the
    lower arc and the flat interface (pointing away from the lens) bound the
    gas (theta1), liquid-2 (theta2) and liquid-3 (theta3) sectors.  Returns
    the angles averaged over both contact points, and the per-point ones."""
    x2, y2 = contour_points_2d(C2)
    x3, y3 = contour_points_2d(C3)
    half = 0.5 * (x2.max() - x2.min())
    side = np.abs(x3 - xc) > half + 3.0 * W
    ys = y3[side]
    yf = float(np.median(ys[ys > ys.mean()]))
    up, lo = y2 > yf + W, y2 < yf - W
    a = kasa_fit(x2[up], y2[up])
    b = kasa_fit(x2[lo], y2[lo])
    ma = np.array([x2[up].mean(), y2[up].mean()])
    mb = np.array([x2[lo].mean(), y2[lo].mean()])
    # circle-circle intersection
    ca, cb = np.array(a[:2]), np.array(b[:2])
    d = np.linalg.norm(cb - ca)
    l = (a[2] ** 2 - b[2] ** 2 + d * d) / (2.0 * d)
    h = math.sqrt(max(a[2] ** 2 - l * l, 0.0))
    e = (cb - ca) / d
    base = ca + l * e
    pts = [base + h * np.array([-e[1], e[0]]), base - h * np.array([-e[1], e[0]])]

    def ray(P, c, m):
        t = np.array([-(P - c)[1], (P - c)[0]])
        t /= np.linalg.norm(t)
        return t if np.dot(t, m - P) > 0 else -t

    def ang(u, v):
        return math.degrees(math.acos(max(-1.0, min(1.0, float(np.dot(u, v))))))

    per = []
    for P in pts:
        ra, rb = ray(P, ca, ma), ray(P, cb, mb)
        rf = np.array([1.0 if P[0] > xc else -1.0, 0.0])
        per.append((ang(ra, rf), ang(ra, rb), ang(rb, rf)))
    mean = tuple(float(np.mean([q[k] for q in per])) for k in range(3))
    return mean, per, yf


def kasa_fit(xs, ys):
    """Algebraic (Kasa) least-squares circle: x^2 + y^2 + D x + E y + F = 0."""
    A = np.stack([xs, ys, np.ones_like(xs)], axis=1)
    rhs = -(xs ** 2 + ys ** 2)
    sol, *_ = np.linalg.lstsq(A, rhs, rcond=None)
    Dd, E, F = sol
    xc, yc = -Dd / 2, -E / 2
    R = math.sqrt(xc ** 2 + yc ** 2 - F)
    return xc, yc, R


def contact_angle_2d(c, wall_y=0.5, exclude=8.0, level=0.5, wall="low"):
    """Contact angle (degrees) measured inside the phase of concentration c for a
    sessile drop on the wall at y = wall_y: circle fit to the c = 0.5 contour
    excluding points within `exclude` of the wall, theta = arccos(-h/R), h the
    centre height above the wall plane (measured into the fluid)."""
    xs, ys = contour_points_2d(c, level)
    if wall == "low":
        keep = ys > wall_y + exclude
    else:
        keep = ys < wall_y - exclude
    xc, yc, R = kasa_fit(xs[keep], ys[keep])
    h = (yc - wall_y) if wall == "low" else (wall_y - yc)
    return math.degrees(math.acos(max(-1.0, min(1.0, -h / R)))), (xc, yc, R)


def contour_points_3d(c, level=0.5):
    """Points where the field c (nz, ny, nx) crosses `level`, by linear
    interpolation along the grid lines of the three axes (no wrap).  Returns
    (x, y, z) arrays in lattice units."""
    a = np.asarray(c, dtype=np.float64) - level
    z, y, x = np.mgrid[0:a.shape[0], 0:a.shape[1], 0:a.shape[2]].astype(np.float64)
    xs, ys, zs = [], [], []
    for ax in (2, 1, 0):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        a0, a1 = a[tuple(lo)], a[tuple(hi)]
        cross = a0 * a1 < 0.0
        t = np.zeros_like(a0)
        t[cross] = a0[cross] / (a0[cross] - a1[cross])
        pos = [x[tuple(lo)], y[tuple(lo)], z[tuple(lo)]]
        pos[2 - ax] = pos[2 - ax] + t
        xs.append(pos[0][cross]); ys.append(pos[1][cross]); zs.append(pos[2][cross])
    return np.concatenate(xs), np.concatenate(ys), np.concatenate(zs)


def kasa_fit_sphere(xs, ys, zs):
    """Algebraic (Kasa) least-squares sphere: x^2 + y^2 + z^2 + D x + E y + F z
    + G = 0."""
    A = np.stack([xs, ys, zs, np.ones_like(xs)], axis=1)
    rhs = -(xs ** 2 + ys ** 2 + zs ** 2)
    sol, *_ = np.linalg.lstsq(A, rhs, rcond=None)
    Dd, E, F, G = sol
    xc, yc, zc = -Dd / 2, -E / 2, -F / 2
    R = math.sqrt(xc ** 2 + yc ** 2 + zc ** 2 - G)
    return xc, yc, zc, R


def contact_angle_3d(c, wall_z=0.5, exclude=8.0, level=0.5, wall="low"):
    """Contact angle (degrees) measured inside the phase of concentration c
    (nz, ny, nx) for a sessile drop on the wall plane z = wall_z: sphere fit
    to the c = 0.5 iso-points farther than `exclude` from the wall plane,
    theta = arccos(-h/R), h the centre height above the wall plane."""
    xs, ys, zs = contour_points_3d(c, level)
    keep = np.abs(zs - wall_z) > exclude
    xc, yc, zc, R = kasa_fit_sphere(xs[keep], ys[keep], zs[keep])
    h = (zc - wall_z) if wall == "low" else (wall_z - zc)
    return math.degrees(math.acos(max(-1.0, min(1.0, -h / R)))), (xc, yc, zc, R)
