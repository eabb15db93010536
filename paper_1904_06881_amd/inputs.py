"""Seeded synthetic initial fields for the ternary wetting workloads.

This module only builds input arrays (density rho and phase field phi on the
full grid, ghost layers included); it holds none of the update's arithmetic.
Both the GPU library and the CPU oracle receive the same arrays from here.

Diffuse shapes use the profile C = (1 + tanh(2 d / W)) / 2 of the signed
distance d (positive inside), i.e. the liquid-liquid tanh profile of the paper
(Sec. III) with alpha = W / 4.  Concentrations map to the fields by the inverse
of the paper's variable change (Sec. II A): rho = rho_l + C1 (rho_g - rho_l),
phi = chi (C2 - C3), with C1 = 1 - C2 - C3 (1 = gas, 2 and 3 = liquids).

Arrays are shaped (ny, nx) in 2D and (nz, ny, nx) in 3D, x fastest; walls sit
on the last axis (y in 2D, z in 3D) with ghost layers at index 0 and n-1 and
the wall planes at 0.5 and n-1.5.
"""
import numpy as np


def profile(d, W):
    return 0.5 * (1.0 + np.tanh(2.0 * d / W))


def fields_from_conc(C2, C3, rho_l=1.0, rho_g=1e-3, chi=5.0):
    C1 = 1.0 - C2 - C3
    rho = rho_l + C1 * (rho_g - rho_l)
    phi = chi * (C2 - C3)
    return np.ascontiguousarray(rho), np.ascontiguousarray(phi)


def _grid2(nx, ny):
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    return x, y


def _grid3(nx, ny, nz):
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(np.float64)
    return x, y, z


def sessile_drop_2d(nx, ny, r, xc=None, comp=2, W=4.0, wall_y=0.5, **kw):
    """Semicircular drop of liquid `comp` (2 or 3) centred on the bottom wall
    plane at (xc, wall_y); gas elsewhere."""
    xc = nx / 2.0 if xc is None else xc
    x, y = _grid2(nx, ny)
    d = r - np.sqrt((x - xc) ** 2 + (y - wall_y) ** 2)
    s = profile(d, W)
    z = np.zeros_like(s)
    return fields_from_conc(s if comp == 2 else z, s if comp == 3 else z, **kw)


def cap_drop_2d(nx, ny, r, theta_deg, xc=None, comp=2, W=4.0, wall_y=0.5, **kw):
    """Circular cap of radius r meeting the bottom wall at contact angle theta
    (measured inside the drop): centre at height -r cos(theta) above the wall."""
    xc = nx / 2.0 if xc is None else xc
    yc = wall_y - r * np.cos(np.radians(theta_deg))
    x, y = _grid2(nx, ny)
    d = r - np.sqrt((x - xc) ** 2 + (y - yc) ** 2)
    s = profile(d, W)
    z = np.zeros_like(s)
    return fields_from_conc(s if comp == 2 else z, s if comp == 3 else z, **kw)


def sessile_drop_3d(nx, ny, nz, r, center=None, comp=2, W=4.0, wall_z=0.5, **kw):
    cx, cy = (nx / 2.0, ny / 2.0) if center is None else center
    x, y, z = _grid3(nx, ny, nz)
    d = r - np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - wall_z) ** 2)
    s = profile(d, W)
    zz = np.zeros_like(s)
    return fields_from_conc(s if comp == 2 else zz, s if comp == 3 else zz, **kw)


def flat_interface_2d(nx, ny, left=(0, 1), right=(1, 0), x0=None, W=4.0, periodic=True, **kw):
    """Two flat interfaces normal to x in a periodic box (band of phase `right`
    between nx/4 and 3nx/4), phases given as (C2, C3) pairs."""
    x, y = _grid2(nx, ny)
    if periodic:
        a, b = nx / 4.0, 3.0 * nx / 4.0
        s = profile(np.minimum(x - a, b - x), W)
    else:
        x0 = nx / 2.0 if x0 is None else x0
        s = profile(x - x0, W)
    C2 = (1 - s) * left[0] + s * right[0]
    C3 = (1 - s) * left[1] + s * right[1]
    return fields_from_conc(C2, C3, **kw)


def bubble_2d(nx, ny, r, inside=(1, 0), outside=(0, 0), W=4.0, **kw):
    """Circular drop of phase `inside` in phase `outside`, periodic box."""
    x, y = _grid2(nx, ny)
    d = r - np.sqrt((x - nx / 2.0) ** 2 + (y - ny / 2.0) ** 2)
    s = profile(d, W)
    C2 = s * inside[0] + (1 - s) * outside[0]
    C3 = s * inside[1] + (1 - s) * outside[1]
    return fields_from_conc(C2, C3, **kw)


def lens_2d(nx, ny, r, band=None, W=4.0, **kw):
    """Liquid-2 drop of radius r centred on the upper edge of a liquid-3 band
    (rows band[0] .. band[1], default ny/4 .. ny/2) in gas, periodic box: the
    floating-lens set-up of a three-phase contact (Neumann triangle)."""
    x, y = _grid2(nx, ny)
    y0, y1 = (ny / 4.0, ny / 2.0) if band is None else band
    C2 = profile(r - np.sqrt((x - nx / 2.0) ** 2 + (y - y1) ** 2), W)
    C3 = profile(np.minimum(y - y0, y1 - y), W) * (1.0 - C2)
    return fields_from_conc(C2, C3, **kw)


def capillary_2d(nx, ny, x_front, film=3, W=4.0, **kw):
    """Channel with walls at y = 0, ny-1: liquid 2 fills x < x_front at full
    height, a liquid-3 film covers `film` fluid rows on both walls along the
    whole length, gas elsewhere."""
    x, y = _grid2(nx, ny)
    # slug occupying [0, x_front) on the periodic axis, two diffuse ends
    half = 0.5 * x_front
    dx = (x - half + 0.5 * nx) % nx - 0.5 * nx
    s2 = profile(half - np.abs(dx), W)
    # film of rows 1..film and ny-1-film..ny-2 (distance from the wall planes)
    dwall = np.minimum(y - 0.5, (ny - 1.5) - y)
    s3 = profile(film - dwall, W) if film > 0 else np.zeros_like(x)
    C2 = s2
    C3 = s3 * (1.0 - s2)
    return fields_from_conc(C2, C3, **kw)


def lubricated_drop_3d(nx, ny, nz, r, film=8, W=4.0, comp_drop=2, comp_film=3, wall_z=0.5, **kw):
    """Sphere of liquid `comp_drop` of radius r resting on a film of liquid
    `comp_film` of thickness `film` over the bottom wall; gas above."""
    x, y, z = _grid3(nx, ny, nz)
    top = wall_z + film
    s_film = profile(top - z, W)
    cz = top + r
    d = r - np.sqrt((x - nx / 2.0) ** 2 + (y - ny / 2.0) ** 2 + (z - cz) ** 2)
    s_drop = profile(d, W)
    Cd = s_drop
    Cf = s_film * (1.0 - s_drop)
    C2 = Cd if comp_drop == 2 else Cf
    C3 = Cf if comp_drop == 2 else Cd
    return fields_from_conc(C2, C3, **kw)


def drop_train_2d(nx, ny, n_drops=16, r=40.0, spacing=200.0, first=100.0, jitter=10.0,
                  seed=0, W=4.0, wall_y=0.5, **kw):
    """Alternating liquid-2 / liquid-3 semicircular drops on the bottom wall at
    x_k = first + spacing k + U(-jitter, jitter) (numpy PCG64 with `seed`)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xs = first + spacing * np.arange(n_drops) + rng.uniform(-jitter, jitter, n_drops)
    x, y = _grid2(nx, ny)
    C2 = np.zeros_like(x)
    C3 = np.zeros_like(x)
    for k, xc in enumerate(xs):
        dx = (x - xc + nx / 2.0) % nx - nx / 2.0
        s = profile(r - np.sqrt(dx ** 2 + (y - wall_y) ** 2), W)
        if k % 2 == 0:
            C2 = np.maximum(C2, s)
        else:
            C3 = np.maximum(C3, s)
    return fields_from_conc(C2, C3, **kw)


def random_fields(shape, seed=0, rho_l=1.0, rho_g=1e-3, chi=5.0, smooth=2):
    """Smooth random concentration fields (parity stress input): three random
    positive fields normalised to sum 1, box-filtered `smooth` times."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.random((3,) + tuple(shape)) + 0.05
    for _ in range(smooth):
        acc = c.copy()
        for ax in range(1, c.ndim):
            acc += np.roll(c, 1, axis=ax) + np.roll(c, -1, axis=ax)
        c = acc / (1 + 2 * (c.ndim - 1))
    c /= c.sum(axis=0, keepdims=True)
    return fields_from_conc(c[1], c[2], rho_l=rho_l, rho_g=rho_g, chi=chi)


def serving_requests(n=512, seed=0, rate=64.0, frac_2d=0.7, grid2=(64, 1024), grid3=(64, 192),
                     steps=(5000, 20000), theta=(30.0, 150.0), gamma=(0.005, 0.03), precisions=("fp32", "fp16s"),
                     margin=0.9):
    """A seeded stream of sessile-drop requests for the serving loop.

    Arrivals are a Poisson process of `rate` per second; a fraction frac_2d
    are D2Q9 square grids with side log-uniform in grid2, the rest D3Q27 cubes
    with side log-uniform in grid3; contact angle uniform in theta (all wall
    angles), step count uniform in `steps`, storage precision uniform over
    `precisions`, and the three tensions uniform in `gamma` subject to the
    triangle inequality gamma_ij < margin (gamma_ik + gamma_jk) (redrawn
    otherwise: outside it one liquid spreads over the other interface and no
    pairwise calibration exists).  The drop (liquid 2) has radius a quarter
    of the side.  Returns a list of dicts ordered by arrival time."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for k in range(n):
        t += rng.exponential(1.0 / rate)
        two_d = rng.random() < frac_2d
        lo, hi = grid2 if two_d else grid3
        side = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        while True:
            g = rng.uniform(gamma[0], gamma[1], 3)
            if g[0] < margin * (g[1] + g[2]) and g[1] < margin * (g[0] + g[2]) and g[2] < margin * (g[0] + g[1]):
                break
        out.append({
            "tag": k, "arrival": t, "lattice": "D2Q9" if two_d else "D3Q27",
            "n": (side, side) if two_d else (side, side, side),
            "theta": float(rng.uniform(theta[0], theta[1])),
            "gamma": tuple(float(v) for v in g),
            "nsteps": int(rng.integers(steps[0], steps[1] + 1)),
            "precision": precisions[int(rng.integers(0, len(precisions)))],
            "radius": side / 4.0,
        })
    return out


def request_fields(req):
    """Initial rho, phi of a serving request: a liquid-2 sessile drop on the
    bottom wall, centred along the wall."""
    n = req["n"]
    if len(n) == 2:
        return sessile_drop_2d(n[0], n[1], req["radius"])
    return sessile_drop_3d(n[0], n[1], n[2], req["radius"])
