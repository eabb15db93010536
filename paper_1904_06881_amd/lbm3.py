"""ctypes binding of the lbm3 C ABI (include/lbm3.h).

Argument marshalling only: every step of the update runs in the HIP library
liblbm3.so.  PyTorch provides the device workspace (a uint8 tensor) and the
stream.  Importing this module loads the library and fails loudly when it is
missing; there is no CPU fallback.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm3.so")

D2Q9, D3Q27 = 9, 27
WET_FORCE, WET_GEOM_INTERP, WET_GEOM_EXTRAP = 0, 1, 2
FP64, FP32, FP16S = 0, 1, 2
NO_COLLIDE, FORCE_ALPHA2, FUSED_3D, STORED_G = 1, 2, 4, 8
OBS_SUMS, OBS_FIELDS, OBS_POPS = 1, 2, 4
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EUNSTABLE", -4: "EDEVICE", -5: "ESTATE",
          -6: "ECALIB"}


class lbm3_params(C.Structure):
    _fields_ = [
        ("lattice", C.c_int32), ("n", C.c_int32 * 3), ("walls", C.c_int32),
        ("rho_l", C.c_double), ("rho_g", C.c_double), ("native", C.c_int32),
        ("lam", C.c_double * 3), ("kap", C.c_double * 3),
        ("gamma12", C.c_double), ("gamma13", C.c_double), ("gamma23", C.c_double),
        ("width", C.c_double), ("chi", C.c_double), ("tau_f", C.c_double),
        ("tau_g", C.c_double), ("Gamma", C.c_double), ("wetting", C.c_int32),
        ("theta_deg", (C.c_double * 3) * 2), ("kw", (C.c_double * 2) * 2),
        ("precision", C.c_int32), ("flags", C.c_uint32), ("alpha_eps", C.c_double),
        ("alpha_tol", C.c_double), ("alpha_maxit", C.c_int32), ("detect_ratio", C.c_double),
    ]


class lbm3_derived(C.Structure):
    _fields_ = [
        ("a", C.c_double), ("b", C.c_double), ("T", C.c_double), ("C", C.c_double),
        ("psi0", C.c_double), ("rho_l", C.c_double), ("rho_g", C.c_double),
        ("lam", C.c_double * 3), ("kap", C.c_double * 3), ("kappa_rr", C.c_double),
        ("kappa_pp", C.c_double), ("kappa_x", C.c_double), ("beta", C.c_double),
        ("cot_theta", (C.c_double * 3) * 2),
    ]


class lbm3_obs(C.Structure):
    _fields_ = [
        ("mass", C.c_double * 3), ("rho_sum", C.c_double), ("phi_sum", C.c_double),
        ("mom", C.c_double * 3), ("kinetic", C.c_double), ("umax", C.c_double),
        ("n_bad", C.c_int64), ("n_newton", C.c_int64), ("n_shortcut", C.c_int64),
        ("n_fallback", C.c_int64), ("step", C.c_int64), ("n_fast", C.c_int64),
    ]


class lbm3_result(C.Structure):
    _fields_ = [
        ("tag", C.c_uint64), ("status", C.c_int32), ("has_fields", C.c_int32),
        ("steps", C.c_int64), ("nodes", C.c_int64),
        ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
        ("bytes", C.c_double), ("obs", lbm3_obs),
    ]


SERVE_FIELDS = 1

EXPORTS = ["lbm3_footprint", "lbm3_resolve", "lbm3_create", "lbm3_init", "lbm3_step",
           "lbm3_step_profiled", "lbm3_observe", "lbm3_contact_angle", "lbm3_destroy",
           "lbm3_last_error", "lbm3_batch_workspace", "lbm3_step_batch",
           "lbm3_server_request_bytes", "lbm3_server_create", "lbm3_server_submit",
           "lbm3_server_run", "lbm3_server_poll", "lbm3_server_fields", "lbm3_server_clock",
           "lbm3_server_destroy", "lbm3_step_batch_static"]


class Lbm3Error(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("lbm3 %s: %s" % (STATUS.get(status, status), msg))
        self.status = status


_lib = None


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("liblbm3.so not built: run __graft_entry__.build() or "
                              "python paper_1904_06881_amd/build.py")
        # torch first: it ships its own HIP and HSA runtimes, and the library's
        # HIP dependency must bind to the ones torch has loaded.  Loaded the
        # other way round, the process holds two HSA runtimes and the
        # library's sees no device.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, dp = C.c_void_p, C.POINTER(C.c_double)
        L.lbm3_footprint.restype = C.c_size_t
        L.lbm3_footprint.argtypes = [C.POINTER(lbm3_params)]
        L.lbm3_resolve.restype = C.c_int
        L.lbm3_resolve.argtypes = [C.POINTER(lbm3_params), C.POINTER(lbm3_derived)]
        L.lbm3_create.restype = C.c_int
        L.lbm3_create.argtypes = [C.POINTER(lbm3_params), vp, C.c_size_t, vp, C.POINTER(vp)]
        L.lbm3_init.restype = C.c_int
        L.lbm3_init.argtypes = [vp, dp, dp]
        L.lbm3_step.restype = C.c_int
        L.lbm3_step.argtypes = [vp, C.c_int64]
        L.lbm3_step_profiled.restype = C.c_int
        L.lbm3_step_profiled.argtypes = [vp, C.c_int64, C.c_int32, dp]
        L.lbm3_observe.restype = C.c_int
        L.lbm3_observe.argtypes = [vp, C.c_uint32, C.POINTER(lbm3_obs), dp, dp, dp, dp]
        L.lbm3_contact_angle.restype = C.c_int
        L.lbm3_contact_angle.argtypes = [vp, C.c_int32, C.c_int32, C.c_double, dp]
        L.lbm3_destroy.restype = C.c_int
        L.lbm3_destroy.argtypes = [vp]
        L.lbm3_last_error.restype = C.c_char_p
        L.lbm3_last_error.argtypes = [vp]
        L.lbm3_batch_workspace.restype = C.c_int
        L.lbm3_batch_workspace.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(C.c_size_t)]
        L.lbm3_step_batch.restype = C.c_int
        L.lbm3_step_batch.argtypes = [C.POINTER(vp), C.c_int32, C.c_int64, vp, vp, C.c_size_t]
        L.lbm3_step_batch_static.restype = C.c_int
        L.lbm3_step_batch_static.argtypes = [C.POINTER(vp), C.c_int32, C.c_int64, vp]
        L.lbm3_server_request_bytes.restype = C.c_size_t
        L.lbm3_server_request_bytes.argtypes = [C.POINTER(lbm3_params)]
        L.lbm3_server_create.restype = C.c_int
        L.lbm3_server_create.argtypes = [vp, C.c_size_t, vp, C.c_int32, C.c_int32, C.POINTER(vp)]
        L.lbm3_server_submit.restype = C.c_int
        L.lbm3_server_submit.argtypes = [vp, C.POINTER(lbm3_params), dp, dp, C.c_int64, C.c_uint64, C.c_uint32]
        L.lbm3_server_run.restype = C.c_int
        L.lbm3_server_run.argtypes = [vp, C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.lbm3_server_poll.restype = C.c_int32
        L.lbm3_server_poll.argtypes = [vp, C.POINTER(lbm3_result)]
        L.lbm3_server_fields.restype = C.c_int
        L.lbm3_server_fields.argtypes = [vp, C.c_uint64, dp, dp]
        L.lbm3_server_clock.restype = C.c_double
        L.lbm3_server_clock.argtypes = [vp]
        L.lbm3_server_destroy.restype = C.c_int
        L.lbm3_server_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(lattice, n, *, walls=True, rho_l=1.0, rho_g=1e-3, lam=None, kap=None,
                gamma=None, width=4.0, chi=5.0, tau_f=1.0, tau_g=1.0, Gamma=1.0,
                wetting=WET_GEOM_INTERP, theta_deg=90.0, kw=((0, 0), (0, 0)), precision=FP64,
                flags=0, alpha_eps=0.0, alpha_tol=0.0, alpha_maxit=0, detect_ratio=0.0):
    """Fill lbm3_params.  Give lam/kap (native) or gamma=(g12, g13, g23) with
    width.  theta_deg: scalar, (theta21, theta31, theta23) or a 2x3 table."""
    p = lbm3_params()
    p.lattice = lattice
    nn = list(n) + [1] * (3 - len(n))
    for k in range(3):
        p.n[k] = int(nn[k])
    p.walls = 1 if walls else 0
    p.rho_l, p.rho_g = rho_l, rho_g
    if lam is not None:
        p.native = 1
        for k in range(3):
            p.lam[k], p.kap[k] = lam[k], kap[k]
    else:
        p.native = 0
        p.gamma12, p.gamma13, p.gamma23 = gamma
        p.width = width
    p.chi, p.tau_f, p.tau_g, p.Gamma = chi, tau_f, tau_g, Gamma
    p.wetting = wetting
    th = np.asarray(theta_deg, dtype=np.float64)
    if th.ndim == 0:
        th = np.full((2, 3), float(th))
    elif th.ndim == 1:
        th = np.stack([th, th])
    for w in range(2):
        for k in range(3):
            p.theta_deg[w][k] = float(th[w][k])
        for k in range(2):
            p.kw[w][k] = float(kw[w][k])
    p.precision = precision
    p.flags = flags
    p.alpha_eps, p.alpha_tol, p.alpha_maxit = alpha_eps, alpha_tol, alpha_maxit
    p.detect_ratio = detect_ratio
    return p


def lbm3_footprint(p):
    return lib().lbm3_footprint(C.byref(p))


def lbm3_resolve(p):
    d = lbm3_derived()
    st = lib().lbm3_resolve(C.byref(p), C.byref(d))
    if st != 0:
        raise Lbm3Error(st, "parameter resolution failed")
    return d


def lbm3_create(p, workspace_ptr, nbytes, stream_ptr):
    h = C.c_void_p()
    st = lib().lbm3_create(C.byref(p), C.c_void_p(workspace_ptr), nbytes, C.c_void_p(stream_ptr),
                           C.byref(h))
    if st != 0:
        raise Lbm3Error(st, lib().lbm3_last_error(None).decode())
    return h


def _check(h, st):
    if st != 0:
        raise Lbm3Error(st, lib().lbm3_last_error(h).decode())


def lbm3_init(h, rho0, phi0):
    r = np.ascontiguousarray(rho0, dtype=np.float64).reshape(-1)
    ph = np.ascontiguousarray(phi0, dtype=np.float64).reshape(-1)
    _check(h, lib().lbm3_init(h, _dp(r), _dp(ph)))


def lbm3_step(h, nsteps):
    _check(h, lib().lbm3_step(h, int(nsteps)))


def lbm3_step_profiled(h, nsteps, sample_every=1):
    """Run nsteps with events around the launches of every sample_every-th
    step; returns the mean device ms per launch of the moments, ghost-layer
    (0 in 2D) and fused kernels (in 3D the stencil pass plus the collide
    kernel, and each of the two alone), the span of the whole run in ms and
    the number of sampled steps."""
    ms = np.zeros(8)
    _check(h, lib().lbm3_step_profiled(h, int(nsteps), int(sample_every), _dp(ms)))
    return {"moments": ms[0], "ghost": ms[1], "fused": ms[2], "span": ms[3], "sampled": int(ms[4]),
            "stencil": ms[5], "collide": ms[6]}


def lbm3_observe(h, what, rho_out=None, phi_out=None, f_out=None, g_out=None, check=True):
    o = lbm3_obs()
    st = lib().lbm3_observe(h, what, C.byref(o), _dp(rho_out), _dp(phi_out), _dp(f_out), _dp(g_out))
    if check and st not in (0, -3):
        _check(h, st)
    return st, o


def lbm3_contact_angle(h, comp, wall, exclude):
    out = np.zeros(6)
    _check(h, lib().lbm3_contact_angle(h, comp, wall, exclude, _dp(out)))
    return out


def lbm3_destroy(h):
    return lib().lbm3_destroy(h)


class Sim:
    """One simulation on a CUDA (HIP) device: owns a torch workspace and uses
    the current torch stream.  Arrays are (ny, nx) or (nz, ny, nx)."""

    def __init__(self, p, device="cuda:0", stream=None):
        import torch
        self.p = p
        self.D = 2 if p.lattice == D2Q9 else 3
        self.Q = p.lattice
        self.shape = (p.n[1], p.n[0]) if self.D == 2 else (p.n[2], p.n[1], p.n[0])
        self.N = int(np.prod(self.shape))
        nbytes = lbm3_footprint(p)
        if nbytes == 0:
            raise Lbm3Error(-1, "invalid parameters")
        self.device = torch.device(device)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = lbm3_create(p, self.ws.data_ptr(), nbytes, self.stream.cuda_stream)
        self.derived = lbm3_resolve(p)

    def close(self):
        if getattr(self, "h", None):
            lbm3_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, rho0, phi0):
        lbm3_init(self.h, rho0, phi0)

    def step(self, n=1):
        lbm3_step(self.h, n)

    def step_profiled(self, n, sample_every=1):
        return lbm3_step_profiled(self.h, n, sample_every)

    def observe(self):
        st, o = lbm3_observe(self.h, OBS_SUMS)
        return {"mass": list(o.mass), "rho_sum": o.rho_sum, "phi_sum": o.phi_sum,
                "mom": list(o.mom), "kinetic": o.kinetic, "umax": o.umax, "n_bad": o.n_bad,
                "n_newton": o.n_newton, "n_shortcut": o.n_shortcut, "n_fallback": o.n_fallback,
                "n_fast": o.n_fast, "step": o.step, "status": st}

    def fields(self):
        r = np.empty(self.N)
        ph = np.empty(self.N)
        lbm3_observe(self.h, OBS_FIELDS, rho_out=r, phi_out=ph)
        return r.reshape(self.shape), ph.reshape(self.shape)

    def pops(self):
        f = np.empty(self.Q * self.N)
        g = np.empty(self.Q * self.N)
        lbm3_observe(self.h, OBS_POPS, f_out=f, g_out=g)
        return f.reshape((self.Q,) + self.shape), g.reshape((self.Q,) + self.shape)

    def contact_angle(self, comp=2, wall=0, exclude=8.0):
        return lbm3_contact_angle(self.h, comp, wall, exclude)


def _obs_dict(o):
    return {"mass": list(o.mass), "rho_sum": o.rho_sum, "phi_sum": o.phi_sum, "mom": list(o.mom),
            "kinetic": o.kinetic, "umax": o.umax, "n_bad": o.n_bad, "n_newton": o.n_newton,
            "n_shortcut": o.n_shortcut, "n_fallback": o.n_fallback, "step": o.step, "n_fast": o.n_fast}


def step_batch(sims, nsteps, stream=None):
    """Advance the Sim objects `sims` (same device) by nsteps each with
    batched launches (lbm3_step_batch) on `stream` (default: the first
    simulation's stream)."""
    import torch
    n = len(sims)
    hs = (C.c_void_p * n)(*[s.h for s in sims])
    nb = C.c_size_t()
    st = lib().lbm3_batch_workspace(hs, n, C.byref(nb))
    if st != 0:
        raise Lbm3Error(st, "bad batch")
    ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=sims[0].device)
    base = (ws.data_ptr() + 255) & ~255
    stream = stream if stream is not None else sims[0].stream
    st = lib().lbm3_step_batch(hs, n, int(nsteps), C.c_void_p(stream.cuda_stream), C.c_void_p(base), nb.value)
    if st != 0:
        raise Lbm3Error(st, "batched step failed")
    return ws  # keep alive until the work is done


def step_batch_static(sims, nsteps, stream=None):
    """As step_batch, with the descriptor image in the library's static device
    array (lbm3_step_batch_static): no workspace is allocated."""
    n = len(sims)
    hs = (C.c_void_p * n)(*[s.h for s in sims])
    stream = stream if stream is not None else sims[0].stream
    st = lib().lbm3_step_batch_static(hs, n, int(nsteps), C.c_void_p(stream.cuda_stream))
    if st != 0:
        raise Lbm3Error(st, lib().lbm3_last_error(hs[0]).decode())


STEP_BATCH_STATIC_MAX_BYTES = 8 << 20  # LBM3_STEP_BATCH_STATIC_MAX_BYTES of include/lbm3.h


def server_request_bytes(p):
    return lib().lbm3_server_request_bytes(C.byref(p))


class Server:
    """Continuous-batching request loop (lbm3_server_*) over a device pool of
    pool_bytes held in a torch tensor, on the current (or given) stream."""

    def __init__(self, pool_bytes, device="cuda:0", max_resident=64, max_skips=4, stream=None):
        import torch
        self.device = torch.device(device)
        self.pool = torch.empty(int(pool_bytes) + 256, dtype=torch.uint8, device=self.device)
        base = (self.pool.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        st = lib().lbm3_server_create(C.c_void_p(base), int(pool_bytes), C.c_void_p(self.stream.cuda_stream),
                                      int(max_resident), int(max_skips), C.byref(h))
        if st != 0:
            raise Lbm3Error(st, "server create failed")
        self.h = h
        self.shapes = {}

    def submit(self, p, rho0, phi0, nsteps, tag, keep_fields=False):
        r = np.ascontiguousarray(rho0, dtype=np.float64).reshape(-1)
        ph = np.ascontiguousarray(phi0, dtype=np.float64).reshape(-1)
        self.shapes[int(tag)] = np.shape(rho0)
        st = lib().lbm3_server_submit(self.h, C.byref(p), _dp(r), _dp(ph), int(nsteps), int(tag),
                                      SERVE_FIELDS if keep_fields else 0)
        if st != 0:
            raise Lbm3Error(st, "submit failed")

    def run(self, quantum):
        nr, nq = C.c_int32(), C.c_int32()
        st = lib().lbm3_server_run(self.h, int(quantum), C.byref(nr), C.byref(nq))
        if st != 0:
            raise Lbm3Error(st, "server round failed")
        return nr.value, nq.value

    def poll(self):
        out = []
        r = lbm3_result()
        while lib().lbm3_server_poll(self.h, C.byref(r)) == 1:
            out.append({"tag": r.tag, "status": r.status, "has_fields": bool(r.has_fields), "steps": r.steps,
                        "nodes": r.nodes, "t_submit": r.t_submit, "t_admit": r.t_admit, "t_done": r.t_done,
                        "bytes": r.bytes, "obs": _obs_dict(r.obs)})
        return out

    def fields(self, tag):
        shape = self.shapes[int(tag)]
        rho = np.empty(shape)
        phi = np.empty(shape)
        st = lib().lbm3_server_fields(self.h, int(tag), _dp(rho), _dp(phi))
        if st != 0:
            raise Lbm3Error(st, "no kept fields for tag %d" % tag)
        return rho, phi

    def clock(self):
        return lib().lbm3_server_clock(self.h)

    def close(self):
        if getattr(self, "h", None):
            lib().lbm3_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
