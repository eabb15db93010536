/*
 * lbm3.h -- C ABI of the MI355X (gfx950) library for the per-timestep update
 * of the ternary high-density-ratio free-energy lattice Boltzmann model with
 * wetting walls (Bala, Pepona, Karlin, Kusumaatmaja, Semprebon,
 * arXiv:1904.06881).
 *
 * One step (Sec. II C and Sec. IV of the paper):
 *   moments rho, phi from the two population sets (density f: entropic
 *   ELBM; phase field g: LBGK) -> ghost layers of the walls (force method
 *   copy, or geometric interpolation / extrapolation toward the prescribed
 *   contact angle) -> isotropic gradient and Laplacian stencils -> chemical
 *   potentials and pressure tensor of the free energy -> interfacial force
 *   F = div(rho c_s^2 I - P) -> entropic collision with exact-difference
 *   forcing for f, LBGK for g -> streaming with halfway bounce-back.
 *
 * Conventions shared by every entry point
 *   - Lattice D2Q9 (2D) or D3Q27 (3D); velocities are {-1,0,1}^D in
 *     lexicographic order, x component most significant: population index
 *     i = sum_a (c_ia + 1) 3^(D-1-a); rest population (Q-1)/2; opposite
 *     Q-1-i.  Weights are products of 2/3 (c = 0) and 1/6 (c = +-1).
 *   - Grid n[0] x n[1] x n[2] (n[2] = 1 in 2D), node index
 *     x + n[0] (y + n[1] z).  Host arrays of fields are FP64 in that order;
 *     host arrays of populations are FP64 [Q][N].
 *   - Walls (walls = 1) sit on the last axis (y in 2D, z in 3D): indices 0
 *     and n-1 of that axis are ghost (solid) layers holding rho and phi only,
 *     the wall planes are half way to the first fluid layer.  Every other
 *     axis is periodic.  walls = 0: fully periodic.
 *   - Components follow the paper: 1 gas, 2 and 3 liquids, phi = chi (C2-C3).
 *   - Device memory: the caller allocates one workspace of lbm3_footprint()
 *     bytes (e.g. a PyTorch uint8 tensor) and owns it; the handle only
 *     sub-allocates from it and never calls the device allocator.  All
 *     device work is enqueued on the caller's HIP stream.
 *   - Errors: every call returns an lbm3_status; no exception crosses the
 *     ABI; lbm3_last_error() gives a message for the last failure on a
 *     handle (or of the last failed create when passed NULL).
 *   - Threading: one handle per stream; calls on one handle must not overlap.
 */
#ifndef LBM3_H
#define LBM3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm3 lbm3;

typedef enum {
    LBM3_OK = 0,
    LBM3_EINVAL = -1,    /* bad shape or parameter */
    LBM3_ENOMEM = -2,    /* workspace smaller than lbm3_footprint() */
    LBM3_EUNSTABLE = -3, /* observe found NaN / rho <= 0, or |u + du| >= 1 */
    LBM3_EDEVICE = -4,   /* HIP runtime error */
    LBM3_ESTATE = -5,    /* e.g. step before init */
    LBM3_ECALIB = -6     /* (gamma, width) -> (lambda, kappa) map failed */
} lbm3_status;

enum { LBM3_D2Q9 = 9, LBM3_D3Q27 = 27 };
enum { LBM3_WET_FORCE = 0, LBM3_WET_GEOM_INTERP = 1, LBM3_WET_GEOM_EXTRAP = 2 };
enum { LBM3_FP64 = 0, LBM3_FP32 = 1, LBM3_FP16S = 2 };
enum {
    LBM3_NO_COLLIDE = 1u,   /* streaming and bounce-back only */
    LBM3_FORCE_ALPHA2 = 2u, /* alpha = 2 everywhere (BGK with 1/tau_f = 2 beta) */
    LBM3_FUSED_3D = 4u,     /* D3Q27: force, collision and streaming in one fused
                               kernel instead of the default stencil pass plus
                               collide kernel (same arithmetic) */
    LBM3_STORED_G = 8u      /* D3Q27 with tau_g = 1: store and stream the 27 g
                               populations instead of the default implicit g
                               (the collision keeps (a, phi, v) of g^eq per
                               node, Eqs. 33-35, in the compute type, and the
                               moments pass rebuilds the streamed g from them);
                               bit-identical results in FP32 and FP64 (with
                               FP16 storage the implicit g is not rounded) */
};

/* Problem statement (paper Sec. II-IV).  Zero-initialise, then set. */
typedef struct {
    int32_t lattice;        /* LBM3_D2Q9 or LBM3_D3Q27 */
    int32_t n[3];           /* nx, ny, nz (nz = 1 for D2Q9); >= 3 on the wall axis;
                               nx ny nz times 8 bytes (FP64) or 4 bytes (FP32,
                               FP16S) below 4 GiB, else LBM3_EINVAL */
    int32_t walls;          /* 1: walls at both ends of the last axis; 0: periodic */
    double  rho_l, rho_g;   /* coexistence densities (Carnahan-Starling, Sec. II A):
                               the temperature follows from rho_l/rho_g at the
                               paper's a/b = 0.185, rescaled to this rho_l */
    int32_t native;         /* 1: use lambda/kappa; 0: derive them from the
                               tensions and the interface width */
    double  lambda[3], kappa[3];            /* free energy, Eqs. 2-3 */
    double  gamma12, gamma13, gamma23;      /* target tensions (native = 0) */
    double  width;          /* 10-90 % interface width, 4 alpha23 (native = 0) */
    double  chi;            /* phi scale (paper: 5) */
    double  tau_f;          /* ELBM: beta = 1/(2 tau_f), nu = (tau_f - 1/2)/3 */
    double  tau_g;          /* LBGK relaxation time of g */
    double  Gamma;          /* mobility M = Gamma (tau_g - 1/2) */
    int32_t wetting;        /* LBM3_WET_* */
    double  theta_deg[2][3];/* per wall (0: index 0, 1: index n-1): theta21,
                               theta31, theta23, degrees, measured in the
                               liquid (liquid 2 at the 2-3 interface), Sec. IV */
    double  kw[2][2];       /* per wall: kappa_rho^w, kappa_phi^w (force method) */
    int32_t precision;      /* LBM3_FP64, LBM3_FP32, LBM3_FP16S (FP32 arithmetic,
                               populations stored in FP16 as density-scaled
                               offsets from the lattice weights) */
    uint32_t flags;         /* LBM3_NO_COLLIDE | LBM3_FORCE_ALPHA2 | LBM3_FUSED_3D |
                               LBM3_STORED_G */
    double  alpha_eps;      /* small-deviation alpha below this max |Delta/f'|
                               (0: 1e-3 FP64, 1e-2 FP32 arithmetic) */
    double  alpha_tol;      /* Newton tolerance (0: 1e-10 FP64, 1e-5 FP32) */
    int32_t alpha_maxit;    /* Newton iteration cap (0: 20) */
    double  detect_ratio;   /* geometric wetting, interface detection (Sec. IV B):
                               a wall node is on the 2-3 interface when
                               |grad_par rho| chi < detect_ratio (rho_l - rho_g)
                               |grad_par phi| (0: the paper's 0.01) */
} lbm3_params;

/* Values the library derives from lbm3_params (lbm3_resolve). */
typedef struct {
    double a, b, T, C, psi0;   /* Carnahan-Starling constants, R = 1 */
    double rho_l, rho_g;
    double lambda[3], kappa[3];
    double kappa_rr, kappa_pp, kappa_x;   /* gradient mixing coefficients */
    double beta, cot_theta[2][3];
} lbm3_derived;

/* Observables of the current state (sums over fluid nodes, FP64). */
typedef struct {
    double  mass[3];        /* sum of C1, C2, C3 */
    double  rho_sum, phi_sum;
    double  mom[3];         /* sum of rho u (bare velocity) */
    double  kinetic;        /* sum of rho |u|^2 / 2 */
    double  umax;           /* max |u| */
    int64_t n_bad;          /* nodes with rho <= 0 or non-finite fields */
    int64_t n_newton, n_shortcut, n_fallback; /* entropic alpha kinds since init */
    int64_t step;
    int64_t n_fast;         /* collisions since init whose velocity u + du had
                               |u + du| >= 1 (u the bare velocity, du = F/rho) */
} lbm3_obs;

enum { LBM3_OBS_SUMS = 1u, LBM3_OBS_FIELDS = 2u, LBM3_OBS_POPS = 4u };

/* Bytes of device workspace a handle with these parameters needs; 0 when
 * the parameters are invalid. */
size_t lbm3_footprint(const lbm3_params *p);

/* Derive the thermodynamic constants and (native = 0) lambda, kappa from the
 * tensions and width.  Host only.  LBM3_EINVAL / LBM3_ECALIB on failure. */
lbm3_status lbm3_resolve(const lbm3_params *p, lbm3_derived *out);

/* Create a handle.  dev_workspace: device pointer to >= lbm3_footprint(p)
 * bytes, 256-byte aligned, owned by the caller and kept alive until
 * lbm3_destroy; hip_stream: a hipStream_t (NULL = default stream).  The
 * parameters are copied. */
lbm3_status lbm3_create(const lbm3_params *p, void *dev_workspace, size_t bytes,
                        void *hip_stream, lbm3 **out);

/* Initial state from host FP64 fields of the full grid (ghost entries are
 * ignored): f = f^eq(rho0, 0) = w rho0; g = g^eq(phi0, mu_phi, 0) with
 * mu_phi from the ghost fill and stencils of the initial fields.  Copies the
 * arrays and returns after the upload has been enqueued and completed. */
lbm3_status lbm3_init(lbm3 *h, const double *rho0, const double *phi0);

/* Enqueue nsteps full updates on the handle's stream (asynchronous). */
lbm3_status lbm3_step(lbm3 *h, int64_t nsteps);

/* As lbm3_step, with HIP events recorded by the kernels of every
 * sample_every-th step (>= 1; LBM3_EINVAL otherwise) from their own dispatch
 * packets (start of a stage's first kernel, end of its last), so that no
 * marker packet enters the stream; synchronises.  kernel_ms (host, 8
 * doubles, may be NULL) receives [0..2] the mean device time per step of the
 * three stages over the sampled steps: moments, ghost layers, and force +
 * collision + streaming (the fused kernel, or in 3D the stencil pass plus
 * the collide kernel, from the first one's start to the second one's end);
 * the ghost-layer entry is 0 in 2D, where the fused kernel fills the ghost
 * layers itself; [3] the time from before the first to after the last step,
 * [4] the number of sampled steps, [5] and [6] the mean time of the stencil
 * pass and of the collide kernel alone (3D two-kernel step; 0 otherwise),
 * [7] 0. */
lbm3_status lbm3_step_profiled(lbm3 *h, int64_t nsteps, int32_t sample_every, double *kernel_ms);

/* Synchronise the stream and report the current state.  what: LBM3_OBS_*
 * bits.  out may be NULL unless LBM3_OBS_SUMS is set.  rho_out/phi_out
 * (N doubles, full grid, ghost layers as last filled) with LBM3_OBS_FIELDS;
 * f_out/g_out (Q*N doubles, [Q][N]) with LBM3_OBS_POPS.  Returns
 * LBM3_EUNSTABLE when the sums found NaN or rho <= 0, or a collision since
 * init had |u + du| >= 1 (n_fast). */
lbm3_status lbm3_observe(lbm3 *h, uint32_t what, lbm3_obs *out, double *rho_out,
                         double *phi_out, double *f_out, double *g_out);

/* Contact angle of the concentration C_k (k = 2 or 3) against wall w (0 or
 * 1): FP64 least-squares circle (2D) / sphere (3D) through the C_k = 1/2
 * iso-points on grid lines more than `exclude` lattice units from the wall
 * plane; theta = arccos(-h/R) with h the centre height over the wall plane
 * measured into the fluid.  out[0] = theta (degrees), out[1..3] = centre
 * (x, y[, z]) , out[4] = radius, out[5] = number of points.  Synchronises the
 * stream. */
lbm3_status lbm3_contact_angle(lbm3 *h, int32_t comp, int32_t wall, double exclude,
                               double *out);

lbm3_status lbm3_destroy(lbm3 *h);
const char *lbm3_last_error(const lbm3 *h);

/* ---------------------------------------------------- batched stepping ---
 * Many simulations advanced in lockstep, every step of all of them one
 * launch per kernel class (moments, 3D ghost layers, fused update per tile
 * class and precision), blocks mapped to simulations through a device table.
 * Each simulation's arithmetic is that of lbm3_step on it alone, so results
 * are bitwise the same alone and in any batch.  This serves many small grids
 * that cannot fill the GPU one at a time (Sec. IV's update, batched). */

/* Device bytes of the descriptor image lbm3_step_batch needs for hs[0..n-1]
 * (*bytes; LBM3_EINVAL for a null, uninitialised or repeated handle). */
lbm3_status lbm3_batch_workspace(lbm3 *const *hs, int32_t n, size_t *bytes);

/* Advance hs[0..n-1] by nsteps each on `stream` (a hipStream_t; every
 * handle's own work must already be ordered before it, e.g. created on the
 * same stream).  ws: device memory of at least lbm3_batch_workspace() bytes,
 * 256-byte aligned, caller-owned and not reused until the steps are done.
 * Uploads the image (synchronising the stream once) and enqueues the steps.
 * LBM3_EINVAL on bad handles, LBM3_ENOMEM for a short workspace,
 * LBM3_EDEVICE on a failed launch. */
lbm3_status lbm3_step_batch(lbm3 *const *hs, int32_t n, int64_t nsteps, void *stream, void *ws,
                            size_t ws_bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * lbm3_step_batch, but the descriptor image goes into a static device array
 * of the library (LBM3_STEP_BATCH_STATIC_MAX_BYTES, 8 MiB, one per GPU,
 * held until the process ends) instead of a caller workspace; no device or
 * host-pinned memory is allocated.  Uses the array of the device
 * current at the call (the handles' device).  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (other threads or
 * streams) race and must be serialised by the caller.  LBM3_EINVAL when the
 * image (lbm3_batch_workspace) exceeds the array or on bad handles,
 * LBM3_EDEVICE on a failed copy or launch. */
#define LBM3_STEP_BATCH_STATIC_MAX_BYTES ((size_t)8 << 20)
lbm3_status lbm3_step_batch_static(lbm3 *const *hs, int32_t n, int64_t nsteps, void *stream);

/* ------------------------------------------------------------- serving ---
 * Continuous batching: requests (parameters, initial fields, step count)
 * queue on the host.  Resident simulations are split by size into lanes
 * (below and from 2^18 nodes), each with its own stream, batch tables and
 * rounds, so small grids are not held to the step time of large ones and the
 * lanes overlap on the GPU.  A lane's round retires its finished
 * simulations, admits queued ones of its size first-come first-served while
 * their device footprint fits the shared pool and, in the large lane, while
 * the lane holds at most 2^23 nodes (one grid is always admitted; larger
 * grids fill the GPU alone) -- later requests may pass one that does not
 * fit, until it has waited max_skips rounds -- and enqueues up
 * to `quantum` batched steps of everything resident in it.  Tension
 * calibration (lbm3_resolve) runs on host worker threads from submission
 * on, while the GPU steps the resident simulations. */
typedef struct lbm3_server lbm3_server;

typedef struct {
    uint64_t tag;           /* the request's tag */
    int32_t  status;        /* LBM3_OK, or why the request failed */
    int32_t  has_fields;    /* final rho, phi kept for lbm3_server_fields */
    int64_t  steps;         /* steps taken */
    int64_t  nodes;         /* lattice nodes of the request */
    double   t_submit, t_admit, t_done;  /* seconds on lbm3_server_clock */
    double   bytes;         /* pool bytes held while resident */
    lbm3_obs obs;           /* observables of the final state */
} lbm3_result;

enum { LBM3_SERVE_FIELDS = 1u };  /* keep the final rho, phi (host copy) */

/* Pool bytes a request with these parameters holds while resident (its
 * lbm3_footprint plus its share of the batch tables); 0 if invalid. */
size_t lbm3_server_request_bytes(const lbm3_params *p);

/* pool: device memory (>= 4 MiB), 256-byte aligned, owned by the caller and
 * used only by the server until lbm3_server_destroy returns; the server's
 * lane streams (default priority) start after the work enqueued on `stream`
 * (a hipStream_t) before this call; max_resident >= 1 simulations at once
 * over all lanes; max_skips >= 0. */
lbm3_status lbm3_server_create(void *pool, size_t pool_bytes, void *stream, int32_t max_resident,
                               int32_t max_skips, lbm3_server **out);

/* Queue a request; rho0, phi0 (host, n[0] n[1] n[2] doubles each, x fastest)
 * are copied.  Parameter failures or a footprint beyond the pool come back
 * at once as a result with that status (the call itself returns LBM3_OK);
 * LBM3_EINVAL only for null arguments or nsteps < 0.  The calibration of
 * (lambda, kappa) from the tensions (lbm3_resolve) runs on the server's
 * worker threads, overlapped with the GPU work; a request is admitted once
 * it is calibrated (requests still calibrating may be overtaken), and a
 * calibration failure comes back as a result with LBM3_ECALIB. */
lbm3_status lbm3_server_submit(lbm3_server *s, const lbm3_params *p, const double *rho0, const double *phi0,
                               int64_t nsteps, uint64_t tag, uint32_t flags);

/* One round of every lane whose previous round has finished (blocking only
 * while every lane with work is still busy).  n_resident, n_queued (may be
 * NULL): simulations on the device / waiting. */
lbm3_status lbm3_server_run(lbm3_server *s, int64_t quantum, int32_t *n_resident, int32_t *n_queued);

/* Pop the oldest finished result into *out: 1 if one was returned, 0 if none,
 * negative lbm3_status on bad arguments. */
int32_t lbm3_server_poll(lbm3_server *s, lbm3_result *out);

/* Copy the kept final fields of result `tag` (n doubles each, may be NULL)
 * and release them.  LBM3_EINVAL when none are kept for that tag. */
lbm3_status lbm3_server_fields(lbm3_server *s, uint64_t tag, double *rho_out, double *phi_out);

/* Seconds since the server was created (the clock of lbm3_result). */
double lbm3_server_clock(const lbm3_server *s);

/* Wait for in-flight work, release every simulation and the server. */
lbm3_status lbm3_server_destroy(lbm3_server *s);

#ifdef __cplusplus
}
#endif
#endif /* LBM3_H */
