/*
 * lbm3_oracle.h -- plain FP64 CPU oracle for the ternary free-energy lattice
 * Boltzmann update with wetting walls (Bala, Pepona, Karlin, Kusumaatmaja,
 * Semprebon, arXiv:1904.06881).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no source,
 * header, table or helper with the GPU library; neither includes the other.
 *
 * Conventions
 *   - D = 2 (D2Q9) or 3 (D3Q27).  Velocities c_i are all of {-1,0,1}^D in
 *     lexicographic order with the x component most significant, so the rest
 *     population is i = (Q-1)/2 and the opposite of i is Q-1-i.
 *   - Node index n = x + nx*(y + ny*z).  Population i of node n lives at
 *     i*N + n (N = nx*ny*nz).
 *   - Walls (when enabled) sit on the last axis (y in 2D, z in 3D): index 0
 *     and n-1 of that axis are solid ghost layers that hold rho and phi only;
 *     the wall planes are half way between a ghost layer and the first fluid
 *     layer (paper Sec. IV).  Every other axis is periodic.
 *   - Component indices follow the paper: 1 = gas, 2 and 3 = liquids,
 *     phi = chi (C2 - C3) (paper Sec. II A).
 */
#ifndef LBM3_ORACLE_H
#define LBM3_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_FORCE = 0, OR_GEOM_INTERP = 1, OR_GEOM_EXTRAP = 2 };

typedef struct {
    int    D;              /* 2 or 3 */
    int    n[3];           /* nx, ny, nz (nz = 1 for D = 2) */
    int    walls;          /* 1: ghost/solid layers at both ends of the last axis */
    /* Carnahan-Starling constants (R = 1) after the coexistence solve */
    double a, b, T, C, psi0, rho_l, rho_g;
    double lambda[3], kappa[3];   /* [0] component 1 (gas), [1] comp. 2, [2] comp. 3 */
    double chi, beta, tau_g, Gamma;
    int    wetting;        /* OR_FORCE, OR_GEOM_INTERP, OR_GEOM_EXTRAP */
    double theta_deg[2][3];/* per wall (0 low, 1 high): theta21, theta31, theta23 */
    double kw[2][2];       /* per wall: kappa_rho^w, kappa_phi^w (force method) */
    double alpha_eps;      /* alpha = 2 shortcut when max|Delta_i/f'_i| < alpha_eps */
    double alpha_tol;      /* Newton stop on |d alpha| */
    int    alpha_maxit;
    int    no_collide;     /* 1: streaming and bounce-back only */
    int    force_alpha2;   /* 1: alpha = 2 everywhere (plain BGK with 1/tau = 2 beta) */
    double detect_ratio;   /* first interface-detection rule (Sec. IV B): the 2-3 interface
                              when |grad rho| chi < detect_ratio drho |grad phi| (0: 0.01) */
    int    wall_par;       /* first-layer tangential derivatives of the force: 0 in-layer
                              central differences, 1 the bulk stencil with the links that
                              point into the wall mirrored to the fluid side (Sec. IV) */
} or_params;

typedef struct or_state or_state;

/* Observables of the current (pre-collision) state.  Sums run over fluid
 * nodes only and use compensated FP64 summation. */
typedef struct {
    double mass[3];        /* sum of C1, C2, C3 */
    double rho_sum, phi_sum;
    double mom[3];         /* sum of rho u (bare velocity) */
    double kinetic;        /* sum of rho |u|^2 / 2 */
    double umax;           /* max |u| */
    int64_t n_bad;         /* nodes with rho <= 0 or a non-finite field */
    int64_t n_newton, n_shortcut, n_fallback;  /* alpha statistics since init */
    int64_t step;
    int64_t n_fast;        /* collisions since init with |u + du| >= 1 (du = F/rho) */
} or_obs;

/* --- thermodynamics ------------------------------------------------------ */
/* Carnahan-Starling free energy density Psi and its derivative (Eqs. 4, 15),
 * R = 1, including the linear constant C. */
double or_psi (double rho, double a, double b, double T, double C);
double or_dpsi(double rho, double a, double b, double T, double C);
/* Maxwell coexistence of the CS EOS at the reference constants a0, b0:
 * finds T such that rho_l/rho_g = ratio, then rescales (a, b) at fixed a/b so
 * that the liquid density equals rho_l_target, and sets C and Psi0 so that
 * Psi(rho_g) = Psi(rho_l) = Psi0 with zero slope at both (Sec. II A).
 * Returns 0 on success. */
int or_coexistence(double a0, double b0, double ratio, double rho_l_target,
                   double *a, double *b, double *T, double *C, double *psi0,
                   double *rho_l, double *rho_g);
/* Critical temperature of the CS EOS for given a, b (R = 1). */
double or_critical_T(double a, double b);

/* --- lattice pieces used by the pins ----------------------------------- */
int  or_lattice(int D, int *c /* Q*3 */, double *w /* Q */);
void or_feq(int D, double rho, const double *u, double *feq);            /* Eq. 25-27 */
void or_geq(int D, double phi, double mu_phi, double Gamma, const double *v,
            double *geq);                                              /* Eq. 34-35 */
/* Entropic alpha for the mirror state fp and direction delta (Eq. 30-32).
 * Returns the kind: 0 shortcut, 1 Newton root, 2 fallback. */
int  or_alpha(int Q, const double *w, const double *fp, const double *delta,
              double eps, double tol, int maxit, double *alpha);
/* Local thermodynamic quantities at one node (Eqs. 11-20, with the signs of
 * the derivation from the free energy). out: mu_rho, mu_phi, P_ab (3x3,
 * row-major). */
void or_local_thermo(const or_params *p, double rho, double phi,
                     const double *grad_rho, const double *grad_phi,
                     double lap_rho, double lap_phi, double *mu_rho,
                     double *mu_phi, double *P);
/* Ghost value of one field by geometric interpolation from the first fluid
 * layer (Eqs. 47-49); exposed for the linear-field pins.  q is the first fluid
 * layer (nx x ny plane, x fastest; ny = 1 in 2D); (i, j) the ghost position;
 * (lx, ly) the interpolation point offset. */
double or_interp2d(const double *q, int nx, int i, double l);
double or_interp3d(const double *q, int nx, int ny, int i, int j, double lx,
                   double ly);

/* --- simulation ---------------------------------------------------------- */
or_state *or_create(const or_params *p);
void      or_destroy(or_state *s);
/* rho0, phi0: full grid including ghost layers (ghost entries are ignored). */
int       or_init(or_state *s, const double *rho0, const double *phi0);
/* Set populations directly (Q*N each); used by the streaming pins. */
int       or_set_pops(or_state *s, const double *f, const double *g);
int       or_step(or_state *s, int64_t nsteps);
/* Copies of the state: rho/phi on the full grid (ghost layers of the current
 * fields),
 * f/g populations (Q*N).  Any pointer may be NULL. */
void      or_get(const or_state *s, double *rho, double *phi, double *f,
                 double *g);
/* Per-node intermediate fields of the most recent step (or of init):
 * which = 0 mu_rho, 1 mu_phi, 2..4 F_x..F_z, 5..7 grad rho, 8..10 grad phi,
 * 11 lap rho, 12 lap phi, 13 alpha. */
void      or_get_field(const or_state *s, int which, double *out);
void      or_observe(const or_state *s, or_obs *o);
int       or_Q(const or_state *s);
int64_t   or_N(const or_state *s);

/* --- calibration --------------------------------------------------------- */
/* Flat interface between two bulk phases relaxed on a 1D lattice of n nodes
 * (spacing 1, fixed bulk values at both ends, interface pinned by holding
 * rho (liquid-gas) or phi (2-3) at the centre node at its mean bulk value)
 * by gradient flow of the
 * free energy; returns its surface tension and, if width != NULL, the 10-90 %
 * width of C1 (liquid-gas pairs) or C2 (pair 23).  pair = 12, 13 or 23. */
double or_flat_tension(const or_params *p, int pair, int n, double *width,
                       double *rho_out, double *phi_out);

/* --- timing ------------------------------------------------------------ */
/* OpenMP threads used by the passes (the results do not depend on it). */
void or_set_threads(int n);
int  or_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
