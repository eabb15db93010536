/*
 * lbm3_oracle.c -- plain FP64 CPU oracle of the per-timestep update of the
 * ternary high-density-ratio free-energy lattice Boltzmann model with wetting
 * walls (arXiv:1904.06881).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline leg of the benchmark; never by the product library.
 *
 * The update is written as a sequence of whole-grid passes in the order the
 * paper describes (Sec. II C and Sec. IV): moments, ghost layer, stencils,
 * chemical potentials, pressure tensor, force, collisions, streaming with
 * bounce-back.  Every pass is a plain loop over nodes.  No blocking, fusion
 * or reordering; clarity over speed.
 *
 * Readings of the paper where it is silent, ambiguous or inconsistent are
 * marked "reading:" at the place they apply.
 *
 * The first-fluid-layer wall rule of the force (pass_force) is pinned by its
 * symmetry (force method without wall force equals the geometric method at
 * 90 degrees, bit for bit) and by the contact angles geometric wetting sets
 * on liquid drops in gas (the CPU pins); nothing else pins it.
 */
#include "lbm3_oracle.h"

#include <float.h>
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define MAXQ 27

struct or_state {
    or_params p;
    int Q, rest;
    int c[MAXQ][3];
    double w[MAXQ];
    int64_t N;
    double *f, *g;            /* pre-collision populations, Q*N */
    double *fs, *gs;          /* post-collision populations, Q*N */
    double *rho, *phi;        /* moments; ghost layers hold the wall values */
    double *u[3];             /* bare velocity sum f c / rho */
    double *grho[3], *gphi[3], *lrho, *lphi;
    double *mur, *mup;
    double *Tt[3][3];         /* -P on fluid nodes */
    double *F[3];
    double *alpha;
    int64_t step;
    int64_t n_newton, n_shortcut, n_fallback;
    int64_t n_fast;           /* collisions with |u + du| >= 1 */
};

/* ------------------------------------------------------------------------ */
/* Lattice: D2Q9 / D3Q27 as the tensor product of D1Q3 with weights 2/3 and
 * 1/6 (Sec. II C, product-form equilibrium). */
int or_lattice(int D, int *c, double *w)
{
    int Q = (D == 2) ? 9 : 27;
    for (int i = 0; i < Q; ++i) {
        int cc[3] = {0, 0, 0};
        int r = i;
        for (int a = D - 1; a >= 0; --a) { cc[a] = (r % 3) - 1; r /= 3; }
        double wi = 1.0;
        for (int a = 0; a < D; ++a) wi *= (cc[a] == 0) ? 2.0 / 3.0 : 1.0 / 6.0;
        for (int a = 0; a < 3; ++a) c[3 * i + a] = cc[a];
        w[i] = wi;
    }
    return Q;
}

/* Product-form equilibrium, Eqs. 25-27:
 * f_i^eq = rho w_i prod_a A(u_a) B(u_a)^{c_ia},
 * A(u) = 2 - sqrt(1+3u^2), B(u) = (2u + sqrt(1+3u^2)) / (1-u). */
void or_feq(int D, double rho, const double *u, double *feq)
{
    int c[MAXQ * 3];
    double w[MAXQ];
    int Q = or_lattice(D, c, w);
    double A[3], B[3];
    for (int a = 0; a < D; ++a) {
        double s = sqrt(1.0 + 3.0 * u[a] * u[a]);
        A[a] = 2.0 - s;
        B[a] = (2.0 * u[a] + s) / (1.0 - u[a]);
    }
    for (int i = 0; i < Q; ++i) {
        double v = rho * w[i];
        for (int a = 0; a < D; ++a) {
            v *= A[a];
            if (c[3 * i + a] == 1) v *= B[a];
            if (c[3 * i + a] == -1) v /= B[a];
        }
        feq[i] = v;
    }
}

/* Phase-field equilibrium, Eqs. 34-35 with c_s^2 = 1/3:
 * g_i = w_i (3 Gamma mu + 3 phi v.c + 9/2 phi (v.c)^2 - 3/2 phi |v|^2), i != 0
 * g_0 = phi - sum_{i != 0} g_i. */
void or_geq(int D, double phi, double mu_phi, double Gamma, const double *v,
            double *geq)
{
    int c[MAXQ * 3];
    double w[MAXQ];
    int Q = or_lattice(D, c, w);
    int rest = (Q - 1) / 2;
    double vv = 0.0;
    for (int a = 0; a < D; ++a) vv += v[a] * v[a];
    double sum = 0.0;
    for (int i = 0; i < Q; ++i) {
        if (i == rest) continue;
        double vc = 0.0;
        for (int a = 0; a < D; ++a) vc += v[a] * c[3 * i + a];
        geq[i] = w[i] * (3.0 * Gamma * mu_phi + 3.0 * phi * vc +
                         4.5 * phi * vc * vc - 1.5 * phi * vv);
        sum += geq[i];
    }
    geq[rest] = phi - sum;
}

/* ------------------------------------------------------------------------ */
/* Carnahan-Starling EOS, Eq. 4 and its derivative (the unnumbered formula
 * after Eq. 14), R = 1. */
double or_psi(double rho, double a, double b, double T, double C)
{
    double br = b * rho;
    return rho * (C - a * rho - 8.0 * T * (br - 6.0) / ((br - 4.0) * (br - 4.0)) +
                  T * log(rho));
}

double or_dpsi(double rho, double a, double b, double T, double C)
{
    double br = b * rho;
    double d = br - 4.0;
    return C - 2.0 * a * rho + T * (1.0 + log(rho)) + 16.0 * T * (br - 12.0) / (d * d * d);
}

/* d^2 Psi / d rho^2, used only to locate the spinodals. */
static double cs_d2psi(double rho, double a, double b, double T)
{
    double br = b * rho;
    double d = br - 4.0;
    return -2.0 * a + T / rho + 16.0 * T * b * (32.0 - 2.0 * br) / (d * d * d * d);
}

/* pressure p = rho dPsi/drho - Psi (C cancels) */
static double cs_p(double rho, double a, double b, double T)
{
    return rho * or_dpsi(rho, a, b, T, 0.0) - or_psi(rho, a, b, T, 0.0);
}

/* Spinodal densities (local max and min of dPsi/drho).  Returns 0 if the
 * isotherm is monotone (T >= Tc).  Plain scan on a log grid plus bisection. */
static int cs_spinodals(double a, double b, double T, double *ra, double *rb)
{
    double rmax = 4.0 / b;
    const int M = 20000;
    double lo = log(rmax * 1e-9), hi = log(rmax * (1.0 - 1e-9));
    double prev_r = exp(lo), prev_s = cs_d2psi(prev_r, a, b, T);
    int found = 0;
    for (int k = 1; k <= M; ++k) {
        double r = exp(lo + (hi - lo) * k / M);
        double s = cs_d2psi(r, a, b, T);
        if ((prev_s > 0.0) != (s > 0.0)) {
            double x0 = prev_r, x1 = r;
            for (int it = 0; it < 200; ++it) {
                double xm = 0.5 * (x0 + x1);
                if ((cs_d2psi(xm, a, b, T) > 0.0) == (prev_s > 0.0)) x0 = xm; else x1 = xm;
            }
            if (found == 0) *ra = 0.5 * (x0 + x1); else *rb = 0.5 * (x0 + x1);
            ++found;
            if (found == 2) return 1;
        }
        prev_r = r;
        prev_s = s;
    }
    return 0;
}

/* root of dPsi(rho) = mu0 in [lo, hi] where dPsi is increasing */
static double cs_branch_root(double a, double b, double T, double mu0, double lo, double hi)
{
    for (int it = 0; it < 300; ++it) {
        double m = 0.5 * (lo + hi);
        if (or_dpsi(m, a, b, T, 0.0) < mu0) lo = m; else hi = m;
    }
    return 0.5 * (lo + hi);
}

/* Maxwell coexistence at temperature T by bisection on the common chemical
 * potential until the two pressures agree. */
static int cs_coex_at(double a, double b, double T, double *rg, double *rl)
{
    double ra, rb;
    if (!cs_spinodals(a, b, T, &ra, &rb)) return 1;
    double rmax = 4.0 / b;
    double mlo = or_dpsi(rb, a, b, T, 0.0), mhi = or_dpsi(ra, a, b, T, 0.0);
    double g = 0, l = 0;
    for (int it = 0; it < 200; ++it) {
        double mu0 = 0.5 * (mlo + mhi);
        g = cs_branch_root(a, b, T, mu0, rmax * 1e-300, ra);
        l = cs_branch_root(a, b, T, mu0, rb, rmax * (1.0 - 1e-15));
        double dp = cs_p(l, a, b, T) - cs_p(g, a, b, T);
        if (dp > 0.0) mhi = mu0; else mlo = mu0;
    }
    *rg = g;
    *rl = l;
    return 0;
}

double or_critical_T(double a, double b)
{
    double lo = 1e-6 * a / b, hi = 2.0 * a / b, ra, rb;
    for (int it = 0; it < 200; ++it) {
        double m = 0.5 * (lo + hi);
        if (cs_spinodals(a, b, m, &ra, &rb)) lo = m; else hi = m;
    }
    return 0.5 * (lo + hi);
}

int or_coexistence(double a0, double b0, double ratio, double rho_l_target,
                   double *a, double *b, double *T, double *C, double *psi0,
                   double *rho_l, double *rho_g)
{
    if (!(ratio > 1.0) || !(rho_l_target > 0.0)) return 1;
    double Tc = or_critical_T(a0, b0);
    double lo = 0.05 * Tc, hi = Tc * (1.0 - 1e-6), rg, rl;
    if (cs_coex_at(a0, b0, lo, &rg, &rl) || rl / rg < ratio) return 2;
    for (int it = 0; it < 100; ++it) {
        double m = 0.5 * (lo + hi);
        if (cs_coex_at(a0, b0, m, &rg, &rl)) { hi = m; continue; }
        if (rl / rg > ratio) lo = m; else hi = m;
    }
    double Tm = 0.5 * (lo + hi);
    if (cs_coex_at(a0, b0, Tm, &rg, &rl)) return 3;
    /* rescale densities by s at fixed a/b and T: rho' = s rho, b' = b/s,
     * a' = a/s keeps b rho and the shape of the isotherm */
    double s = rho_l_target / rl;
    *a = a0 / s;
    *b = b0 / s;
    *T = Tm;
    *rho_l = rl * s;
    *rho_g = rg * s;
    *C = -or_dpsi(*rho_g, *a, *b, Tm, 0.0);
    *psi0 = or_psi(*rho_g, *a, *b, Tm, *C);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Local thermodynamics.  Concentrations from Eqs. 5-7; bulk chemical
 * potentials from Eqs. 11-12; gradient parts and the pressure tensor from
 * Eqs. 13-20.
 * reading: the bulk chemical potential of rho is taken as the derivative of
 * f_Bulk, (lambda2 g(C2) + lambda3 g(C3)) / Delta_rho, since dC2/drho =
 * dC3/drho = 1/(2 Delta_rho); the sign printed on the lambda2 term is not
 * that derivative.
 * reading: one cross coefficient k_x = (kappa2 - kappa3)/(4 chi Delta_rho),
 * from expanding f_Inter in (rho, phi), enters mu_rho, mu_phi and P with the
 * same sign. */
static double gfun(double x) { return x * (x - 0.5) * (x - 1.0); }

typedef struct {
    double drho, krr, kpp, kx;
} derived_k;

static derived_k derive_k(const or_params *p)
{
    derived_k d;
    d.drho = p->rho_l - p->rho_g;
    d.krr = p->kappa[0] + (p->kappa[1] + p->kappa[2]) / (4.0 * d.drho * d.drho);
    d.kpp = (p->kappa[1] + p->kappa[2]) / (4.0 * p->chi * p->chi);
    d.kx = (p->kappa[1] - p->kappa[2]) / (4.0 * p->chi * d.drho);
    return d;
}

static void bulk_terms(const or_params *p, double rho, double phi,
                       double *mur_b, double *mup_b, double *fb)
{
    double drho = p->rho_l - p->rho_g;
    double C1 = (rho - p->rho_l) / (p->rho_g - p->rho_l);
    double C2 = 0.5 * (1.0 + phi / p->chi - C1);
    double C3 = 0.5 * (1.0 - phi / p->chi - C1);
    *mur_b = 0.5 * p->lambda[0] * or_dpsi(rho, p->a, p->b, p->T, p->C) +
             (p->lambda[1] * gfun(C2) + p->lambda[2] * gfun(C3)) / drho;
    *mup_b = (p->lambda[1] * gfun(C2) - p->lambda[2] * gfun(C3)) / p->chi;
    *fb = 0.5 * p->lambda[0] * (or_psi(rho, p->a, p->b, p->T, p->C) - p->psi0) +
          0.5 * p->lambda[1] * C2 * C2 * (1.0 - C2) * (1.0 - C2) +
          0.5 * p->lambda[2] * C3 * C3 * (1.0 - C3) * (1.0 - C3);
}

void or_local_thermo(const or_params *p, double rho, double phi,
                     const double *G, const double *H, double Lr, double Lp,
                     double *mu_rho, double *mu_phi, double *P)
{
    derived_k k = derive_k(p);
    double mrb, mpb, fb;
    bulk_terms(p, rho, phi, &mrb, &mpb, &fb);
    *mu_rho = mrb - k.krr * Lr - k.kx * Lp;
    *mu_phi = mpb - k.kpp * Lp - k.kx * Lr;
    double p0 = rho * mrb + phi * mpb - fb;
    double GG = 0, HH = 0, GH = 0;
    for (int a = 0; a < p->D; ++a) {
        GG += G[a] * G[a];
        HH += H[a] * H[a];
        GH += G[a] * H[a];
    }
    double iso = p0 - k.krr * (rho * Lr + 0.5 * GG) - k.kpp * (phi * Lp + 0.5 * HH) -
                 k.kx * (rho * Lp + phi * Lr + GH);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) P[3 * a + b] = 0.0;
    for (int a = 0; a < p->D; ++a)
        for (int b = 0; b < p->D; ++b)
            P[3 * a + b] = (a == b ? iso : 0.0) + k.krr * G[a] * G[b] +
                           k.kpp * H[a] * H[b] + k.kx * (G[a] * H[b] + H[a] * G[b]);
}

/* ------------------------------------------------------------------------ */
/* Entropic alpha: non-trivial root of H(f' + alpha Delta) = H(f') with
 * H(f) = sum f ln(f/w) (Eqs. 30-32), Delta = f^eq(rho, u + du) - f'.
 * Writing x_i = Delta_i / f'_i and using that ln(f^eq_i / w_i) is linear in
 * c_i while Delta carries no mass and no momentum (sum Delta = sum Delta c = 0),
 * the equation is G(alpha) = 0 with
 *   G(alpha) = sum_i f'_i [(1 + alpha x_i) log1p(alpha x_i)
 *                          - alpha x_i (1 + log1p(x_i))],
 *   G'(alpha) = sum_i f'_i x_i [log1p(alpha x_i) - log1p(x_i)].
 * (The term alpha sum Delta, zero by conservation, is left out: kept, its
 * rounding alone would move the root by ~1e-16 / x^2.)
 * reading (the paper gives only the equation):
 *   - a non-positive mirror population: alpha = 2 (fallback);
 *   - max |x_i| < eps: the small-deviation root from expanding G about
 *     alpha = 2, alpha = 2 + (S3 - 2 S4) / (3 S2 - 4 S3), S_k = sum f' x^k
 *     (alpha = 2 when S2 = 0);
 *   - otherwise Newton from min(2, (1 + alpha_max)/2), alpha_max =
 *     min_{Delta_i<0} -f'_i/Delta_i the positivity limit; an iterate that
 *     leaves (1, alpha_max) is replaced by the midpoint towards the violated
 *     bound; stop when |step| < tol, or when a step below 10 tol fails to
 *     halve the previous one (the root is resolved to rounding); no
 *     convergence within maxit (or a non-positive slope) ->
 *     alpha = min(2, alpha_max) (fallback). */
int or_alpha(int Q, const double *w, const double *fp, const double *delta,
             double eps, double tol, int maxit, double *alpha)
{
    (void)w;
    double x[MAXQ], l1x[MAXQ];
    for (int i = 0; i < Q; ++i) {
        if (!(fp[i] > 0.0)) { *alpha = 2.0; return 2; }
    }
    double xmax = 0.0;
    for (int i = 0; i < Q; ++i) {
        x[i] = delta[i] / fp[i];
        if (fabs(x[i]) > xmax) xmax = fabs(x[i]);
    }
    if (xmax < eps) {
        double S2 = 0, S3 = 0, S4 = 0;
        for (int i = 0; i < Q; ++i) {
            double x2 = x[i] * x[i];
            S2 += fp[i] * x2;
            S3 += fp[i] * x2 * x[i];
            S4 += fp[i] * x2 * x2;
        }
        double den = 3.0 * S2 - 4.0 * S3;
        *alpha = (den > 0.0) ? 2.0 + (S3 - 2.0 * S4) / den : 2.0;
        return 0;
    }
    double amax = INFINITY;
    for (int i = 0; i < Q; ++i)
        if (delta[i] < 0.0 && -fp[i] / delta[i] < amax) amax = -fp[i] / delta[i];
    for (int i = 0; i < Q; ++i) l1x[i] = log1p(x[i]);
    double a = (2.0 < amax) ? 2.0 : 0.5 * (1.0 + amax);
    double prev = INFINITY;
    for (int it = 0; it < maxit; ++it) {
        double G = 0.0, dG = 0.0;
        for (int i = 0; i < Q; ++i) {
            double la = log1p(a * x[i]);
            G += fp[i] * ((1.0 + a * x[i]) * la - a * x[i] * (1.0 + l1x[i]));
            dG += fp[i] * x[i] * (la - l1x[i]);
        }
        if (!(dG > 0.0)) break;
        double an = a - G / dG;
        if (an >= amax) an = 0.5 * (a + amax);
        if (an <= 1.0) an = 0.5 * (a + 1.0);
        double st = fabs(an - a);
        if (st < tol || (st < 10.0 * tol && st > 0.5 * prev)) { *alpha = an; return 1; }
        prev = st;
        a = an;
    }
    *alpha = (2.0 < amax) ? 2.0 : amax;
    return 2;
}

/* ------------------------------------------------------------------------ */
/* Geometric interpolation of a ghost value, Eq. 47 (2D) and Eqs. 48-49 (3D).
 * q is the first fluid layer, periodic along its axes. */
static int wrap(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

double or_interp2d(const double *q, int nx, int i, double l)
{
    double l0 = floor(l), l1 = l0 + 1.0;
    /* integer shift: the exact lattice copy of the special-angle table */
    if (l == l0) return q[wrap(i + (int)l0, nx)];
    double q0 = q[wrap(i + (int)l0, nx)];
    double q1 = q[wrap(i + (int)l1, nx)];
    return (q1 - q0) * l + (l1 * q0 - l0 * q1);
}

double or_interp3d(const double *q, int nx, int ny, int i, int j, double lx, double ly)
{
    double x0 = floor(lx), y0 = floor(ly);
    double fx = lx - x0, fy = ly - y0;
    static const int cx[4] = {0, 1, 0, 1}, cy[4] = {0, 0, 1, 1};
    /* reading: keep the three corners of the unit cell nearest to the point
     * (drop the farthest; first in this order on a tie), i.e. the triangle
     * that contains it. */
    int drop = 0;
    double dmax = -1.0;
    for (int k = 0; k < 4; ++k) {
        double d = (fx - cx[k]) * (fx - cx[k]) + (fy - cy[k]) * (fy - cy[k]);
        if (d > dmax) { dmax = d; drop = k; }
    }
    double X[3], Y[3], Cv[3];
    int m = 0;
    for (int k = 0; k < 4; ++k) {
        if (k == drop) continue;
        X[m] = x0 + cx[k];
        Y[m] = y0 + cy[k];
        Cv[m] = q[wrap(i + (int)X[m], nx) + (int64_t)nx * wrap(j + (int)Y[m], ny)];
        ++m;
    }
    double x1 = X[0], x2 = X[1], x3 = X[2], y1 = Y[0], y2 = Y[1], y3 = Y[2];
    double c1 = Cv[0], c2 = Cv[1], c3 = Cv[2];
    double A = y2 * c1 - y3 * c1 - y1 * c2 + y3 * c2 + y1 * c3 - y2 * c3;
    double B = -x2 * c1 + x3 * c1 + x1 * c2 - x3 * c2 - x1 * c3 + x2 * c3;
    double Cc = -x3 * y2 * c1 + x2 * y3 * c1 + x3 * y1 * c2 - x1 * y3 * c2 -
                x2 * y1 * c3 + x1 * y2 * c3;
    double Dd = -x2 * y1 + x3 * y1 + x1 * y2 - x3 * y2 - x1 * y3 + x2 * y3;
    return (A * lx + B * ly + Cc) / Dd;
}

/* ------------------------------------------------------------------------ */
static int64_t idx(const or_state *s, int x, int y, int z)
{
    return (int64_t)x + (int64_t)s->p.n[0] * ((int64_t)y + (int64_t)s->p.n[1] * z);
}

static void coords(const or_state *s, int64_t n, int *x, int *y, int *z)
{
    *x = (int)(n % s->p.n[0]);
    *y = (int)((n / s->p.n[0]) % s->p.n[1]);
    *z = (int)(n / ((int64_t)s->p.n[0] * s->p.n[1]));
}

static int wall_axis(const or_state *s) { return s->p.D - 1; }

static int is_fluid(const or_state *s, int x, int y, int z)
{
    if (!s->p.walls) return 1;
    int ax = wall_axis(s);
    int v = (ax == 1) ? y : z;
    return v >= 1 && v <= s->p.n[ax] - 2;
}

/* neighbour of (x,y,z) along c, periodic on every non-wall axis; on the wall
 * axis the coordinate is returned unwrapped (callers check it). */
static void neighbour(const or_state *s, int x, int y, int z, const int *c,
                      int *xn, int *yn, int *zn)
{
    int ax = wall_axis(s);
    int v[3] = {x + c[0], y + c[1], z + c[2]};
    for (int a = 0; a < s->p.D; ++a) {
        if (s->p.walls && a == ax) continue;
        v[a] = wrap(v[a], s->p.n[a]);
    }
    *xn = v[0];
    *yn = v[1];
    *zn = v[2];
}

static double *alloc(int64_t n)
{
    double *p = (double *)calloc((size_t)n, sizeof(double));
    return p;
}

or_state *or_create(const or_params *p)
{
    if (p->D != 2 && p->D != 3) return NULL;
    or_state *s = (or_state *)calloc(1, sizeof(or_state));
    s->p = *p;
    if (p->D == 2) s->p.n[2] = 1;
    int cc[MAXQ * 3];
    s->Q = or_lattice(p->D, cc, s->w);
    s->rest = (s->Q - 1) / 2;
    for (int i = 0; i < s->Q; ++i)
        for (int a = 0; a < 3; ++a) s->c[i][a] = cc[3 * i + a];
    s->N = (int64_t)s->p.n[0] * s->p.n[1] * s->p.n[2];
    int64_t QN = (int64_t)s->Q * s->N;
    s->f = alloc(QN);
    s->g = alloc(QN);
    s->fs = alloc(QN);
    s->gs = alloc(QN);
    s->rho = alloc(s->N);
    s->phi = alloc(s->N);
    for (int a = 0; a < 3; ++a) {
        s->u[a] = alloc(s->N);
        s->grho[a] = alloc(s->N);
        s->gphi[a] = alloc(s->N);
        s->F[a] = alloc(s->N);
        for (int b = 0; b < 3; ++b) s->Tt[a][b] = alloc(s->N);
    }
    s->lrho = alloc(s->N);
    s->lphi = alloc(s->N);
    s->mur = alloc(s->N);
    s->mup = alloc(s->N);
    s->alpha = alloc(s->N);
    return s;
}

void or_destroy(or_state *s)
{
    if (!s) return;
    free(s->f); free(s->g); free(s->fs); free(s->gs);
    free(s->rho); free(s->phi);
    for (int a = 0; a < 3; ++a) {
        free(s->u[a]); free(s->grho[a]); free(s->gphi[a]); free(s->F[a]);
        for (int b = 0; b < 3; ++b) free(s->Tt[a][b]);
    }
    free(s->lrho); free(s->lphi); free(s->mur); free(s->mup); free(s->alpha);
    free(s);
}

int or_Q(const or_state *s) { return s->Q; }
int64_t or_N(const or_state *s) { return s->N; }

/* ---- pass 1: moments (Sec. II C: rho u = sum f c, bare velocity) ------- */
static void pass_moments(or_state *s)
{
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < s->N; ++n) {
        int x, y, z;
        coords(s, n, &x, &y, &z);
        if (!is_fluid(s, x, y, z)) continue;
        double r = 0, ph = 0, j[3] = {0, 0, 0};
        for (int i = 0; i < s->Q; ++i) {
            double fi = s->f[(int64_t)i * s->N + n];
            r += fi;
            ph += s->g[(int64_t)i * s->N + n];
            for (int a = 0; a < 3; ++a) j[a] += fi * s->c[i][a];
        }
        s->rho[n] = r;
        s->phi[n] = ph;
        for (int a = 0; a < 3; ++a) s->u[a][n] = j[a] / r;
    }
}

/* ---- pass 2: ghost layers (Sec. IV) ------------------------------------ */
/* reading: interface detection is the cascade of the paper's rules in the
 * order printed, the first three exclusive (rule 1 evaluated cross-multiplied
 * as |grad rho| chi < 0.01 Delta_rho |grad phi|), then rules 4 and 5 override.
 * Returns 0 for interface 1-2 (theta21), 1 for 1-3 (theta31), 2 for 2-3
 * (theta23). */
static int classify(const or_params *p, double ngr, double ngp, double dot,
                    double r, double ph)
{
    double drho = p->rho_l - p->rho_g;
    int k;
    const double ratio = p->detect_ratio > 0.0 ? p->detect_ratio : 0.01;
    if (ngr * p->chi < ratio * drho * ngp) k = 2;
    else if (dot < 0.0) k = 1;
    else k = 0;
    if (r > 0.5 * p->rho_l && ph < -0.95 * p->chi) k = 1;
    if (r > 0.5 * p->rho_l && ph > 0.95 * p->chi) k = 0;
    return k;
}

/* cot(theta) with the special angles of the lattice-copy table exact:
 * values within 1e-9 of an integer are snapped to it. */
static double cot_deg(double deg)
{
    double t = deg * M_PI / 180.0;
    double c = cos(t) / sin(t);
    double r = nearbyint(c);
    if (fabs(c - r) < 1e-9) c = r;
    return c;
}

static void pass_ghost(or_state *s)
{
    if (!s->p.walls) return;
    const or_params *p = &s->p;
    int nx = p->n[0], ny = p->n[1], nz = p->n[2];
    int D = p->D;
    int nw = (D == 2) ? ny : nz;           /* extent of the wall axis */
    int np1 = nx, np2 = (D == 2) ? 1 : ny; /* plane extents */
    double drho = p->rho_l - p->rho_g;
    double *lr = alloc((int64_t)np1 * np2), *lp = alloc((int64_t)np1 * np2);
    for (int wall = 0; wall < 2; ++wall) {
        int kg = wall == 0 ? 0 : nw - 1;   /* ghost layer */
        int kf = wall == 0 ? 1 : nw - 2;   /* first fluid layer */
        for (int j = 0; j < np2; ++j)
            for (int i = 0; i < np1; ++i) {
                int64_t n = (D == 2) ? idx(s, i, kf, 0) : idx(s, i, j, kf);
                lr[i + (int64_t)np1 * j] = s->rho[n];
                lp[i + (int64_t)np1 * j] = s->phi[n];
            }
        for (int j = 0; j < np2; ++j)
            for (int i = 0; i < np1; ++i) {
                int64_t ng = (D == 2) ? idx(s, i, kg, 0) : idx(s, i, j, kg);
                int64_t pi = i + (int64_t)np1 * j;
                double r0 = lr[pi], p0 = lp[pi];
                if (p->wetting == OR_FORCE) {
                    /* force method: ghost = copy of the first fluid layer */
                    s->rho[ng] = r0;
                    s->phi[ng] = p0;
                    continue;
                }
                /* in-layer central gradients */
                double gr[2] = {0, 0}, gp[2] = {0, 0};
                gr[0] = 0.5 * (lr[wrap(i + 1, np1) + (int64_t)np1 * j] - lr[wrap(i - 1, np1) + (int64_t)np1 * j]);
                gp[0] = 0.5 * (lp[wrap(i + 1, np1) + (int64_t)np1 * j] - lp[wrap(i - 1, np1) + (int64_t)np1 * j]);
                if (D == 3) {
                    gr[1] = 0.5 * (lr[i + (int64_t)np1 * wrap(j + 1, np2)] - lr[i + (int64_t)np1 * wrap(j - 1, np2)]);
                    gp[1] = 0.5 * (lp[i + (int64_t)np1 * wrap(j + 1, np2)] - lp[i + (int64_t)np1 * wrap(j - 1, np2)]);
                }
                double ngr = sqrt(gr[0] * gr[0] + gr[1] * gr[1]);
                double ngp = sqrt(gp[0] * gp[0] + gp[1] * gp[1]);
                if (ngr < 1e-12 * drho && ngp < 1e-12 * drho) {
                    s->rho[ng] = r0;
                    s->phi[ng] = p0;
                    continue;
                }
                double dot = gr[0] * gp[0] + gr[1] * gp[1];
                int k = classify(p, ngr, ngp, dot, r0, p0);
                double ct = cot_deg(p->theta_deg[wall][k]);
                /* c = phi at the liquid-liquid interface, rho otherwise; it
                 * increases into the phase in which the angle is measured */
                const double *gc = (k == 2) ? gp : gr;
                double ngc = (k == 2) ? ngp : ngr;
                if (p->wetting == OR_GEOM_EXTRAP) {
                    /* Eqs. 45-46: c_ghost = c_first + grad_perp c, with
                     * grad_perp c = cot(theta) |grad_par c| toward the wall.
                     * reading: each field q gets cot(theta) (grad_par q . m),
                     * m the unit in-plane direction of grad c.
                     * reading (the extrapolation is unbounded; at density
                     * ratio 1000 and |cot theta| near 1 it can give a negative
                     * ghost density on the gas side): each value is kept
                     * within the bulk range widened to the first-layer value,
                     * rho in [min(rho_1, rho_g), max(rho_1, rho_l)], phi in
                     * [min(phi_1, -chi), max(phi_1, chi)]; inside that range
                     * it is the plain extrapolation. */
                    if (ngc == 0.0) { s->rho[ng] = r0; s->phi[ng] = p0; continue; }
                    double m0 = gc[0] / ngc, m1 = gc[1] / ngc;
                    double re = r0 + ct * (gr[0] * m0 + gr[1] * m1);
                    double pe = p0 + ct * (gp[0] * m0 + gp[1] * m1);
                    double rlo = fmin(r0, p->rho_g), rhi = fmax(r0, p->rho_l);
                    double plo = fmin(p0, -p->chi), phi_ = fmax(p0, p->chi);
                    s->rho[ng] = re < rlo ? rlo : (re > rhi ? rhi : re);
                    s->phi[ng] = pe < plo ? plo : (pe > phi_ ? phi_ : pe);
                    continue;
                }
                /* geometric interpolation.  reading: the sampling point is
                 * shifted by cot(theta) toward the measuring phase, i.e. along
                 * +grad c (Eq. 47 with the measuring phase at lower i is the
                 * case grad c < 0). */
                if (D == 2) {
                    double sg = (gc[0] > 0.0) ? 1.0 : (gc[0] < 0.0 ? -1.0 : 0.0);
                    double l = sg * ct;
                    s->rho[ng] = or_interp2d(lr, np1, i, l);
                    s->phi[ng] = or_interp2d(lp, np1, i, l);
                } else {
                    if (ngc == 0.0) { s->rho[ng] = r0; s->phi[ng] = p0; continue; }
                    double lx = ct * gc[0] / ngc, ly = ct * gc[1] / ngc;
                    s->rho[ng] = or_interp3d(lr, np1, np2, i, j, lx, ly);
                    s->phi[ng] = or_interp3d(lp, np1, np2, i, j, lx, ly);
                }
            }
    }
    free(lr);
    free(lp);
}

/* ---- pass 3: stencils ---------------------------------------------------
 * reading (stencils are not printed): isotropic lattice stencils
 *   grad q = (1/c_s^2) sum_i w_i c_i q(x + c_i),
 *   lap q  = (2/c_s^2) sum_i w_i (q(x + c_i) - q(x)),  c_s^2 = 1/3,
 * using the ghost layers next to walls (Sec. IV, Fig. 4a). */
static void pass_stencils(or_state *s)
{
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < s->N; ++n) {
        int x, y, z;
        coords(s, n, &x, &y, &z);
        if (!is_fluid(s, x, y, z)) continue;
        double G[3] = {0, 0, 0}, H[3] = {0, 0, 0}, Lr = 0, Lp = 0;
        for (int i = 0; i < s->Q; ++i) {
            int xn, yn, zn;
            neighbour(s, x, y, z, s->c[i], &xn, &yn, &zn);
            int64_t m = idx(s, xn, yn, zn);
            for (int a = 0; a < 3; ++a) {
                G[a] += 3.0 * s->w[i] * s->c[i][a] * s->rho[m];
                H[a] += 3.0 * s->w[i] * s->c[i][a] * s->phi[m];
            }
            Lr += 6.0 * s->w[i] * (s->rho[m] - s->rho[n]);
            Lp += 6.0 * s->w[i] * (s->phi[m] - s->phi[n]);
        }
        for (int a = 0; a < 3; ++a) { s->grho[a][n] = G[a]; s->gphi[a][n] = H[a]; }
        s->lrho[n] = Lr;
        s->lphi[n] = Lp;
    }
}

/* ---- passes 4-5: chemical potentials and pressure tensor ---------------- */
static void pass_thermo(or_state *s)
{
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < s->N; ++n) {
        int x, y, z;
        coords(s, n, &x, &y, &z);
        if (!is_fluid(s, x, y, z)) continue;
        double G[3] = {s->grho[0][n], s->grho[1][n], s->grho[2][n]};
        double H[3] = {s->gphi[0][n], s->gphi[1][n], s->gphi[2][n]};
        double P[9];
        or_local_thermo(&s->p, s->rho[n], s->phi[n], G, H, s->lrho[n], s->lphi[n],
                        &s->mur[n], &s->mup[n], P);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                s->Tt[a][b][n] = -P[3 * a + b];
    }
}

/* ---- pass 6: force F = div(rho c_s^2 I - P), Eq. 29 --------------------
 * The divergence of -P uses the isotropic gradient stencil of pass 3 on each
 * column of P.
 * reading (the paper only says the force comes from numerically
 * differentiating the pressure tensor): the ideal part div(rho c_s^2 I) is
 * the lattice divergence of a link pressure,
 *   F_id(x) = sum_i 6 w_i c_i Pi(x, x + c_i),
 *   Pi(x, y) = 2 rho_x rho_y / (rho_x + rho_y + 4 sqrt(rho_x rho_y)),
 * which equals rho/3 for equal densities (so it reduces to the isotropic
 * stencil of rho/3 to first order), is symmetric (momentum is conserved
 * exactly) and makes a static profile rho ~ exp(k x) an exact steady state of
 * the exact-difference ELBM with the product-form equilibrium: per link the
 * streamed-in populations are then f^eq at the constant bare velocity -U with
 * B(U)^2 = rho_y/rho_x (B of Eq. 27), for any alpha and beta.  The plain
 * isotropic stencil of rho/3 lets the soft gas phase run away at large
 * density ratios.
 * reading of the wall rule (Sec. IV): on the first fluid layer the pressure
 * tensor, which is not defined on the solid nodes, has its wall-normal
 * derivatives dropped and its in-layer derivatives taken as central
 * differences within the layer; the ideal part needs only rho, which the
 * ghost nodes hold, and uses the axis links including the wall-normal one,
 * sum_b [Pi(x, x + e_b) - Pi(x, x - e_b)] e_b (the wetting ghost values so
 * enter the momentum balance of the contact line).
 * Force method (Eq. 43): on the second fluid layer
 *   F_s = rho_rel (kw_rho + phi_rel kw_phi) sum_i w_i s(x + 2 c_i) c_i
 *       = -(1/6) rho_rel (kw_rho + phi_rel kw_phi) n_wall,
 * n_wall the unit normal pointing into the fluid.
 * reading: s marks the solid as seen two lattice links away, so the lattice
 * sum is over the links that point at the wall (weight 1/6 in D2Q9 and
 * D3Q27); positive kw attracts the phase to the wall. */
static double link_pressure(double rx, double ry)
{
    return 2.0 * rx * ry / (rx + ry + 4.0 * sqrt(rx * ry));
}

static void pass_force(or_state *s)
{
    const or_params *p = &s->p;
    int ax = wall_axis(s);
    int nw = p->n[ax];
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < s->N; ++n) {
        int x, y, z;
        coords(s, n, &x, &y, &z);
        if (!is_fluid(s, x, y, z)) continue;
        int k = (ax == 1) ? y : z;
        int first = p->walls && (k == 1 || k == nw - 2);
        double F[3] = {0, 0, 0};
        if (first && p->wall_par == 1) {
            /* reading (the alternative of Sec. IV and Fig. 4b, a stencil for the
             * tangential derivatives of P that excludes solid nodes): the
             * bulk stencil of the tangential terms with every link that
             * points into the wall replaced by its mirror image on the fluid
             * side; the wall-normal derivative of P dropped and the
             * wall-normal ideal link kept, as in the default reading */
            const int into = (k == 1) ? -1 : 1;
            double r0 = s->rho[n];
            for (int i = 0; i < s->Q; ++i) {
                int c[3] = {s->c[i][0], s->c[i][1], s->c[i][2]};
                if (c[ax] == into) c[ax] = -into;
                int xn, yn, zn;
                neighbour(s, x, y, z, c, &xn, &yn, &zn);
                int64_t m = idx(s, xn, yn, zn);
                double pl = link_pressure(r0, s->rho[m]);
                for (int b = 0; b < p->D; ++b) {
                    if (b == ax) continue;
                    for (int a = 0; a < p->D; ++a)
                        F[a] += 3.0 * s->w[i] * s->c[i][b] * s->Tt[a][b][m];
                    F[b] += 6.0 * s->w[i] * s->c[i][b] * pl;
                }
            }
            int cp[3] = {0, 0, 0}, cm[3] = {0, 0, 0};
            cp[ax] = 1;
            cm[ax] = -1;
            int xp, yp, zp, xm, ym, zm;
            neighbour(s, x, y, z, cp, &xp, &yp, &zp);
            neighbour(s, x, y, z, cm, &xm, &ym, &zm);
            F[ax] += link_pressure(s->rho[n], s->rho[idx(s, xp, yp, zp)]) -
                     link_pressure(s->rho[n], s->rho[idx(s, xm, ym, zm)]);
        } else if (first) {
            for (int b = 0; b < p->D; ++b) {
                if (b == ax) continue;
                int cp[3] = {0, 0, 0}, cm[3] = {0, 0, 0};
                cp[b] = 1;
                cm[b] = -1;
                int xp, yp, zp, xm, ym, zm;
                neighbour(s, x, y, z, cp, &xp, &yp, &zp);
                neighbour(s, x, y, z, cm, &xm, &ym, &zm);
                int64_t np_ = idx(s, xp, yp, zp), nm = idx(s, xm, ym, zm);
                for (int a = 0; a < p->D; ++a)
                    F[a] += 0.5 * (s->Tt[a][b][np_] - s->Tt[a][b][nm]);
                F[b] += link_pressure(s->rho[n], s->rho[np_]) -
                        link_pressure(s->rho[n], s->rho[nm]);
            }
            /* wall-normal link of the ideal part, across to the ghost node */
            int cp[3] = {0, 0, 0}, cm[3] = {0, 0, 0};
            cp[ax] = 1;
            cm[ax] = -1;
            int xp, yp, zp, xm, ym, zm;
            neighbour(s, x, y, z, cp, &xp, &yp, &zp);
            neighbour(s, x, y, z, cm, &xm, &ym, &zm);
            F[ax] += link_pressure(s->rho[n], s->rho[idx(s, xp, yp, zp)]) -
                     link_pressure(s->rho[n], s->rho[idx(s, xm, ym, zm)]);
        } else {
            double r0 = s->rho[n];
            for (int i = 0; i < s->Q; ++i) {
                int xn, yn, zn;
                neighbour(s, x, y, z, s->c[i], &xn, &yn, &zn);
                int64_t m = idx(s, xn, yn, zn);
                for (int a = 0; a < p->D; ++a)
                    for (int b = 0; b < p->D; ++b)
                        F[a] += 3.0 * s->w[i] * s->c[i][b] * s->Tt[a][b][m];
                double pl = link_pressure(r0, s->rho[m]);
                for (int a = 0; a < p->D; ++a)
                    F[a] += 6.0 * s->w[i] * s->c[i][a] * pl;
            }
        }
        if (p->walls && p->wetting == OR_FORCE) {
            for (int wall = 0; wall < 2; ++wall) {
                int second = (wall == 0) ? 2 : nw - 3;
                if (k != second) continue;
                double rrel = (s->rho[n] - p->rho_g) / (p->rho_l - p->rho_g);
                double prel = s->phi[n] / p->chi;
                double mag = rrel * (p->kw[wall][0] + prel * p->kw[wall][1]);
                double nrm = (wall == 0) ? 1.0 : -1.0;
                F[ax] += -(1.0 / 6.0) * mag * nrm;
            }
        }
        for (int a = 0; a < 3; ++a) s->F[a][n] = F[a];
    }
}

/* ---- passes 7-8: collisions -------------------------------------------- */
/* f: ELBM with exact-difference forcing (Eqs. 24-32):
 *   du = F / rho;  f' = f + f^eq(rho, u + du) - f^eq(rho, u);
 *   Delta = f^eq(rho, u + du) - f';  f* = f' + alpha beta Delta.
 * g: LBGK (Eqs. 33-35) with v = u + du / 2 and the same-step mu_phi. */
static void pass_collide(or_state *s)
{
    const or_params *p = &s->p;
    int Q = s->Q;
    int64_t nn = 0, ns = 0, nf = 0, nq = 0;
#pragma omp parallel for schedule(static) reduction(+ : nn, ns, nf, nq)
    for (int64_t n = 0; n < s->N; ++n) {
        int x, y, z;
        coords(s, n, &x, &y, &z);
        if (!is_fluid(s, x, y, z)) continue;
        if (p->no_collide) {
            for (int i = 0; i < Q; ++i) {
                s->fs[(int64_t)i * s->N + n] = s->f[(int64_t)i * s->N + n];
                s->gs[(int64_t)i * s->N + n] = s->g[(int64_t)i * s->N + n];
            }
            continue;
        }
        double r = s->rho[n];
        double u[3], ud[3], v[3];
        for (int a = 0; a < 3; ++a) {
            u[a] = s->u[a][n];
            double du = s->F[a][n] / r;
            ud[a] = u[a] + du;
            v[a] = u[a] + 0.5 * du;
        }
        /* the velocity the collision uses has reached the lattice speed */
        if (ud[0] * ud[0] + ud[1] * ud[1] + ud[2] * ud[2] >= 1.0) nq += 1;
        double fe[MAXQ], fed[MAXQ], fp[MAXQ], dl[MAXQ];
        or_feq(p->D, r, u, fe);
        or_feq(p->D, r, ud, fed);
        for (int i = 0; i < Q; ++i) {
            double fi = s->f[(int64_t)i * s->N + n];
            fp[i] = fi + fed[i] - fe[i];
            dl[i] = fed[i] - fp[i];
        }
        double al = 2.0;
        if (!p->force_alpha2) {
            int kind = or_alpha(Q, s->w, fp, dl, p->alpha_eps, p->alpha_tol,
                                p->alpha_maxit, &al);
            if (kind == 0) ++ns; else if (kind == 1) ++nn; else ++nf;
        }
        s->alpha[n] = al;
        for (int i = 0; i < Q; ++i)
            s->fs[(int64_t)i * s->N + n] = fp[i] + al * p->beta * dl[i];
        double ge[MAXQ];
        or_geq(p->D, s->phi[n], s->mup[n], p->Gamma, v, ge);
        for (int i = 0; i < Q; ++i) {
            double gi = s->g[(int64_t)i * s->N + n];
            s->gs[(int64_t)i * s->N + n] = gi + (ge[i] - gi) / p->tau_g;
        }
    }
    s->n_newton += nn;
    s->n_shortcut += ns;
    s->n_fast += nq;
    s->n_fallback += nf;
}

/* ---- pass 9: streaming with halfway bounce-back (Sec. IV) --------------
 * f_i(x + c_i) <- f*_i(x) when x + c_i is fluid, else f_{-i}(x) <- f*_i(x). */
static void pass_stream(or_state *s)
{
    int Q = s->Q;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < s->N; ++n) {
        int x, y, z;
        coords(s, n, &x, &y, &z);
        if (!is_fluid(s, x, y, z)) continue;
        for (int i = 0; i < Q; ++i) {
            int xn, yn, zn;
            neighbour(s, x, y, z, s->c[i], &xn, &yn, &zn);
            double vf = s->fs[(int64_t)i * s->N + n];
            double vg = s->gs[(int64_t)i * s->N + n];
            if (is_fluid(s, xn, yn, zn)) {
                int64_t m = idx(s, xn, yn, zn);
                s->f[(int64_t)i * s->N + m] = vf;
                s->g[(int64_t)i * s->N + m] = vg;
            } else {
                int o = Q - 1 - i;
                s->f[(int64_t)o * s->N + n] = vf;
                s->g[(int64_t)o * s->N + n] = vg;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
int or_init(or_state *s, const double *rho0, const double *phi0)
{
    /* reading (initial state not stated): f = f^eq(rho0, 0) = w rho0;
     * g = g^eq(phi0, mu_phi(rho0, phi0), 0) with mu_phi from the ghost fill
     * and stencils of the initial fields. */
    memcpy(s->rho, rho0, sizeof(double) * (size_t)s->N);
    memcpy(s->phi, phi0, sizeof(double) * (size_t)s->N);
    for (int a = 0; a < 3; ++a) memset(s->u[a], 0, sizeof(double) * (size_t)s->N);
    pass_ghost(s);
    pass_stencils(s);
    pass_thermo(s);
    memset(s->f, 0, sizeof(double) * (size_t)(s->Q * s->N));
    memset(s->g, 0, sizeof(double) * (size_t)(s->Q * s->N));
    double zero[3] = {0, 0, 0};
    for (int64_t n = 0; n < s->N; ++n) {
        int x, y, z;
        coords(s, n, &x, &y, &z);
        if (!is_fluid(s, x, y, z)) continue;
        double ge[MAXQ];
        or_geq(s->p.D, s->phi[n], s->mup[n], s->p.Gamma, zero, ge);
        for (int i = 0; i < s->Q; ++i) {
            s->f[(int64_t)i * s->N + n] = s->w[i] * s->rho[n];
            s->g[(int64_t)i * s->N + n] = ge[i];
        }
    }
    s->step = 0;
    s->n_newton = s->n_shortcut = s->n_fallback = s->n_fast = 0;
    pass_moments(s);
    pass_ghost(s);
    return 0;
}

int or_set_pops(or_state *s, const double *f, const double *g)
{
    memcpy(s->f, f, sizeof(double) * (size_t)(s->Q * s->N));
    memcpy(s->g, g, sizeof(double) * (size_t)(s->Q * s->N));
    pass_moments(s);
    return 0;
}

int or_step(or_state *s, int64_t nsteps)
{
    for (int64_t t = 0; t < nsteps; ++t) {
        pass_moments(s);
        if (!s->p.no_collide) {
            pass_ghost(s);
            pass_stencils(s);
            pass_thermo(s);
            pass_force(s);
        }
        pass_collide(s);
        pass_stream(s);
        s->step++;
    }
    /* moments and ghost layers of the state reached (reported by or_get) */
    pass_moments(s);
    pass_ghost(s);
    return 0;
}

void or_get(const or_state *s, double *rho, double *phi, double *f, double *g)
{
    if (rho) memcpy(rho, s->rho, sizeof(double) * (size_t)s->N);
    if (phi) memcpy(phi, s->phi, sizeof(double) * (size_t)s->N);
    if (f) memcpy(f, s->f, sizeof(double) * (size_t)(s->Q * s->N));
    if (g) memcpy(g, s->g, sizeof(double) * (size_t)(s->Q * s->N));
}

void or_get_field(const or_state *s, int which, double *out)
{
    const double *src = NULL;
    switch (which) {
    case 0: src = s->mur; break;
    case 1: src = s->mup; break;
    case 2: case 3: case 4: src = s->F[which - 2]; break;
    case 5: case 6: case 7: src = s->grho[which - 5]; break;
    case 8: case 9: case 10: src = s->gphi[which - 8]; break;
    case 11: src = s->lrho; break;
    case 12: src = s->lphi; break;
    case 13: src = s->alpha; break;
    default: return;
    }
    memcpy(out, src, sizeof(double) * (size_t)s->N);
}

/* compensated (Neumaier) accumulation */
typedef struct { double s, c; } ksum;
static void kadd(ksum *k, double v)
{
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v; else k->c += (v - t) + k->s;
    k->s = t;
}
static double kval(const ksum *k) { return k->s + k->c; }

void or_observe(const or_state *s, or_obs *o)
{
    const or_params *p = &s->p;
    ksum m[3] = {{0, 0}, {0, 0}, {0, 0}}, rs = {0, 0}, ps = {0, 0}, ke = {0, 0};
    ksum mo[3] = {{0, 0}, {0, 0}, {0, 0}};
    double umax = 0.0;
    int64_t bad = 0;
    for (int64_t n = 0; n < s->N; ++n) {
        int x, y, z;
        coords(s, n, &x, &y, &z);
        if (!is_fluid(s, x, y, z)) continue;
        double r = s->rho[n], ph = s->phi[n];
        if (!(r > 0.0) || !isfinite(r) || !isfinite(ph)) { ++bad; continue; }
        double C1 = (r - p->rho_l) / (p->rho_g - p->rho_l);
        double C2 = 0.5 * (1.0 + ph / p->chi - C1);
        double C3 = 0.5 * (1.0 - ph / p->chi - C1);
        kadd(&m[0], C1);
        kadd(&m[1], C2);
        kadd(&m[2], C3);
        kadd(&rs, r);
        kadd(&ps, ph);
        double uu = 0.0;
        for (int a = 0; a < 3; ++a) {
            kadd(&mo[a], r * s->u[a][n]);
            uu += s->u[a][n] * s->u[a][n];
        }
        kadd(&ke, 0.5 * r * uu);
        if (sqrt(uu) > umax) umax = sqrt(uu);
    }
    for (int k = 0; k < 3; ++k) { o->mass[k] = kval(&m[k]); o->mom[k] = kval(&mo[k]); }
    o->rho_sum = kval(&rs);
    o->phi_sum = kval(&ps);
    o->kinetic = kval(&ke);
    o->umax = umax;
    o->n_bad = bad;
    o->n_newton = s->n_newton;
    o->n_shortcut = s->n_shortcut;
    o->n_fallback = s->n_fallback;
    o->n_fast = s->n_fast;
    o->step = s->step;
}

/* ------------------------------------------------------------------------ */
/* 1D flat interface by gradient flow of the free energy (used to calibrate
 * lambda, kappa against target tensions).  Discrete 3-point Laplacian and
 * central gradient, matching the lattice stencils along one axis.  The
 * tension is the integral of the normal minus the tangential pressure,
 * sum_x [krr rho'^2 + kpp phi'^2 + 2 kx rho' phi'] (from Eq. 19). */
double or_flat_tension(const or_params *p, int pair, int n, double *width,
                       double *rho_out, double *phi_out)
{
    derived_k k = derive_k(p);
    double rA, pA, rB, pB;
    if (pair == 12) { rA = p->rho_g; pA = 0.0; rB = p->rho_l; pB = p->chi; }
    else if (pair == 13) { rA = p->rho_g; pA = 0.0; rB = p->rho_l; pB = -p->chi; }
    else { rA = p->rho_l; pA = p->chi; rB = p->rho_l; pB = -p->chi; }
    double *r = alloc(n), *ph = alloc(n), *mr = alloc(n), *mp = alloc(n);
    for (int x = 0; x < n; ++x) {
        double t = 0.5 * (1.0 + tanh((x - 0.5 * (n - 1)) / 2.0));
        r[x] = rA + (rB - rA) * t;
        ph[x] = pA + (pB - pA) * t;
    }
    /* explicit step bounded by the stiffest local curvature */
    double stiff = 0.5 * fabs(p->lambda[0]) * (p->T / p->rho_g + 2.0 * fabs(p->a)) +
                   (fabs(p->lambda[1]) + fabs(p->lambda[2])) / (k.drho * k.drho) +
                   4.0 * (fabs(k.krr) + fabs(k.kx)) + 0.0;
    double stiffp = (fabs(p->lambda[1]) + fabs(p->lambda[2])) / (p->chi * p->chi) +
                    4.0 * (fabs(k.kpp) + fabs(k.kx));
    double dt = 0.4 / (stiff > stiffp ? stiff : stiffp);
    /* reading: the interface position is a neutral mode of the flat
     * problem; it is pinned by holding the field that changes across it (rho
     * for the liquid-gas pairs, phi for 2-3) at the centre node at the mean of
     * its two bulk values */
    const int pin = n / 2;
    const int pin_phi = (pair == 23);
    if (pin_phi) ph[pin] = 0.5 * (pA + pB); else r[pin] = 0.5 * (rA + rB);
    for (int it = 0; it < 20000000; ++it) {
        double res = 0.0;
        for (int x = 1; x < n - 1; ++x) {
            double Lr = r[x + 1] + r[x - 1] - 2.0 * r[x];
            double Lp = ph[x + 1] + ph[x - 1] - 2.0 * ph[x];
            double mrb, mpb, fb;
            bulk_terms(p, r[x], ph[x], &mrb, &mpb, &fb);
            mr[x] = (x == pin && !pin_phi) ? 0.0 : mrb - k.krr * Lr - k.kx * Lp;
            mp[x] = (x == pin && pin_phi) ? 0.0 : mpb - k.kpp * Lp - k.kx * Lr;
            double e = fabs(mr[x]) + fabs(mp[x]);
            if (e > res) res = e;
        }
        for (int x = 1; x < n - 1; ++x) {
            r[x] -= dt * mr[x];
            ph[x] -= dt * mp[x];
        }
        if (res < 1e-13) break;
    }
    double gam = 0.0;
    for (int x = 1; x < n - 1; ++x) {
        double dr = 0.5 * (r[x + 1] - r[x - 1]);
        double dp = 0.5 * (ph[x + 1] - ph[x - 1]);
        gam += k.krr * dr * dr + k.kpp * dp * dp + 2.0 * k.kx * dr * dp;
    }
    if (width) {
        /* 10-90 % width of the concentration that changes across the
         * interface: C1 for the liquid-gas pairs, C2 for 2-3 */
        double lo = -1, hi = -1;
        for (int x = 0; x < n - 1; ++x) {
            double c0, c1;
            if (pair == 23) {
                double a0 = (r[x] - p->rho_l) / (p->rho_g - p->rho_l);
                double a1 = (r[x + 1] - p->rho_l) / (p->rho_g - p->rho_l);
                c0 = 0.5 * (1.0 + ph[x] / p->chi - a0);
                c1 = 0.5 * (1.0 + ph[x + 1] / p->chi - a1);
            } else {
                c0 = (r[x] - p->rho_l) / (p->rho_g - p->rho_l);
                c1 = (r[x + 1] - p->rho_l) / (p->rho_g - p->rho_l);
            }
            /* monotone profile: record the crossing positions of 0.9 and 0.1 */
            double t9 = 0.9, t1 = 0.1;
            if ((c0 - t9) * (c1 - t9) <= 0.0 && c0 != c1 && lo < 0) lo = x + (t9 - c0) / (c1 - c0);
            if ((c0 - t1) * (c1 - t1) <= 0.0 && c0 != c1 && hi < 0) hi = x + (t1 - c0) / (c1 - c0);
        }
        *width = (lo >= 0 && hi >= 0) ? fabs(hi - lo) : NAN;
    }
    if (rho_out) memcpy(rho_out, r, sizeof(double) * (size_t)n);
    if (phi_out) memcpy(phi_out, ph, sizeof(double) * (size_t)n);
    free(r); free(ph); free(mr); free(mp);
    return gam;
}

/* OpenMP threads of the passes (timing only; the results do not depend on
 * it: no pass reduces in floating point across threads). */
void or_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int  or_get_threads(void) { return omp_get_max_threads(); }
