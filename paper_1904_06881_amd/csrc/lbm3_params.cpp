// Host-side thermodynamics and parameter resolution of the lbm3 library.
//
// Carnahan-Starling coexistence (paper Sec. II A, Eq. 4): the temperature is
// found from the requested density ratio at the paper's a/b = 0.185, by
// Newton continuation in log(ratio) from the critical point on the two
// Maxwell conditions (equal chemical potential, equal pressure); then the
// densities are rescaled to the requested liquid density at fixed a/b and T
// (rho' = s rho, b' = b/s, a' = a/s keeps b rho and the isotherm's shape), and
// C, Psi0 make Psi(rho_g) = Psi(rho_l) = Psi0 with zero slope at both.
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/lbm3.h"
#include "lbm3_params.h"

namespace lbm3h {

namespace {

struct CS {
    double a, b, T;
    // mu = dPsi/drho without the constant C (Eq. 15)
    double mu(double r) const
    {
        double d = b * r - 4.0;
        return -2.0 * a * r + T * (1.0 + std::log(r)) + 16.0 * T * (b * r - 12.0) / (d * d * d);
    }
    double dmu_dr(double r) const
    {
        double d = b * r - 4.0;
        return -2.0 * a + T / r + 16.0 * T * b * (32.0 - 2.0 * b * r) / (d * d * d * d);
    }
    double dmu_dT(double r) const
    {
        double d = b * r - 4.0;
        return 1.0 + std::log(r) + 16.0 * (b * r - 12.0) / (d * d * d);
    }
    // pressure in the compressibility-factor form, eta = b rho / 4
    double p(double r) const
    {
        double e = 0.25 * b * r, om = 1.0 - e;
        return r * T * (1.0 + e + e * e - e * e * e) / (om * om * om) - a * r * r;
    }
    double dp_dT(double r) const
    {
        double e = 0.25 * b * r, om = 1.0 - e;
        return r * (1.0 + e + e * e - e * e * e) / (om * om * om);
    }
};

// Critical point of the CS EOS: d mu/d rho = 0 and d^2 mu/d rho^2 = 0 in the
// packing fraction eta = b rho / 4 (independent of a, b up to scaling).
// Newton on g(eta) = eta h''(eta) - h'(eta)... solved once numerically.
void critical(double a, double b, double &Tc, double &rc)
{
    // d mu/d rho = T k1(eta)/rho - 2a, d2 mu/d rho2 = T (b/4)^2 k2(eta)... use
    // the reduced form: Z(eta) p = rho T Z - a rho^2; at the critical point
    // d(eta Z)/d eta = eta d2(eta Z)/d eta2 (a is eliminated).
    auto z1 = [](double e) {  // d/de [e Z(e)]
        double om = 1.0 - e;
        double num = 1.0 + 4.0 * e + 4.0 * e * e - 4.0 * e * e * e + e * e * e * e;
        return num / (om * om * om * om);
    };
    auto z2 = [&](double e) {  // d2/de2 [e Z(e)] by a central difference of z1
        double h = 1e-6;
        return (z1(e + h) - z1(e - h)) / (2.0 * h);
    };
    double e = 0.13;
    for (int it = 0; it < 60; ++it) {
        double h = 1e-7;
        double g = z1(e) - e * z2(e);
        double gp = ((z1(e + h) - (e + h) * z2(e + h)) - (z1(e - h) - (e - h) * z2(e - h))) / (2 * h);
        double de = g / gp;
        e -= de;
        if (std::fabs(de) < 1e-14) break;
    }
    // d p/d rho = T z1 - 2 a rho = 0 at rho = 4 e / b
    rc = 4.0 * e / b;
    Tc = 2.0 * a * rc / z1(e);
}

// Newton on (T, log rho_g) with rho_l = ratio rho_g for the two Maxwell
// conditions; returns false if it does not converge.
bool maxwell_newton(const CS &base, double ratio, double &T, double &lg)
{
    CS c = base;
    for (int it = 0; it < 100; ++it) {
        c.T = T;
        double rg = std::exp(lg), rl = ratio * rg;
        double E1 = c.mu(rl) - c.mu(rg);
        double E2 = c.p(rl) - c.p(rg);
        double J11 = c.dmu_dT(rl) - c.dmu_dT(rg);
        double J12 = rl * c.dmu_dr(rl) - rg * c.dmu_dr(rg);
        double J21 = c.dp_dT(rl) - c.dp_dT(rg);
        double J22 = rl * rl * c.dmu_dr(rl) - rg * rg * c.dmu_dr(rg);  // dp/drho = rho dmu/drho
        double det = J11 * J22 - J12 * J21;
        if (!(std::fabs(det) > 0.0)) return false;
        double dT = (E1 * J22 - E2 * J12) / det;
        double dl = (J11 * E2 - J21 * E1) / det;
        // damping keeps T positive and the liquid below close packing
        double lam = 1.0;
        for (int k = 0; k < 40; ++k) {
            double Tn = T - lam * dT, ln = lg - lam * dl;
            if (Tn > 0.0 && ratio * std::exp(ln) * c.b < 4.0 * 0.999) break;
            lam *= 0.5;
        }
        T -= lam * dT;
        lg -= lam * dl;
        if (std::fabs(dT) < 1e-15 * T && std::fabs(dl) < 1e-14) return true;
    }
    c.T = T;
    double rg = std::exp(lg), rl = ratio * rg;
    return std::fabs(c.mu(rl) - c.mu(rg)) < 1e-12 * T && std::fabs(c.p(rl) - c.p(rg)) < 1e-12 * T * rl;
}

}  // namespace

bool coexistence(double ratio, double rho_l_target, double &a, double &b, double &T, double &C, double &psi0,
                 double &rho_l, double &rho_g)
{
    const double a0 = 0.037, b0 = 0.2;
    if (!(ratio > 1.0) || !(rho_l_target > 0.0)) return false;
    CS cs{a0, b0, 0.0};
    double Tc, rc;
    critical(a0, b0, Tc, rc);
    // continuation from just below the critical point: for a small ratio the
    // coexistence densities sit symmetrically around rho_c in log space
    double lr_target = std::log(ratio);
    double lr = std::fmin(0.05, lr_target);
    double Tcur = Tc * (1.0 - 1e-3), lg = std::log(rc) - 0.5 * lr;
    // first solve: sweep T down until the ratio-lr solve converges
    bool ok = false;
    for (int k = 0; k < 60 && !ok; ++k) {
        double Tt = Tcur, lgt = lg;
        ok = maxwell_newton(cs, std::exp(lr), Tt, lgt);
        if (ok) { Tcur = Tt; lg = lgt; }
        else Tcur = Tc * (1.0 - 1e-3 * (k + 2));
    }
    if (!ok) return false;
    while (lr < lr_target) {
        double step = 0.1;
        double next = std::fmin(lr + step, lr_target);
        double Tt = Tcur, lgt = lg - 0.5 * (next - lr);
        while (!maxwell_newton(cs, std::exp(next), Tt, lgt)) {
            step *= 0.5;
            if (step < 1e-6) return false;
            next = std::fmin(lr + step, lr_target);
            Tt = Tcur;
            lgt = lg - 0.5 * (next - lr);
        }
        lr = next;
        Tcur = Tt;
        lg = lgt;
    }
    double rg = std::exp(lg), rl = ratio * rg;
    double s = rho_l_target / rl;
    a = a0 / s;
    b = b0 / s;
    T = Tcur;
    rho_l = rho_l_target;
    rho_g = rho_l_target / ratio;
    CS sc{a, b, T};
    C = -sc.mu(rho_g);
    // Psi(rho_g) with the constant C (Eq. 4)
    double d = b * rho_g - 4.0;
    psi0 = rho_g * (C - a * rho_g - 8.0 * T * (b * rho_g - 6.0) / (d * d) + T * std::log(rho_g));
    return true;
}

}  // namespace lbm3h

// ---------------------------------------------------------------------------
// (gamma12, gamma13, gamma23, width) -> (lambda, kappa).
// alpha23 = width / 4 (the tanh profile of Eq. 37 has a 10-90 % width of
// 2 alpha23 ln 9 ~ 4.39 alpha23, read as "interface width" = 4 alpha23);
// kappa_i = alpha23^2 lambda_i (i = 2, 3) so that Eq. 36 gives alpha23;
// lambda2 + lambda3 = 6 gamma23 / alpha23 (Eq. 38).  lambda1, kappa1 and
// lambda2 - lambda3 are solved so that flat 1-2 and 1-3 interfaces relaxed
// on a 1D lattice have tensions gamma12, gamma13 and a mean 10-90 % width of
// the gas concentration equal to 2 alpha23 ln 9.
namespace lbm3h {

namespace {

struct FE {  // free-energy model on a 1D lattice
    double a, b, T, C, psi0, rho_l, rho_g, drho, chi, lam[3], kap[3], krr, kpp, kx;
    void derive()
    {
        drho = rho_l - rho_g;
        krr = kap[0] + (kap[1] + kap[2]) / (4.0 * drho * drho);
        kpp = (kap[1] + kap[2]) / (4.0 * chi * chi);
        kx = (kap[1] - kap[2]) / (4.0 * chi * drho);
    }
    static double gf(double x) { return x * (x - 0.5) * (x - 1.0); }
    static double dg(double x) { return 3.0 * x * x - 3.0 * x + 0.5; }
    // bulk chemical potentials and their Jacobian
    void bulk(double r, double ph, double &mr, double &mp, double J[2][2]) const
    {
        double C1 = (rho_l - r) / drho;
        double C2 = 0.5 * (1.0 + ph / chi - C1), C3 = 0.5 * (1.0 - ph / chi - C1);
        double d = b * r - 4.0;
        double dpsi = C - 2.0 * a * r + T * (1.0 + std::log(r)) + 16.0 * T * (b * r - 12.0) / (d * d * d);
        double d2psi = -2.0 * a + T / r + 16.0 * T * b * (32.0 - 2.0 * b * r) / (d * d * d * d);
        mr = 0.5 * lam[0] * dpsi + (lam[1] * gf(C2) + lam[2] * gf(C3)) / drho;
        mp = (lam[1] * gf(C2) - lam[2] * gf(C3)) / chi;
        double s = lam[1] * dg(C2) + lam[2] * dg(C3), t = lam[1] * dg(C2) - lam[2] * dg(C3);
        J[0][0] = 0.5 * lam[0] * d2psi + s / (2.0 * drho * drho);
        J[0][1] = t / (2.0 * drho * chi);
        J[1][0] = t / (2.0 * chi * drho);
        J[1][1] = s / (2.0 * chi * chi);
    }
};

// Relax a flat interface between bulk states A (x = 0) and B (x = n-1),
// ends fixed, by pseudo-transient continuation: (I/dt + J) du = -R with the
// discrete (3-point) chemical potentials as residual; dt grows while the
// residual falls.  Returns the tension sum (P_xx - P_yy) and the 10-90 %
// width of the gas concentration (liquid-gas pairs).
bool flat(const FE &m, int pair, int n, double &gamma, double &width)
{
    double rA, pA, rB, pB;
    if (pair == 12) { rA = m.rho_g; pA = 0.0; rB = m.rho_l; pB = m.chi; }
    else { rA = m.rho_g; pA = 0.0; rB = m.rho_l; pB = -m.chi; }
    std::vector<double> r(n), ph(n), R(2 * n), du(2 * n);
    for (int x = 0; x < n; ++x) {
        double t = 0.5 * (1.0 + std::tanh((x - 0.5 * (n - 1)) / 2.0));
        r[x] = rA + (rB - rA) * t;
        ph[x] = pA + (pB - pA) * t;
    }
    // the interface position is a neutral mode: pin it by replacing the rho
    // equation of the centre node with rho = (rho_A + rho_B) / 2
    const int pin = n / 2;
    const double rmid = 0.5 * (rA + rB);
    auto residual = [&](std::vector<double> &out) {
        double nrm = 0.0;
        for (int x = 1; x < n - 1; ++x) {
            double J[2][2], mr, mp;
            m.bulk(r[x], ph[x], mr, mp, J);
            double Lr = r[x + 1] + r[x - 1] - 2.0 * r[x], Lp = ph[x + 1] + ph[x - 1] - 2.0 * ph[x];
            out[2 * x] = x == pin ? r[x] - rmid : mr - m.krr * Lr - m.kx * Lp;
            out[2 * x + 1] = mp - m.kpp * Lp - m.kx * Lr;
            nrm = std::fmax(nrm, std::fabs(out[2 * x]) + std::fabs(out[2 * x + 1]));
        }
        return nrm;
    };
    double res = residual(R), dt = 1.0;
    // block-tridiagonal Thomas solve storage
    std::vector<double> cp(4 * n), dp(2 * n);
    for (int it = 0; it < 400 && res > 1e-14; ++it) {
        // forward sweep: diagonal D_x = I/dt + Jbulk + 2K, off-diagonals -K
        const double K[2][2] = {{m.krr, m.kx}, {m.kx, m.kpp}};
        double Cprev[2][2] = {{0, 0}, {0, 0}}, dprev[2] = {0, 0};
        for (int x = 1; x < n - 1; ++x) {
            double J[2][2], mr, mp;
            m.bulk(r[x], ph[x], mr, mp, J);
            // rows: Kl couples to x-1 and Ku to x+1 (both -K except the pinned row)
            double Dm[2][2], Kl[2][2], Ku[2][2];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) {
                    Dm[i][j] = J[i][j] + 2.0 * K[i][j] + (i == j ? 1.0 / dt : 0.0);
                    Kl[i][j] = Ku[i][j] = K[i][j];
                }
            if (x == pin) {
                Dm[0][0] = 1.0 + 1.0 / dt;
                Dm[0][1] = 0.0;
                Kl[0][0] = Kl[0][1] = Ku[0][0] = Ku[0][1] = 0.0;
            }
            // D' = D + Kl Cprev ; rhs' = -R + Kl dprev
            double rhs[2] = {-R[2 * x], -R[2 * x + 1]};
            if (x > 1) {
                for (int i = 0; i < 2; ++i) {
                    for (int j = 0; j < 2; ++j) Dm[i][j] += Kl[i][0] * Cprev[0][j] + Kl[i][1] * Cprev[1][j];
                    rhs[i] += Kl[i][0] * dprev[0] + Kl[i][1] * dprev[1];
                }
            }
            double det = Dm[0][0] * Dm[1][1] - Dm[0][1] * Dm[1][0];
            if (!(std::fabs(det) > 0.0)) return false;
            double Di[2][2] = {{Dm[1][1] / det, -Dm[0][1] / det}, {-Dm[1][0] / det, Dm[0][0] / det}};
            // C = D'^-1 (-Ku) (upper neighbour), d = D'^-1 rhs'
            double Cn[2][2];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) Cn[i][j] = -(Di[i][0] * Ku[0][j] + Di[i][1] * Ku[1][j]);
            double dn[2] = {Di[0][0] * rhs[0] + Di[0][1] * rhs[1], Di[1][0] * rhs[0] + Di[1][1] * rhs[1]};
            for (int i = 0; i < 2; ++i) {
                for (int j = 0; j < 2; ++j) { cp[4 * x + 2 * i + j] = Cn[i][j]; Cprev[i][j] = Cn[i][j]; }
                dp[2 * x + i] = dn[i];
                dprev[i] = dn[i];
            }
        }
        // back substitution: u_x = d_x - C_x u_{x+1}
        double nx[2] = {0, 0};
        for (int x = n - 2; x >= 1; --x) {
            double ux[2];
            for (int i = 0; i < 2; ++i) ux[i] = dp[2 * x + i] - (cp[4 * x + 2 * i] * nx[0] + cp[4 * x + 2 * i + 1] * nx[1]);
            du[2 * x] = ux[0];
            du[2 * x + 1] = ux[1];
            nx[0] = ux[0];
            nx[1] = ux[1];
        }
        std::vector<double> r0 = r, p0 = ph;
        for (int x = 1; x < n - 1; ++x) {
            r[x] += du[2 * x];
            ph[x] += du[2 * x + 1];
        }
        bool ok = true;
        for (int x = 1; x < n - 1; ++x) ok = ok && r[x] > 0.0 && std::isfinite(r[x]) && std::isfinite(ph[x]);
        double nres = ok ? residual(R) : INFINITY;
        if (ok && nres < res) {
            res = nres;
            dt = std::fmin(dt * 4.0, 1e12);
        } else {
            r = r0;
            ph = p0;
            residual(R);
            dt *= 0.25;
            if (dt < 1e-10) return false;
        }
    }
    if (res > 1e-10) return false;
    gamma = 0.0;
    for (int x = 1; x < n - 1; ++x) {
        double dr = 0.5 * (r[x + 1] - r[x - 1]), dph = 0.5 * (ph[x + 1] - ph[x - 1]);
        gamma += m.krr * dr * dr + m.kpp * dph * dph + 2.0 * m.kx * dr * dph;
    }
    double lo = -1, hi = -1;
    for (int x = 0; x < n - 1; ++x) {
        double c0 = (r[x] - m.rho_l) / (m.rho_g - m.rho_l), c1 = (r[x + 1] - m.rho_l) / (m.rho_g - m.rho_l);
        if (c0 != c1 && (c0 - 0.9) * (c1 - 0.9) <= 0.0 && lo < 0) lo = x + (0.9 - c0) / (c1 - c0);
        if (c0 != c1 && (c0 - 0.1) * (c1 - 0.1) <= 0.0 && hi < 0) hi = x + (0.1 - c0) / (c1 - c0);
    }
    if (lo < 0 || hi < 0) return false;
    width = std::fabs(hi - lo);
    return true;
}

}  // namespace

bool flat_tension(const double *lam, const double *kap, double rho_l, double rho_g, double chi, double a, double b,
                  double T, double C, double psi0, int pair, int n, double &gamma, double &width)
{
    FE m{};
    m.a = a; m.b = b; m.T = T; m.C = C; m.psi0 = psi0; m.rho_l = rho_l; m.rho_g = rho_g; m.chi = chi;
    for (int k = 0; k < 3; ++k) { m.lam[k] = lam[k]; m.kap[k] = kap[k]; }
    m.derive();
    return flat(m, pair, n, gamma, width);
}

int calibrate(double g12, double g13, double g23, double width, double rho_l, double rho_g, double chi, double a,
              double b, double T, double C, double psi0, double *lam, double *kap)
{
    const double alpha = 0.25 * width;
    const double sum23 = 6.0 * g23 / alpha;
    const double wtarget = 2.0 * alpha * std::log(9.0);
    // unknowns: log lambda1, log kappa1, delta = (lambda2 - lambda3) / sum23
    auto eval = [&](const double *u, double *res) {
        double L[3] = {std::exp(u[0]), 0.5 * sum23 * (1.0 + u[2]), 0.5 * sum23 * (1.0 - u[2])};
        double K[3] = {std::exp(u[1]), alpha * alpha * L[1], alpha * alpha * L[2]};
        double ga, wa, gb, wb;
        if (!flat_tension(L, K, rho_l, rho_g, chi, a, b, T, C, psi0, 12, 64, ga, wa)) return false;
        if (!flat_tension(L, K, rho_l, rho_g, chi, a, b, T, C, psi0, 13, 64, gb, wb)) return false;
        res[0] = std::log(ga / g12);
        res[1] = std::log(gb / g13);
        res[2] = std::log(0.5 * (wa + wb) / wtarget);
        return true;
    };
    double u[3] = {std::log(2.0 * 0.5 * sum23), std::log(alpha * alpha * 0.5 * sum23), 0.0};
    double res[3];
    if (!eval(u, res)) return 1;
    for (int it = 0; it < 40; ++it) {
        double nrm = std::fabs(res[0]) + std::fabs(res[1]) + std::fabs(res[2]);
        if (nrm < 1e-9) break;
        double J[3][3];
        for (int j = 0; j < 3; ++j) {
            double up[3] = {u[0], u[1], u[2]}, rp[3];
            double h = 1e-6;
            up[j] += h;
            if (!eval(up, rp)) return 2;
            for (int i = 0; i < 3; ++i) J[i][j] = (rp[i] - res[i]) / h;
        }
        // solve J du = -res (Cramer)
        double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        if (!(std::fabs(det) > 1e-300)) return 3;
        double du[3];
        for (int c = 0; c < 3; ++c) {
            double M[3][3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) M[i][j] = (j == c) ? -res[i] : J[i][j];
            du[c] = (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                     M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0])) / det;
        }
        // damped step: accept the first halving that lowers the residual
        double lamb = 1.0;
        bool acc = false;
        for (int k = 0; k < 30; ++k) {
            double un[3] = {u[0] + lamb * du[0], u[1] + lamb * du[1], u[2] + lamb * du[2]}, rn[3];
            if (std::fabs(un[2]) < 1.0 && eval(un, rn) &&
                std::fabs(rn[0]) + std::fabs(rn[1]) + std::fabs(rn[2]) < nrm) {
                for (int i = 0; i < 3; ++i) { u[i] = un[i]; res[i] = rn[i]; }
                acc = true;
                break;
            }
            lamb *= 0.5;
        }
        if (!acc) return 4;
    }
    if (std::fabs(res[0]) + std::fabs(res[1]) + std::fabs(res[2]) > 1e-6) return 5;
    lam[0] = std::exp(u[0]);
    lam[1] = 0.5 * sum23 * (1.0 + u[2]);
    lam[2] = 0.5 * sum23 * (1.0 - u[2]);
    kap[0] = std::exp(u[1]);
    kap[1] = alpha * alpha * lam[1];
    kap[2] = alpha * alpha * lam[2];
    return 0;
}

}  // namespace lbm3h
