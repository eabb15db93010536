// Host-side thermodynamics of the lbm3 library (internal).
#pragma once

namespace lbm3h {

// Carnahan-Starling coexistence at density ratio `ratio` (paper's a/b kept),
// rescaled to liquid density rho_l_target.  Returns false if no solution.
bool coexistence(double ratio, double rho_l_target, double &a, double &b, double &T, double &C, double &psi0,
                 double &rho_l, double &rho_g);

}  // namespace lbm3h

namespace lbm3h {
// Flat-interface tension and 10-90 % gas width (pair 12 or 13) on a 1D
// lattice of n nodes; false if the relaxation fails.
bool flat_tension(const double *lam, const double *kap, double rho_l, double rho_g, double chi, double a, double b,
                  double T, double C, double psi0, int pair, int n, double &gamma, double &width);
// (gamma12, gamma13, gamma23, width) -> lambda[3], kappa[3]; 0 on success.
int calibrate(double g12, double g13, double g23, double width, double rho_l, double rho_g, double chi, double a,
              double b, double T, double C, double psi0, double *lam, double *kap);
}  // namespace lbm3h
