// Host-side solver set-up of relpic (internal).
#pragma once

#include <vector>

namespace relpic {

bool fit_axial_coefficients(double kappa, int M, int p, double wk1, double nsg, int nq, std::vector<double> &C);
double axial_symbol_max(const double *C, int M);
double courant_number(int ndim, const double *dx, double dt, const double *C, int M);
bool correction_taps(const double *C, int M, double tol, int max_taps, std::vector<double> &taps);

}  // namespace relpic
