// Host-side solver set-up of relpic (internal).
#pragma once

#include <vector>

namespace relpic {

// target_kind 0: [k1]_t (App. C); 1: [k1]_t^2 / [k]_Yee (operator on E, Yee on B)
bool fit_axial_coefficients(double kappa, int M, int p, double wk1, double nsg, int nq, std::vector<double> &C,
                            int target_kind = 0);
double axial_symbol_max(const double *C, int M);
double courant_number(int ndim, const double *dx, double dt, const double *C, int M);
// (dt/2) sqrt(max [k]_E1 [k]_B1 + sum_d [k]_d^2) with different axial operators on E and on B
double courant_number2(int ndim, const double *dx, double dt, const double *CE, const double *CB, int M);
double axial_product_max(const double *CE, const double *CB, int M);
bool correction_taps(const double *C, int M, double tol, int max_taps, std::vector<double> &taps);

}  // namespace relpic
