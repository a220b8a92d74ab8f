// Host-side FP64 helpers (no HIP).
#pragma once

#include <stdint.h>

namespace rmh {

void jackson_factors(int32_t D, double* g);
int cheb_window_coefficients(int32_t D, int32_t nw, const double* edges, int32_t kernel, double* coef);
void trace_moments_free(const int32_t L[4], int32_t D, double* tau);
int rational_from_quadratics(int32_t n, const double* a0, const double* a1, const double* b0, const double* b1,
                             double* r, double* sigma);
int rational_kappa(double kappa, int32_t n, double* c, double* r, double* sigma);
// Partial fractions of 1/R for R(l) = c + sum_j r_j / (l + sigma_j) with c >= 0, r_j > 0 and distinct
// sigma_j > 0: 1/R(l) = a l + b + sum_k rho_k / (l + tau_k), k < m (m = n - 1 for c = 0, n for c > 0),
// tau_k > 0 the negated zeros of R (one between each pair of neighbouring poles, and for c > 0 one
// below the lowest), rho_k = 1 / R'(-tau_k) < 0.  Returns 0, or -1 when R has no such form.
int rational_inverse(double c, int32_t n, const double* r, const double* sigma, double* a, double* b, double* rho,
                     double* tau, int32_t* m);

}  // namespace rmh
