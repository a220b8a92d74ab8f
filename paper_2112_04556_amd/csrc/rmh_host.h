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

}  // namespace rmh
