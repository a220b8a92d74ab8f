// Host-side FP64 arithmetic of the library: Chebyshev window coefficients with Jackson
// damping (section 2), the exact free-field trace moments, moment -> window combination
// (Eq. 4), and the rational pole sets of the mass term (section 3, Eq. 6).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "rmh_host.h"

namespace rmh {

static const double kPi = 3.14159265358979323846;

// Jackson kernel factors for degree D (N = D + 1 moments), Weisse et al. 2006:
// g_k = [(N-k+1) cos(pi k/(N+1)) + sin(pi k/(N+1)) cot(pi/(N+1))] / (N+1).
void jackson_factors(int32_t D, double* g) {
  const double N = D + 1;
  const double q = kPi / (N + 1.0);
  const double cotq = cos(q) / sin(q);
  for (int32_t k = 0; k <= D; ++k) g[k] = ((N - k + 1.0) * cos(q * k) + sin(q * k) * cotq) / (N + 1.0);
}

// coef[w][k] = g_k c^w_k, with c^w the Chebyshev series of the indicator of
// [e_w, e_{w+1}] in x = lambda/8 - 1:  theta = arccos x,
// c_0 = (theta_lo - theta_hi)/pi,  c_k = 2 (sin(k theta_lo) - sin(k theta_hi)) / (k pi).
int cheb_window_coefficients(int32_t D, int32_t nw, const double* edges, int32_t kernel, double* coef) {
  std::vector<double> e(nw + 1);
  for (int32_t w = 0; w <= nw; ++w) e[w] = edges ? edges[w] : 16.0 * w / nw;
  for (int32_t w = 0; w < nw; ++w)
    if (!(e[w] < e[w + 1]) || e[w] < 0.0 || e[w + 1] > 16.0) return -1;
  std::vector<double> g(D + 1, 1.0);
  if (kernel == 1) jackson_factors(D, g.data());
  for (int32_t w = 0; w < nw; ++w) {
    double xl = e[w] / 8.0 - 1.0, xh = e[w + 1] / 8.0 - 1.0;
    xl = xl < -1.0 ? -1.0 : (xl > 1.0 ? 1.0 : xl);
    xh = xh < -1.0 ? -1.0 : (xh > 1.0 ? 1.0 : xh);
    const double tl = acos(xl), th = acos(xh);
    double* c = coef + (size_t)w * (D + 1);
    c[0] = g[0] * (tl - th) / kPi;
    for (int32_t k = 1; k <= D; ++k) c[k] = g[k] * 2.0 * (sin(k * tl) - sin(k * th)) / (k * kPi);
  }
  return 0;
}

// Tr T_k(Delta/8 - 1) over the link-field space at U = 1: the spectrum of Delta is
// 4 sum_mu sin^2(pi n_mu / L_mu) on each of 8 colours x 4 directions.
void trace_moments_free(const int32_t L[4], int32_t D, double* tau) {
  for (int32_t k = 0; k <= D; ++k) tau[k] = 0.0;
  std::vector<double> s[4];
  for (int mu = 0; mu < 4; ++mu) {
    s[mu].resize(L[mu]);
    for (int32_t n = 0; n < L[mu]; ++n) {
      const double h = sin(kPi * n / L[mu]);
      s[mu][n] = 4.0 * h * h;
    }
  }
  for (int32_t n3 = 0; n3 < L[3]; ++n3)
    for (int32_t n2 = 0; n2 < L[2]; ++n2)
      for (int32_t n1 = 0; n1 < L[1]; ++n1)
        for (int32_t n0 = 0; n0 < L[0]; ++n0) {
          const double lam = s[0][n0] + s[1][n1] + s[2][n2] + s[3][n3];
          double x = lam / 8.0 - 1.0;
          x = x < -1.0 ? -1.0 : (x > 1.0 ? 1.0 : x);
          // T_k(x) by the three-term recursion
          double t0 = 1.0, t1 = x;
          tau[0] += 32.0;
          if (D >= 1) tau[1] += 32.0 * t1;
          for (int32_t k = 2; k <= D; ++k) {
            const double t2 = 2.0 * x * t1 - t0;
            tau[k] += 32.0 * t2;
            t0 = t1;
            t1 = t2;
          }
        }
}

// (a0 + a1 L) / (b0 + b1 L + L^2) = rho1/(L + s1) + rho2/(L + s2) with s1 + s2 = b1,
// s1 s2 = b0; in Delta = 16 L units: r = 16 rho, sigma = 16 s.
int rational_from_quadratics(int32_t n, const double* a0, const double* a1, const double* b0,
                             const double* b1, double* r, double* sigma) {
  for (int32_t i = 0; i < n; ++i) {
    const double disc = b1[i] * b1[i] - 4.0 * b0[i];
    if (!(disc > 0.0)) return -1;
    const double q = sqrt(disc);
    const double s1 = 0.5 * (b1[i] - q), s2 = 0.5 * (b1[i] + q);
    if (!(s1 > 0.0) || !(s2 > 0.0)) return -1;
    r[2 * i] = 16.0 * (a0[i] - a1[i] * s1) / (s2 - s1);
    sigma[2 * i] = 16.0 * s1;
    r[2 * i + 1] = 16.0 * (a0[i] - a1[i] * s2) / (s1 - s2);
    sigma[2 * i + 1] = 16.0 * s2;
  }
  return 0;
}

// Midpoint rule on y^{-1/2} = (2/pi) sqrt(s) int_0^{pi/2} dt / (s sin^2 t + y cos^2 t),
// y = 1 - kappa + kappa Delta, nodes t_j = (2j - 1) pi / (4n):
// y^{-1/2} ~ sum_j sqrt(s)/(n cos^2 t_j) / (s tan^2 t_j + y).
int rational_kappa(double kappa, int32_t n, double* c, double* r, double* sigma) {
  if (!(kappa > 0.0 && kappa < 1.0) || n < 1) return -1;
  const double s = sqrt((1.0 - kappa) * (1.0 + 15.0 * kappa));
  *c = 0.0;
  for (int32_t j = 1; j <= n; ++j) {
    const double t = (2.0 * j - 1.0) * kPi / (4.0 * n);
    const double ct = cos(t), tt = tan(t);
    r[j - 1] = sqrt(s) / (n * kappa * ct * ct);
    sigma[j - 1] = (1.0 - kappa + s * tt * tt) / kappa;
  }
  return 0;
}

int rational_inverse(double c, int32_t n, const double* r, const double* sigma, double* a, double* b, double* rho,
                     double* tau, int32_t* m) {
  if (n < 1 || !(c >= 0.0)) return -1;
  std::vector<double> sg(sigma, sigma + n), rr(r, r + n);
  // poles sorted by sigma (ascending), each with its residue
  std::vector<int> ord(n);
  for (int j = 0; j < n; ++j) ord[j] = j;
  std::sort(ord.begin(), ord.end(), [&](int i, int j) { return sg[i] < sg[j]; });
  std::vector<double> s_(n), r_(n);
  for (int j = 0; j < n; ++j) {
    s_[j] = sg[ord[j]];
    r_[j] = rr[ord[j]];
    if (!(r_[j] > 0.0) || !(s_[j] > 0.0)) return -1;
    if (j && !(s_[j] > s_[j - 1])) return -1;
  }
  auto R = [&](double l) {
    double v = c;
    for (int j = 0; j < n; ++j) v += r_[j] / (l + s_[j]);
    return v;
  };
  auto dR = [&](double l) {
    double v = 0.0;
    for (int j = 0; j < n; ++j) v -= r_[j] / ((l + s_[j]) * (l + s_[j]));
    return v;
  };
  // R decreases strictly between neighbouring poles, from +inf to -inf: one zero in each gap
  // (-s_{j+1}, -s_j), found by bisection to the last bit; for c > 0 one more below -s_{n-1}
  std::vector<double> z;
  auto bisect = [&](double lo, double hi) {   // R(lo) > 0 > R(hi)
    for (int it = 0; it < 400; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (R(mid) > 0.0)
        lo = mid;
      else
        hi = mid;
    }
    return 0.5 * (lo + hi);
  };
  for (int j = 0; j + 1 < n; ++j) {
    const double w = s_[j + 1] - s_[j];
    double lo = -s_[j + 1] + 1e-300, hi = -s_[j] - 1e-300;
    // step inside the gap until the signs are established
    double e = w * 1e-3;
    while (!(R(-s_[j + 1] + e) > 0.0) && e > 1e-300) e *= 0.5;
    lo = -s_[j + 1] + e;
    e = w * 1e-3;
    while (!(R(-s_[j] - e) < 0.0) && e > 1e-300) e *= 0.5;
    hi = -s_[j] - e;
    if (!(R(lo) > 0.0 && R(hi) < 0.0)) return -1;
    z.push_back(bisect(lo, hi));
  }
  if (c > 0.0) {
    // below the lowest pole R -> c > 0 at -inf and -> -inf at -s_{n-1}
    double e = 1e-3 * s_[n - 1];
    while (!(R(-s_[n - 1] - e) < 0.0) && e > 1e-300) e *= 0.5;
    const double hi = -s_[n - 1] - e;
    double lo = hi - 1.0;
    while (!(R(lo) > 0.0)) {
      lo = hi - 2.0 * (hi - lo);
      if (lo < -1e300) return -1;
    }
    if (!(R(hi) < 0.0)) return -1;
    z.push_back(bisect(lo, hi));
  }
  *m = (int32_t)z.size();
  for (size_t k = 0; k < z.size(); ++k) {
    tau[k] = -z[k];
    rho[k] = 1.0 / dR(z[k]);
    if (!(tau[k] > 0.0) || !(rho[k] < 0.0)) return -1;
  }
  // polynomial part: 1/R(l) - sum_k rho_k/(l + tau_k) = a l + b; for c = 0, a = 1/S1 and
  // b = S2/S1^2 + sum ... fixed by the values at two points instead (exact for a polynomial of degree 1)
  auto rest = [&](double l) {
    double v = 1.0 / R(l);
    for (size_t k = 0; k < z.size(); ++k) v -= rho[k] / (l + tau[k]);
    return v;
  };
  const double f0 = rest(0.0), f16 = rest(16.0);
  *a = (f16 - f0) / 16.0;
  *b = f0;
  if (c > 0.0) *a = 0.0;
  // the form must reproduce 1/R across the spectrum [0, 16]
  for (int q = 0; q <= 32; ++q) {
    const double l = 0.5 * q;
    double v = *a * l + *b;
    for (size_t k = 0; k < z.size(); ++k) v += rho[k] / (l + tau[k]);
    const double ref = 1.0 / R(l);
    if (!(std::fabs(v - ref) <= 1e-11 * std::fabs(ref))) return -1;
  }
  return 0;
}

}  // namespace rmh
