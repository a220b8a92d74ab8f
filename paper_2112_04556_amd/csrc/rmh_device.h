// Device-side building blocks of the adjoint-Laplacian library (gfx950).
//
// Layouts (structure of arrays, site index s = x0 + L0*(x1 + L1*(x2 + L2*x3))):
//   links   U[mu][18][V]  : U_mu(x)_ij, component 2*(3i+j) = Re, 2*(3i+j)+1 = Im
//   fields  P[v][8][V]    : v runs over (rhs, nu) pairs, component a of the su(3)
//                           element sum_a P^a T^a, T^a = lambda^a/2 (Gell-Mann a+1)
//
// The adjoint action U phi U^dag of a link on an su(3) element is the 8x8
// orthogonal matrix R^{ab}(U) = 2 Tr(T^a U T^b U^dag) acting on the components;
// U^dag phi U uses R(U)^T.  R is built here from bilinears of U's columns,
// exploiting that every T^b has at most three non-zero entries.
//
// All functions are __host__ __device__ so the arithmetic can also be compiled
// and exercised on the CPU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rmh {

#define RMH_HD __host__ __device__ __forceinline__

constexpr double kInvSqrt3 = 0.57735026918962576451;

// Lattice geometry passed by value to kernels.
struct Geom {
  int32_t L0, L1, L2, L3;
  int32_t V;
};

// Flat index of x + mu (sign = +1) or x - mu (sign = -1) from coordinates.
RMH_HD int32_t site_shift(const Geom& g, int32_t s, int32_t x[4], int mu, int sign) {
  const int32_t Ls[4] = {g.L0, g.L1, g.L2, g.L3};
  const int32_t stride[4] = {1, g.L0, g.L0 * g.L1, g.L0 * g.L1 * g.L2};
  int32_t xm = x[mu];
  if (sign > 0) return (xm == Ls[mu] - 1) ? s - (Ls[mu] - 1) * stride[mu] : s + stride[mu];
  return (xm == 0) ? s + (Ls[mu] - 1) * stride[mu] : s - stride[mu];
}

RMH_HD void site_coords(const Geom& g, int32_t s, int32_t x[4]) {
  int32_t r = s;
  x[0] = r % g.L0; r /= g.L0;
  x[1] = r % g.L1; r /= g.L1;
  x[2] = r % g.L2;
  x[3] = r / g.L2;
}

// R^{ab}(U) = 2 Tr(T^a U T^b U^dag), written into R[a*8+b] (row a, column b).
// u[2*(3i+j)] + i u[2*(3i+j)+1] = U_ij.
//
// Column b is the component vector of Y_b = U T^b U^dag.  With u_k the k-th
// column of U, M = u_k u_l^dag (M_ij = U_ik conj(U_jl)):
//   pair (k,l) symmetric generator:      Y = (M + M^dag)/2
//   pair (k,l) antisymmetric generator:  Y = -i (M - M^dag)/2
//   T^3 = (E00 - E11)/2,  T^8 = (E00 + E11 - 2 E22)/(2 sqrt 3): Y from N_k = u_k u_k^dag.
// Components of a Hermitian Y: pair (i,j) -> (2 Re Y_ij, -2 Im Y_ij);
// a=3 -> Y00 - Y11; a=8 -> (Y00 + Y11 - 2 Y22)/sqrt 3.
template <typename T>
RMH_HD void adjoint_matrix(const T* u, T* R) {
  // generator index of the (symmetric, antisymmetric) pair for (0,1), (0,2), (1,2)
  constexpr int pr_i[3] = {0, 0, 1};
  constexpr int pr_j[3] = {1, 2, 2};
  constexpr int pr_s[3] = {0, 3, 5};  // symmetric generator (lambda 1, 4, 6); antisymmetric = +1
#define URE(i, k) u[2 * (3 * (i) + (k))]
#define UIM(i, k) u[2 * (3 * (i) + (k)) + 1]
  // Columns of the off-diagonal generators.
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int k = pr_i[q], l = pr_j[q];
    T mre[3][3], mim[3][3];  // M_ij = U_ik conj(U_jl)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        mre[i][j] = URE(i, k) * URE(j, l) + UIM(i, k) * UIM(j, l);
        mim[i][j] = UIM(i, k) * URE(j, l) - URE(i, k) * UIM(j, l);
      }
    const int bs = pr_s[q], ba = pr_s[q] + 1;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const int i = pr_i[p], j = pr_j[p];
      const int as = pr_s[p], aa = pr_s[p] + 1;
      R[as * 8 + bs] = mre[i][j] + mre[j][i];
      R[aa * 8 + bs] = mim[j][i] - mim[i][j];
      R[as * 8 + ba] = mim[i][j] + mim[j][i];
      R[aa * 8 + ba] = mre[i][j] - mre[j][i];
    }
    R[2 * 8 + bs] = mre[0][0] - mre[1][1];
    R[7 * 8 + bs] = (mre[0][0] + mre[1][1] - T(2) * mre[2][2]) * T(kInvSqrt3);
    R[2 * 8 + ba] = mim[0][0] - mim[1][1];
    R[7 * 8 + ba] = (mim[0][0] + mim[1][1] - T(2) * mim[2][2]) * T(kInvSqrt3);
  }
  // Columns of T^3 and T^8 from N_k = u_k u_k^dag (Hermitian).
  T nre[3][3][3], nim[3][3];  // nre[k][i][j] for i<=j used; nim[k][pair]
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int i = 0; i < 3; ++i) nre[k][i][i] = URE(i, k) * URE(i, k) + UIM(i, k) * UIM(i, k);
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const int i = pr_i[p], j = pr_j[p];
      nre[k][i][j] = URE(i, k) * URE(j, k) + UIM(i, k) * UIM(j, k);
      nim[k][p] = UIM(i, k) * URE(j, k) - URE(i, k) * UIM(j, k);
    }
  }
  // Y3 = (N0 - N1)/2, Y8 = (N0 + N1 - 2 N2)/(2 sqrt 3)
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const int i = pr_i[p], j = pr_j[p];
    const int as = pr_s[p], aa = pr_s[p] + 1;
    const T d3re = nre[0][i][j] - nre[1][i][j];
    const T d3im = nim[0][p] - nim[1][p];
    const T d8re = (nre[0][i][j] + nre[1][i][j] - T(2) * nre[2][i][j]) * T(kInvSqrt3);
    const T d8im = (nim[0][p] + nim[1][p] - T(2) * nim[2][p]) * T(kInvSqrt3);
    R[as * 8 + 2] = d3re;   // 2 Re Y_ij with Y = (N0 - N1)/2
    R[aa * 8 + 2] = -d3im;
    R[as * 8 + 7] = d8re;
    R[aa * 8 + 7] = -d8im;
  }
  {
    T y3[3], y8[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      y3[i] = T(0.5) * (nre[0][i][i] - nre[1][i][i]);
      y8[i] = T(0.5) * T(kInvSqrt3) * (nre[0][i][i] + nre[1][i][i] - T(2) * nre[2][i][i]);
    }
    R[2 * 8 + 2] = y3[0] - y3[1];
    R[7 * 8 + 2] = (y3[0] + y3[1] - T(2) * y3[2]) * T(kInvSqrt3);
    R[2 * 8 + 7] = y8[0] - y8[1];
    R[7 * 8 + 7] = (y8[0] + y8[1] - T(2) * y8[2]) * T(kInvSqrt3);
  }
#undef URE
#undef UIM
}

// acc += R phi   (forward hop: U phi U^dag)
template <typename T>
RMH_HD void adj_apply(const T* R, const T* phi, T* acc) {
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    T s = acc[a];
#pragma unroll
    for (int b = 0; b < 8; ++b) s += R[a * 8 + b] * phi[b];
    acc[a] = s;
  }
}

// acc += R^T phi (backward hop: U^dag phi U)
template <typename T>
RMH_HD void adj_apply_t(const T* R, const T* phi, T* acc) {
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const T p = phi[b];
#pragma unroll
    for (int a = 0; a < 8; ++a) acc[a] += R[b * 8 + a] * p;
  }
}

// Fundamental-representation form of the same hop: acc += comps(U Phi U^dag)
// (dagger = false) or comps(U^dag Phi U) (dagger = true), Phi = sum_a phi^a T^a.
template <typename T, bool kDagger>
RMH_HD void mat_hop(const T* u, const T* phi, T* acc) {
  // Phi (Hermitian): diagonal d[i], upper off-diagonal o[p] for pairs (0,1),(0,2),(1,2)
  const T h = T(0.5);
  T dre[3], ore[3], oim[3];
  dre[0] = h * phi[2] + h * T(kInvSqrt3) * phi[7];
  dre[1] = -h * phi[2] + h * T(kInvSqrt3) * phi[7];
  dre[2] = -T(kInvSqrt3) * phi[7];
  ore[0] = h * phi[0]; oim[0] = -h * phi[1];
  ore[1] = h * phi[3]; oim[1] = -h * phi[4];
  ore[2] = h * phi[5]; oim[2] = -h * phi[6];
  // full Phi as 3x3 complex
  T pre[3][3], pim[3][3];
  pre[0][0] = dre[0]; pim[0][0] = 0;
  pre[1][1] = dre[1]; pim[1][1] = 0;
  pre[2][2] = dre[2]; pim[2][2] = 0;
  pre[0][1] = ore[0]; pim[0][1] = oim[0]; pre[1][0] = ore[0]; pim[1][0] = -oim[0];
  pre[0][2] = ore[1]; pim[0][2] = oim[1]; pre[2][0] = ore[1]; pim[2][0] = -oim[1];
  pre[1][2] = ore[2]; pim[1][2] = oim[2]; pre[2][1] = ore[2]; pim[2][1] = -oim[2];
  // A = U (or U^dag) as explicit 3x3
  T are[3][3], aim[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      if (!kDagger) {
        are[i][j] = u[2 * (3 * i + j)];
        aim[i][j] = u[2 * (3 * i + j) + 1];
      } else {
        are[i][j] = u[2 * (3 * j + i)];
        aim[i][j] = -u[2 * (3 * j + i) + 1];
      }
    }
  // W = A Phi
  T wre[3][3], wim[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      T sr = 0, si = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        sr += are[i][k] * pre[k][j] - aim[i][k] * pim[k][j];
        si += are[i][k] * pim[k][j] + aim[i][k] * pre[k][j];
      }
      wre[i][j] = sr;
      wim[i][j] = si;
    }
  // Y = W A^dag : Y_ij = sum_k W_ik conj(A_jk); only the diagonal (real) and upper part
  T yd[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T sr = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) sr += wre[i][k] * are[i][k] + wim[i][k] * aim[i][k];
    yd[i] = sr;
  }
  constexpr int pi_[3] = {0, 0, 1};
  constexpr int pj_[3] = {1, 2, 2};
  constexpr int ps_[3] = {0, 3, 5};
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const int i = pi_[p], j = pj_[p];
    T sr = 0, si = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      sr += wre[i][k] * are[j][k] + wim[i][k] * aim[j][k];
      si += wim[i][k] * are[j][k] - wre[i][k] * aim[j][k];
    }
    acc[ps_[p]] += T(2) * sr;
    acc[ps_[p] + 1] += -T(2) * si;
  }
  acc[2] += yd[0] - yd[1];
  acc[7] += (yd[0] + yd[1] - T(2) * yd[2]) * T(kInvSqrt3);
}

}  // namespace rmh
