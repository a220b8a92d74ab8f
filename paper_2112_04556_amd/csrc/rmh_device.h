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

// Every multiply-add of the per-site arithmetic is an explicit fused multiply-add and the
// library is compiled with -ffp-contract=off, so the rounding of a result is fixed by the
// source alone (identical for every launch configuration of one form).
RMH_HD double fmadd(double a, double b, double c) { return fma(a, b, c); }
RMH_HD float fmadd(float a, float b, float c) { return fmaf(a, b, c); }

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
        mre[i][j] = fmadd(URE(i, k), URE(j, l), UIM(i, k) * UIM(j, l));
        mim[i][j] = fmadd(UIM(i, k), URE(j, l), -(URE(i, k) * UIM(j, l)));
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
    R[7 * 8 + bs] = fmadd(T(-2), mre[2][2], mre[0][0] + mre[1][1]) * T(kInvSqrt3);
    R[2 * 8 + ba] = mim[0][0] - mim[1][1];
    R[7 * 8 + ba] = fmadd(T(-2), mim[2][2], mim[0][0] + mim[1][1]) * T(kInvSqrt3);
  }
  // Columns of T^3 and T^8 from N_k = u_k u_k^dag (Hermitian).
  T nre[3][3][3], nim[3][3];  // nre[k][i][j] for i<=j used; nim[k][pair]
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int i = 0; i < 3; ++i) nre[k][i][i] = fmadd(URE(i, k), URE(i, k), UIM(i, k) * UIM(i, k));
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const int i = pr_i[p], j = pr_j[p];
      nre[k][i][j] = fmadd(URE(i, k), URE(j, k), UIM(i, k) * UIM(j, k));
      nim[k][p] = fmadd(UIM(i, k), URE(j, k), -(URE(i, k) * UIM(j, k)));
    }
  }
  // Y3 = (N0 - N1)/2, Y8 = (N0 + N1 - 2 N2)/(2 sqrt 3)
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const int i = pr_i[p], j = pr_j[p];
    const int as = pr_s[p], aa = pr_s[p] + 1;
    const T d3re = nre[0][i][j] - nre[1][i][j];
    const T d3im = nim[0][p] - nim[1][p];
    const T d8re = fmadd(T(-2), nre[2][i][j], nre[0][i][j] + nre[1][i][j]) * T(kInvSqrt3);
    const T d8im = fmadd(T(-2), nim[2][p], nim[0][p] + nim[1][p]) * T(kInvSqrt3);
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
      y8[i] = T(0.5) * T(kInvSqrt3) * fmadd(T(-2), nre[2][i][i], nre[0][i][i] + nre[1][i][i]);
    }
    R[2 * 8 + 2] = y3[0] - y3[1];
    R[7 * 8 + 2] = fmadd(T(-2), y3[2], y3[0] + y3[1]) * T(kInvSqrt3);
    R[2 * 8 + 7] = y8[0] - y8[1];
    R[7 * 8 + 7] = fmadd(T(-2), y8[2], y8[0] + y8[1]) * T(kInvSqrt3);
  }
#undef URE
#undef UIM
}

// The two columns of R(U) that belong to generator group q, written into c1[8], c2[8]:
// q = 0, 1, 2: the symmetric / antisymmetric generators of the pair (0,1), (0,2), (1,2)
// (columns 0/1, 3/4, 5/6); q = 3: the diagonal generators T^3, T^8 (columns 2 and 7).
// Same bilinears of the columns of U as adjoint_matrix, one group at a time.
template <typename T, int q>
RMH_HD void adjoint_columns(const T* u, T* c1, T* c2) {
  constexpr int pr_i[3] = {0, 0, 1};
  constexpr int pr_j[3] = {1, 2, 2};
  constexpr int pr_s[3] = {0, 3, 5};
#define URE(i, k) u[2 * (3 * (i) + (k))]
#define UIM(i, k) u[2 * (3 * (i) + (k)) + 1]
  if (q < 3) {
    constexpr int k = pr_i[q < 3 ? q : 0], l = pr_j[q < 3 ? q : 0];
    T mre[3][3], mim[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        mre[i][j] = fmadd(URE(i, k), URE(j, l), UIM(i, k) * UIM(j, l));
        mim[i][j] = fmadd(UIM(i, k), URE(j, l), -(URE(i, k) * UIM(j, l)));
      }
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const int i = pr_i[p], j = pr_j[p];
      const int as = pr_s[p], aa = pr_s[p] + 1;
      c1[as] = mre[i][j] + mre[j][i];
      c1[aa] = mim[j][i] - mim[i][j];
      c2[as] = mim[i][j] + mim[j][i];
      c2[aa] = mre[i][j] - mre[j][i];
    }
    c1[2] = mre[0][0] - mre[1][1];
    c1[7] = fmadd(T(-2), mre[2][2], mre[0][0] + mre[1][1]) * T(kInvSqrt3);
    c2[2] = mim[0][0] - mim[1][1];
    c2[7] = fmadd(T(-2), mim[2][2], mim[0][0] + mim[1][1]) * T(kInvSqrt3);
  } else {
    T nd[3][3], nre[3][3], nim[3][3];  // [k][i] diagonal |U_ik|^2; [k][pair] off-diagonal of u_k u_k^dag
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
#pragma unroll
      for (int i = 0; i < 3; ++i) nd[kk][i] = fmadd(URE(i, kk), URE(i, kk), UIM(i, kk) * UIM(i, kk));
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        const int i = pr_i[p], j = pr_j[p];
        nre[kk][p] = fmadd(URE(i, kk), URE(j, kk), UIM(i, kk) * UIM(j, kk));
        nim[kk][p] = fmadd(UIM(i, kk), URE(j, kk), -(URE(i, kk) * UIM(j, kk)));
      }
    }
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const int as = pr_s[p], aa = pr_s[p] + 1;
      c1[as] = nre[0][p] - nre[1][p];
      c1[aa] = -(nim[0][p] - nim[1][p]);
      c2[as] = fmadd(T(-2), nre[2][p], nre[0][p] + nre[1][p]) * T(kInvSqrt3);
      c2[aa] = -fmadd(T(-2), nim[2][p], nim[0][p] + nim[1][p]) * T(kInvSqrt3);
    }
    T y3[3], y8[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      y3[i] = T(0.5) * (nd[0][i] - nd[1][i]);
      y8[i] = T(0.5) * T(kInvSqrt3) * fmadd(T(-2), nd[2][i], nd[0][i] + nd[1][i]);
    }
    c1[2] = y3[0] - y3[1];
    c1[7] = fmadd(T(-2), y3[2], y3[0] + y3[1]) * T(kInvSqrt3);
    c2[2] = y8[0] - y8[1];
    c2[7] = fmadd(T(-2), y8[2], y8[0] + y8[1]) * T(kInvSqrt3);
  }
#undef URE
#undef UIM
}

// Row 2 of an SU(3) matrix from rows 0 and 1 (u as in adjoint_matrix): for a unitary matrix of
// unit determinant each row is the complex conjugate of the cross product of the other two,
// U_2j = conj(U_0k U_1l - U_0l U_1k) with (j, k, l) a cyclic permutation of (0, 1, 2).
template <typename T>
RMH_HD void su3_row2(T* u) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int k = (j + 1) % 3, l = (j + 2) % 3;
    const T ar = u[2 * k], ai = u[2 * k + 1];            // U_0k
    const T br = u[6 + 2 * l], bi = u[6 + 2 * l + 1];    // U_1l
    const T cr = u[2 * l], ci = u[2 * l + 1];            // U_0l
    const T dr = u[6 + 2 * k], di = u[6 + 2 * k + 1];    // U_1k
    u[12 + 2 * j] = (ar * br - ai * bi) - (cr * dr - ci * di);
    u[12 + 2 * j + 1] = (cr * di + ci * dr) - (ar * bi + ai * br);
  }
}

// Column indices of group q (see adjoint_columns).
template <int q>
struct ColPair {
  static constexpr int b1 = q == 0 ? 0 : q == 1 ? 3 : q == 2 ? 5 : 2;
  static constexpr int b2 = q == 0 ? 1 : q == 1 ? 4 : q == 2 ? 6 : 7;
};

// Streamed adjoint action on NV vectors: acc += R phi (kT = false) or acc += R^T phi (kT = true),
// building R two columns at a time so the 8x8 matrix is never held in registers.
template <typename T, int NV, bool kT, int q>
RMH_HD void adj_stream_group(const T* u, const T (*phi)[8], T (*acc)[8]) {
  T c1[8], c2[8];
  adjoint_columns<T, q>(u, c1, c2);
  constexpr int b1 = ColPair<q>::b1, b2 = ColPair<q>::b2;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if (!kT) {
#pragma unroll
      for (int a = 0; a < 8; ++a) acc[v][a] = fmadd(c2[a], phi[v][b2], fmadd(c1[a], phi[v][b1], acc[v][a]));
    } else {
      T s1 = acc[v][b1], s2 = acc[v][b2];
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        s1 = fmadd(c1[a], phi[v][a], s1);
        s2 = fmadd(c2[a], phi[v][a], s2);
      }
      acc[v][b1] = s1;
      acc[v][b2] = s2;
    }
  }
}

template <typename T, int NV, bool kT>
RMH_HD void adj_stream(const T* u, const T (*phi)[8], T (*acc)[8]) {
  adj_stream_group<T, NV, kT, 0>(u, phi, acc);
  adj_stream_group<T, NV, kT, 1>(u, phi, acc);
  adj_stream_group<T, NV, kT, 2>(u, phi, acc);
  adj_stream_group<T, NV, kT, 3>(u, phi, acc);
}

// acc += R phi   (forward hop: U phi U^dag)
template <typename T>
RMH_HD void adj_apply(const T* R, const T* phi, T* acc) {
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    T s = acc[a];
#pragma unroll
    for (int b = 0; b < 8; ++b) s = fmadd(R[a * 8 + b], phi[b], s);
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
    for (int a = 0; a < 8; ++a) acc[a] = fmadd(R[b * 8 + a], p, acc[a]);
  }
}

// Fundamental-representation form of the same hop: acc += comps(U Phi U^dag)
// (dagger = false) or comps(U^dag Phi U) (dagger = true), Phi = sum_a phi^a T^a.
template <typename T, bool kDagger>
RMH_HD void mat_hop(const T* u, const T* phi, T* acc) {
  // Phi (Hermitian): diagonal d[i], upper off-diagonal o[p] for pairs (0,1),(0,2),(1,2)
  const T h = T(0.5);
  T dre[3], ore[3], oim[3];
  dre[0] = fmadd(h, phi[2], h * T(kInvSqrt3) * phi[7]);
  dre[1] = fmadd(-h, phi[2], h * T(kInvSqrt3) * phi[7]);
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
  // W = A Phi (the diagonal of Phi is real: its imaginary terms are left out)
  T wre[3][3], wim[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      T sr = 0, si = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (k == j) {
          sr = fmadd(are[i][k], pre[k][j], sr);
          si = fmadd(aim[i][k], pre[k][j], si);
        } else {
          sr = fmadd(are[i][k], pre[k][j], fmadd(-aim[i][k], pim[k][j], sr));
          si = fmadd(are[i][k], pim[k][j], fmadd(aim[i][k], pre[k][j], si));
        }
      }
      wre[i][j] = sr;
      wim[i][j] = si;
    }
  // Y = W A^dag : Y_ij = sum_k W_ik conj(A_jk); only the diagonal (real) and upper part; Y is
  // traceless with Phi, so Y_22 = -(Y_00 + Y_11)
  T yd[3];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    T sr = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) sr = fmadd(wre[i][k], are[i][k], fmadd(wim[i][k], aim[i][k], sr));
    yd[i] = sr;
  }
  yd[2] = -(yd[0] + yd[1]);
  constexpr int pi_[3] = {0, 0, 1};
  constexpr int pj_[3] = {1, 2, 2};
  constexpr int ps_[3] = {0, 3, 5};
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const int i = pi_[p], j = pj_[p];
    T sr = 0, si = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      sr = fmadd(wre[i][k], are[j][k], fmadd(wim[i][k], aim[j][k], sr));
      si = fmadd(wim[i][k], are[j][k], fmadd(-wre[i][k], aim[j][k], si));
    }
    acc[ps_[p]] = fmadd(T(2), sr, acc[ps_[p]]);
    acc[ps_[p] + 1] = fmadd(T(-2), si, acc[ps_[p] + 1]);
  }
  acc[2] += yd[0] - yd[1];
  acc[7] = fmadd(fmadd(T(-2), yd[2], yd[0] + yd[1]), T(kInvSqrt3), acc[7]);
}

}  // namespace rmh
