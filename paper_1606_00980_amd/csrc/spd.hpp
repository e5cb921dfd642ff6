// Inverse of a small symmetric positive definite block held packed (lower
// triangle, row-major) in registers: Cholesky A = L L', then
// A^{-1} = L^{-T} L^{-1}.
#pragma once
#include "common.hpp"

namespace gp {

// Writes the packed inverse of the packed SPD block a into inv and returns
// whether every pivot was positive and finite.  A failed pivot is replaced by
// one so that the arithmetic stays finite.
template <int K>
__device__ inline bool spd_inverse(const double (&a)[K * (K + 1) / 2], double (&inv)[K * (K + 1) / 2]) {
  constexpr int NB = K * (K + 1) / 2;
  double L[NB];
  bool ok = true;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    double dj = a[pk(j, j)];
#pragma unroll
    for (int l = 0; l < j; ++l) dj -= L[pk(j, l)] * L[pk(j, l)];
    ok = ok && (dj > 0.0) && (dj == dj);
    const double ljj = sqrt(dj > 0.0 ? dj : 1.0);
    L[pk(j, j)] = ljj;
#pragma unroll
    for (int i = j + 1; i < K; ++i) {
      double v = a[pk(i, j)];
#pragma unroll
      for (int l = 0; l < j; ++l) v -= L[pk(i, l)] * L[pk(j, l)];
      L[pk(i, j)] = v / ljj;
    }
  }
  double Li[NB];   // lower-triangular inverse of L, by forward substitution per column
#pragma unroll
  for (int c = 0; c < K; ++c) {
#pragma unroll
    for (int i = c; i < K; ++i) {
      double v = (i == c) ? 1.0 : 0.0;
#pragma unroll
      for (int l = c; l < i; ++l) v -= L[pk(i, l)] * Li[pk(l, c)];
      Li[pk(i, c)] = v / L[pk(i, i)];
    }
  }
#pragma unroll
  for (int i = 0; i < K; ++i) {
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      double v = 0.0;
#pragma unroll
      for (int l = i; l < K; ++l) v += Li[pk(l, i)] * Li[pk(l, j)];
      inv[pk(i, j)] = v;
    }
  }
  return ok;
}

// Blocks above this K are factored by the rolled routines below (runtime K,
// arrays in scratch memory): the set-up kernels run once per change of the
// blocks or alpha, and fully unrolled O(K^3) code for larger K would take
// minutes to compile.
constexpr int KREG = 16;

// In-place lower Cholesky factor of the packed SPD block a (runtime K); a
// failed pivot is replaced by one.  Returns whether every pivot was positive.
__device__ inline bool cholesky_dyn(int K, double* a) {
  bool ok = true;
#pragma unroll 1
  for (int j = 0; j < K; ++j) {
    double dj = a[pk(j, j)];
#pragma unroll 1
    for (int l = 0; l < j; ++l) dj -= a[pk(j, l)] * a[pk(j, l)];
    ok = ok && (dj > 0.0) && (dj == dj);
    const double ljj = sqrt(dj > 0.0 ? dj : 1.0);
    a[pk(j, j)] = ljj;
#pragma unroll 1
    for (int i = j + 1; i < K; ++i) {
      double v = a[pk(i, j)];
#pragma unroll 1
      for (int l = 0; l < j; ++l) v -= a[pk(i, l)] * a[pk(j, l)];
      a[pk(i, j)] = v / ljj;
    }
  }
  return ok;
}

// The packed inverse of the packed SPD block a (runtime K), written to inv;
// a is overwritten (Cholesky factor, then its inverse).
__device__ inline bool spd_inverse_dyn(int K, double* a, double* inv) {
  const bool ok = cholesky_dyn(K, a);
  // L^{-1} into inv, column by column by forward substitution
#pragma unroll 1
  for (int c = 0; c < K; ++c) {
#pragma unroll 1
    for (int i = c; i < K; ++i) {
      double v = (i == c) ? 1.0 : 0.0;
#pragma unroll 1
      for (int l = c; l < i; ++l) v -= a[pk(i, l)] * inv[pk(l, c)];
      inv[pk(i, c)] = v / a[pk(i, i)];
    }
  }
  // A^{-1} = L^{-T} L^{-1} back into a, then copied to inv
#pragma unroll 1
  for (int i = 0; i < K; ++i) {
#pragma unroll 1
    for (int j = 0; j <= i; ++j) {
      double v = 0.0;
#pragma unroll 1
      for (int l = i; l < K; ++l) v += inv[pk(l, i)] * inv[pk(l, j)];
      a[pk(i, j)] = v;
    }
  }
  const int NB = K * (K + 1) / 2;
#pragma unroll 1
  for (int e = 0; e < NB; ++e) inv[e] = a[e];
  return ok;
}

// The packed inverse of a packed SPD block held in registers: unrolled up to
// K = KREG, through the rolled routine above.
template <int K>
__device__ inline bool spd_inverse_any(double (&a)[K * (K + 1) / 2], double (&inv)[K * (K + 1) / 2]) {
  if constexpr (K <= KREG)
    return spd_inverse<K>(a, inv);
  else
    return spd_inverse_dyn(K, a, inv);
}

}  // namespace gp
