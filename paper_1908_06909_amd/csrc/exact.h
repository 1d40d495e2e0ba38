// Exact sign of 3x3 determinants of float32 point differences.
//
// Used for every decision of the walk that a floating-point estimate cannot
// certify: orientation of tetrahedra and faces at mesh creation, and the
// edge signs of rays through vertices, along edges or inside face planes
// (the near-degenerate cases the paper's Section II-C-1 and Fig. 9 show
// breaking float32 intersection code).
//
// Method: error-free transformations on float64 (Knuth's two-sum; the fused
// multiply-add two-product), accumulated into a non-overlapping expansion
// with zero elimination (Shewchuk 1997, "Adaptive precision floating-point
// arithmetic and fast robust geometric predicates").  Inputs are float32, so
// the product of two coordinates is exact in float64 and the product of three
// is exactly the sum of two float64 values; the determinant of differences is
// expanded by multilinearity into at most 48 such triple products and summed
// exactly.  The sign of a non-overlapping expansion is the sign of its
// largest component.
#pragma once

#include <hip/hip_runtime.h>

namespace tct {

__host__ __device__ inline void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bv = s - a;
  double av = s - bv;
  e = (a - av) + (b - bv);
}

__host__ __device__ inline void two_prod(double a, double b, double& p, double& e) {
  p = a * b;
  e = fma(a, b, -p);
}

// e[0..n) is non-overlapping with increasing magnitude; add b in place.
__host__ __device__ inline int expansion_grow(double* e, int n, double b) {
  double q = b;
  int k = 0;
  for (int i = 0; i < n; ++i) {
    double s, h;
    two_sum(q, e[i], s, h);
    if (h != 0.0) e[k++] = h;
    q = s;
  }
  if (q != 0.0) e[k++] = q;
  return k;
}

__host__ __device__ inline int expansion_add_triple(double* e, int n, float x, float y, float z, bool negate) {
  double xy = (double)x * (double)y;  // exact: 24 + 24 significant bits
  double p, r;
  two_prod(xy, (double)z, p, r);
  if (negate) {
    p = -p;
    r = -r;
  }
  n = expansion_grow(e, n, r);
  return expansion_grow(e, n, p);
}

// det[X, Y, Z] (columns) added exactly into the expansion, times sgn.
__host__ __device__ inline int expansion_add_det(double* e, int n, const float* X, const float* Y, const float* Z,
                                                 bool neg) {
  // + X0 Y1 Z2 - X0 Y2 Z1 - X1 Y0 Z2 + X1 Y2 Z0 + X2 Y0 Z1 - X2 Y1 Z0
  n = expansion_add_triple(e, n, X[0], Y[1], Z[2], neg);
  n = expansion_add_triple(e, n, X[0], Y[2], Z[1], !neg);
  n = expansion_add_triple(e, n, X[1], Y[0], Z[2], !neg);
  n = expansion_add_triple(e, n, X[1], Y[2], Z[0], neg);
  n = expansion_add_triple(e, n, X[2], Y[0], Z[1], neg);
  n = expansion_add_triple(e, n, X[2], Y[1], Z[0], !neg);
  return n;
}

// Exact sign of det[A1 - A0, B1 - B0, C1 - C0].  A null pointer stands for the
// zero vector.  By multilinearity the determinant is the signed sum of
// det[X, Y, Z] over X in {A1, A0}, Y in {B1, B0}, Z in {C1, C0}, the sign
// being (-1)^(number of *0 picks); picks of a null pointer or of the same
// point twice contribute exactly zero and are skipped.
__host__ __device__ inline int exact_det_diff_sign(const float* A1, const float* A0, const float* B1,
                                                   const float* B0, const float* C1, const float* C0) {
  double e[96];
  int n = 0;
  const float* As[2] = {A1, A0};
  const float* Bs[2] = {B1, B0};
  const float* Cs[2] = {C1, C0};
  for (int ia = 0; ia < 2; ++ia)
    for (int ib = 0; ib < 2; ++ib)
      for (int ic = 0; ic < 2; ++ic) {
        const float *X = As[ia], *Y = Bs[ib], *Z = Cs[ic];
        if (!X || !Y || !Z || X == Y || Y == Z || X == Z) continue;
        n = expansion_add_det(e, n, X, Y, Z, ((ia + ib + ic) & 1) != 0);
      }
  if (n == 0) return 0;
  return e[n - 1] > 0.0 ? 1 : -1;
}

// Float64 estimate of the same determinant with a certified error bound.
// det = A . (B x C); every one of its six monomials goes through at most
// eight roundings (three input differences, the product and difference
// inside B x C, the product with A, two additions), so
// |computed - exact| <= gamma_8 * sum|monomials| < 9 * 2^-53 * perm; 12 * 2^-53
// is used.  Returns 2 when the estimate cannot decide.
__host__ __device__ inline int filtered_det_diff_sign(const float* A1, const float* A0, const float* B1,
                                                      const float* B0, const float* C1, const float* C0) {
  double A[3], B[3], C[3];
  for (int i = 0; i < 3; ++i) {
    A[i] = (double)A1[i] - (A0 ? (double)A0[i] : 0.0);
    B[i] = (double)B1[i] - (B0 ? (double)B0[i] : 0.0);
    C[i] = (double)C1[i] - (C0 ? (double)C0[i] : 0.0);
  }
  double cx = B[1] * C[2] - B[2] * C[1];
  double cy = B[2] * C[0] - B[0] * C[2];
  double cz = B[0] * C[1] - B[1] * C[0];
  double det = A[0] * cx + A[1] * cy + A[2] * cz;
  double px = fabs(B[1] * C[2]) + fabs(B[2] * C[1]);
  double py = fabs(B[2] * C[0]) + fabs(B[0] * C[2]);
  double pz = fabs(B[0] * C[1]) + fabs(B[1] * C[0]);
  double perm = fabs(A[0]) * px + fabs(A[1]) * py + fabs(A[2]) * pz;
  const double bound = 12.0 * 1.1102230246251565e-16 * perm;  // 12 * 2^-53 * perm
  if (det > bound) return 1;
  if (det < -bound) return -1;
  return 2;
}

enum SignFlags : unsigned { kFlagExact = 1u, kFlagPerturbed = 2u };

__host__ __device__ inline int det_diff_sign(const float* A1, const float* A0, const float* B1, const float* B0,
                                             const float* C1, const float* C0, unsigned* flags) {
  int s = filtered_det_diff_sign(A1, A0, B1, B0, C1, C0);
  if (s != 2) return s;
  if (flags) *flags |= kFlagExact;
  return exact_det_diff_sign(A1, A0, B1, B0, C1, C0);
}

// orient3d(a, b, c, d) = sign det[b - a, c - a, d - a].
__host__ __device__ inline int orient3d_sign(const float* a, const float* b, const float* c, const float* d) {
  return det_diff_sign(b, a, c, a, d, a, nullptr);
}

// Sign of the edge (p, q) seen by the ray S -> P translated by eps U + eps^2 V:
// det[P - S, p - S, q - S], else det[P - S, U, p - q], else det[P - S, V, p - q].
// Zero only for an edge parallel to P - S.
__host__ __device__ inline int perturbed_edge_sign(const float* S, const float* P, const float* U, const float* V,
                                                   const float* p, const float* q, unsigned* flags) {
  int s = det_diff_sign(P, S, p, S, q, S, flags);
  if (s != 0) return s;
  if (flags) *flags |= kFlagPerturbed;
  s = det_diff_sign(P, S, U, nullptr, p, q, flags);
  if (s != 0) return s;
  return det_diff_sign(P, S, V, nullptr, p, q, flags);
}

}  // namespace tct
