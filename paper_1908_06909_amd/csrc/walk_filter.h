// Float32 sign filters of the walk (Section II-C-1: the intersection test
// in higher precision than the data; here float32 decides only when a
// certified error bound says its sign is right, and the uncertain cases go
// to float64 and exact arithmetic).  Everything here is __host__ __device__
// so that tests can run the very same code on the CPU and check every sign
// it certifies against exact arithmetic.
#pragma once

#include "common.h"

#ifndef TCT_FILTER_BOUND_SCALE
#define TCT_FILTER_BOUND_SCALE 1.0f
#endif

namespace tct {
namespace {

__host__ __device__ __forceinline__ float3 f3sub(float3 a, float3 b) {
  return make_float3(a.x - b.x, a.y - b.y, a.z - b.z);
}
// Dot and cross products with fused multiply-adds (the library is built
// without automatic contraction): each monomial meets no more roundings than
// in the plain order, so the error bounds stated where they are used hold.
__host__ __device__ __forceinline__ float f3dot(float3 a, float3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }
__host__ __device__ __forceinline__ float3 f3cross(float3 a, float3 b) {
  return make_float3(fmaf(a.y, b.z, -(a.z * b.y)), fmaf(a.z, b.x, -(a.x * b.z)), fmaf(a.x, b.y, -(a.y * b.x)));
}
__host__ __device__ __forceinline__ float3 f3abs(float3 a) { return make_float3(fabsf(a.x), fabsf(a.y), fabsf(a.z)); }

// Entry-test filter constants: every monomial of (q-p).((P-S)x(p-S)) carries
// at most 8 roundings (three input differences, product and difference in
// the cross product, the outer product, two additions); with the bound
// itself evaluated in float32 from rounded magnitudes, 10 * 2^-24 * perm
// covers gamma_8 * perm of the exact inputs.  The absolute term covers
// underflow.
constexpr float kFilterRel = 10.0f * 5.9604644775390625e-8f * TCT_FILTER_BOUND_SCALE;
constexpr float kFilterAbs = 7.888609052210118e-31f;  // 2^-100

// Walk filter.  With w = fl(d_hi x D) and e = fl(a - v), the exact edge value
// E(v, a) = (a - v) . (d x (v - S)) = (a - v) . (d x (v - Q)) differs from
// fl(e . w) by at most |e|_1 |d|_inf (20.5 u |D|_inf + 57.2 u^2 R): six
// roundings per monomial of e.(d_hi x D), the d_lo x D term, and the error of
// D itself.  The step measures edges by |e|_inf (one max of magnitudes, no
// rounding) and |e|_1 <= 3 |e|_inf, so the constants carry a factor 3:
// 72 u = 3 x 24 u and 192 u^2 = 3 x 64 u^2, where 24 u and 64 u^2 leave room
// for the rounding of the bound's own evaluation.
constexpr float kWalkRel = 72.0f * 5.9604644775390625e-8f * TCT_FILTER_BOUND_SCALE;
constexpr float kWalkAbs2 = 192.0f * 3.552713678800501e-15f * TCT_FILTER_BOUND_SCALE;  // 192 u^2

// The crossing is recomputed in float64 when |d . n| < sqrt(3) |d| |n|_inf /
// 128, which takes in every face whose normal makes cos < 1/128 with the ray
// (|n|_2 <= sqrt(3) |n|_inf) and at most sqrt(3) times that angle.  With the
// vertex offset D accurate to a few ulps of |D| (offset_from_ray), the
// float32 crossing moves by about c u h / cos (h the face diameter, c ~ 5
// from the rounded normal), i.e. 4e-5 h at cos = 1/128; well under one
// segment in ten thousand is that oblique, so the bound on a projection, a
// sum over some hundred segments, stays near 1e-7 of it.
constexpr float kGrazingBound = 1.7320509f / 128.0f;

// The ray leaves through the face (v, a_{k+1}, a_{k+2}) opposite entry slot
// k (indices mod 3) for which E(v, a_{k+1}) < 0 < E(v, a_{k+2}), the first of
// k = 2, 0, 1 that qualifies.  When the three signs are certain (nonzero)
// this is a table on n = neg0 | neg1 << 1 | neg2 << 2, two bits per entry;
// 3 = none (all three signs equal: the walk has failed).
constexpr unsigned kExitFace = 0xD90Bu;

struct Ray {
  float3 S, P, U, V;
  float3 d;    // d_hi = fl(P - S)
  float3 ad;   // |d_hi|
  double dx64, dy64, dz64;  // P - S (exact in float64)
  double Mx64, My64, Mz64;  // the ray point at t = 1/2
  float dn;    // |d| (Euclidean)
  float gd;    // sqrt(3) |d| / 128 (grazing test)
  float kA;    // |d|_inf 72 u        walk filter: K = kA |D|_inf + kB
  float kB;    // |d|_inf 192 u^2 R, R bounding every coordinate met on this ray
};

// The ray is carried with d_hi = fl(P - S) for the float32 filters and, in
// float64, with the exact direction P - S and the point M at t = 1/2 (one
// float64 rounding), so positions on it near the mesh can be formed to a
// relative accuracy set by their distance to the mesh features rather than
// by the distance to the source.
__host__ __device__ __forceinline__ void finish_ray(Ray& r, float mesh_extent) {
  r.d = f3sub(r.P, r.S);
  r.dx64 = (double)r.P.x - r.S.x;
  r.dy64 = (double)r.P.y - r.S.y;
  r.dz64 = (double)r.P.z - r.S.z;
  r.Mx64 = r.S.x + 0.5 * r.dx64;
  r.My64 = r.S.y + 0.5 * r.dy64;
  r.Mz64 = r.S.z + 0.5 * r.dz64;
  r.ad = f3abs(r.d);
  const float dd = r.d.x * r.d.x + r.d.y * r.d.y + r.d.z * r.d.z;
  r.dn = sqrtf(dd);
  r.gd = kGrazingBound * r.dn;
  const float dinf = fmaxf(r.ad.x, fmaxf(r.ad.y, r.ad.z));
  float sp = fmaxf(fmaxf(fmaxf(fabsf(r.S.x), fabsf(r.S.y)), fmaxf(fabsf(r.S.z), fabsf(r.P.x))),
                   fmaxf(fabsf(r.P.y), fabsf(r.P.z)));
  float R = (fmaxf(sp, mesh_extent) + dinf) * 1.0001f;
  r.kA = dinf * kWalkRel;
  r.kB = dinf * (kWalkAbs2 * R);  // |d|_inf 192 u^2 R with u = 2^-24
}

// True when every point of the cube [-extent, extent]^3, which holds the
// mesh, lies before the ray's end point P by more than 2^-10 of the ray
// parameter: max over the cube of (X - P).d = extent |d|_1 - P.d.  A walk
// inside the mesh then never reaches t = 1, and its segments need no clamp
// at the end point.  Float64 from the exact direction.
__host__ __device__ __forceinline__ bool ends_beyond_mesh(const Ray& r, float extent) {
  const double d1 = fabs(r.dx64) + fabs(r.dy64) + fabs(r.dz64);
  const double dd = r.dx64 * r.dx64 + r.dy64 * r.dy64 + r.dz64 * r.dz64;
  const double pd = (double)r.P.x * r.dx64 + (double)r.P.y * r.dy64 + (double)r.P.z * r.dz64;
  return pd - (double)extent * d1 > 0x1p-10 * dd;
}

// D = v - Q for the ray point Q = M + s d, in float64: M, v - M and the
// fused s d term each carry one float64 rounding of the source-distance
// scale R, so with the final rounding to float32
// |D - (v - Q)| <= u |D| + 2^-51 R componentwise, inside the allowance
// 3.1 u |D| + 28 u^2 R the walk filter is built on.
__host__ __device__ __forceinline__ float3 offset_from_ray(const Ray& r, double s, float3 v) {
  return make_float3((float)fma(-s, r.dx64, (double)v.x - r.Mx64), (float)fma(-s, r.dy64, (double)v.y - r.My64),
                     (float)fma(-s, r.dz64, (double)v.z - r.Mz64));
}

// Float32 estimate of sigma(p, q) = (q - p) . w with w = d x (p - S) and
// W = |d| x |p - S| (the cross-product magnitudes); 2 = uncertain.
__host__ __device__ __forceinline__ int fast_sign(float3 e, float3 w, float3 W) {
  float E = e.x * w.x + e.y * w.y + e.z * w.z;
  float B = kFilterRel * (fabsf(e.x) * W.x + fabsf(e.y) * W.y + fabsf(e.z) * W.z) + kFilterAbs;
  return E > B ? 1 : (E < -B ? -1 : 2);
}

__host__ __device__ __forceinline__ void cross_pair(const Ray& r, float3 p, float3& w, float3& W) {
  float3 pv = f3sub(p, r.S);
  w = f3cross(r.d, pv);
  float3 apv = f3abs(pv);
  W = make_float3(r.ad.y * apv.z + r.ad.z * apv.y, r.ad.z * apv.x + r.ad.x * apv.z, r.ad.x * apv.y + r.ad.y * apv.x);
}

// Float32 estimate of sigma(p, q) with its certification (the entry test's
// filter): 1 / -1 when certain, 2 when uncertain.
__host__ __device__ __forceinline__ int entry_edge_sign(const Ray& r, float3 p, float3 q) {
  float3 w, W;
  cross_pair(r, p, w, W);
  return fast_sign(f3sub(q, p), w, W);
}

// The three edge values of one walk step: the current tetrahedron's fourth
// vertex v against the entry-face slots a0, a1, a2, from the offset D of v to
// the ray point at parameter s (the entry point).
struct StepEdges {
  float3 D;           // v - Q, rounded to float32
  float3 e0, e1, e2;  // a_k - v
  float E0, E1, E2;   // float32 estimates of E(v, a_k)
  float m0, m1, m2;   // |e_k|_inf
  float K;            // |d|_inf (72 u |D|_inf + 192 u^2 R): bound per unit of |e|_inf
};

__host__ __device__ __forceinline__ void step_edges(const Ray& r, double s, float3 v, float3 a0, float3 a1, float3 a2,
                                                    StepEdges& g) {
  g.D = offset_from_ray(r, s, v);
  const float3 wv = f3cross(r.d, g.D);
  g.K = fmaf(fmaxf(fabsf(g.D.x), fmaxf(fabsf(g.D.y), fabsf(g.D.z))), r.kA, r.kB);
  g.e0 = f3sub(a0, v);
  g.e1 = f3sub(a1, v);
  g.e2 = f3sub(a2, v);
  g.E0 = f3dot(g.e0, wv);
  g.E1 = f3dot(g.e1, wv);
  g.E2 = f3dot(g.e2, wv);
  g.m0 = fmaxf(fabsf(g.e0.x), fmaxf(fabsf(g.e0.y), fabsf(g.e0.z)));
  g.m1 = fmaxf(fabsf(g.e1.x), fmaxf(fabsf(g.e1.y), fabsf(g.e1.z)));
  g.m2 = fmaxf(fabsf(g.e2.x), fmaxf(fabsf(g.e2.y), fabsf(g.e2.z)));
}

// One bound from the longest edge settles all three signs in the common
// case: returns the exit slot (0..2; 3 when all three signs agree, a failed
// walk), or -1 when some sign is uncertain under that bound.
__host__ __device__ __forceinline__ int step_exit_common(const StepEdges& g) {
  if (fminf(fabsf(g.E0), fminf(fabsf(g.E1), fabsf(g.E2))) > fmaf(fmaxf(g.m0, fmaxf(g.m1, g.m2)), g.K, kFilterAbs)) {
    const unsigned n = (__builtin_bit_cast(unsigned, g.E0) >> 31) | ((__builtin_bit_cast(unsigned, g.E1) >> 31) << 1) |
                       ((__builtin_bit_cast(unsigned, g.E2) >> 31) << 2);
    return (int)((kExitFace >> (2 * n)) & 3u);
  }
  return -1;
}

// Each edge under its own bound: 1 / -1 when certain, 0 when not.
__host__ __device__ __forceinline__ int step_edge_certified(float E, float m, float K) {
  return fabsf(E) - fmaf(m, K, kFilterAbs) > 0.f ? (E > 0.f ? 1 : -1) : 0;
}

// Exit slot from three decided signs (same rule as the table).
__host__ __device__ __forceinline__ int exit_slot(int s0, int s1, int s2) {
  return (s0 < 0 && s1 > 0) ? 2 : (s1 < 0 && s2 > 0) ? 0 : (s2 < 0 && s0 > 0) ? 1 : 3;
}

}  // namespace
}  // namespace tct
