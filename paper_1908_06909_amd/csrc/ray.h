// Device helpers shared by the ray walk and the element-driven
// backprojection: the pixel ray endpoint and the exact perturbed edge sign
// (small vector operations come from walk_filter.h).  Both kernels must see identical rays and
// identical signs, so they take them from here.
#pragma once

#include "common.h"
#include "exact.h"
#include "walk_filter.h"

namespace tct {
namespace {

__device__ __forceinline__ float3 xyz(float4 a) { return make_float3(a.y, a.z, a.w); }

// Detector point of pixel (u, v) for one angle's frame f = {S, D, U, V}:
// P = fl(fl(D + fl(u U)) + fl(v V)) per component, with no contraction, so
// that every kernel forms bit-identical rays (one ray per detector pixel
// centre, Section II-A).
__device__ __forceinline__ float3 pixel_point(const float* f, float u, float v) {
  float3 P;
  P.x = __fadd_rn(__fadd_rn(f[3], __fmul_rn(u, f[6])), __fmul_rn(v, f[9]));
  P.y = __fadd_rn(__fadd_rn(f[4], __fmul_rn(u, f[7])), __fmul_rn(v, f[10]));
  P.z = __fadd_rn(__fadd_rn(f[5], __fmul_rn(u, f[8])), __fmul_rn(v, f[11]));
  return P;
}

// Exact perturbed sign of the edge (p, q): returns sign + 1 in bits 0-1 and
// the exact.h flags in bits 2-3.
__device__ __noinline__ int slow_edge_sign(float3 S, float3 P, float3 U, float3 V, float3 p, float3 q) {
  float s[3] = {S.x, S.y, S.z}, pp[3] = {P.x, P.y, P.z}, u[3] = {U.x, U.y, U.z}, v[3] = {V.x, V.y, V.z};
  float a[3] = {p.x, p.y, p.z}, b[3] = {q.x, q.y, q.z};
  unsigned flags = 0;
  int sg = perturbed_edge_sign(s, pp, u, v, a, b, &flags);
  return (sg + 1) | (int)(flags << 2);
}

}  // namespace
}  // namespace tct
