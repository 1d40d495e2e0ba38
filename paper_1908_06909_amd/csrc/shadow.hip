// Element-driven backprojection: A^T y computed one tetrahedron at a time
// from implicit ray lists.
//
// The backprojection of Eq. (3) sums, for every element, a_ij y_j over the
// rays j that cross it.  Instead of scattering from the rays (Algorithm 1 run
// with atomic updates, Section II-F), each lane owns one tetrahedron and, for
// every angle, enumerates the detector pixels inside the tetrahedron's
// central projection (its "shadow"), decides exactly whether each pixel's ray
// crosses it, and if so adds the chord length times y_j.  Every element is
// written once, so the result needs no atomics and is bitwise reproducible:
// the sum runs in float64 over rays in increasing ray id (angle, row, column),
// except for the few elements the exact pass takes over, which it sums per
// angle in a fixed order across one wavefront.
//
// Crossing test.  With sigma(p, q) the exact sign of det[P - S, p - S, q - S]
// for the ray translated by eps U + eps^2 V (the same perturbed predicate the
// walk uses, so both see the same tetrahedra on every ray), the translated
// ray crosses the tetrahedron iff one face, taken with outward orientation
// (a, b, c), has sigma(a, b) = sigma(b, c) = sigma(c, a) = -1 (the entry
// face); then exactly one other face has all three +1 (the exit face).  An
// edge parallel to the ray has sigma = 0 and makes no face qualify, matching
// a ray that runs parallel to the faces through that edge.
//
// Two passes.  The fast pass evaluates the six signs in the detector plane:
// with w_k the central projections of the vertices and P' where the ray meets
// the plane, det[P - S, p - S, q - S] has the sign of the 2-D cross product
// (w_p - P') x (w_q - P') times the sign of (D - S) . (U x V), because every
// factor between them is a positive depth ratio.  The 2-D values are cheap
// (the vertices are projected once per angle in float64) and carry a
// certified bound that covers the float32 evaluation and the rounding of the
// pixel point; values inside the bound are recomputed in float64 in 3-D, and a
// tetrahedron where that is still uncertain (a tie at a vertex or an edge) is
// handed whole to the exact pass, which resolves the six signs with the exact
// expansion and the perturbation.
//
// Chord length.  From the exit and entry faces, L = |d| (t_x - t_e) with
// t_f = ((a_f - S) . n_f) / (d . n_f) for face f through vertex a_f with
// normal n_f, all in float64 (fast pass); the exact pass uses the crossing
// points X = (E_bc a + E_ca b + E_ab c) / (E_ab + E_bc + E_ca) given by the
// float64 edge values E (Plücker coordinates).
#include "common.h"
#include "exact.h"
#include "kernels.h"
#include "ray.h"

namespace tct {

namespace {

constexpr int kShadowThreads = 256;
constexpr int kShadowLdsTable = 2048;  // detector tables up to this many entries live in LDS
constexpr int kShadowTargetWaves = 8192;
constexpr float kUnit = 5.9604644775390625e-8f;  // 2^-24

// Float64 filter for E = d . (r x e), d = P - S, r = p - S, e = q - p formed
// in float64 from float32 inputs: at most eight roundings of 2^-53 per
// monomial, so |E - E*| <= 2^-50 |d|_inf |r|_1 |e|_1.  The test compares the
// float32 image of E with 2^-44 |d|_inf m_e (m_e = |r|_1 |e|_1 rounded in
// float32), a 64-fold margin that absorbs the float32 rounding of both sides;
// 2^-100 guards against underflow.
constexpr float kShadowRel = 5.684341886080802e-14f;  // 2^-44
constexpr float kShadowAbs = 7.888609052210118e-31f;  // 2^-100

struct ShadowArgs {
  MeshView M;
  GeomView G;
  const float* proj;  // [na][nv][nu]
  float* xhat;        // [nt], written when partial is null
  double* partial;    // [chunks][nt] float64 partial sums, or null
  int a0, na, chunk_len;
  int accumulate;
  float u0, inv_du;  // pixel column coordinate of detector abscissa u: (u - u0) * inv_du
  float v0, inv_dv;
  float margin;      // pixels added around each shadow
  float du, dv;      // pixel pitch: local coordinates are (i - i0) du, (j - j0) dv
  float eps_p;       // bound on the detector-plane distance between a pixel's ray and the pixel centre
  int* dirty_count;  // items (chunk * nt + t) left to the exact pass
  int* dirty;
};

struct ShadowStats {
  int hits = 0, fp64 = 0, slow = 0, exact = 0, pert = 0;
};

// Per-angle frame in float64 (uniform across the wave).
struct FrameD {
  float3 S, U, V;
  const float* f;
  double Sx, Sy, Sz, SDx, SDy, SDz;  // S and S - D
  double Nx, Ny, Nz;                 // U x V
  double hN;                         // (D - S) . N
  double g00, g01, g11;              // inverse Gram matrix of (U, V)
};

__device__ __forceinline__ FrameD load_frame(const float* frame, int a) {
  FrameD F;
  const float* f = frame + 12 * a;
  F.f = f;
  F.S = make_float3(f[0], f[1], f[2]);
  F.U = make_float3(f[6], f[7], f[8]);
  F.V = make_float3(f[9], f[10], f[11]);
  F.Sx = f[0];
  F.Sy = f[1];
  F.Sz = f[2];
  F.SDx = (double)f[0] - f[3];
  F.SDy = (double)f[1] - f[4];
  F.SDz = (double)f[2] - f[5];
  double Ux = f[6], Uy = f[7], Uz = f[8], Vx = f[9], Vy = f[10], Vz = f[11];
  F.Nx = Uy * Vz - Uz * Vy;
  F.Ny = Uz * Vx - Ux * Vz;
  F.Nz = Ux * Vy - Uy * Vx;
  F.hN = -(F.SDx * F.Nx + F.SDy * F.Ny + F.SDz * F.Nz);
  double uu = Ux * Ux + Uy * Uy + Uz * Uz, uv = Ux * Vx + Uy * Vy + Uz * Vz, vv = Vx * Vx + Vy * Vy + Vz * Vz;
  double det = uu * vv - uv * uv;
  F.g00 = vv / det;
  F.g01 = -uv / det;
  F.g11 = uu / det;
  return F;
}

// Detector coordinates (alpha, beta) of the central projection of p, in
// float64: S + tau (p - S) = D + alpha U + beta V.
__device__ __forceinline__ void project_vertex(const FrameD& F, float3 p, double& al, double& be) {
  double rx = (double)p.x - F.Sx, ry = (double)p.y - F.Sy, rz = (double)p.z - F.Sz;
  double tau = F.hN / (rx * F.Nx + ry * F.Ny + rz * F.Nz);
  double Xx = F.SDx + tau * rx, Xy = F.SDy + tau * ry, Xz = F.SDz + tau * rz;
  const float* f = F.f;
  double xu = Xx * f[6] + Xy * f[7] + Xz * f[8];
  double xv = Xx * f[9] + Xy * f[10] + Xz * f[11];
  al = F.g00 * xu + F.g01 * xv;
  be = F.g01 * xu + F.g11 * xv;
}

__device__ __forceinline__ float3 tet_vertex(const float4* tq, int k) {
  const float* c = (const float*)tq + 3 * k;
  return make_float3(c[0], c[1], c[2]);
}

// Entry face from the six signs (exit face: swap the masks).  Faces with
// outward orientation: f0 (1,2,3), f1 (0,3,2), f2 (0,1,3), f3 (0,2,1); entry
// = its three edge signs all -1.  Bits 0:01 1:02 2:03 3:12 4:13 5:23.
__device__ __forceinline__ bool face_all(int lo, int hi, int m1, int m2) {
  return ((lo & m1) == m1) && ((hi & m2) == m2);
}
__device__ __forceinline__ int entry_face(int neg, int pos) {
  if (face_all(neg, pos, 0x28, 0x10)) return 0;  // -12 -23 +13
  if (face_all(neg, pos, 0x04, 0x22)) return 1;  // -03 +23 +02
  if (face_all(neg, pos, 0x11, 0x04)) return 2;  // -01 -13 +03
  if (face_all(neg, pos, 0x02, 0x09)) return 3;  // -02 +12 +01
  return -1;
}

// Float64 3-D edge value E(p, q) = d . ((p - S) x (q - p)) with its filter;
// returns +1 / -1 when certain, 0 when not.
__device__ __forceinline__ int edge_sign_fp64(const FrameD& F, double dx, double dy, double dz, float dinf, float3 p,
                                              float3 q, double* Eout) {
  double rx = (double)p.x - F.Sx, ry = (double)p.y - F.Sy, rz = (double)p.z - F.Sz;
  double ex = (double)q.x - p.x, ey = (double)q.y - p.y, ez = (double)q.z - p.z;
  double cx = ry * ez - rz * ey, cy = rz * ex - rx * ez, cz = rx * ey - ry * ex;
  double E = fma(dx, cx, fma(dy, cy, dz * cz));
  if (Eout) *Eout = E;
  float3 rf = f3sub(p, F.S), ef = f3sub(q, p);
  float m = (fabsf(rf.x) + fabsf(rf.y) + fabsf(rf.z)) * (fabsf(ef.x) + fabsf(ef.y) + fabsf(ef.z));
  float B = fmaf(dinf * kShadowRel, m, kShadowAbs);
  float Ef = (float)E;
  return Ef > B ? 1 : (Ef < -B ? -1 : 0);
}

// Pixel ranges of the shadow of vertices (al, be) (float64 detector
// coordinates); false when it misses the detector.
__device__ __forceinline__ bool shadow_box(const ShadowArgs& A, const double* al, const double* be, int& i0, int& i1,
                                           int& j0, int& j1) {
  float cmin = 3.0e38f, cmax = -3.0e38f, rmin = 3.0e38f, rmax = -3.0e38f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    float pu = ((float)al[k] - A.u0) * A.inv_du, pv = ((float)be[k] - A.v0) * A.inv_dv;
    cmin = fminf(cmin, pu);
    cmax = fmaxf(cmax, pu);
    rmin = fminf(rmin, pv);
    rmax = fmaxf(rmax, pv);
  }
  const float mg = A.margin;
  // Clamped in float before conversion, so out-of-range or non-finite values
  // give an empty or a full range, never an overflowed index.
  j0 = (int)ceilf(fminf(fmaxf(rmin - mg, 0.f), (float)A.G.nv));
  j1 = (int)floorf(fmaxf(fminf(rmax + mg, (float)(A.G.nv - 1)), -1.f));
  i0 = (int)ceilf(fminf(fmaxf(cmin - mg, 0.f), (float)A.G.nu));
  i1 = (int)floorf(fmaxf(fminf(cmax + mg, (float)(A.G.nu - 1)), -1.f));
  return j0 <= j1 && i0 <= i1;
}

__device__ __forceinline__ void flush_shadow_stats(const MeshView& M, const ShadowStats& st) {
  int vals[5] = {st.hits, st.fp64, st.exact, st.pert, st.slow};
  const int slots[5] = {kSegments, kGrazing, kExactStage, kPerturbed, kFp64Stage};
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    int x = vals[k];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    if ((threadIdx.x & 63) == 0 && x) atomicAdd(M.counters + slots[k], (unsigned long long)x);
  }
}

__device__ __forceinline__ void store_result(const ShadowArgs& A, int chunk, int t, double acc) {
  if (A.partial) {
    A.partial[(size_t)chunk * A.M.nt + t] = acc;
  } else {
    double base = A.accumulate ? (double)A.xhat[t] : 0.0;
    A.xhat[t] = (float)(base + acc);
  }
}

// ---------------------------------------------------------------- fast pass

// Edge e joins local vertices (p, q), p < q: 0 = (0,1), 1 = (0,2), 2 = (0,3),
// 3 = (1,2), 4 = (1,3), 5 = (2,3).  Face f is opposite vertex f; its outward
// edge values are those listed in entry_face.
constexpr int kEdgeP[6] = {0, 0, 0, 1, 1, 2};
constexpr int kEdgeQ[6] = {1, 2, 3, 2, 3, 3};
// The two faces containing edge e (those opposite its other two vertices)
// and the edge's sign in the first one's outward edge values.
constexpr int kEdgeFaceA[6] = {2, 1, 1, 0, 0, 0};
constexpr int kEdgeFaceB[6] = {3, 3, 2, 3, 2, 1};
constexpr float kEdgeSignA[6] = {1.f, -1.f, 1.f, 1.f, -1.f, 1.f};

// Largest (smallest) outward edge value of each face: the face is the entry
// (exit) face of the ray iff this is negative (positive).
__device__ __forceinline__ void face_max(const float* E, float* g) {
  g[0] = fmaxf(fmaxf(E[3], E[5]), -E[4]);
  g[1] = fmaxf(fmaxf(E[2], -E[5]), -E[1]);
  g[2] = fmaxf(fmaxf(E[0], E[4]), -E[2]);
  g[3] = fmaxf(fmaxf(E[1], -E[3]), -E[0]);
}
__device__ __forceinline__ void face_min(const float* E, float* g) {
  g[0] = fminf(fminf(E[3], E[5]), -E[4]);
  g[1] = fminf(fminf(E[2], -E[5]), -E[1]);
  g[2] = fminf(fminf(E[0], E[4]), -E[2]);
  g[3] = fminf(fminf(E[1], -E[3]), -E[0]);
}

// One lane per tetrahedron and angle chunk.  Per angle the six 2-D edge
// values are affine in the pixel position, E_e = C_e + x A_e + y B_e in
// coordinates local to the shadow's first pixel, evaluated as one fused
// multiply-add per pixel on a per-row value.  A pixel is decided when the
// smallest over faces of the largest outward edge value is certainly
// positive (no entry face: miss) or, for a hit, certainly negative with an
// exit face whose smallest value is certainly positive; anything else takes
// the per-edge route (float64 3-D values, then the exact pass).
template <bool kLdsTable>
__global__ __launch_bounds__(kShadowThreads, 4) void shadow_fast_kernel(ShadowArgs A) {
  // Face planes of each lane's tetrahedron, float64: (n_x, n_y) and
  // (n_z, (a_f - S) . n_f) for face f through vertex a_f.
  __shared__ double2 s_plane[4][2][kShadowThreads];
  __shared__ float s_ut[kLdsTable ? kShadowLdsTable : 1];
  const int nu = A.G.nu, nv = A.G.nv;
  if constexpr (kLdsTable) {
    for (int k = threadIdx.x; k < nu; k += kShadowThreads) s_ut[k] = A.G.ut[k];
    __syncthreads();
  }
  const float* ut = kLdsTable ? s_ut : A.G.ut;
  const float* vt = A.G.vt;
  const int nt = A.M.nt;
  const int lane = threadIdx.x;
  // XCD-aware order (xcd_block): each die takes one contiguous run of
  // tetrahedra (neighbours in the mesh order), whose shadows cover one region
  // of the detector, so its L2 holds that region's projection values.
  const int64_t nblk = (int64_t)gridDim.x * gridDim.y;
  const int64_t blk = xcd_block((int64_t)blockIdx.y * gridDim.x + blockIdx.x, nblk);
  const int t = (int)(blk % gridDim.x) * kShadowThreads + lane;
  const int chunk = (int)(blk / gridDim.x);
  const int a_begin = A.a0 + chunk * A.chunk_len;
  const int a_end = min(A.a0 + A.na, a_begin + A.chunk_len);
  ShadowStats st;
  if (t < nt) {
    const float4* tq = A.M.tetxyz + 3 * (size_t)t;
    // Face normals (angle independent), vertices in increasing order.
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const int ia = f == 0 ? 1 : 0, ib = f <= 1 ? 2 : 1, ic = f == 3 ? 2 : 3;
      const float3 pa = tet_vertex(tq, ia), pb = tet_vertex(tq, ib), pc = tet_vertex(tq, ic);
      double bx = (double)pb.x - pa.x, by = (double)pb.y - pa.y, bz = (double)pb.z - pa.z;
      double cx = (double)pc.x - pa.x, cy = (double)pc.y - pa.y, cz = (double)pc.z - pa.z;
      s_plane[f][0][lane] = make_double2(by * cz - bz * cy, bz * cx - bx * cz);
      s_plane[f][1][lane] = make_double2(bx * cy - by * cx, 0.0);
    }
    double acc = 0.0;
    bool deferred = false;
#pragma unroll 1
    for (int a = a_begin; a < a_end && !deferred; ++a) {
      FrameD F = load_frame(A.G.frame, a);
      double al[4], be[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) project_vertex(F, tet_vertex(tq, k), al[k], be[k]);
      int i0, i1, j0, j1;
      if (!shadow_box(A, al, be, i0, i1, j0, j1)) continue;
      // Local detector coordinates around the pixel centre (i0, j0).
      const float ao = ut[i0], bo = vt[j0];
      float xk[4], yk[4];
      float Lb = fmaxf(fmaxf(ut[i1] - ao, vt[j1] - bo), fmaxf((float)(i1 - i0) * A.du, (float)(j1 - j0) * A.dv));
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        xk[k] = (float)(al[k] - (double)ao);
        yk[k] = (float)(be[k] - (double)bo);
        Lb = fmaxf(Lb, fmaxf(fabsf(xk[k]), fabsf(yk[k])));
      }
      // E'_pq = (x_p - x)(y_q - y) - (y_p - y)(x_q - x) differs from its
      // exact value at the pixel centre by at most 34 u Lb^2 for the
      // rounding of the local coordinates (vertices and pixel) and of the
      // affine evaluation; the ray meets the plane within eps_p of the
      // centre, which moves E' by at most 4 eps_p Lb.
      const float bound = fmaf(64.0f * kUnit * Lb, Lb, fmaf(4.5f * A.eps_p, Lb, kShadowAbs));
      const float sg = F.hN > 0.0 ? 1.0f : -1.0f;
      // E = sg E' = cC + kx cA + y cB with kx = i - i0 and y = (j - j0) dv.
      float cA[6], cB[6], cC[6];
#pragma unroll
      for (int e = 0; e < 6; ++e) {
        const int p = kEdgeP[e], q = kEdgeQ[e];
        cA[e] = sg * ((yk[p] - yk[q]) * A.du);
        cB[e] = sg * (xk[q] - xk[p]);
        cC[e] = sg * fmaf(xk[p], yk[q], -(yk[p] * xk[q]));
      }
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const float3 pa = tet_vertex(tq, f == 0 ? 1 : 0);
        const double2 n0 = s_plane[f][0][lane];
        double2 n1 = s_plane[f][1][lane];
        n1.y = ((double)pa.x - F.Sx) * n0.x + ((double)pa.y - F.Sy) * n0.y + ((double)pa.z - F.Sz) * n1.x;
        s_plane[f][1][lane] = n1;
      }
      // Row spans.  The shadow is bounded by the silhouette edges: those
      // between a face the rays enter by (its outward edge values are all
      // negative inside it, so their constant sum S_f is negative) and one
      // they leave by.  For a silhouette edge with outward sign s in its
      // entry face the whole shadow has s E_e <= 0, so a pixel with
      // s E_e > bound is no hit; in a row that bounds kx from one side:
      // kx <= t or kx >= t with t = (s bound - R_e) / cA_e.  With a face seen
      // nearly edge-on (|S_f| <= bound) the silhouette is uncertain and the
      // whole box is scanned; near-horizontal edges (|cA_e| < bound / 1024)
      // are not used.  Skipping pixels never changes a decision: every
      // scanned pixel is still classified as above.
      const float Sf[4] = {cC[3] + cC[5] - cC[4], cC[2] - cC[5] - cC[1], cC[0] + cC[4] - cC[2],
                           cC[1] - cC[3] - cC[0]};
      const bool spans = fminf(fminf(fabsf(Sf[0]), fabsf(Sf[1])), fminf(fabsf(Sf[2]), fabsf(Sf[3]))) > bound;
      float rA[6], sb[6];
      bool upper[6], lower[6];
#pragma unroll
      for (int e = 0; e < 6; ++e) {
        const bool fa = Sf[kEdgeFaceA[e]] < 0.f, fb = Sf[kEdgeFaceB[e]] < 0.f;
        const float sgn = fa ? kEdgeSignA[e] : -kEdgeSignA[e];
        const float g = sgn * cA[e];
        const bool use = spans && fa != fb && fabsf(cA[e]) * 1024.0f >= bound;
        upper[e] = use && g > 0.f;
        lower[e] = use && g < 0.f;
        rA[e] = use ? 1.0f / cA[e] : 0.f;
        sb[e] = sgn * bound;
      }
      const float box_hi = (float)(i1 - i0);
      const float* yrow = A.proj + (size_t)a * nv * nu;
#pragma unroll 1
      for (int j = j0; j <= j1 && !deferred; ++j) {
        const float vv = vt[j];
        const float y = (float)(j - j0) * A.dv;
        const float* yr = yrow + (size_t)j * nu;
        float R[6];
#pragma unroll
        for (int e = 0; e < 6; ++e) R[e] = fmaf(y, cB[e], cC[e]);
        float lo = 0.f, hi = box_hi;
#pragma unroll
        for (int e = 0; e < 6; ++e) {
          const float t = (sb[e] - R[e]) * rA[e];
          hi = upper[e] ? fminf(hi, t) : hi;
          lo = lower[e] ? fmaxf(lo, t) : lo;
        }
        // Slack for the rounding of t (relative) and of the comparison.
        hi = fmaxf(hi + fmaf(fabsf(hi), 0x1p-22f, 0x1p-10f), -1.0f);
        lo = fminf(lo - fmaf(fabsf(lo), 0x1p-22f, 0x1p-10f), box_hi + 1.0f);
        const int ilo = i0 + max(0, (int)ceilf(lo)), ihi = i0 + min(i1 - i0, (int)floorf(hi));
#pragma unroll 1
        for (int i = ilo; i <= ihi; ++i) {
          // Issued first so that their latency overlaps the classification.
          const float yv = yr[i];
          const float uu = ut[i];
          const float kx = (float)(i - i0);
          float E[6];
#pragma unroll
          for (int e = 0; e < 6; ++e) E[e] = fmaf(kx, cA[e], R[e]);
          float g[4];
          face_max(E, g);
          const float m = fminf(fminf(g[0], g[1]), fminf(g[2], g[3]));
          if (m > bound) continue;
          float h[4];
          face_min(E, h);
          const float M = fmaxf(fmaxf(h[0], h[1]), fmaxf(h[2], h[3]));
          int fe = 3, fx = 3;
          fe = g[2] == m ? 2 : fe;
          fe = g[1] == m ? 1 : fe;
          fe = g[0] == m ? 0 : fe;
          fx = h[2] == M ? 2 : fx;
          fx = h[1] == M ? 1 : fx;
          fx = h[0] == M ? 0 : fx;
          fx = (m < -bound && M > bound) ? fx : -1;
          const float3 P = pixel_point(F.f, uu, vv);
          const double dx = (double)P.x - F.Sx, dy = (double)P.y - F.Sy, dz = (double)P.z - F.Sz;
          if (fx < 0) {
            // Per-edge route: certain float signs, float64 3-D values for
            // the rest, the exact pass for what float64 cannot decide.
            int pos = 0, neg = 0;
#pragma unroll
            for (int e = 0; e < 6; ++e) {
              pos |= (E[e] > bound) << e;
              neg |= (E[e] < -bound) << e;
            }
            int unk = 0x3f & ~(pos | neg);
            if (unk) {
              const float3 df = f3sub(P, F.S);
              const float dinf = fmaxf(fabsf(df.x), fmaxf(fabsf(df.y), fabsf(df.z)));
              while (unk) {
                const int e = __ffs(unk) - 1;
                unk &= unk - 1;
                const int pe = (0x211000 >> (4 * e)) & 3, qe = (0x332321 >> (4 * e)) & 3;
                const int s = edge_sign_fp64(F, dx, dy, dz, dinf, tet_vertex(tq, pe), tet_vertex(tq, qe), nullptr);
                st.fp64++;
                if (s == 0) {
                  deferred = true;
                  break;
                }
                pos |= (s > 0) << e;
                neg |= (s < 0) << e;
              }
              if (deferred) break;
            }
            fe = entry_face(neg, pos);
            if (fe < 0) continue;
            fx = entry_face(pos, neg);
            if (fx < 0) continue;  // cannot happen for a valid tetrahedron
          }
          st.hits++;
          const double2 e0 = s_plane[fe][0][lane], e1 = s_plane[fe][1][lane];
          const double2 x0 = s_plane[fx][0][lane], x1 = s_plane[fx][1][lane];
          const double de = fma(dx, e0.x, fma(dy, e0.y, dz * e1.x));
          const double dxx = fma(dx, x0.x, fma(dy, x0.y, dz * x1.x));
          // t_x - t_e = (n_x d_e - n_e d_x) / (d_x d_e); the float64
          // numerator keeps the cancellation harmless.
          const double num = fma(x1.y, de, -(e1.y * dxx));
          const float3 df = f3sub(P, F.S);
          const float dn = __builtin_amdgcn_sqrtf(fmaf(df.x, df.x, fmaf(df.y, df.y, df.z * df.z)));
          float L = (float)num * dn * __builtin_amdgcn_rcpf((float)(dxx * de));
          L = fmaxf(L, 0.f);
          acc = fma((double)L, (double)yv, acc);
        }
      }
    }
    if (deferred) {
      int k = atomicAdd(A.dirty_count, 1);
      A.dirty[k] = chunk * nt + t;
    } else {
      store_result(A, chunk, t, acc);
    }
  }
  flush_shadow_stats(A.M, st);
}

// ---------------------------------------------------------------- exact pass

// One lane per deferred item, all six signs per candidate pixel in float64
// with the exact expansion behind the filter.
template <bool kLdsTables>
__global__ __launch_bounds__(kShadowThreads) void shadow_exact_kernel(ShadowArgs A) {
  __shared__ float s_ut[kLdsTables ? kShadowLdsTable : 1];
  __shared__ float s_vt[kLdsTables ? kShadowLdsTable : 1];
  const int nu = A.G.nu, nv = A.G.nv;
  if constexpr (kLdsTables) {
    for (int k = threadIdx.x; k < nu; k += kShadowThreads) s_ut[k] = A.G.ut[k];
    for (int k = threadIdx.x; k < nv; k += kShadowThreads) s_vt[k] = A.G.vt[k];
    __syncthreads();
  }
  const float* ut = kLdsTables ? s_ut : A.G.ut;
  const float* vt = kLdsTables ? s_vt : A.G.vt;
  const int nt = A.M.nt;
  const int count = *A.dirty_count;
  ShadowStats st;
  // One wavefront per deferred item; lane l takes the angles a_begin + l,
  // a_begin + l + 64, ... in order, and the 64 partial sums are combined in
  // a fixed butterfly order (lane 0's result is stored), so the sum is the
  // same on every run.
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * kShadowThreads + threadIdx.x) >> 6;
  const int nwaves = (gridDim.x * kShadowThreads) >> 6;
  for (int k = wave; k < count; k += nwaves) {
    const int item = __builtin_amdgcn_readfirstlane(A.dirty[k]);
    const int chunk = item / nt, t = item - chunk * nt;
    const int a_begin = A.a0 + chunk * A.chunk_len;
    const int a_end = min(A.a0 + A.na, a_begin + A.chunk_len);
    const float4* tq = A.M.tetxyz + 3 * (size_t)t;
    float3 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = tet_vertex(tq, q);
    double acc = 0.0;
#pragma unroll 1
    for (int a = a_begin + lane; a < a_end; a += 64) {
      FrameD F = load_frame(A.G.frame, a);
      double al[4], be[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) project_vertex(F, v[q], al[q], be[q]);
      int i0, i1, j0, j1;
      if (!shadow_box(A, al, be, i0, i1, j0, j1)) continue;
      const float* yrow = A.proj + (size_t)a * nv * nu;
#pragma unroll 1
      for (int j = j0; j <= j1; ++j) {
        const float vv = vt[j];
#pragma unroll 1
        for (int i = i0; i <= i1; ++i) {
          const float3 P = pixel_point(F.f, ut[i], vv);
          const double dx = (double)P.x - F.Sx, dy = (double)P.y - F.Sy, dz = (double)P.z - F.Sz;
          const float3 df = f3sub(P, F.S);
          const float dinf = fmaxf(fabsf(df.x), fmaxf(fabsf(df.y), fabsf(df.z)));
          float E[6];
          int pos = 0, neg = 0;
#pragma unroll
          for (int e = 0; e < 6; ++e) {
            const int pe = e < 3 ? 0 : (e < 5 ? 1 : 2);
            const int qe = e < 3 ? e + 1 : (e < 5 ? e - 1 : 3);
            double Ed;
            int s = edge_sign_fp64(F, dx, dy, dz, dinf, v[pe], v[qe], &Ed);
            E[e] = (float)Ed;
            pos |= (s > 0) << e;
            neg |= (s < 0) << e;
          }
          int unk = 0x3f & ~(pos | neg);
          while (unk) {
            // One call site; the two vertices re-read from memory.
            const int e = __ffs(unk) - 1;
            unk &= unk - 1;
            const int pe = (0x211000 >> (4 * e)) & 3, qe = (0x332321 >> (4 * e)) & 3;
            const int res = slow_edge_sign(F.S, P, F.U, F.V, tet_vertex(tq, pe), tet_vertex(tq, qe));
            const int s = (res & 3) - 1;
            st.slow++;
            if (res & (kFlagExact << 2)) st.exact++;
            if (res & (kFlagPerturbed << 2)) st.pert++;
            pos |= (s > 0) << e;
            neg |= (s < 0) << e;
          }
          const int fe = entry_face(neg, pos);
          if (fe < 0) continue;
          const int fx = entry_face(pos, neg);
          if (fx < 0) continue;
          st.hits++;
          // Crossing points from the edge values: for face (a, b, c) the
          // weight of a is E(b, c).  With lambda_k = (v_k - v0) . d the
          // chord is (sum_k w^x_k lambda_k / W_x - sum_k w^e_k lambda_k / W_e) / |d|.
          const float3 d = df;
          const float l1 = f3dot(f3sub(v[1], v[0]), d), l2 = f3dot(f3sub(v[2], v[0]), d),
                      l3 = f3dot(f3sub(v[3], v[0]), d);
          float Nf[4], Wf[4];
          Nf[0] = E[5] * l1 - E[4] * l2 + E[3] * l3;
          Wf[0] = E[5] - E[4] + E[3];
          Nf[1] = E[2] * l2 - E[1] * l3;
          Wf[1] = E[2] - E[5] - E[1];
          Nf[2] = E[0] * l3 - E[2] * l1;
          Wf[2] = E[4] - E[2] + E[0];
          Nf[3] = E[1] * l1 - E[0] * l2;
          Wf[3] = E[1] - E[3] - E[0];
          const float ne = fe == 0 ? Nf[0] : fe == 1 ? Nf[1] : fe == 2 ? Nf[2] : Nf[3];
          const float we = fe == 0 ? Wf[0] : fe == 1 ? Wf[1] : fe == 2 ? Wf[2] : Wf[3];
          const float nx = fx == 0 ? Nf[0] : fx == 1 ? Nf[1] : fx == 2 ? Nf[2] : Nf[3];
          const float wx = fx == 0 ? Wf[0] : fx == 1 ? Wf[1] : fx == 2 ? Wf[2] : Wf[3];
          float L = (nx / wx - ne / we) * __frsqrt_rn(f3dot(d, d));
          L = fmaxf(L, 0.f);
          acc = fma((double)L, (double)yrow[(size_t)j * nu + i], acc);
        }
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) store_result(A, chunk, t, acc);
  }
  flush_shadow_stats(A.M, st);
}

// xhat[t] = (accumulate ? xhat[t] : 0) + sum over chunks, in chunk order.
__global__ void shadow_reduce_kernel(const double* partial, int chunks, int nt, float* xhat, int accumulate) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  double s = accumulate ? (double)xhat[t] : 0.0;
  for (int k = 0; k < chunks; ++k) s += partial[(size_t)k * nt + t];
  xhat[t] = (float)s;
}

__global__ void zero_int_kernel(int* p) { *p = 0; }

}  // namespace

tct_status backproject_shadow(const tct_mesh* m, const tct_geom* g, const float* proj, float* xhat, int accumulate,
                              int a_begin, int a_count, hipStream_t s) {
  if (m->nt <= 0) return TCT_OK;
  if (a_count <= 0) {
    if (!accumulate) return launch_fill(xhat, m->nt, 0.f, s);
    return TCT_OK;
  }
  ShadowArgs A;
  A.M = m->view();
  A.G = g->view();
  A.proj = proj;
  A.xhat = xhat;
  A.partial = nullptr;
  A.a0 = a_begin;
  A.na = a_count;
  A.accumulate = accumulate;
  const tct_cone& c = g->cone;
  A.u0 = g->ut[0];
  A.v0 = g->vt[0];
  A.inv_du = (float)(1.0 / c.du);
  A.inv_dv = (float)(1.0 / c.dv);
  // Pixel points: each coordinate of P = fl(fl(D + fl(u U)) + fl(v V)) is
  // within u (|u U_c| + |v V_c| + 2 |P_c|) of D + u U + v V; the ray meets
  // the detector plane within (1 + tan) of that, tan being the angle between
  // the ray and the plane normal.  Bounded over the detector corners of every
  // angle (the terms are convex in the pixel position), in the detector's
  // own units, with a 25% margin.
  double R = 0.0, eps = 0.0;
  const double u = std::ldexp(1.0, -24);
  const float us[2] = {g->ut.front(), g->ut.back()}, vs[2] = {g->vt.front(), g->vt.back()};
  for (int a = 0; a < g->na; ++a) {
    const float* f = &g->frame[12 * (size_t)a];
    double r = 0.0;
    for (int k = 0; k < 6; ++k) r = std::max(r, (double)std::fabs(f[k]));
    R = std::max(R, 2.0 * r);
    double N[3] = {(double)f[7] * f[11] - (double)f[8] * f[10], (double)f[8] * f[9] - (double)f[6] * f[11],
                   (double)f[6] * f[10] - (double)f[7] * f[9]};
    double nn = std::sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
    double umin = std::min(std::sqrt((double)f[6] * f[6] + (double)f[7] * f[7] + (double)f[8] * f[8]),
                           std::sqrt((double)f[9] * f[9] + (double)f[10] * f[10] + (double)f[11] * f[11]));
    for (int cu = 0; cu < 2; ++cu)
      for (int cv = 0; cv < 2; ++cv) {
        double err = 0.0, d[3], P[3];
        for (int k = 0; k < 3; ++k) {
          P[k] = f[3 + k] + (double)us[cu] * f[6 + k] + (double)vs[cv] * f[9 + k];
          d[k] = P[k] - f[k];
          err += std::fabs((double)us[cu] * f[6 + k]) + std::fabs((double)vs[cv] * f[9 + k]) + 2.0 * std::fabs(P[k]);
        }
        double dn = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double cosv = std::fabs(d[0] * N[0] + d[1] * N[1] + d[2] * N[2]) / (dn * nn);
        double tanv = std::sqrt(std::max(0.0, 1.0 - cosv * cosv)) / std::max(cosv, 1e-300);
        eps = std::max(eps, u * err * (1.0 + tanv) / umin);
      }
  }
  // The pixel tables are float32 roundings of affine values: the local
  // coordinates (i - i0) du used by the fast pass differ from the tables'
  // differences by at most 2u max|table| (the product's rounding is in the
  // kernel's bound).
  const double tmax = std::max(std::max(std::fabs((double)g->ut.front()), std::fabs((double)g->ut.back())),
                               std::max(std::fabs((double)g->vt.front()), std::fabs((double)g->vt.back())));
  A.eps_p = (float)(1.25 * (eps + 2.0 * u * (tmax + std::max(c.du, c.dv))));
  A.du = (float)c.du;
  A.dv = (float)c.dv;
  R += std::max(std::max(std::fabs((double)g->ut.front()), std::fabs((double)g->ut.back())),
                std::max(std::fabs((double)g->vt.front()), std::fabs((double)g->vt.back())));
  // Shadow margin: rounding of the pixel points and of the projected vertices
  // is a few float32 ulps of the coordinates involved; 2^-15 of their size in
  // pixels plus 1/32 pixel covers it many times over.
  A.margin = (float)(1.0 / 32 + std::ldexp(R, -15) * std::max(1.0 / c.du, 1.0 / c.dv));
  int64_t blocks = ((int64_t)m->nt + kShadowThreads - 1) / kShadowThreads;
  int64_t waves = blocks * (kShadowThreads / 64);
  int chunks = (int)std::max<int64_t>(1, std::min<int64_t>(a_count, (kShadowTargetWaves + waves - 1) / waves));
  A.chunk_len = (a_count + chunks - 1) / chunks;
  chunks = (a_count + A.chunk_len - 1) / A.chunk_len;
  // Scratch: [counter][pad][deferred items: chunks * nt][float64 partials when chunked].
  size_t items = (size_t)chunks * m->nt;
  size_t off_part = ((16 + 4 * items) + 255) & ~(size_t)255;
  size_t bytes = off_part + (chunks > 1 ? sizeof(double) * items : 0);
  void* scratch = nullptr;
  TCT_HIP(hipMallocAsync(&scratch, bytes, s));
  A.dirty_count = (int*)scratch;
  A.dirty = (int*)((char*)scratch + 16);
  A.partial = chunks > 1 ? (double*)((char*)scratch + off_part) : nullptr;
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, s, A.dirty_count);
  const bool lds = g->cone.nu <= kShadowLdsTable && g->cone.nv <= kShadowLdsTable;
  dim3 grid((unsigned)blocks, (unsigned)chunks), block(kShadowThreads);
  if (lds)
    hipLaunchKernelGGL(shadow_fast_kernel<true>, grid, block, 0, s, A);
  else
    hipLaunchKernelGGL(shadow_fast_kernel<false>, grid, block, 0, s, A);
  // The exact pass reads the deferred count on the device: a fixed grid
  // strides over however many items the fast pass left.
  const int64_t waves_per_block = kShadowThreads / 64;
  unsigned xgrid = (unsigned)std::min<int64_t>(1024, (int64_t)(items + waves_per_block - 1) / waves_per_block);
  if (lds)
    hipLaunchKernelGGL(shadow_exact_kernel<true>, dim3(xgrid), block, 0, s, A);
  else
    hipLaunchKernelGGL(shadow_exact_kernel<false>, dim3(xgrid), block, 0, s, A);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && A.partial) {
    hipLaunchKernelGGL(shadow_reduce_kernel, dim3((unsigned)((m->nt + 255) / 256)), dim3(256), 0, s,
                       (const double*)A.partial, chunks, m->nt, xhat, accumulate);
    e = hipGetLastError();
  }
  (void)hipFreeAsync(scratch, s);
  if (e != hipSuccess) return hip_fail(e, "shadow backprojection launch");
  return TCT_OK;
}

}  // namespace tct
