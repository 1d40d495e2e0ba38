// Paper-faithful propagation (Algorithms 1 and 2 of Section II), for
// comparison with the exact walk: per tetrahedron four Moller-Trumbore
// ray-triangle tests with the safety parameter eps, escalated by x10 until
// two faces are hit, then a step to the neighbour across the face of the
// larger intersection parameter.  Templated on the arithmetic type (the
// paper's single versus double precision experiment, Section III-C).
//
// Readings where the algorithms leave a choice:
//   * the second barycentric coordinate is v = f (d . r) (the printed cross
//     product would not be a scalar);
//   * the parallel test is the printed absolute |a| < 1e-8;
//   * eps starts at 1e-9 for every tetrahedron and is multiplied by 10 after
//     each failure; past eps = 1 the ray is declared halted;
//   * of the faces hit, t1 is the smallest parameter and the exit is the
//     face with the largest one other than the face the ray came in by
//     (never step back; the check of Algorithm 2 that exchanges the hits), lowest index on
//     ties;
//   * a ray that takes more than kPaperStepCap steps is declared looping;
//   * the ray enters through the boundary face found by the exact entry
//     search (initialisation is not part of this comparison).
// Face k of a tetrahedron is opposite its vertex k, with the other three
// vertices in increasing local order; the local order is the vertex table's
// (ascending node ids, the last two swapped if that order is negatively
// oriented).  All arithmetic is written out in a fixed order without fused
// multiply-add, so the CPU reference reproduces it bit for bit.
#include "common.h"
#include "kernels.h"
#include "ray.h"

namespace tct {

namespace {

constexpr int kPaperStepCap = 16384;

template <typename T>
struct Vec3 {
  T x, y, z;
};

template <typename T>
__device__ __forceinline__ Vec3<T> vsub(const Vec3<T>& a, const Vec3<T>& b) {
  return {a.x - b.x, a.y - b.y, a.z - b.z};
}
template <typename T>
__device__ __forceinline__ T vdot(const Vec3<T>& a, const Vec3<T>& b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename T>
__device__ __forceinline__ Vec3<T> vcross(const Vec3<T>& a, const Vec3<T>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename T>
__device__ __forceinline__ Vec3<T> vcast(float3 p) {
  return {(T)p.x, (T)p.y, (T)p.z};
}

// Algorithm 1: Moller-Trumbore with the safety parameter eps.
template <typename T>
__device__ __forceinline__ bool mt_hit(const Vec3<T>& R1, const Vec3<T>& d, const Vec3<T>& P1, const Vec3<T>& P2,
                                       const Vec3<T>& P3, T eps, T& t) {
  const Vec3<T> E1 = vsub(P2, P1), E2 = vsub(P3, P1);
  const Vec3<T> q = vcross(d, E2);
  const T a = vdot(E1, q);
  const T tiny = (T)1e-8;
  if (a > -tiny && a < tiny) return false;
  const T f = (T)1 / a;
  const Vec3<T> s = vsub(R1, P1);
  const T u = f * vdot(s, q);
  if (u < (T)0 - eps) return false;
  const Vec3<T> r = vcross(s, E1);
  const T v = f * vdot(d, r);
  if (v < (T)0 - eps || u + v > (T)1 + eps) return false;
  t = f * vdot(E2, r);
  return true;
}

struct PaperStats {
  int steps = 0, escalations = 0, halted = 0, looped = 0;
};

// Algorithm 2 for one ray; returns the line integral in T.
template <typename T>
__device__ T paper_walk(const MeshView& M, const float* x, float3 S, float3 P, int tet, int entry_face,
                        PaperStats& st) {
  const Vec3<T> R1 = vcast<T>(S), R2 = vcast<T>(P);
  const Vec3<T> d = vsub(R2, R1);
  const T l = sqrt(vdot(d, d));
  T sum = 0;
  int prev_face = entry_face;
  for (int step = 0;; ++step) {
    if (step >= kPaperStepCap) {
      st.looped++;
      break;
    }
    st.steps++;
    const float* c = (const float*)(M.tetxyz + 3 * (size_t)tet);
    Vec3<T> v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = {(T)c[3 * k], (T)c[3 * k + 1], (T)c[3 * k + 2]};
    T eps = (T)1e-9;
    T t1 = 0, t2 = 0;
    int exit = -1;
    bool halted = false;
    for (;;) {
      T th[4];
      bool hit[4];
      hit[0] = mt_hit(R1, d, v[1], v[2], v[3], eps, th[0]);
      hit[1] = mt_hit(R1, d, v[0], v[2], v[3], eps, th[1]);
      hit[2] = mt_hit(R1, d, v[0], v[1], v[3], eps, th[2]);
      hit[3] = mt_hit(R1, d, v[0], v[1], v[2], eps, th[3]);
      const int nhit = (int)hit[0] + (int)hit[1] + (int)hit[2] + (int)hit[3];
      if (nhit >= 2) {
        bool first = true;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (!hit[k]) continue;
          if (first || th[k] < t1) t1 = th[k];
          first = false;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (!hit[k] || k == prev_face) continue;
          if (exit < 0 || th[k] > t2) {
            t2 = th[k];
            exit = k;
          }
        }
        if (exit >= 0) break;
      }
      eps = eps * (T)10;
      st.escalations++;
      if (eps > (T)1) {
        halted = true;
        break;
      }
    }
    if (halted) {
      st.halted++;
      break;
    }
    sum = sum + l * (t2 - t1) * (T)x[tet];
    const int next = M.tetnbr[4 * (size_t)tet + exit];
    if (next < 0) break;
    // The face of `next` shared with `tet`.
    int back = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (M.tetnbr[4 * (size_t)next + k] == tet) back = k;
    prev_face = back;
    tet = next;
  }
  return sum;
}

template <typename T>
__global__ __launch_bounds__(256) void paper_forward_kernel(MeshView M, GeomView G, const float* x,
                                                            const int32_t* entry, float* proj,
                                                            unsigned long long* stats, int64_t nrays) {
  const int64_t rid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  PaperStats st;
  int ray = 0;
  if (rid < nrays) {
    const int i = (int)(rid % G.nu);
    const int j = (int)((rid / G.nu) % G.nv);
    const int a = (int)(rid / ((int64_t)G.nu * G.nv));
    const float* f = G.frame + 12 * a;
    const float3 S = make_float3(f[0], f[1], f[2]);
    const float3 P = pixel_point(f, G.ut[i], G.vt[j]);
    const int e = entry[rid];
    float out = 0.f;
    if (e >= 0) {
      ray = 1;
      const float4* bq = M.bfaces + 4 * (size_t)e;
      const int tet = __float_as_int(bq[0].w);
      const float4 opp = bq[3];
      // Local index of the owner's vertex opposite the entry face.
      const float* c = (const float*)(M.tetxyz + 3 * (size_t)tet);
      int ef = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (c[3 * k] == opp.x && c[3 * k + 1] == opp.y && c[3 * k + 2] == opp.z) ef = k;
      out = (float)paper_walk<T>(M, x, S, P, tet, ef, st);
    }
    proj[rid] = out;
  }
  int vals[5] = {ray, st.steps, st.escalations, st.halted, st.looped};
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    int v = vals[k];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(stats + k, (unsigned long long)v);
  }
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
  const int k = threadIdx.x;
  if (k < n) p[k] = 0ull;
}

}  // namespace

tct_status forward_paper(const tct_mesh* m, const tct_geom* g, const float* x, float* proj, const int32_t* entry,
                         int precision, tct_paper_stats* stats, hipStream_t s) {
  const int64_t n = g->nrays();
  unsigned long long* d_stats = nullptr;
  TCT_HIP(hipMallocAsync(&d_stats, 8 * sizeof(unsigned long long), s));
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, d_stats, 8);
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (precision == 64)
    hipLaunchKernelGGL(paper_forward_kernel<double>, grid, block, 0, s, m->view(), g->view(), x, entry, proj, d_stats,
                       n);
  else
    hipLaunchKernelGGL(paper_forward_kernel<float>, grid, block, 0, s, m->view(), g->view(), x, entry, proj, d_stats,
                       n);
  hipError_t e = hipGetLastError();
  unsigned long long h[8] = {0};
  if (e == hipSuccess && stats) {
    e = hipMemcpyAsync(h, d_stats, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  (void)hipFreeAsync(d_stats, s);
  if (e != hipSuccess) return hip_fail(e, "paper-faithful forward");
  if (stats) {
    stats->rays = (int64_t)h[0];
    stats->steps = (int64_t)h[1];
    stats->escalations = (int64_t)h[2];
    stats->halted = (int64_t)h[3];
    stats->looped = (int64_t)h[4];
  }
  return TCT_OK;
}

}  // namespace tct
