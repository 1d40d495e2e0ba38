// Ray walk kernels for gfx950.
//
// One lane per detector ray (Algorithm 2 launches one thread per pixel); a
// wavefront covers a tile of tile_u x tile_v = 64 pixels of one angle, so
// neighbouring rays, which cross nearby tetrahedra, share a wave and its
// cache lines (the paper found small square pixel blocks fastest, Section
// II-F).
//
// Per ray: find the boundary face it enters by (a BVH over boundary faces
// replaces the paper's R*-tree, Section II-E), then step from tetrahedron to
// neighbour.  The state carried from step to step is the face the ray came
// in by, as three vertex slots (a0, a1, a2) ordered so that all three edge
// signs sigma(a0,a1), sigma(a1,a2), sigma(a2,a0) are -1 (the ray enters
// through it), plus the current tetrahedron's fourth vertex v.  With
// s_k = sigma(v, a_k), the ray leaves
//   through the face opposite a2 iff s0 = -1 and s1 = +1,
//   through the face opposite a0 iff s1 = -1 and s2 = +1,
//   through the face opposite a1 iff s2 = -1 and s0 = +1,
// and the next entry face is the current one with slot k replaced by v.  One
// 16-byte record per (tetrahedron, face) gives the neighbour, its local index
// of the vertex opposite the shared face, and that vertex's coordinates, so a
// step costs one dependent load (plus x for the forward projection).
//
// sigma(p, q) is the exact sign of det[P - S, p - S, q - S] for the ray
// S -> P translated by eps U + eps^2 V (eps -> 0+), which makes the walk
// well defined through vertices, edges and face planes (the failure cases of
// Section II-C, Fig. 3) without the paper's escalating epsilon.  It is first
// estimated in float32 as (q - p) . ((P - S) x (p - S)) with a certified
// error bound; the rare uncertain cases go to a non-inlined float64 /
// exact-expansion routine (exact.h).
#include <mutex>
#include <type_traits>

#include "common.h"
#include "exact.h"
#include "kernels.h"
#include "ray.h"

namespace tct {

namespace {

// Pointers into LDS (32-bit addresses; atomics through them are native LDS
// atomics, not flat ones).
typedef __attribute__((address_space(3))) unsigned lds_u32;
typedef __attribute__((address_space(3))) int lds_i32;
typedef __attribute__((address_space(3))) long long lds_i64;

// The wavefront index within the block, as a wave-uniform (scalar) value.
__device__ __forceinline__ int wave_in_block() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// Walk statistics, in two forms with the same interface.  RegStats keeps
// every count in a lane register (the forward, trace and entry walks, where
// a register costs nothing and a branch per step would).  LdsStats keeps
// only the step count per lane and adds the rare events (zero-length
// passages, float64 and exact sign evaluations, perturbed ties, failures,
// float64 crossings) straight to the wavefront's own counters in LDS, which
// frees the registers the scatter walks need for their table.  flush_stats
// adds either to the mesh's counters once per wavefront.
enum Event { kEvZero = 0, kEvFp64, kEvExact, kEvPert, kEvFailed, kEvGrazing, kEvRays, kEvSteps, kEvents };

__device__ __forceinline__ void lds_add_u32(lds_u32* p, unsigned v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

struct RegStats {
  int steps = 0, zero = 0, fp64 = 0, exact = 0, pert = 0, failed = 0, grazing = 0;
  __device__ __forceinline__ explicit RegStats(lds_u32*) {}
  __device__ __forceinline__ void add_zero() { zero++; }
  __device__ __forceinline__ void add_grazing() { grazing++; }
  __device__ __forceinline__ void add_fp64() { fp64++; }
  __device__ __forceinline__ void add_exact() { exact++; }
  __device__ __forceinline__ void add_pert() { pert++; }
  __device__ __forceinline__ void add_failed() { failed++; }
};

struct LdsStats {
  int steps = 0;
  lds_u32* ev;  // this wavefront's kEvents counters in LDS
  __device__ __forceinline__ explicit LdsStats(lds_u32* wave_counters) : ev(wave_counters) {}
  __device__ __forceinline__ void add_zero() { lds_add_u32(ev + kEvZero, 1u); }
  __device__ __forceinline__ void add_grazing() { lds_add_u32(ev + kEvGrazing, 1u); }
  __device__ __forceinline__ void add_fp64() { lds_add_u32(ev + kEvFp64, 1u); }
  __device__ __forceinline__ void add_exact() { lds_add_u32(ev + kEvExact, 1u); }
  __device__ __forceinline__ void add_pert() { lds_add_u32(ev + kEvPert, 1u); }
  __device__ __forceinline__ void add_failed() { lds_add_u32(ev + kEvFailed, 1u); }
};

// The calling wavefront's event counters in the block's table `all`
// (kEvents per wavefront), cleared.
__device__ __forceinline__ lds_u32* wave_counters(unsigned* all) {
  lds_u32* ev = (lds_u32*)all + kEvents * wave_in_block();
  if ((threadIdx.x & 63) < kEvents) ev[threadIdx.x & 63] = 0u;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  return ev;
}

// Pixel ray S -> P(u, v) of one angle's frame.
__device__ __forceinline__ Ray cone_ray(const GeomView& g, float mesh_extent, int a, int i, int j) {
  const float* f = g.frame + 12 * a;
  float u = g.ut[i], v = g.vt[j];
  Ray r;
  r.S = make_float3(f[0], f[1], f[2]);
  r.U = make_float3(f[6], f[7], f[8]);
  r.V = make_float3(f[9], f[10], f[11]);
  r.P = pixel_point(f, u, v);
  finish_ray(r, mesh_extent);
  return r;
}

// Where the walk's rare exact paths find the ray's endpoints and
// tie-breaking axes.  Keeping them out of the step loop's live registers
// matters: for pixel rays they are re-read from the angle's frame (uniform
// across the block) and the pixel tables; listed rays carry them.
struct PixelSrc {
  const float* f;  // frame {S, D, U, V} of the ray's angle
  float u, v;      // pixel abscissa and ordinate
  __device__ __forceinline__ float3 S() const { return make_float3(f[0], f[1], f[2]); }
  __device__ __forceinline__ float3 P() const { return pixel_point(f, u, v); }
  __device__ __forceinline__ float3 U() const { return make_float3(f[6], f[7], f[8]); }
  __device__ __forceinline__ float3 V() const { return make_float3(f[9], f[10], f[11]); }
};
struct RegSrc {
  float3 s, p, uu, vv;
  __device__ __forceinline__ float3 S() const { return s; }
  __device__ __forceinline__ float3 P() const { return p; }
  __device__ __forceinline__ float3 U() const { return uu; }
  __device__ __forceinline__ float3 V() const { return vv; }
};

__device__ __forceinline__ PixelSrc pixel_src(const GeomView& g, int a, int i, int j) {
  return PixelSrc{g.frame + 12 * a, g.ut[i], g.vt[j]};
}

// Ray parameter s = t - 1/2 where S + t (P - S) meets the plane through
// `on` with normal (a - on) x (b - on), in float64 from the exact float32
// inputs.  Used when the crossing is ill-conditioned (the face is nearly
// parallel to the ray), where float32 rounding of any point on the ray is
// amplified by 1 / cos(angle between ray and normal).
__device__ __noinline__ double crossing_s_fp64(float3 S, float3 P, float3 on, float3 a, float3 b) {
  double dx = (double)P.x - S.x, dy = (double)P.y - S.y, dz = (double)P.z - S.z;
  double ax = (double)a.x - on.x, ay = (double)a.y - on.y, az = (double)a.z - on.z;
  double bx = (double)b.x - on.x, by = (double)b.y - on.y, bz = (double)b.z - on.z;
  double nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
  double ox = (double)on.x - S.x, oy = (double)on.y - S.y, oz = (double)on.z - S.z;
  return (ox * nx + oy * ny + oz * nz) / (dx * nx + dy * ny + dz * nz) - 0.5;
}


template <class St>
__device__ __forceinline__ int resolve(int fast, const Ray& r, float3 p, float3 q, St& st) {
  if (fast != 2) return fast;
  int res = slow_edge_sign(r.S, r.P, r.U, r.V, p, q);
  st.add_fp64();
  if (res & (kFlagExact << 2)) st.add_exact();
  if (res & (kFlagPerturbed << 2)) st.add_pert();
  return (res & 3) - 1;
}

template <class Src, class St>
__device__ __forceinline__ int resolve_src(const Src& q, float3 a, float3 b, St& st) {
  int res = slow_edge_sign(q.S(), q.P(), q.U(), q.V(), a, b);
  st.add_fp64();
  if (res & (kFlagExact << 2)) st.add_exact();
  if (res & (kFlagPerturbed << 2)) st.add_pert();
  return (res & 3) - 1;
}

// Exact entry test for boundary face b (slots in outward order).
template <class St>
__device__ bool enters_face(const MeshView& M, const Ray& r, int b, St& st) {
  const float4* q = M.bfaces + 4 * (size_t)b;
  float4 q0 = q[0], q1 = q[1], q2 = q[2];
  float3 a0 = make_float3(q0.x, q0.y, q0.z), a1 = make_float3(q1.x, q1.y, q1.z), a2 = make_float3(q2.x, q2.y, q2.z);
  float3 w, W;
  cross_pair(r, a0, w, W);
  int s0 = fast_sign(f3sub(a1, a0), w, W);
  if (s0 == 1) return false;
  cross_pair(r, a1, w, W);
  int s1 = fast_sign(f3sub(a2, a1), w, W);
  if (s1 == 1) return false;
  cross_pair(r, a2, w, W);
  int s2 = fast_sign(f3sub(a0, a2), w, W);
  if (s2 == 1) return false;
  if (resolve(s0, r, a0, a1, st) != -1) return false;
  if (resolve(s1, r, a1, a2, st) != -1) return false;
  return resolve(s2, r, a2, a0, st) == -1;
}

// Slab test against a padded box over the whole line (conservative).
__device__ __forceinline__ bool line_hits_box(const Ray& r, float3 inv, const BvhNode& nd) {
  float tmin = -INFINITY, tmax = INFINITY;
  const float s[3] = {r.S.x, r.S.y, r.S.z};
  const float d[3] = {r.d.x, r.d.y, r.d.z};
  const float iv[3] = {inv.x, inv.y, inv.z};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (d[k] == 0.0f) {
      if (s[k] < nd.lo[k] || s[k] > nd.hi[k]) return false;
    } else {
      float t0 = (nd.lo[k] - s[k]) * iv[k];
      float t1 = (nd.hi[k] - s[k]) * iv[k];
      tmin = fmaxf(tmin, fminf(t0, t1));
      tmax = fminf(tmax, fmaxf(t0, t1));
    }
  }
  return tmin <= tmax;
}

// Depth-first scan of a preorder tree with skip links (no stack) from
// `node` until `end` (-1: the end of the array): the convex hull is entered
// through exactly one face, so the first face passing the exact entry test
// is the answer.  BVH leaves hold a contiguous range of faces
// (first * 8 + count); R*-tree leaves index a face list (first * 16 + count).
template <bool kRstar, class St>
__device__ int scan_tree(const MeshView& M, const BvhNode* tree, const Ray& r, float3 inv, int node, int end,
                         St& st) {
  while (node >= 0 && node != end) {
    const float4* np = reinterpret_cast<const float4*>(tree + node);
    float4 n0 = np[0], n1 = np[1];
    BvhNode nd;
    nd.lo[0] = n0.x;
    nd.lo[1] = n0.y;
    nd.lo[2] = n0.z;
    nd.skip = __float_as_int(n0.w);
    nd.hi[0] = n1.x;
    nd.hi[1] = n1.y;
    nd.hi[2] = n1.z;
    nd.leaf = __float_as_int(n1.w);
    if (line_hits_box(r, inv, nd)) {
      if (nd.leaf >= 0) {
        if constexpr (kRstar) {
          const int first = nd.leaf >> 4, cnt = nd.leaf & 15;
          for (int i = 0; i < cnt; ++i) {
            const int f = M.rstar_faces[first + i];
            if (enters_face(M, r, f, st)) return f;
          }
        } else {
          const int first = nd.leaf >> 3, cnt = nd.leaf & 7;
          for (int i = 0; i < cnt; ++i)
            if (enters_face(M, r, first + i, st)) return first + i;
        }
        node = nd.skip;
      } else {
        node = node + 1;
      }
    } else {
      node = nd.skip;
    }
  }
  return -1;
}

// Entry search (Section II-E) through the boundary BVH, or the R*-tree
// (kRstar).  The BVH is split into groups of faces by the axis of their
// outward normal; a ray enters only through a face with d . n < 0, so a
// group is skipped when the smallest d . n over its normals' bounding box is
// positive (beyond the rounding of that bound: products of |n| <= 1 with d,
// three of them summed, err below 3u |d|_1; the margin is 1e-6 |d|_1).
template <bool kRstar = false, class St>
__device__ int find_entry(const MeshView& M, const Ray& r, St& st) {
  float3 inv = make_float3(1.0f / r.d.x, 1.0f / r.d.y, 1.0f / r.d.z);
  if constexpr (kRstar) {
    return scan_tree<true>(M, M.rstar, r, inv, 0, -1, st);
  } else {
    const float4* h = reinterpret_cast<const float4*>(M.bvh);
    const float l1 = fabsf(r.d.x) + fabsf(r.d.y) + fabsf(r.d.z);
    const int ng = __float_as_int(h[0].w);
    for (int g = 1; g <= ng; ++g) {
      const float4 lo = h[2 * g], hi = h[2 * g + 1];  // normal bounds; lo.w = end node, hi.w = root node
      const float m = fminf(r.d.x * lo.x, r.d.x * hi.x) + fminf(r.d.y * lo.y, r.d.y * hi.y) +
                      fminf(r.d.z * lo.z, r.d.z * hi.z);
      if (m > 1e-6f * l1) continue;
      const int f = scan_tree<false>(M, M.bvh, r, inv, __float_as_int(hi.w), __float_as_int(lo.w), st);
      if (f >= 0) return f;
    }
    return -1;
  }
}

// Per-wavefront accumulation tables for the backprojections.  Neighbouring
// rays of a pixel tile cross mostly the same tetrahedra (at the benchmark
// pitch an 8 x 8 tile spans about one element), so scattering every segment
// with a global atomic makes dozens of lanes update one address at once.
// Instead each wavefront sums its segments per tetrahedron in its own LDS
// open-addressing table (key = tetrahedron, linear probing) and adds one
// global atomic (or, for the explicit lists, writes one record) per distinct
// tetrahedron when it flushes the table.  The rays advance in windows of a
// fixed number of steps and the wavefront flushes its table after each
// window, so the table only holds the tetrahedra of one window of its ray
// bundle (an 8 x 8 bundle meets about 170 tetrahedra per 32 steps, 300 per
// 64 steps on the benchmark mesh); a segment that finds no slot within
// kLdsProbes probes goes straight to global memory.  Tables are private to a
// wavefront, so a window ends without any block-wide barrier and each
// wavefront runs at its own pace.  The scatters use small tables and short
// windows (kScatterSlots, kScatterWindow: fewer registers and less LDS, four
// wavefronts per SIMD); the explicit lists use longer windows, which make
// fewer records per segment.
//
// The tables sum in 64-bit fixed point: LDS integer atomics run several
// times faster than float ones on this chip.  Each term t = L y_j |d| is
// rounded to a multiple of 2^-50 2^e, 2^e the next power of two above the
// wavefront's largest |y_j| |d|, and at most 64 terms (one per ray of the
// wavefront) meet in a slot per window, so the integer sum stays below 2^56
// and is exact; the flush converts it back (or records it as it is).  Every
// term keeps an absolute error below 2^-51 2^e, far below a float32 rounding
// of the terms that matter.  Terms below 2^51 in magnitude are converted to
// integers with one float64 addition (round_to_i64).
constexpr int kScatterSlots = 384;
constexpr int kScatterWindow = 28;
constexpr int kListSlots = 768;
constexpr int kListWindow = 64;
constexpr int kLdsProbes = 8;
constexpr int kBlockWaves = 4;

template <int MODE>
struct TableShape {
  static constexpr int slots = MODE == kModeGatherFill ? kListSlots : kScatterSlots;
  static constexpr int window = MODE == kModeGatherFill ? kListWindow : kScatterWindow;
};

// Claims an empty slot (-1) for key `tet`; returns the key found there before.
__device__ __forceinline__ int lds_cas(lds_i32* p, int tet) {
  int expected = -1;
  __hip_atomic_compare_exchange_strong(p, &expected, tet, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WAVEFRONT);
  return expected;
}

// Multiplicative (Fibonacci) hash in 24 bits, since 24-bit multiplies run
// at full rate and 32-bit ones at a quarter: the low 24 bits of k A, A the
// golden-ratio fraction of 2^24, are the fractional part of k times 0.618,
// which spreads consecutive keys over the table; its top 20 bits are scaled
// to the table size.
template <int kSlots>
__device__ __forceinline__ unsigned table_home(int tet) {
  static_assert(kSlots < (1 << 12), "slot index times 2^20 must fit 32 bits");
  const unsigned h = __umul24((unsigned)tet & 0xFFFFFFu, 0x9E3779u);
  return (((h >> 4) & 0xFFFFFu) * (unsigned)kSlots) >> 20;
}

// x rounded to the nearest integer (ties to even), |x| < 2^51: in float64,
// x + 1.5 2^52 falls in [2^52, 2^53), where consecutive values are 1 apart,
// so the addition rounds x to an integer and the sum's bit pattern exceeds
// that of 1.5 2^52 (0x4338000000000000, low word zero) by exactly that
// integer.
__device__ __forceinline__ long long round_to_i64(float x) {
  const double y = (double)x + 0x1.8p52;
  const int hi = __double2hiint(y) - 0x43380000;
  const unsigned lo = (unsigned)__double2loint(y);
  return (long long)(((unsigned long long)(unsigned)hi << 32) | lo);
}

// Adds the fixed-point term m to the slot of `tet`; false when the
// tetrahedron finds no slot within kLdsProbes probes (the caller then adds
// the term elsewhere).  `slot` is the key's home slot and `claimed` what the
// compare-and-swap that claimed it for `tet` returned, issued when the ray
// entered the tetrahedron (a slot keeps its key until the window's flush):
// -1 or `tet` mean the home slot is the tetrahedron's.
template <int kSlots>
__device__ __forceinline__ bool lds_accumulate(lds_i32* keys, lds_i64* vals, int tet, long long m, unsigned slot,
                                               int claimed) {
  int k = claimed;
  if (k != -1 && k != tet) {
    // The first probe is written out: it settles nearly every displaced key,
    // and the loop's bookkeeping then only runs when it fails.
    slot = slot + 1 == (unsigned)kSlots ? 0u : slot + 1;
    k = lds_cas(keys + slot, tet);
    if (k != -1 && k != tet) {
#pragma unroll 1
      for (int p = 2; p < kLdsProbes; ++p) {
        slot = slot + 1 == (unsigned)kSlots ? 0u : slot + 1;
        k = lds_cas(keys + slot, tet);
        if (k == -1 || k == tet) break;
      }
      if (k != -1 && k != tet) return false;
    }
  }
  __hip_atomic_fetch_add(vals + slot, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
  return true;
}

// The record region of this workgroup: a multiplicative hash of the block
// index, so that every region gets a fair share of the detector's central
// (long-ray) and outer blocks whatever the tiling.
__device__ __forceinline__ unsigned gather_group() {
  static_assert(kGatherGroups == 64, "the region is the hash's top 6 bits");
  return ((unsigned)blockIdx.x * 2654435761u) >> 26;
}

// Record number p of this workgroup's region.
__device__ __forceinline__ void gather_record(const GatherOut& g, int64_t p, int tet, int scale, long long m) {
  if (p < g.gcap) g.rec[(int64_t)gather_group() * g.gcap + p] = GatherRecord{m, tet, scale};
  // Counted here, where the atomic's latency hides behind the walk (a
  // separate pass over the records took three times as long).
  atomicAdd(g.counts + tet, 1);
}

template <int MODE>
struct WalkOut {
  // FWD
  const float* x = nullptr;
  double acc = 0.0;
  // BWD / GATHER_FILL: weight = y_j * |d|; the table walks hold it times
  // lds_scale, so that a segment's fixed-point term is one product away
  float weight = 0.f;
  float* xhat = nullptr;
  lds_i32* lds_keys = nullptr;  // the wavefront's accumulation table (BWD)
  lds_i64* lds_vals = nullptr;
  float lds_scale = 1.f;  // fixed-point scale of the table (a power of two)
  unsigned long long* acc64 = nullptr;  // fixed-point result (reproducible mode), else null
  // GATHER_FILL: records of the explicit lists; key of the current window
  GatherOut gather{};
  int scale_exp = 0;  // log2 of lds_scale
  // TRACE output cursor
  int32_t* out_tet = nullptr;
  float* out_len = nullptr;
  int64_t cursor = 0;
  const int* perm = nullptr;
  // COUNT
  int64_t count = 0;
};

// Walk state between steps: the entry face as three vertex slots, the
// fourth vertex v, the current tetrahedron and the ray parameter where the
// ray entered it.  `loc` holds the local indices (0..3 within the current
// tetrahedron) of slots 0, 1, 2 and of v: in four 2-bit fields of one byte
// for the walks that remap it through the LDS table (loc_table), in four
// 4-bit fields for the bit-parallel remap of the others.
//
// Crossing face f (the face opposite local vertex f) into a neighbour whose
// opposite vertex has local index `back` there, the three shared vertices
// keep their order: local indices are sorted the same way in both elements,
// so a shared vertex of rank r among the face's vertices has local index
// r + (r >= back) in the neighbour, with r = p - (p > f).  walk_step applies
// this to all four fields at once.
struct WalkState {
  float3 a0, a1, a2, v;
  int tet;
  unsigned loc;
  double s_in;  // ray parameter where the ray entered the current tetrahedron
  float xcur;  // forward projection: x of the current tetrahedron
  int claim;   // table walks: old key returned by the claim of the tetrahedron's home slot
  unsigned home;  // table walks: that home slot, kept from the claim for the step's accumulation
  int steps;
  // Every ray of the wavefront ends beyond the mesh (ends_beyond_mesh), so
  // segments need no clamp at the end point; the same for the whole
  // wavefront, hence a scalar branch per step.
  bool far;
};

// Local-index remap as a table of loc_remap_entry (common.h), one byte per
// (loc, k, back), copied into each block's LDS by the walks that use it.
struct alignas(4) LocRemap {
  unsigned char v[kLocRemapEntries];
};

constexpr LocRemap make_loc_remap() {
  LocRemap t{};
  for (unsigned i = 0; i < (unsigned)kLocRemapEntries; ++i) t.v[i] = (unsigned char)loc_remap_entry(i);
  return t;
}

__constant__ LocRemap kLocRemap = make_loc_remap();

// The walks that look the remap up in LDS (a read per step in place of about
// fifteen vector instructions); the others keep the bit-parallel remap.
constexpr bool loc_table(int MODE) {
  return MODE == kModeForward || MODE == kModeBackAtomic || MODE == kModeBackFixed || MODE == kModeGatherFill;
}

__shared__ __align__(4) unsigned char s_loc_remap[kLocRemapEntries];

// Copies the remap table into the block's LDS; every thread of the block
// calls it before its first step.
__device__ __forceinline__ void load_loc_remap() {
  const unsigned* src = reinterpret_cast<const unsigned*>(kLocRemap.v);
  unsigned* dst = reinterpret_cast<unsigned*>(s_loc_remap);
  for (int i = threadIdx.x; i < kLocRemapEntries / 4; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
}

// Enter the mesh through boundary face `entry`.
template <int MODE, class Src>
__device__ __forceinline__ void walk_start(const MeshView& M, const Ray& r, const Src& q, int entry, WalkState& w,
                                           const WalkOut<MODE>& o, bool far) {
  w.far = far;
  const float4* bq = M.bfaces + 4 * (size_t)entry;
  float4 q0 = bq[0], q1 = bq[1], q2 = bq[2], q3 = bq[3];
  w.tet = __float_as_int(q0.w);
  unsigned lp = (unsigned)__float_as_int(q1.w);
  if constexpr (loc_table(MODE))
    w.loc = lp & 0xFFu;
  else
    w.loc = (lp & 3u) | ((lp & 12u) << 2) | ((lp & 48u) << 4) | ((lp & 192u) << 6);
  w.a0 = make_float3(q0.x, q0.y, q0.z);
  w.a1 = make_float3(q1.x, q1.y, q1.z);
  w.a2 = make_float3(q2.x, q2.y, q2.z);
  w.v = make_float3(q3.x, q3.y, q3.z);
  // Ray parameters are kept in float64 as s = t - 1/2 around the reference
  // point M.  Each step forms D = v - Q for the current entry point
  // Q = M + s_in d in float64 (offset_from_ray), so both the exit-face signs
  // and the crossing are evaluated from a vector of element size whose error
  // is a few ulps of itself, not of the source distance.  Each segment's
  // float32 length is added to s_in in float64, so the entry points do not
  // drift by a rounding of the parameter per step.
  const double s_in = crossing_s_fp64(q.S(), q.P(), w.a0, w.a1, w.a2);
  w.s_in = fmin(fmax(s_in, -0.5), 0.5);
  w.xcur = 0.f;
  if constexpr (MODE == kModeForward) w.xcur = o.x[w.tet];
  w.steps = 0;
}

// One step: leave the current tetrahedron, apply the mode's action for its
// segment, move to the neighbour.  Returns false once the ray has left the
// mesh (or the walk failed).  kLimit: the step bounds the walk itself (a ray
// never crosses more than nt elements); the windowed walks bound it once per
// window instead.
template <int MODE, bool kLimit = true, class Src, class St>
__device__ __forceinline__ bool walk_step(const MeshView& M, const Ray& r, const Src& q, WalkState& w,
                                          WalkOut<MODE>& o, St& st) {
  if (kLimit && w.steps > M.nt) {
    st.add_failed();
    st.steps += w.steps;
    return false;
  }
  const float3 v = w.v;
  StepEdges g;
  step_edges(r, w.s_in, v, w.a0, w.a1, w.a2, g);
  const float3 D = g.D, e0 = g.e0, e1 = g.e1, e2 = g.e2;
  // One bound from the longest edge settles all three signs in the common
  // case; otherwise each edge gets its own bound before any float64 work.
  int k = step_exit_common(g);
  if (k < 0) {
    int s0 = step_edge_certified(g.E0, g.m0, g.K);
    int s1 = step_edge_certified(g.E1, g.m1, g.K);
    int s2 = step_edge_certified(g.E2, g.m2, g.K);
    if (s0 == 0) s0 = resolve_src(q, v, w.a0, st);
    if (s1 == 0) s1 = resolve_src(q, v, w.a1, st);
    if (s2 == 0) s2 = resolve_src(q, v, w.a2, st);
    k = exit_slot(s0, s1, s2);
  }
  if (k == 3) {
    st.add_failed();
    st.steps += w.steps;
    return false;
  }
  w.steps++;
  // Next tetrahedron across the exit face (local face index loc[k]): the
  // record's load is issued as soon as the face is known, so that its
  // latency overlaps the crossing and the segment's accumulation.
  const int tet = w.tet;
  const unsigned sh = (loc_table(MODE) ? 2u : 4u) * (unsigned)k;
  unsigned f = (w.loc >> sh) & 3u;
  float4 rec = M.faces[(size_t)(((unsigned)tet << 2) | f)];
  const bool k0 = k == 0, k2 = k == 2;
  const float3 ei = make_float3(k2 ? e0.x : (k0 ? e1.x : e2.x), k2 ? e0.y : (k0 ? e1.y : e2.y),
                                k2 ? e0.z : (k0 ? e1.z : e2.z));
  const float3 ej = make_float3(k2 ? e1.x : (k0 ? e2.x : e0.x), k2 ? e1.y : (k0 ? e2.y : e0.y),
                                k2 ? e1.z : (k0 ? e2.z : e0.z));
  float3 n = f3cross(ei, ej);
  float den = f3dot(r.d, n);
  float dt;
  if (fabsf(den) > r.gd * fmaxf(fabsf(n.x), fmaxf(fabsf(n.y), fabsf(n.z)))) {
    dt = f3dot(D, n) * __builtin_amdgcn_rcpf(den);  // v_rcp_f32, about 1 ulp
  } else {
    st.add_grazing();
    const float3 ai = make_float3(k2 ? w.a0.x : (k0 ? w.a1.x : w.a2.x), k2 ? w.a0.y : (k0 ? w.a1.y : w.a2.y),
                                  k2 ? w.a0.z : (k0 ? w.a1.z : w.a2.z));
    const float3 aj = make_float3(k2 ? w.a1.x : (k0 ? w.a2.x : w.a0.x), k2 ? w.a1.y : (k0 ? w.a2.y : w.a0.y),
                                  k2 ? w.a1.z : (k0 ? w.a2.z : w.a0.z));
    dt = (float)(crossing_s_fp64(q.S(), q.P(), v, ai, aj) - w.s_in);
  }
  if (w.far)  // (1, the whole ray's parameter range, is an inline constant)
    dt = __builtin_amdgcn_fmed3f(dt, 0.0f, 1.0f);
  else
    dt = __builtin_amdgcn_fmed3f(dt, 0.0f, (float)fmax(0.5 - w.s_in, 0.0));
  if (dt == 0.f) st.add_zero();
  if constexpr (MODE == kModeForward) {
    o.acc = fma((double)dt, (double)w.xcur, o.acc);  // the product is exact
  } else if constexpr (MODE == kModeBackAtomic || MODE == kModeBackFixed || MODE == kModeGatherFill) {
    // Every segment goes into the table, a zero-length one as 0 (dt is never
    // negative or NaN after the clamp): adding zero costs less than a branch
    // per step, and the step's claim is then consumed on every path.
    const float v = dt * o.weight;  // in units of 2^-scale_exp
    const long long m = round_to_i64(v);
    if (!lds_accumulate<TableShape<MODE>::slots>(o.lds_keys, o.lds_vals, tet, m,
                                                 w.home, w.claim)) {
      if constexpr (MODE == kModeBackFixed) {
        atomicAdd(o.acc64 + tet, (unsigned long long)m);
      } else if constexpr (MODE == kModeGatherFill) {
        const int64_t p = (int64_t)atomicAdd(o.gather.cursor + gather_group(), 1ull);
        gather_record(o.gather, p, tet, o.scale_exp, m);
      } else {
        unsafeAtomicAdd(o.xhat + tet, ldexpf(v, -o.scale_exp));
      }
    }
  } else if constexpr (MODE == kModeBackDirect) {
    if (dt > 0.f) unsafeAtomicAdd(o.xhat + tet, dt * o.weight);
  } else if constexpr (MODE == kModeCountAll) {
    o.count++;
  } else if constexpr (MODE == kModeTrace) {
    o.out_tet[o.cursor] = o.perm[tet];
    o.out_len[o.cursor] = dt * r.dn;
    o.cursor++;
  }
  // What does not need the record is done while it is in flight: the entry
  // slots (slot k takes v), the ray parameter, and the first half of the
  // local-index remap: the table row (loc, k), or, bit-parallel, all four
  // index fields at once: adding 7 - f to a field sets its bit 3 exactly
  // when p > f, and adding 8 - back to the rank sets it exactly when r >=
  // back; the fields hold at most 10, so no carry crosses into the next.
  // (The field of slot k, whose vertex is not on the face, is replaced.)
  const unsigned L = w.loc;
  const unsigned R = loc_table(MODE) ? (L * 3u + (unsigned)k) * 4u
                                     : L - (((L + 0x7777u - f * 0x1111u) >> 3) & 0x1111u);
  w.a0 = make_float3(k == 0 ? v.x : w.a0.x, k == 0 ? v.y : w.a0.y, k == 0 ? v.z : w.a0.z);
  w.a1 = make_float3(k == 1 ? v.x : w.a1.x, k == 1 ? v.y : w.a1.y, k == 1 ? v.z : w.a1.z);
  w.a2 = make_float3(k == 2 ? v.x : w.a2.x, k == 2 ? v.y : w.a2.y, k == 2 ? v.z : w.a2.z);
  w.s_in += (double)dt;  // float64: no rounding drift along the ray
  unsigned Rk = R;
  // (An empty statement that takes these values, so the compiler computes
  // them here rather than sinking them behind the wait for the record.)
  asm volatile("" : "+v"(w.a0.x), "+v"(w.a0.y), "+v"(w.a0.z), "+v"(w.a1.x), "+v"(w.a1.y), "+v"(w.a1.z),
               "+v"(w.a2.x), "+v"(w.a2.y), "+v"(w.a2.z), "+v"(w.s_in), "+v"(Rk));
  // Keep the record one 16-byte load consumed here; otherwise the compiler
  // splits it into four loads sunk into the next step, which serialises the
  // dependent fetch behind the next step's arithmetic.
  asm volatile("" : "+v"(rec.x), "+v"(rec.y), "+v"(rec.z), "+v"(rec.w));
  int packed = __float_as_int(rec.x);
  if (packed < 0) {
    st.steps += w.steps;
    return false;
  }
  unsigned back = (unsigned)packed & 3u;
  if constexpr (loc_table(MODE)) {
    // Read back while the next step computes; needed at its exit face.
    w.loc = s_loc_remap[Rk + back];
  } else {
    const unsigned N = Rk + (((Rk + 0x8888u - back * 0x1111u) >> 3) & 0x1111u);
    // Slot k takes v's new index; the neighbour's opposite vertex is `back`.
    const unsigned fieldk = 0xFu << sh;
    w.loc = (((N & 0xFFFu) & ~fieldk) | ((N >> 12) << sh)) | (back << 12);
  }
  w.v = xyz(rec);
  w.tet = packed >> 2;
  // Table walks claim the new tetrahedron's home slot now; the old key comes
  // back while the next step computes, and is needed only at its end.
  if constexpr (MODE == kModeBackAtomic || MODE == kModeBackFixed || MODE == kModeGatherFill) {
    w.home = table_home<TableShape<MODE>::slots>(w.tet);
    w.claim = lds_cas(o.lds_keys + w.home, w.tet);
  }
  if constexpr (MODE == kModeForward) w.xcur = o.x[w.tet];
  return true;
}

// Walk one ray from boundary face `entry` to the boundary.
template <int MODE, class Src, class St>
__device__ __forceinline__ void walk_ray(const MeshView& M, const Ray& r, const Src& q, int entry, WalkOut<MODE>& o,
                                         St& st) {
  WalkState w;
  // Called by the lanes that walk: the vote is over them.
  walk_start<MODE>(M, r, q, entry, w, o, __all(ends_beyond_mesh(r, M.extent)) != 0);
  while (walk_step<MODE>(M, r, q, w, o, st)) {
  }
}

// Adds a wavefront's counts to the mesh's counters: a shuffle reduction of
// the lane registers, or (LdsStats) every lane's ray and step counts added to
// the wavefront's LDS counters; then one lane per counter adds it to global
// memory.
__device__ __forceinline__ void flush_stats(const MeshView& M, RegStats& st, int active) {
  int v[8] = {active, st.steps, st.zero, st.fp64, st.exact, st.pert, st.failed, st.grazing};
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    int x = v[c];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    v[c] = x;
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (v[c]) atomicAdd(M.counters + c, (unsigned long long)v[c]);
  }
}

__device__ __forceinline__ void flush_stats(const MeshView& M, LdsStats& st, int active) {
  if (active) lds_add_u32(st.ev + kEvRays, 1u);
  if (st.steps) lds_add_u32(st.ev + kEvSteps, (unsigned)st.steps);
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const int lane = threadIdx.x & 63;
  if (lane < kEvents) {
    const unsigned v = st.ev[lane];
    const int slot = lane == kEvRays ? kRays : lane == kEvSteps ? kSegments : kZeroLen + lane;
    if (v) atomicAdd(M.counters + slot, (unsigned long long)v);
  }
}

// Pixel blocks: a 256-thread block is four wavefronts arranged 2 x 2, each
// covering a tile of tu x tv = 64 pixels of one angle (8 x 8 by default), so a
// block covers (2 tu) x (2 tv) pixels.
struct TileMap {
  int nbu, nbv;  // blocks along u and v
  int tu, tv;    // wave tile
};

__device__ __forceinline__ bool tile_ray(const GeomView& g, const TileMap& tm, int64_t block, int tid, int a0,
                                         int na_chunk, int* a, int* i, int* j) {
  int64_t per_angle = (int64_t)tm.nbu * tm.nbv;
  int64_t aa = block / per_angle;
  int64_t rem = block - aa * per_angle;
  int bv = (int)(rem / tm.nbu), bu = (int)(rem - (int64_t)bv * tm.nbu);
  int wave = tid >> 6, lane = tid & 63;
  *a = a0 + (int)aa;
  *i = bu * 2 * tm.tu + (wave & 1) * tm.tu + lane % tm.tu;
  *j = bv * 2 * tm.tv + (wave >> 1) * tm.tv + lane / tm.tu;
  return aa < na_chunk && *i < g.nu && *j < g.nv;
}

// Inputs and outputs of one pixel-block walk (which fields are used depends on the mode).
struct BlockIO {
  const int32_t* entry;
  const float* in;
  float* out_f32;
  int32_t* out_i32;
  GatherOut gather;  // kModeGatherFill
  int lds_table;
  unsigned long long* acc64;  // kModeBackFixed: fixed-point sums [nt]
  const int* scale_exp;       // kModeBackFixed: log2 of their scale
};

// Walk the rays of pixel block `block` (of angles [a0, a0 + na_chunk)).
//   kModeEntry:      out_i32[rid] = entry face (or -1)
//   kModeEntryRstar: the same, searched through the R*-tree
//   kModeForward:    out_f32[rid] = sum_i a_ij x_i
//   kModeBackAtomic: xhat[i] += a_ij y_j through the block's LDS table
//   kModeBackFixed:  acc64[i] += a_ij y_j 2^scale_exp, exact integer sums
//   kModeBackDirect: xhat[i] += a_ij y_j, one global atomic per segment
//   kModeGatherFill: records of the explicit per-tetrahedron lists
// Every thread of the block must call it.
// kCached: every ray's entry face comes from io.entry (the launch has an
// entry cache), so the kernel carries no tree search.
template <int MODE, bool kLeanSrc = false, bool kCached = false>
__device__ __forceinline__ void walk_block(const MeshView& M, const GeomView& G, const TileMap& tm, int64_t block,
                                           int a0, int na_chunk, const BlockIO& io, int* tkeys,
                                           long long* tvals) {
  int a, i, j;
  bool active = tile_ray(G, tm, block, threadIdx.x, a0, na_chunk, &a, &i, &j);
  // The scatter walks keep their rare counts in LDS, the others in registers.
  constexpr bool kTable = MODE == kModeBackAtomic || MODE == kModeBackFixed || MODE == kModeGatherFill;
  using St = typename std::conditional<kTable, LdsStats, RegStats>::type;
  __shared__ unsigned s_ev[kTable ? kBlockWaves * kEvents : 1];
  St st(kTable ? wave_counters(s_ev) : nullptr);
  if constexpr (kTable) {
    const int lane = threadIdx.x & 63;
    constexpr int kSlots = TableShape<MODE>::slots, kWindow = TableShape<MODE>::window;
    lds_i32* keys = (lds_i32*)tkeys + kSlots * wave_in_block();
    lds_i64* vals = (lds_i64*)tvals + kSlots * wave_in_block();
    for (int k = lane; k < kSlots; k += 64) {
      keys[k] = -1;
      vals[k] = 0;
    }
    Ray r;
    PixelSrc q{};
    WalkOut<MODE> o;
    o.xhat = io.out_f32;
    o.lds_keys = keys;
    o.lds_vals = vals;
    WalkState w;
    bool alive = false;
    bool ends_far = true;
    if (active) {
      int64_t rid = ((int64_t)a * G.nv + j) * G.nu + i;
      r = cone_ray(G, M.extent, a, i, j);
      q = pixel_src(G, a, i, j);
      ends_far = ends_beyond_mesh(r, M.extent);
      int e;
      if constexpr (kCached)
        e = io.entry[rid];
      else
        e = io.entry ? io.entry[rid] : find_entry(M, r, st);
      o.weight = io.in[rid] * r.dn;
      if (e >= 0 && o.weight != 0.f) {
        walk_start<MODE>(M, r, q, e, w, o, false);
        alive = true;
      }
    }
    w.far = __all(ends_far) != 0;
    if constexpr (MODE == kModeBackFixed) {
      // One scale for the whole launch, so that every sum is an exact
      // integer whatever the order of the additions.
      o.scale_exp = *io.scale_exp;
      o.lds_scale = ldexpf(1.0f, o.scale_exp);
      o.acc64 = io.acc64;
    } else {
      if constexpr (MODE == kModeGatherFill) o.gather = io.gather;
      // Fixed-point scale from the wavefront's largest ray weight (a max over
      // the float bits, which order like the values for non-negative floats).
      __shared__ unsigned s_wmax[kBlockWaves];
      lds_u32* wm = (lds_u32*)s_wmax + wave_in_block();
      if (lane == 0) *wm = 0u;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (alive)
        __hip_atomic_fetch_max(wm, __float_as_uint(fabsf(o.weight)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      int ex = 0;
      (void)frexpf(__uint_as_float(*wm), &ex);
      o.scale_exp = min(50 - ex, 120);
      o.lds_scale = ldexpf(1.0f, o.scale_exp);
    }
    o.weight *= o.lds_scale;  // a power of two: exact
    // The wavefront's rays start together and every live one takes one step
    // per iteration, so all of them have taken `taken` steps at a window's
    // start: the step bound is checked there, once per window.
    int taken = 0;
    // The wavefront's rays advance together in windows of kWindow
    // steps; after each window its table is added to xhat and cleared, so it
    // only ever holds the tetrahedra of one window of the ray bundle.
    for (;;) {
      // Each step claims the slot of the tetrahedron it enters (walk_step);
      // the flush has cleared the table, so the current ones claim again.
      if (alive) {
        w.home = table_home<kSlots>(w.tet);
        w.claim = lds_cas(keys + w.home, w.tet);
      }
      if (taken > M.nt && alive) {
        st.add_failed();
        st.steps += w.steps;
        alive = false;
      }
#pragma unroll 1
      for (int k = 0; k < kWindow && alive; ++k) alive = walk_step<MODE, false>(M, r, q, w, o, st);
      taken += kWindow;
      // LDS operations of one wavefront complete in order: the flush sees
      // every add of the window.
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if constexpr (MODE == kModeGatherFill) {
        // One record per occupied slot, at consecutive positions reserved
        // with one atomic for the wavefront.  (Slots claimed ahead by a
        // window's last step hold zero and are only cleared.)
        unsigned total = 0;
        for (int k = lane; k < kSlots; k += 64) total += __popcll(__ballot(keys[k] >= 0 && vals[k] != 0));
        unsigned long long base = 0;
        if (lane == 0 && total)
          base = atomicAdd(o.gather.cursor + gather_group(), (unsigned long long)total);
        base = ((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(base >> 32)) << 32) |
               (unsigned)__builtin_amdgcn_readfirstlane((int)base);
        for (int k = lane; k < kSlots; k += 64) {
          const int key = keys[k];
          const long long v = vals[k];
          const unsigned long long m = __ballot(key >= 0 && v != 0);
          if (key >= 0) {
            if (v != 0) {
              const int64_t p = (int64_t)base + __popcll(m & ((1ull << lane) - 1ull));
              gather_record(o.gather, p, key, o.scale_exp, v);
            }
            keys[k] = -1;
            vals[k] = 0;
          }
          base += __popcll(m);
        }
      } else {
        for (int k = lane; k < kSlots; k += 64) {
          const int key = keys[k];
          if (key >= 0) {
            const long long v = vals[k];
            if (v != 0) {
              if constexpr (MODE == kModeBackFixed)
                atomicAdd(io.acc64 + key, (unsigned long long)v);
              else
                unsafeAtomicAdd(io.out_f32 + key, (float)ldexp((double)v, -o.scale_exp));
            }
            keys[k] = -1;
            vals[k] = 0;
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (__ballot(alive) == 0) break;
    }
  } else if (active) {
    int64_t rid = ((int64_t)a * G.nv + j) * G.nu + i;
    Ray r = cone_ray(G, M.extent, a, i, j);
    // The single-problem walks have registers to spare, so their exact paths
    // read the ray from registers; the batched ones (and the windowed
    // backprojection) re-read it from the frame.
    using Src = typename std::conditional<kLeanSrc, PixelSrc, RegSrc>::type;
    Src q;
    if constexpr (kLeanSrc)
      q = pixel_src(G, a, i, j);
    else
      q = RegSrc{r.S, r.P, r.U, r.V};
    int e;
    if constexpr (MODE == kModeEntryRstar)
      e = find_entry<true>(M, r, st);
    else if constexpr (kCached && MODE != kModeEntry)
      e = io.entry[rid];
    else
      e = (io.entry && MODE != kModeEntry) ? io.entry[rid] : find_entry(M, r, st);
    if constexpr (MODE == kModeEntry || MODE == kModeEntryRstar) {
      io.out_i32[rid] = e;
    } else if constexpr (MODE == kModeForward) {
      WalkOut<MODE> o;
      o.x = io.in;
      if (e >= 0) walk_ray<MODE>(M, r, q, e, o, st);
      io.out_f32[rid] = (float)(o.acc * (double)r.dn);
    } else if constexpr (MODE == kModeBackDirect) {
      WalkOut<MODE> o;
      o.xhat = io.out_f32;
      o.weight = io.in[rid] * r.dn;
      if (e >= 0 && o.weight != 0.f) walk_ray<MODE>(M, r, q, e, o, st);
    }
  }
  flush_stats(M, st, active ? 1 : 0);
}

}  // namespace

// ---------------------------------------------------------------- kernels

template <int MODE, bool kCached>
__global__ __launch_bounds__(256, 4) void pixel_walk_kernel(MeshView M, GeomView G, TileMap tm, int a0, int na_chunk,
                                                         BlockIO io) {
  if constexpr (loc_table(MODE)) load_loc_remap();
  if constexpr (MODE == kModeBackAtomic || MODE == kModeBackFixed || MODE == kModeGatherFill) {
    __shared__ int tkeys[kBlockWaves * TableShape<MODE>::slots];
    __shared__ long long tvals[kBlockWaves * TableShape<MODE>::slots];
    walk_block<MODE, false, kCached>(M, G, tm, xcd_block(blockIdx.x, gridDim.x), a0, na_chunk, io, tkeys, tvals);
  } else {
    walk_block<MODE, false, kCached>(M, G, tm, xcd_block(blockIdx.x, gridDim.x), a0, na_chunk, io, nullptr,
                                     nullptr);
  }
}

// Entry faces by projecting the boundary (an alternative to the tree
// searches that gives the same faces).  For one angle, the rays are the lines
// from the source S through the pixel points; a boundary face can only be
// entered by them when S lies on the outer side of its plane.  Such a face is
// projected centrally onto the detector plane in float64, and the pixels
// whose abscissa and ordinate fall inside the bounding box of the projection,
// widened by a twentieth of the pitch, are tested with the exact entry test
// of the tree searches on their own float32 rays.  The widening covers the
// rounding of the pixel points (about 1e-4 of the pitch), so every pixel
// whose ray enters through the face is tested; a convex mesh is entered
// through exactly one face per ray, so each pixel is written at most once
// and the result equals the tree searches'.  Faces whose plane nearly
// contains S, and vertices at or behind S's plane parallel to the detector,
// fall back to testing the whole detector for that face.
//
// A wavefront takes 64 boundary faces of one angle: each lane classifies one
// face, then the wavefront walks the candidate faces one by one with a lane
// per pixel of the face's box.  When faces and angles are too few to fill
// the chip (coarse meshes, single projections), gridDim.z wavefronts share
// each face's box, taking interleaved runs of 64 pixels.
constexpr int kRasterWaves = 4;

__device__ __forceinline__ void raster_box(const GeomView& G, const float* f, float3 a0, float3 a1, float3 a2,
                                           int* i0, int* i1, int* j0, int* j1) {
  const double Sx = f[0], Sy = f[1], Sz = f[2], Cx = f[3], Cy = f[4], Cz = f[5];
  const double Ux = f[6], Uy = f[7], Uz = f[8], Vx = f[9], Vy = f[10], Vz = f[11];
  // Outward normal of the face and the side of its plane S is on.
  const double e1x = (double)a1.x - a0.x, e1y = (double)a1.y - a0.y, e1z = (double)a1.z - a0.z;
  const double e2x = (double)a2.x - a0.x, e2y = (double)a2.y - a0.y, e2z = (double)a2.z - a0.z;
  const double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
  const double wx = (double)a0.x - Sx, wy = (double)a0.y - Sy, wz = (double)a0.z - Sz;
  const double side = wx * nx + wy * ny + wz * nz;
  const double scale = sqrt((wx * wx + wy * wy + wz * wz) * (nx * nx + ny * ny + nz * nz));
  *i0 = 0;
  *i1 = -1;
  *j0 = 0;
  *j1 = -1;
  if (side > 1e-9 * scale) return;  // S on the inner side: no ray enters here
  const int nu = G.nu, nv = G.nv;
  bool whole = !(side < -1e-9 * scale);
  // Detector plane normal and the source's distance to that plane.
  const double Nx = Uy * Vz - Uz * Vy, Ny = Uz * Vx - Ux * Vz, Nz = Ux * Vy - Uy * Vx;
  const double cs = (Cx - Sx) * Nx + (Cy - Sy) * Ny + (Cz - Sz) * Nz;
  const double uu = Ux * Ux + Uy * Uy + Uz * Uz, vv = Vx * Vx + Vy * Vy + Vz * Vz;
  double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
  const float3 pts[3] = {a0, a1, a2};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double px = (double)pts[k].x - Sx, py = (double)pts[k].y - Sy, pz = (double)pts[k].z - Sz;
    const double den = px * Nx + py * Ny + pz * Nz;
    if (!(den * cs > 0.0) || !(fabs(den) > 1e-9 * fabs(cs))) whole = true;
    const double lam = cs / den;
    const double xx = Sx + lam * px - Cx, xy = Sy + lam * py - Cy, xz = Sz + lam * pz - Cz;
    const double u = (xx * Ux + xy * Uy + xz * Uz) / uu, v = (xx * Vx + xy * Vy + xz * Vz) / vv;
    umin = fmin(umin, u);
    umax = fmax(umax, u);
    vmin = fmin(vmin, v);
    vmax = fmax(vmax, v);
  }
  if (whole) {
    *i0 = 0;
    *i1 = nu - 1;
    *j0 = 0;
    *j1 = nv - 1;
    return;
  }
  // Pixel abscissae are affine in the index up to float rounding.
  const double u0 = G.ut[0], du = nu > 1 ? ((double)G.ut[nu - 1] - u0) / (nu - 1) : 1.0;
  const double v0 = G.vt[0], dv = nv > 1 ? ((double)G.vt[nv - 1] - v0) / (nv - 1) : 1.0;
  double ia = (umin - u0) / du, ib = (umax - u0) / du, ja = (vmin - v0) / dv, jb = (vmax - v0) / dv;
  if (ia > ib) {
    const double t = ia;
    ia = ib;
    ib = t;
  }
  if (ja > jb) {
    const double t = ja;
    ja = jb;
    jb = t;
  }
  // Clamped in double before the conversion, so far-off boxes stay empty.
  *i0 = (int)fmin((double)nu, fmax(0.0, ceil(ia - 0.05)));
  *i1 = (int)fmax(-1.0, fmin((double)(nu - 1), floor(ib + 0.05)));
  *j0 = (int)fmin((double)nv, fmax(0.0, ceil(ja - 0.05)));
  *j1 = (int)fmax(-1.0, fmin((double)(nv - 1), floor(jb + 0.05)));
}

__global__ __launch_bounds__(64 * kRasterWaves) void entry_raster_kernel(MeshView M, GeomView G, int a0,
                                                                         int32_t* entry) {
  const int lane = threadIdx.x & 63;
  const int group = blockIdx.x * kRasterWaves + (threadIdx.x >> 6);
  const int a = a0 + (int)blockIdx.y;
  const float* f = G.frame + 12 * (size_t)a;
  const int b = group * 64 + lane;
  int i0 = 0, i1 = -1, j0 = 0, j1 = -1;
  if (b < M.nb) {
    const float4* q = M.bfaces + 4 * (size_t)b;
    const float4 q0 = q[0], q1 = q[1], q2 = q[2];
    raster_box(G, f, make_float3(q0.x, q0.y, q0.z), make_float3(q1.x, q1.y, q1.z), make_float3(q2.x, q2.y, q2.z),
               &i0, &i1, &j0, &j1);
  }
  RegStats st(nullptr);
  unsigned long long todo = __ballot(i0 <= i1 && j0 <= j1);
  while (todo) {
    const int src = __ffsll((long long)todo) - 1;
    todo &= todo - 1;
    const int fb = __shfl(b, src, 64), fi0 = __shfl(i0, src, 64), fi1 = __shfl(i1, src, 64);
    const int fj0 = __shfl(j0, src, 64), fj1 = __shfl(j1, src, 64);
    const int w = fi1 - fi0 + 1;
    const int64_t n = (int64_t)w * (fj1 - fj0 + 1);
    const int z = (int)blockIdx.z, nz = (int)gridDim.z;
    if (n < 0x7fff0000) {  // 32-bit indices (k + 64 gridDim.z cannot overflow) unless the box is huge
      for (int k = lane + 64 * z; k < (int)n; k += 64 * nz) {
        const int row = k / w;
        const int i = fi0 + (k - row * w), j = fj0 + row;
        const Ray r = cone_ray(G, M.extent, a, i, j);
        if (enters_face(M, r, fb, st)) entry[((int64_t)a * G.nv + j) * G.nu + i] = fb;
      }
    } else {
      for (int64_t k = lane + 64 * z; k < n; k += 64 * nz) {
        const int64_t row = k / w;
        const int i = fi0 + (int)(k - row * w), j = fj0 + (int)row;
        const Ray r = cone_ray(G, M.extent, a, i, j);
        if (enters_face(M, r, fb, st)) entry[((int64_t)a * G.nv + j) * G.nu + i] = fb;
      }
    }
  }
  flush_stats(M, st, 0);
}

// Batched problems: one persistent launch pulls pixel blocks of every
// problem from device work lists.  Problems are listed most expensive block
// first, so long walks start early and short ones fill the tail.  As in the
// single-problem launches (xcd_block), each problem's blocks are split into
// kXcds contiguous runs, one per die: list x holds run x of every problem in
// problem order, and a workgroup takes from the list of its own die (block
// b runs on die b mod kXcds) until that list is empty, then from the others.
struct BatchDesc {
  MeshView M;
  GeomView G;
  TileMap tm;
  int64_t items;  // pixel blocks of this problem
  const int32_t* entry;
  int user;  // index of the problem in the caller's lists
  int lds_table;
};

// Run x of a problem of n blocks: first block and length (as xcd_block).
__host__ __device__ __forceinline__ int64_t xcd_run_begin(int64_t n, int x) {
  const int64_t per = n / kXcds, rem = n % kXcds;
  return x * per + (x < rem ? x : rem);
}
__host__ __device__ __forceinline__ int64_t xcd_run_length(int64_t n, int x) {
  return n / kXcds + (x < n % kXcds ? 1 : 0);
}

template <int MODE>
__global__ __launch_bounds__(256, 4) void batch_walk_kernel(const BatchDesc* __restrict__ D, int nprob,
                                                         const int64_t* __restrict__ lists,
                                                         unsigned long long* counters, int chunk,
                                                         const float* const* __restrict__ ins,
                                                         float* const* __restrict__ outs) {
  // lists[x (nprob + 1) + p]: position of problem p's run in list x (its
  // last entry is the list's length); counters[x]: next free position.
  // Thread 0 fetches `chunk` positions at a time and resolves each to a
  // (problem, pixel block) for the whole block; its state lives in LDS so
  // that nothing of the queue stays live in registers during the walk.
  if constexpr (loc_table(MODE)) load_loc_remap();
  __shared__ long long s_k, s_end, s_block;
  __shared__ int s_list, s_prob;
  const int home = (int)(blockIdx.x % kXcds);
  if (threadIdx.x == 0) {
    s_k = 0;
    s_end = 0;
    s_list = home;
  }
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) {
      long long k = s_k, end = s_end;
      int x = s_list;
      if (k >= end) {
        k = -1;
        for (int g = 0; g < kXcds; ++g) {
          const int y = (home + g) % kXcds;
          const long long len = lists[y * (nprob + 1) + nprob];
          const long long c = (long long)atomicAdd(counters + y, (unsigned long long)chunk);
          if (c < len) {
            k = c;
            end = c + chunk < len ? c + chunk : len;
            x = y;
            break;
          }
        }
      }
      if (k < 0) {
        s_prob = -1;
      } else {
        // The problem whose run holds position k: the last p with
        // pos[p] <= k (runs may be empty, so several p share a position).
        const int64_t* pos = lists + x * (nprob + 1);
        int lo = 0, hi = nprob - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (pos[mid] <= k)
            lo = mid;
          else
            hi = mid - 1;
        }
        s_prob = lo;
        s_block = xcd_run_begin(D[lo].items, x) + (k - pos[lo]);
        s_k = k + 1;
        s_end = end;
        s_list = x;
      }
    }
    __syncthreads();
    // The same for the whole block; saying so lets the descriptor below be
    // read with scalar loads into scalar registers, as kernel arguments are
    // in the single-problem kernel.
    const int p = __builtin_amdgcn_readfirstlane(s_prob);
    if (p < 0) break;
    const long long raw = s_block;
    const long long block = (long long)(((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(raw >> 32))
                                         << 32) |
                                        (unsigned)__builtin_amdgcn_readfirstlane((int)raw));
    // A reference into the constant address space: the descriptor's fields
    // are invariant, so the compiler may reload them with scalar loads
    // instead of spilling them around the walk (which it did with a copy).
    // (The host pass, which only checks the kernel, has no such space.)
#if defined(__HIP_DEVICE_COMPILE__)
    typedef __attribute__((address_space(4))) const BatchDesc cdesc;
#else
    typedef const BatchDesc cdesc;
#endif
    cdesc& d = ((cdesc*)D)[p];
    BlockIO io{};
    io.entry = d.entry;
    io.in = ins[d.user];
    io.out_f32 = outs[d.user];
    io.lds_table = d.lds_table;
    if constexpr (MODE == kModeBackAtomic) {
      __shared__ int tkeys[kBlockWaves * TableShape<MODE>::slots];
      __shared__ long long tvals[kBlockWaves * TableShape<MODE>::slots];
      walk_block<MODE, true, true>(d.M, d.G, d.tm, block, 0, d.G.na, io, tkeys, tvals);
    } else {
      walk_block<MODE, true, true>(d.M, d.G, d.tm, block, 0, d.G.na, io, nullptr, nullptr);
    }
  }
}

__global__ void reset_counters_kernel(unsigned long long* c, int n) {
  if ((int)threadIdx.x < n) c[threadIdx.x] = 0ull;
}

// Listed rays (trace): either pixel ray ids, or explicit S/P/U/V arrays.
template <int MODE>
__global__ __launch_bounds__(256) void list_walk_kernel(MeshView M, GeomView G, const int64_t* ids, const float* S,
                                                        const float* P, const float* U, const float* V, int32_t n,
                                                        int64_t* counts, const int64_t* offsets, int32_t* tets,
                                                        float* lens) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  RegStats st(nullptr);
  bool active = k < n;
  if (active) {
    Ray r;
    if (ids) {
      int64_t rid = ids[k];
      int i = (int)(rid % G.nu);
      int j = (int)((rid / G.nu) % G.nv);
      int a = (int)(rid / ((int64_t)G.nu * G.nv));
      r = cone_ray(G, M.extent, a, i, j);
    } else {
      r.S = make_float3(S[3 * k], S[3 * k + 1], S[3 * k + 2]);
      r.P = make_float3(P[3 * k], P[3 * k + 1], P[3 * k + 2]);
      r.U = make_float3(U[3 * k], U[3 * k + 1], U[3 * k + 2]);
      r.V = make_float3(V[3 * k], V[3 * k + 1], V[3 * k + 2]);
      finish_ray(r, M.extent);
    }
    // {P - S, U, V} must be a basis for the tie-breaking translation.
    float s3[3] = {r.S.x, r.S.y, r.S.z}, p3[3] = {r.P.x, r.P.y, r.P.z}, u3[3] = {r.U.x, r.U.y, r.U.z},
          v3[3] = {r.V.x, r.V.y, r.V.z};
    bool basis = det_diff_sign(p3, s3, u3, nullptr, v3, nullptr, nullptr) != 0;
    int e = basis ? find_entry(M, r, st) : -1;
    if (!basis) st.add_failed();
    const RegSrc q{r.S, r.P, r.U, r.V};
    WalkOut<MODE> o;
    if constexpr (MODE == kModeTrace) {
      o.out_tet = tets;
      o.out_len = lens;
      o.perm = M.perm;
      o.cursor = offsets[k];
    }
    if (e >= 0) walk_ray<MODE>(M, r, q, e, o, st);
    if constexpr (MODE == kModeCountAll) counts[k] = o.count;
  }
  flush_stats(M, st, active ? 1 : 0);
}

// Reproducible scatter: the largest |y_j| of the launch (as float bits,
// which order like the values for non-negative floats), the scale exponent
// derived from it, the zeroed integer sums and their conversion at the end.
__global__ void max_abs_kernel(const float* y, int64_t n, unsigned* out) {
  float m = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, fabsf(y[i]));
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

__global__ void fixed_scale_kernel(const unsigned* max_bits, float max_dlen, int K, int* exp_out) {
  const float w = __uint_as_float(*max_bits) * max_dlen;
  int e = 0;
  if (w > 0.f && w < INFINITY) (void)frexpf(w, &e);
  *exp_out = min(max(K - e, -120), 120);
}

__global__ void zero_u64_kernel(unsigned long long* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

__global__ void fixed_finish_kernel(const unsigned long long* acc, const int* scale_exp, float* xhat, int n,
                                    int accumulate) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = ldexp((double)(long long)acc[i], -*scale_exp);
  xhat[i] = accumulate ? (float)((double)xhat[i] + v) : (float)v;
}

__global__ void fill_f32_kernel(float* p, int64_t n, float v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void permute_kernel(const float* in, float* out, const int32_t* perm, int n, int scatter) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (scatter)
    out[perm[i]] = in[i];
  else
    out[i] = in[perm[i]];
}

// ---------------------------------------------------------------- launchers

static TileMap make_tiles(const GeomView& g, int tile_u) {
  TileMap t;
  if (tile_u != 4 && tile_u != 8 && tile_u != 16 && tile_u != 32 && tile_u != 64) tile_u = 8;
  t.tu = tile_u;
  t.tv = 64 / tile_u;
  t.nbu = (g.nu + 2 * t.tu - 1) / (2 * t.tu);
  t.nbv = (g.nv + 2 * t.tv - 1) / (2 * t.tv);
  return t;
}

int64_t pixel_walk_waves(const tct_geom* g, int na_chunk, int tile_u) {
  const TileMap tm = make_tiles(g->view(), tile_u);
  return (int64_t)tm.nbu * tm.nbv * na_chunk * 4;
}

tct_status launch_pixel_walk(int mode, const tct_mesh* m, const tct_geom* g, int a0, int na_chunk,
                             const int32_t* entry, const float* in, float* out_f32, int32_t* out_i32,
                             const GatherOut* gather, int tile_u, hipStream_t s, int lds_table,
                             unsigned long long* acc64, const int* scale_exp) {
  MeshView M = m->view();
  GeomView G = g->view();
  TileMap tm = make_tiles(G, tile_u);
  int64_t blocks = (int64_t)tm.nbu * tm.nbv * na_chunk;
  if (blocks <= 0) return TCT_OK;
  if (blocks > 0x7fffffff) {
    set_error("too many rays in one launch");
    return TCT_E_ARG;
  }
  BlockIO io{entry, in, out_f32, out_i32, gather ? *gather : GatherOut{}, lds_table, acc64, scale_exp};
  dim3 grid((unsigned)blocks), block(256);
#define TCT_LAUNCH(MODE_)                                                                              \
  do {                                                                                                 \
    if (entry)                                                                                         \
      hipLaunchKernelGGL((pixel_walk_kernel<MODE_, true>), grid, block, 0, s, M, G, tm, a0, na_chunk, io);  \
    else                                                                                               \
      hipLaunchKernelGGL((pixel_walk_kernel<MODE_, false>), grid, block, 0, s, M, G, tm, a0, na_chunk, io); \
  } while (0)
  switch (mode) {
    case kModeEntry:
      hipLaunchKernelGGL((pixel_walk_kernel<kModeEntry, false>), grid, block, 0, s, M, G, tm, a0, na_chunk, io);
      break;
    case kModeEntryRstar:
      hipLaunchKernelGGL((pixel_walk_kernel<kModeEntryRstar, false>), grid, block, 0, s, M, G, tm, a0, na_chunk, io);
      break;
    case kModeForward:
      TCT_LAUNCH(kModeForward);
      break;
    case kModeBackAtomic:
      if (lds_table)
        TCT_LAUNCH(kModeBackAtomic);
      else
        TCT_LAUNCH(kModeBackDirect);
      break;
    case kModeBackFixed:
      TCT_LAUNCH(kModeBackFixed);
      break;
    case kModeGatherFill:
      TCT_LAUNCH(kModeGatherFill);
      break;
    default:
      set_error("bad walk mode");
      return TCT_E_ARG;
  }
#undef TCT_LAUNCH
  TCT_HIP(hipGetLastError());
  return TCT_OK;
}

tct_status launch_list_walk(int mode, const tct_mesh* m, const tct_geom* g, const int64_t* ids, const float* S,
                            const float* P, const float* U, const float* V, int32_t n, int64_t* counts,
                            const int64_t* offsets, int32_t* tets, float* lens, hipStream_t s) {
  if (n <= 0) return TCT_OK;
  MeshView M = m->view();
  GeomView G{};
  if (g) G = g->view();
  dim3 grid((n + 255) / 256), block(256);
  if (mode == kModeCountAll)
    hipLaunchKernelGGL(list_walk_kernel<kModeCountAll>, grid, block, 0, s, M, G, ids, S, P, U, V, n, counts, offsets,
                       tets, lens);
  else
    hipLaunchKernelGGL(list_walk_kernel<kModeTrace>, grid, block, 0, s, M, G, ids, S, P, U, V, n, counts, offsets,
                       tets, lens);
  TCT_HIP(hipGetLastError());
  return TCT_OK;
}

tct_status launch_fill(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return TCT_OK;
  hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  TCT_HIP(hipGetLastError());
  return TCT_OK;
}

tct_status backproject_atomic(const tct_mesh* m, const tct_geom* g, const float* proj, float* xhat, int accumulate,
                              const int32_t* entry, int tile_u, int lds_table, hipStream_t s) {
  if (!accumulate) {
    tct_status st = launch_fill(xhat, m->nt, 0.f, s);
    if (st != TCT_OK) return st;
  }
  return launch_pixel_walk(kModeBackAtomic, m, g, 0, g->na, entry, proj, xhat, nullptr, nullptr, tile_u, s,
                           lds_table);
}

// Reproducible scatter (TCT_BP_FIXED).  Every term L y_j |d_j| is rounded
// to a multiple of 2^-scale_exp, one scale for the launch: 2^e bounds the
// largest |y_j| |d_j| (|d_j| <= the longest pixel ray of the angle range)
// and K = min(50, 62 - ceil(log2(rays))), so each term is below 2^K in
// magnitude (within the range of the walk's float-to-integer rounding) and
// no tetrahedron's sum of at most `rays` terms can reach 2^62.  The block
// tables and the global sums then add integers, exactly, in any order.
// Scratch layout of the reproducible scatter: [max |y| bits, scale exponent,
// pad to 256 B][nt int64 sums].
static size_t fixed_scratch_bytes(int nt) { return 256 + 8 * (size_t)nt; }

static tct_status backproject_fixed_in(const tct_mesh* m, const tct_geom* g, const float* proj, float* xhat,
                                       int accumulate, const int32_t* entry, int tile_u, int a_begin, int a_count,
                                       hipStream_t s, char* scratch) {
  const int64_t per_angle = (int64_t)g->cone.nu * g->cone.nv;
  const int64_t nrays = per_angle * a_count;
  if (nrays <= 0) return accumulate ? TCT_OK : launch_fill(xhat, m->nt, 0.f, s);
  // Longest pixel ray |P - S| over the angle range: the distance is convex
  // in the pixel position, so a detector corner attains it.
  double dmax = 0.0;
  const float us[2] = {g->ut.front(), g->ut.back()}, vs[2] = {g->vt.front(), g->vt.back()};
  for (int a = a_begin; a < a_begin + a_count; ++a) {
    const float* f = &g->frame[12 * (size_t)a];
    for (float u : us)
      for (float v : vs) {
        double d2 = 0.0;
        for (int k = 0; k < 3; ++k) {
          const double c = (double)f[3 + k] + (double)u * f[6 + k] + (double)v * f[9 + k] - f[k];
          d2 += c * c;
        }
        dmax = std::max(dmax, std::sqrt(d2));
      }
  }
  int bits = 1;
  while (bits < 62 && ((int64_t)1 << bits) < nrays) ++bits;
  const int K = std::min(50, 62 - bits);
  unsigned long long* acc = nullptr;
  unsigned* max_bits = (unsigned*)scratch;
  int* scale_exp = (int*)(scratch + 4);
  acc = (unsigned long long*)(scratch + 256);
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, (unsigned long long*)scratch, (int64_t)1);
  hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)((m->nt + 255) / 256)), dim3(256), 0, s, acc, (int64_t)m->nt);
  const float* y = proj + per_angle * a_begin;
  const unsigned mgrid = (unsigned)std::min<int64_t>(4096, (nrays + 255) / 256);
  hipLaunchKernelGGL(max_abs_kernel, dim3(mgrid), dim3(256), 0, s, y, nrays, max_bits);
  hipLaunchKernelGGL(fixed_scale_kernel, dim3(1), dim3(1), 0, s, (const unsigned*)max_bits,
                     (float)(dmax * 1.0001), K, scale_exp);
  hipError_t e = hipGetLastError();
  tct_status st = TCT_OK;
  if (e == hipSuccess)
    st = launch_pixel_walk(kModeBackFixed, m, g, a_begin, a_count, entry, proj, xhat, nullptr, nullptr, tile_u,
                           s, 1, acc, scale_exp);
  if (e == hipSuccess && st == TCT_OK) {
    hipLaunchKernelGGL(fixed_finish_kernel, dim3((unsigned)((m->nt + 255) / 256)), dim3(256), 0, s,
                       (const unsigned long long*)acc, (const int*)scale_exp, xhat, m->nt, accumulate);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return hip_fail(e, "reproducible scatter launch");
  return st;
}

tct_status backproject_fixed(const tct_mesh* m, const tct_geom* g, const float* proj, float* xhat, int accumulate,
                             const int32_t* entry, int tile_u, int a_begin, int a_count, hipStream_t s) {
  if (m->nt <= 0) return TCT_OK;
  char* scratch = nullptr;
  TCT_HIP(hipMallocAsync((void**)&scratch, fixed_scratch_bytes(m->nt), s));
  const tct_status st = backproject_fixed_in(m, g, proj, xhat, accumulate, entry, tile_u, a_begin, a_count, s,
                                             scratch);
  (void)hipFreeAsync(scratch, s);
  return st;
}

// The allocation-free reproducible scatter keeps its scratch in one static
// device array per GPU, sized for TCT_NOALLOC_MAX_TETS tetrahedra; it lives
// until the process ends.  In host code `scratch` names a host-side stand-in,
// not device memory: kernels get the per-device address that
// hipGetSymbolAddress returns, looked up once per device with that device
// current.  Every call on a GPU reuses the same array; the scatter clears
// what it needs at the start of each call, and calls that overlap in time on
// one GPU race on it.
static __device__ __align__(256) unsigned char scratch[256 + 8 * (size_t)TCT_NOALLOC_MAX_TETS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static tct_status static_scratch(int device, char** out) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("allocation-free scatter: device id out of range");
    return TCT_E_ARG;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[device] = (char*)ptr;
  }
  *out = g_scratch_ptr[device];
  return TCT_OK;
}

tct_status backproject_fixed_noalloc(const tct_mesh* m, const tct_geom* g, const float* proj, float* xhat,
                                     int accumulate, const int32_t* entry, int tile_u, hipStream_t s) {
  if (m->nt <= 0) return TCT_OK;
  if ((int64_t)m->nt > (int64_t)TCT_NOALLOC_MAX_TETS) {
    set_error("tct_backproject_fixed_noalloc: the mesh has " + std::to_string(m->nt) +
              " tetrahedra, more than the static scratch holds (TCT_NOALLOC_MAX_TETS = " +
              std::to_string((long long)TCT_NOALLOC_MAX_TETS) + ")");
    return TCT_E_ARG;
  }
  char* ptr = nullptr;
  const tct_status st = static_scratch(m->device, &ptr);
  if (st != TCT_OK) return st;
  return backproject_fixed_in(m, g, proj, xhat, accumulate, entry, tile_u, 0, g->na, s, ptr);
}

tct_status entry_raster(const tct_mesh* m, const tct_geom* g, int32_t* entry, hipStream_t s) {
  const int64_t nrays = (int64_t)g->na * g->cone.nu * g->cone.nv;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((nrays + 255) / 256)), dim3(256), 0, s, entry, nrays, -1);
  if (m->nb > 0) {
    MeshView M = m->view();
    GeomView G = g->view();
    const unsigned gx = (unsigned)((m->nb + 64 * kRasterWaves - 1) / (64 * kRasterWaves));
    // Split each face's box over several wavefronts when fewer than about
    // 32 per compute unit would run otherwise.
    const int64_t waves = (int64_t)gx * kRasterWaves * g->na;
    const unsigned nz = (unsigned)std::max<int64_t>(1, std::min<int64_t>(64, (8192 + waves - 1) / waves));
    for (int a0 = 0; a0 < g->na; a0 += 65535) {
      const unsigned ny = (unsigned)std::min(65535, g->na - a0);
      hipLaunchKernelGGL(entry_raster_kernel, dim3(gx, ny, nz), dim3(64 * kRasterWaves), 0, s, M, G, a0, entry);
    }
  }
  TCT_HIP(hipGetLastError());
  return TCT_OK;
}

// ---------------------------------------------------------------- batches

tct_status batch_build(const tct_mesh* const* meshes, const tct_geom* const* geoms, int32_t n, const int32_t* tile_u,
                       int32_t* const* entries, tct_batch** out) {
  *out = nullptr;
  tct_batch* b = new tct_batch();
  b->n = n;
  b->device = meshes[0]->device;
  std::vector<BatchDesc> desc(n);
  std::vector<double> cost(n);
  for (int p = 0; p < n; ++p) {
    b->meshes.push_back(meshes[p]);
    b->geoms.push_back(geoms[p]);
    b->tile_u.push_back(tile_u ? tile_u[p] : default_tile_u());
    BatchDesc& d = desc[p];
    d.M = meshes[p]->view();
    d.G = geoms[p]->view();
    d.tm = make_tiles(d.G, b->tile_u[p]);
    d.entry = entries ? entries[p] : nullptr;
    d.user = p;
    d.lds_table = 1;
    // Walk length per ray grows like the mesh's linear resolution.
    cost[p] = std::cbrt((double)meshes[p]->nt);
  }
  std::vector<int> order(n);
  for (int p = 0; p < n; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  std::vector<BatchDesc> sorted(n);
  int64_t item = 0;
  for (int k = 0; k < n; ++k) {
    sorted[k] = desc[order[k]];
    sorted[k].items = (int64_t)sorted[k].tm.nbu * sorted[k].tm.nbv * sorted[k].G.na;
    item += sorted[k].items;
  }
  b->total_items = item;
  // Per-die work lists: run x of every problem, in problem order.
  std::vector<int64_t> lists((size_t)kXcds * (n + 1));
  for (int x = 0; x < kXcds; ++x) {
    int64_t at = 0;
    for (int k = 0; k < n; ++k) {
      lists[(size_t)x * (n + 1) + k] = at;
      at += xcd_run_length(sorted[k].items, x);
    }
    lists[(size_t)x * (n + 1) + n] = at;
  }
  auto fail = [&](hipError_t e, const char* what) {
    batch_free(b);
    return hip_fail(e, what);
  };
  hipError_t e;
  // The batched kernels read every entry face from a cache: problems given
  // without one get a batch-owned cache, filled here by boundary projection.
  for (int k = 0; k < n; ++k) {
    if (sorted[k].entry) continue;
    const int p = sorted[k].user;
    const int64_t nrays = (int64_t)geoms[p]->na * geoms[p]->cone.nu * geoms[p]->cone.nv;
    int32_t* cache = nullptr;
    if ((e = hipMalloc((void**)&cache, sizeof(int32_t) * (size_t)std::max<int64_t>(1, nrays))) != hipSuccess)
      return fail(e, "hipMalloc(batch entry cache)");
    b->owned_entries.push_back(cache);
    const tct_status st = entry_raster(meshes[p], geoms[p], cache, nullptr);
    if (st != TCT_OK) {
      batch_free(b);
      return st;
    }
    sorted[k].entry = cache;
  }
  if ((e = hipDeviceSynchronize()) != hipSuccess) return fail(e, "batch entry caches");
  if ((e = hipMalloc(&b->d_desc, sizeof(BatchDesc) * (size_t)n)) != hipSuccess) return fail(e, "hipMalloc(batch)");
  if ((e = hipMemcpy(b->d_desc, sorted.data(), sizeof(BatchDesc) * (size_t)n, hipMemcpyHostToDevice)) != hipSuccess)
    return fail(e, "hipMemcpy(batch)");
  if ((e = hipMalloc((void**)&b->d_lists, sizeof(int64_t) * lists.size())) != hipSuccess)
    return fail(e, "hipMalloc(batch lists)");
  if ((e = hipMemcpy(b->d_lists, lists.data(), sizeof(int64_t) * lists.size(), hipMemcpyHostToDevice)) !=
      hipSuccess)
    return fail(e, "hipMemcpy(batch lists)");
  if ((e = hipMalloc((void**)&b->d_counter, sizeof(unsigned long long) * kXcds)) != hipSuccess)
    return fail(e, "hipMalloc(batch counters)");
  int cus = 0, occ_f = 0, occ_b = 0;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device)) != hipSuccess)
    return fail(e, "hipDeviceGetAttribute");
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_f, batch_walk_kernel<kModeForward>, 256, 0)) !=
      hipSuccess)
    return fail(e, "occupancy");
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_b, batch_walk_kernel<kModeBackAtomic>, 256, 0)) !=
      hipSuccess)
    return fail(e, "occupancy");
  b->grid_fwd = std::max(1, cus * std::max(1, occ_f));
  b->grid_bwd = std::max(1, cus * std::max(1, occ_b));
  *out = b;
  return TCT_OK;
}

void batch_free(tct_batch* b) {
  if (!b) return;
  if (b->d_desc) (void)hipFree(b->d_desc);
  if (b->d_counter) (void)hipFree(b->d_counter);
  if (b->d_lists) (void)hipFree(b->d_lists);
  for (int32_t* p : b->owned_entries) (void)hipFree(p);
  delete b;
}

tct_status batch_walk(tct_batch* b, int mode, const tct_vecset* in, const tct_vecset* out, hipStream_t s) {
  // A kernel, not a memset, clears the counters: the launch may be captured
  // into a graph and replayed.
  hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, s, b->d_counter, kXcds);
  const BatchDesc* D = (const BatchDesc*)b->d_desc;
  if (mode == kModeForward) {
    hipLaunchKernelGGL(batch_walk_kernel<kModeForward>, dim3(b->grid_fwd), dim3(256), 0, s, D, b->n, b->d_lists,
                       b->d_counter, b->queue_chunk, (const float* const*)in->d_ptrs, out->d_ptrs);
  } else if (mode == kModeBackAtomic) {
    hipLaunchKernelGGL(batch_walk_kernel<kModeBackAtomic>, dim3(b->grid_bwd), dim3(256), 0, s, D, b->n,
                       b->d_lists, b->d_counter, b->queue_chunk, (const float* const*)in->d_ptrs, out->d_ptrs);
  } else {
    set_error("batch_walk: unsupported mode");
    return TCT_E_ARG;
  }
  TCT_HIP(hipGetLastError());
  return TCT_OK;
}

tct_status launch_permute(const float* in, float* out, const int32_t* perm, int n, int scatter, hipStream_t s) {
  if (n <= 0) return TCT_OK;
  hipLaunchKernelGGL(permute_kernel, dim3((n + 255) / 256), dim3(256), 0, s, in, out, perm, n, scatter);
  TCT_HIP(hipGetLastError());
  return TCT_OK;
}

}  // namespace tct
