// Internal types shared by the host and device parts of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tetct.h"

#ifndef TCT_XCD_REMAP
#define TCT_XCD_REMAP 1
#endif

namespace tct {

// One bounding-volume-hierarchy node over boundary faces, 32 bytes, stored
// in depth-first preorder: an interior node's first child is the next node;
// `skip` is the node after its whole subtree (-1 past the end).  `leaf` is
// -1 for interior nodes, else first_face * 8 + count (count <= 7).  The
// boundary BVH starts with a header (node 0, skip = number of groups) and
// one record per group of faces with a common outward-normal axis (nodes
// 1..ng: normal bounds in lo/hi, skip = the node after the group's tree,
// leaf = the group's root node); the group trees follow.
struct BvhNode {
  float lo[3];
  int skip;
  float hi[3];
  int leaf;
};

// Device view of a mesh.  Each tetrahedron has its four vertex ids sorted
// ascending (ids are only used at creation); face f is opposite its f-th
// vertex.  faces[4 t + f] describes the tetrahedron across face f:
//   .x  bits: (neighbour << 2) | back, where `back` is the neighbour's local
//       index of its vertex not on the shared face; -1 on the boundary
//   .yzw coordinates of that vertex.
// Because both tetrahedra list their vertices in ascending id order, the
// shared face's three vertices appear in the same relative order in both,
// which fixes the map between the two local numberings.
// bfaces[4 b + 0..3] describes boundary face b with its owner:
//   [0] xyz vertex slot 0, w = owner (int bits)
//   [1] xyz vertex slot 1, w = slot local indices (bits 0-1, 2-3, 4-5) | face << 6
//   [2] xyz vertex slot 2
//   [3] xyz owner's vertex opposite the face
// with slots ordered so that (slot1 - slot0) x (slot2 - slot0) points out of the mesh.
struct MeshView {
  const float4* faces;
  const float4* bfaces;
  const BvhNode* bvh;
  const int* perm;  // internal -> user tetrahedron id
  int nt;
  int nb;
  unsigned long long* counters;  // tct_stats fields, int64 each
  float extent;                  // largest |coordinate| of any node
  // tetxyz[3 t + 0..2]: the four vertices of tetrahedron t as 12 floats
  // (v0.xyz v1.xyz v2.xyz v3.xyz), ordered so that
  // det[v1 - v0, v2 - v0, v3 - v0] > 0.
  const float4* tetxyz;
  const int32_t* tetnbr;  // [nt][4] neighbour across the face opposite tetxyz vertex k, -1 = boundary
  // R*-tree over the boundary faces in the same preorder node format, leaf
  // field first * 16 + count into rstar_faces (null when not built).
  const BvhNode* rstar;
  const int32_t* rstar_faces;
};

// Cone-beam frames: frame[12 a + 0..11] = S, D, U, V of angle a.
struct GeomView {
  const float* frame;
  const float* ut;
  const float* vt;
  int na, nu, nv;
};

// Stats slots in MeshView::counters (same order as tct_stats).
enum Counter {
  kRays = 0,
  kSegments,
  kZeroLen,
  kFp64Stage,
  kExactStage,
  kPerturbed,
  kFailed,
  kGrazing,
  kNumCounters = 8
};

// XCD-aware block order.  The chip's 256 compute units sit in 8 dies
// (XCDs), each with its own L2, and the dispatcher hands workgroup b to die
// b mod 8.  Launches whose neighbouring blocks share data renumber their
// blocks so that each die takes one contiguous run of the logical order
// instead of every eighth block: die x (0..7) processes logical blocks
// [x per + min(x, rem), ...) with per = n / 8 and rem = n mod 8, the first
// rem dies one block more.  A bijection on [0, n) for any n.
constexpr int kXcds = 8;
__host__ __device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t n) {
#if TCT_XCD_REMAP
  const int64_t per = n / kXcds, rem = n % kXcds;
  const int64_t x = b % kXcds, i = b / kXcds;
  return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
#else
  (void)n;
  return b;
#endif
}

// Local-index remap, tabulated for the walk.  The walk keeps the local indices of its
// three entry-face slots and of v in 2-bit fields of one byte (slot j in bits
// 2j, v in bits 6-7).  Leaving through the face opposite slot k into a
// neighbour whose opposite vertex has local index `back`, every index p
// becomes r + (r >= back) with r = p - (p > f), f = the index in slot k; slot
// k then takes v's new index and v's field takes `back`.  The entry for
// (byte, k, back) sits at (byte * 3 + k) * 4 + back; bytes that are not
// permutations map to values the walk never reads.
constexpr int kLocRemapEntries = 256 * 3 * 4;

constexpr unsigned loc_remap_entry(unsigned i) {
  const unsigned L = i / 12u, k = (i / 4u) % 3u, back = i % 4u;
  const unsigned f = (L >> (2u * k)) & 3u;
  unsigned out = 0;
  for (unsigned s = 0; s < 4; ++s) {
    const unsigned p = (L >> (2u * s)) & 3u;
    const unsigned r = p - (p > f ? 1u : 0u);
    out |= ((r + (r >= back ? 1u : 0u)) & 3u) << (2u * s);
  }
  const unsigned vnew = (out >> 6) & 3u;
  out = (out & ~(3u << (2u * k))) | (vnew << (2u * k));
  return (out & 0x3Fu) | (back << 6);
}

void set_error(const std::string& msg);
tct_status hip_fail(hipError_t e, const char* what);

#define TCT_HIP(call)                                             \
  do {                                                            \
    hipError_t _e = (call);                                       \
    if (_e != hipSuccess) return ::tct::hip_fail(_e, #call);      \
  } while (0)

}  // namespace tct

// Opaque handles.
struct tct_mesh {
  int device = 0;
  int nv = 0, nt = 0, nb = 0;
  bool host_only = false;
  std::vector<int32_t> perm;       // internal -> user
  std::vector<int32_t> inv_perm;   // user -> internal
  std::vector<int32_t> user_nbrs;  // [nt][4] user numbering
  float lo[3], hi[3];              // bounding box of the nodes
  float4* d_faces = nullptr;
  float4* d_bfaces = nullptr;
  float4* d_tetxyz = nullptr;
  int32_t* d_tetnbr = nullptr;
  tct::BvhNode* d_bvh = nullptr;
  tct::BvhNode* d_rstar = nullptr;
  int32_t* d_rstar_faces = nullptr;
  int32_t* d_perm = nullptr;
  int32_t* d_inv_perm = nullptr;
  unsigned long long* d_counters = nullptr;
  int nbvh = 0;
  bool has_rstar = false;
  std::vector<tct::BvhNode> rstar_nodes;  // host copy of the R*-tree (preorder)
  std::vector<int32_t> rstar_list;        // its leaf face ids
  int rstar_height = 0;
  std::vector<float> bface_xyz;           // [nb][3][3] boundary faces in entry-id order
  std::vector<int32_t> bface_owner;       // [nb] user owner tetrahedron
  int64_t device_bytes = 0;
  tct::MeshView view() const {
    tct::MeshView v;
    v.faces = d_faces;
    v.bfaces = d_bfaces;
    v.bvh = d_bvh;
    v.perm = d_perm;
    v.nt = nt;
    v.nb = nb;
    v.counters = d_counters;
    v.tetxyz = d_tetxyz;
    v.tetnbr = d_tetnbr;
    v.rstar = d_rstar;
    v.rstar_faces = d_rstar_faces;
    v.extent = 0.f;
    for (int k = 0; k < 3; ++k) v.extent = std::max(v.extent, std::max(std::fabs(lo[k]), std::fabs(hi[k])));
    return v;
  }
};

struct tct_vecset {
  int device = 0;
  int n = 0;
  std::vector<float*> ptrs;
  std::vector<int64_t> lens;
  float** d_ptrs = nullptr;
  int64_t* d_lens = nullptr;
};

struct tct_batch {
  int device = 0;
  int n = 0;
  std::vector<const tct_mesh*> meshes;
  std::vector<const tct_geom*> geoms;
  std::vector<int> tile_u;
  void* d_desc = nullptr;  // device BatchDesc[n], most expensive blocks first
  int64_t total_items = 0;
  unsigned long long* d_counter = nullptr;  // [kXcds] next free position of each die's work list
  int64_t* d_lists = nullptr;               // [kXcds][n + 1] positions of the problems' runs in the lists
  int grid_fwd = 0, grid_bwd = 0;  // persistent grid sizes
  int queue_chunk = 1;             // pixel blocks handed out per queue fetch
  std::vector<int32_t*> owned_entries;  // entry caches made for problems given without one
};

struct tct_geom {
  int device = 0;
  tct_cone cone;
  int na = 0;
  std::vector<double> angles;
  std::vector<float> frame;  // [na][12]
  std::vector<float> ut, vt;
  float* d_frame = nullptr;
  float* d_ut = nullptr;
  float* d_vt = nullptr;
  tct::GeomView view() const {
    tct::GeomView v;
    v.frame = d_frame;
    v.ut = d_ut;
    v.vt = d_vt;
    v.na = na;
    v.nu = cone.nu;
    v.nv = cone.nv;
    return v;
  }
  int64_t nrays() const { return (int64_t)na * cone.nu * cone.nv; }
};
