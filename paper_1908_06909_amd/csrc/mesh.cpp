// Mesh creation on the host: validation, face neighbours, boundary, convexity,
// spatial reordering, per-face records for the walk and the boundary BVH.
//
// The element graph follows the paper's Section II-B (Fig. 1): every element
// keeps its nodes and its ordered face neighbours, plus the list of boundary
// elements used to start rays (Section II-E).  The method requires a convex
// mesh (Section II-D), which is checked exactly here.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "common.h"
#include "exact.h"
#include "kernels.h"
#include "rstar.h"

namespace tct {

thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

tct_status hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? TCT_E_NOMEM : TCT_E_HIP;
}

namespace {

struct FaceKey {
  int32_t a, b, c;
  int32_t tf;  // tet * 4 + local face (sorted-vertex numbering)
  bool operator<(const FaceKey& o) const {
    if (a != o.a) return a < o.a;
    if (b != o.b) return b < o.b;
    if (c != o.c) return c < o.c;
    return tf < o.tf;
  }
  bool same(const FaceKey& o) const { return a == o.a && b == o.b && c == o.c; }
};

struct DirEdge {
  int32_t from, to, face, third;
  bool operator<(const DirEdge& o) const {
    if (from != o.from) return from < o.from;
    return to < o.to;
  }
};

uint64_t spread21(uint64_t v) {
  v &= 0x1fffff;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}

struct BuildItem {
  float lo[3], hi[3], c[3];
  int id;
};

void bvh_build(std::vector<BuildItem>& it, int begin, int end, float pad, std::vector<BvhNode>& nodes,
               std::vector<int>& order) {
  int me = (int)nodes.size();
  nodes.push_back(BvhNode());
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int i = begin; i < end; ++i)
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], it[i].lo[k]);
      hi[k] = std::max(hi[k], it[i].hi[k]);
      clo[k] = std::min(clo[k], it[i].c[k]);
      chi[k] = std::max(chi[k], it[i].c[k]);
    }
  for (int k = 0; k < 3; ++k) {
    nodes[me].lo[k] = lo[k] - pad;
    nodes[me].hi[k] = hi[k] + pad;
  }
  int count = end - begin;
  if (count <= 4) {
    nodes[me].leaf = (int)order.size() * 8 + count;
    for (int i = begin; i < end; ++i) order.push_back(it[i].id);
  } else {
    int ax = 0;
    for (int k = 1; k < 3; ++k)
      if (chi[k] - clo[k] > chi[ax] - clo[ax]) ax = k;
    int mid = (begin + end) / 2;
    std::nth_element(it.begin() + begin, it.begin() + mid, it.begin() + end,
                     [ax](const BuildItem& p, const BuildItem& q) {
                       if (p.c[ax] != q.c[ax]) return p.c[ax] < q.c[ax];
                       return p.id < q.id;
                     });
    nodes[me].leaf = -1;
    bvh_build(it, begin, mid, pad, nodes, order);
    bvh_build(it, mid, end, pad, nodes, order);
  }
  nodes[me].skip = (int)nodes.size();
}

template <typename T>
tct_status upload(const std::vector<T>& h, T** d, int64_t* bytes) {
  size_t n = h.size() * sizeof(T);
  if (n == 0) n = sizeof(T);
  TCT_HIP(hipMalloc((void**)d, n));
  if (!h.empty()) TCT_HIP(hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  *bytes += (int64_t)n;
  return TCT_OK;
}

}  // namespace

tct_status mesh_build(const float* verts, int32_t nv, const int32_t* tets, int32_t nt, const int32_t* nbrs,
                      uint32_t flags, int device, tct_mesh** out) {
  *out = nullptr;
  if (!verts || !tets || nv <= 0 || nt <= 0) {
    set_error("tct_mesh_create: null input or empty mesh");
    return TCT_E_ARG;
  }
  if (nt >= (1 << 29)) {
    set_error("tct_mesh_create: more than 2^29 tetrahedra");
    return TCT_E_ARG;
  }
  auto P = [&](int v) { return verts + 3 * (size_t)v; };
  for (int64_t i = 0; i < 3 * (int64_t)nv; ++i)
    if (!std::isfinite(verts[i])) {
      set_error("tct_mesh_create: non-finite coordinate");
      return TCT_E_ARG;
    }
  // Sorted vertex ids per tetrahedron; local face f is opposite Ts[t][f].
  std::vector<int32_t> Ts(4 * (size_t)nt);
  for (int t = 0; t < nt; ++t) {
    for (int k = 0; k < 4; ++k) {
      int v = tets[4 * (size_t)t + k];
      if (v < 0 || v >= nv) {
        set_error("tct_mesh_create: tetrahedron " + std::to_string(t) + " has a vertex id out of range");
        return TCT_E_ARG;
      }
      Ts[4 * (size_t)t + k] = v;
    }
    std::sort(&Ts[4 * (size_t)t], &Ts[4 * (size_t)t] + 4);
    const int32_t* q = &Ts[4 * (size_t)t];
    if (q[0] == q[1] || q[1] == q[2] || q[2] == q[3] ||
        orient3d_sign(P(q[0]), P(q[1]), P(q[2]), P(q[3])) == 0) {
      set_error("tct_mesh_create: tetrahedron " + std::to_string(t) + " has zero volume");
      return TCT_E_MESH_DEGENERATE;
    }
  }
  // Face neighbours: sort the 4 nt faces by vertex triple and pair equal keys.
  std::vector<FaceKey> keys(4 * (size_t)nt);
  for (int t = 0; t < nt; ++t) {
    const int32_t* q = &Ts[4 * (size_t)t];
    for (int f = 0; f < 4; ++f) {
      int32_t w[3], n = 0;
      for (int j = 0; j < 4; ++j)
        if (j != f) w[n++] = q[j];
      keys[4 * (size_t)t + f] = {w[0], w[1], w[2], 4 * t + f};
    }
  }
  std::sort(keys.begin(), keys.end());
  std::vector<int32_t> nbr(4 * (size_t)nt, -1), back(4 * (size_t)nt, -1);
  std::vector<int32_t> bface_tf;
  for (size_t i = 0; i < keys.size();) {
    size_t j = i + 1;
    while (j < keys.size() && keys[j].same(keys[i])) ++j;
    if (j - i > 2) {
      set_error("tct_mesh_create: a face is shared by more than two tetrahedra");
      return TCT_E_MESH_NONMANIFOLD;
    }
    if (j - i == 2) {
      int t0 = keys[i].tf >> 2, f0 = keys[i].tf & 3, t1 = keys[i + 1].tf >> 2, f1 = keys[i + 1].tf & 3;
      if (t0 == t1) {
        set_error("tct_mesh_create: a tetrahedron repeats a face");
        return TCT_E_MESH_NONMANIFOLD;
      }
      nbr[4 * (size_t)t0 + f0] = t1;
      back[4 * (size_t)t0 + f0] = f1;
      nbr[4 * (size_t)t1 + f1] = t0;
      back[4 * (size_t)t1 + f1] = f0;
    } else {
      bface_tf.push_back(keys[i].tf);
    }
    i = j;
  }
  keys.clear();
  keys.shrink_to_fit();
  // Neighbours in the caller's numbering (face k opposite the user's vertex k).
  std::vector<int32_t> user_nbrs(4 * (size_t)nt);
  for (int t = 0; t < nt; ++t)
    for (int k = 0; k < 4; ++k) {
      int v = tets[4 * (size_t)t + k];
      int f = (int)(std::find(&Ts[4 * (size_t)t], &Ts[4 * (size_t)t] + 4, v) - &Ts[4 * (size_t)t]);
      user_nbrs[4 * (size_t)t + k] = nbr[4 * (size_t)t + f];
    }
  if (nbrs) {
    for (size_t i = 0; i < user_nbrs.size(); ++i)
      if (nbrs[i] != user_nbrs[i]) {
        set_error("tct_mesh_create: the given neighbour table disagrees with the connectivity (tetrahedron " +
                  std::to_string(i / 4) + ")");
        return TCT_E_MESH_NONMANIFOLD;
      }
  }
  // Boundary faces with outward vertex order: (b - a) x (c - a) must point
  // away from the owner's fourth vertex.
  const int nb = (int)bface_tf.size();
  if (nb < 4) {
    set_error("tct_mesh_create: no closed boundary");
    return TCT_E_MESH_NONMANIFOLD;
  }
  std::vector<int32_t> slot(3 * (size_t)nb), sloc(3 * (size_t)nb);
  for (int b = 0; b < nb; ++b) {
    int t = bface_tf[b] >> 2, f = bface_tf[b] & 3;
    const int32_t* q = &Ts[4 * (size_t)t];
    int l[3], n = 0;
    for (int j = 0; j < 4; ++j)
      if (j != f) l[n++] = j;
    if (orient3d_sign(P(q[l[0]]), P(q[l[1]]), P(q[l[2]]), P(q[f])) > 0) std::swap(l[1], l[2]);
    for (int s = 0; s < 3; ++s) {
      slot[3 * (size_t)b + s] = q[l[s]];
      sloc[3 * (size_t)b + s] = l[s];
    }
  }
  // Convexity and connectivity of the boundary surface: at each boundary
  // edge (a, b) of face (a, b, c), the far vertex d of the face across the
  // edge must not lie strictly outside plane (a, b, c).  A closed, connected,
  // consistently oriented surface that is convex at every edge bounds a
  // convex body.
  {
    std::vector<DirEdge> e(3 * (size_t)nb);
    for (int b = 0; b < nb; ++b)
      for (int s = 0; s < 3; ++s)
        e[3 * (size_t)b + s] = {slot[3 * (size_t)b + s], slot[3 * (size_t)b + (s + 1) % 3], b,
                                slot[3 * (size_t)b + (s + 2) % 3]};
    std::sort(e.begin(), e.end());
    for (size_t i = 1; i < e.size(); ++i)
      if (e[i].from == e[i - 1].from && e[i].to == e[i - 1].to) {
        set_error("tct_mesh_create: boundary edge used twice in one direction");
        return TCT_E_MESH_NONMANIFOLD;
      }
    std::vector<int> parent(nb);
    std::iota(parent.begin(), parent.end(), 0);
    auto find = [&](int x) {
      while (parent[x] != x) x = parent[x] = parent[parent[x]];
      return x;
    };
    for (const DirEdge& de : e) {
      DirEdge key{de.to, de.from, 0, 0};
      auto it = std::lower_bound(e.begin(), e.end(), key);
      if (it == e.end() || it->from != de.to || it->to != de.from) {
        set_error("tct_mesh_create: open boundary (edge without a twin)");
        return TCT_E_MESH_NONMANIFOLD;
      }
      if (orient3d_sign(P(de.from), P(de.to), P(de.third), P(it->third)) > 0) {
        set_error("tct_mesh_create: the mesh is not convex");
        return TCT_E_MESH_NONCONVEX;
      }
      parent[find(de.face)] = find(it->face);
    }
    for (int b = 0; b < nb; ++b)
      if (find(b) != find(0)) {
        set_error("tct_mesh_create: the boundary has several components");
        return TCT_E_MESH_DISCONNECTED;
      }
  }
  tct_mesh* m = new tct_mesh();
  m->device = device;
  m->nv = nv;
  m->nt = nt;
  m->nb = nb;
  m->host_only = (flags & TCT_MESH_HOST_ONLY) != 0;
  m->user_nbrs.swap(user_nbrs);
  for (int k = 0; k < 3; ++k) {
    m->lo[k] = INFINITY;
    m->hi[k] = -INFINITY;
  }
  for (int v = 0; v < nv; ++v)
    for (int k = 0; k < 3; ++k) {
      m->lo[k] = std::min(m->lo[k], P(v)[k]);
      m->hi[k] = std::max(m->hi[k], P(v)[k]);
    }
  // Internal order: Morton curve of the tetrahedron centroids.
  m->perm.resize(nt);
  std::iota(m->perm.begin(), m->perm.end(), 0);
  if (!(flags & TCT_MESH_NO_REORDER)) {
    std::vector<std::pair<uint64_t, int32_t>> code(nt);
    double ext[3], lo3[3];
    for (int k = 0; k < 3; ++k) {
      lo3[k] = m->lo[k];
      ext[k] = std::max(1e-30, (double)m->hi[k] - m->lo[k]);
    }
    for (int t = 0; t < nt; ++t) {
      uint64_t c = 0;
      for (int k = 0; k < 3; ++k) {
        double s = 0;
        for (int j = 0; j < 4; ++j) s += P(Ts[4 * (size_t)t + j])[k];
        double u = (s / 4 - lo3[k]) / ext[k];
        uint64_t q = (uint64_t)std::min(2097151.0, std::max(0.0, u * 2097152.0));
        c |= spread21(q) << k;
      }
      code[t] = {c, t};
    }
    std::sort(code.begin(), code.end());
    for (int i = 0; i < nt; ++i) m->perm[i] = code[i].second;
  }
  m->inv_perm.resize(nt);
  for (int i = 0; i < nt; ++i) m->inv_perm[m->perm[i]] = i;
  // Boundary BVH (entry search, Section II-E) over face bounding boxes.
  std::vector<BvhNode> nodes;
  std::vector<int> order;
  {
    std::vector<BuildItem> items(nb);
    float ext = 0;
    for (int k = 0; k < 3; ++k) ext = std::max(ext, m->hi[k] - m->lo[k]);
    for (int b = 0; b < nb; ++b) {
      BuildItem& it = items[b];
      it.id = b;
      for (int k = 0; k < 3; ++k) {
        float x0 = P(slot[3 * (size_t)b])[k], x1 = P(slot[3 * (size_t)b + 1])[k], x2 = P(slot[3 * (size_t)b + 2])[k];
        it.lo[k] = std::min(x0, std::min(x1, x2));
        it.hi[k] = std::max(x0, std::max(x1, x2));
        it.c[k] = (it.lo[k] + it.hi[k]) * 0.5f;
      }
    }
    // Faces are grouped by the dominant axis of their outward normal (+x, -x,
    // +y, -y, +z, -z), one BVH per group under a common root.  A ray enters
    // only through a face it meets from outside (d . n < 0), so the search
    // skips every group whose normals all face away from it: for a convex
    // mesh that is about half of the boundary, the side the ray leaves by.
    std::vector<int> grp(nb);
    std::vector<double> nrm(3 * (size_t)nb);
    for (int b = 0; b < nb; ++b) {
      const float* p0 = P(slot[3 * (size_t)b]);
      const float* p1 = P(slot[3 * (size_t)b + 1]);
      const float* p2 = P(slot[3 * (size_t)b + 2]);
      double e1[3], e2[3];
      for (int k = 0; k < 3; ++k) {
        e1[k] = (double)p1[k] - p0[k];
        e2[k] = (double)p2[k] - p0[k];
      }
      double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
      const double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      int ax = 0;
      for (int k = 0; k < 3; ++k) {
        n[k] /= len;
        nrm[3 * (size_t)b + k] = n[k];
        if (std::fabs(n[k]) > std::fabs(n[ax])) ax = k;
      }
      grp[b] = 2 * ax + (n[ax] < 0 ? 1 : 0);
    }
    std::stable_sort(items.begin(), items.end(),
                     [&](const BuildItem& a, const BuildItem& b) { return grp[a.id] < grp[b.id]; });
    const float pad = 1e-4f * ext + 1e-30f;
    std::vector<std::pair<int, int>> ranges;
    for (int begin = 0, g = 0; g < 6; ++g) {
      int end = begin;
      while (end < nb && grp[items[end].id] == g) ++end;
      if (end > begin) ranges.push_back({begin, end});
      begin = end;
    }
    // Node 0 is a header (skip = number of groups), nodes 1..ng the group
    // records (normal bounds in lo/hi, skip = the node after the group's
    // tree, leaf = the group's root node); the trees follow.
    const int ng = (int)ranges.size();
    nodes.resize(1 + ng);
    nodes[0] = BvhNode();
    nodes[0].skip = ng;
    nodes[0].leaf = -1;
    for (int gi = 0; gi < ng; ++gi) {
      double lo[3] = {1, 1, 1}, hi[3] = {-1, -1, -1};
      for (int i = ranges[gi].first; i < ranges[gi].second; ++i)
        for (int k = 0; k < 3; ++k) {
          lo[k] = std::min(lo[k], nrm[3 * (size_t)items[i].id + k]);
          hi[k] = std::max(hi[k], nrm[3 * (size_t)items[i].id + k]);
        }
      const int root = (int)nodes.size();
      bvh_build(items, ranges[gi].first, ranges[gi].second, pad, nodes, order);
      BvhNode& rec = nodes[1 + gi];
      // Normal bounds, widened by 1e-6 against the float rounding of the box.
      for (int k = 0; k < 3; ++k) {
        rec.lo[k] = (float)lo[k] - 1e-6f;
        rec.hi[k] = (float)hi[k] + 1e-6f;
      }
      rec.skip = (int)nodes.size();
      rec.leaf = root;
    }
    for (auto& nd : nodes)
      if (nd.skip >= (int)nodes.size()) nd.skip = -1;
    // Boundary faces in entry-id order, and the R*-tree over them when asked.
    m->bface_xyz.resize(9 * (size_t)nb);
    m->bface_owner.resize(nb);
    std::vector<float> flo(3 * (size_t)nb), fhi(3 * (size_t)nb);
    for (int j = 0; j < nb; ++j) {
      const int b = order[j];
      for (int sl = 0; sl < 3; ++sl)
        for (int k = 0; k < 3; ++k) m->bface_xyz[9 * (size_t)j + 3 * sl + k] = P(slot[3 * (size_t)b + sl])[k];
      m->bface_owner[j] = bface_tf[b] >> 2;
      for (int k = 0; k < 3; ++k) {
        const float x0 = P(slot[3 * (size_t)b])[k], x1 = P(slot[3 * (size_t)b + 1])[k],
                    x2 = P(slot[3 * (size_t)b + 2])[k];
        flo[3 * (size_t)j + k] = std::min(x0, std::min(x1, x2));
        fhi[3 * (size_t)j + k] = std::max(x0, std::max(x1, x2));
      }
    }
    if (flags & TCT_MESH_RSTAR) {
      RstarTree tree;
      rstar_build(flo.data(), fhi.data(), nb, 1e-4f * ext + 1e-30f, tree);
      m->rstar_nodes = std::move(tree.nodes);
      m->rstar_list = std::move(tree.faces);
      m->rstar_height = tree.height;
      m->has_rstar = true;
    }
  }
  m->nbvh = (int)nodes.size();
  if (m->host_only) {
    *out = m;
    return TCT_OK;
  }
  // Per-face walk records and boundary-face records.
  std::vector<float4> faces(4 * (size_t)nt);
  for (int i = 0; i < nt; ++i) {
    int t = m->perm[i];
    for (int f = 0; f < 4; ++f) {
      float4 r;
      int nb_user = nbr[4 * (size_t)t + f];
      if (nb_user < 0) {
        int32_t packed = -1;
        std::memcpy(&r.x, &packed, 4);
        r.y = r.z = r.w = 0.f;
      } else {
        int bk = back[4 * (size_t)t + f];
        int32_t packed = (m->inv_perm[nb_user] << 2) | bk;
        std::memcpy(&r.x, &packed, 4);
        const float* o = P(Ts[4 * (size_t)nb_user + bk]);
        r.y = o[0];
        r.z = o[1];
        r.w = o[2];
      }
      faces[4 * (size_t)i + f] = r;
    }
  }
  std::vector<float4> bfaces(4 * (size_t)nb);
  for (int j = 0; j < nb; ++j) {
    int b = order[j];
    int t = bface_tf[b] >> 2, f = bface_tf[b] & 3;
    for (int s = 0; s < 3; ++s) {
      const float* p = P(slot[3 * (size_t)b + s]);
      bfaces[4 * (size_t)j + s] = make_float4(p[0], p[1], p[2], 0.f);
    }
    int32_t owner = m->inv_perm[t];
    int32_t locs = sloc[3 * (size_t)b] | (sloc[3 * (size_t)b + 1] << 2) | (sloc[3 * (size_t)b + 2] << 4) | (f << 6);
    std::memcpy(&bfaces[4 * (size_t)j].w, &owner, 4);
    std::memcpy(&bfaces[4 * (size_t)j + 1].w, &locs, 4);
    const float* o = P(Ts[4 * (size_t)t + f]);
    bfaces[4 * (size_t)j + 3] = make_float4(o[0], o[1], o[2], 0.f);
  }
  // Vertex coordinates per tetrahedron for the element-driven kernels, in
  // positive orientation (v2 and v3 swapped when the sorted order is negative).
  // tetnbr[4 i + k]: internal neighbour across the face opposite tetxyz
  // vertex k (-1 on the boundary), for the element-table walk of the
  // paper-faithful mode.
  std::vector<float4> tetxyz(3 * (size_t)nt);
  std::vector<int32_t> tetnbr(4 * (size_t)nt);
  for (int i = 0; i < nt; ++i) {
    const int32_t* q = &Ts[4 * (size_t)m->perm[i]];
    int idx[4] = {q[0], q[1], q[2], q[3]};
    const bool flip = orient3d_sign(P(idx[0]), P(idx[1]), P(idx[2]), P(idx[3])) < 0;
    if (flip) std::swap(idx[2], idx[3]);
    for (int k = 0; k < 4; ++k) {
      const int f = flip && k >= 2 ? 5 - k : k;  // sorted-order face of local face k
      const int nb_user = nbr[4 * (size_t)m->perm[i] + f];
      tetnbr[4 * (size_t)i + k] = nb_user < 0 ? -1 : m->inv_perm[nb_user];
    }
    float c[12];
    for (int k = 0; k < 4; ++k)
      for (int x = 0; x < 3; ++x) c[3 * k + x] = P(idx[k])[x];
    for (int w = 0; w < 3; ++w) tetxyz[3 * (size_t)i + w] = make_float4(c[4 * w], c[4 * w + 1], c[4 * w + 2], c[4 * w + 3]);
  }
  tct_status st;
  auto fail = [&](tct_status s) {
    mesh_free_device(m);
    delete m;
    return s;
  };
  if (hipSetDevice(device) != hipSuccess) {
    set_error("tct_mesh_create: hipSetDevice failed");
    delete m;
    return TCT_E_HIP;
  }
  if ((st = upload(faces, &m->d_faces, &m->device_bytes)) != TCT_OK) return fail(st);
  if ((st = upload(bfaces, &m->d_bfaces, &m->device_bytes)) != TCT_OK) return fail(st);
  if ((st = upload(tetxyz, &m->d_tetxyz, &m->device_bytes)) != TCT_OK) return fail(st);
  if ((st = upload(tetnbr, &m->d_tetnbr, &m->device_bytes)) != TCT_OK) return fail(st);
  if ((st = upload(nodes, &m->d_bvh, &m->device_bytes)) != TCT_OK) return fail(st);
  if (m->has_rstar) {
    if ((st = upload(m->rstar_nodes, &m->d_rstar, &m->device_bytes)) != TCT_OK) return fail(st);
    if ((st = upload(m->rstar_list, &m->d_rstar_faces, &m->device_bytes)) != TCT_OK) return fail(st);
  }
  if ((st = upload(m->perm, &m->d_perm, &m->device_bytes)) != TCT_OK) return fail(st);
  if ((st = upload(m->inv_perm, &m->d_inv_perm, &m->device_bytes)) != TCT_OK) return fail(st);
  std::vector<unsigned long long> zeros(kNumCounters, 0ull);
  if ((st = upload(zeros, &m->d_counters, &m->device_bytes)) != TCT_OK) return fail(st);
  *out = m;
  return TCT_OK;
}

void mesh_free_device(tct_mesh* m) {
  if (!m) return;
  if (m->d_faces) (void)hipFree(m->d_faces);
  if (m->d_bfaces) (void)hipFree(m->d_bfaces);
  if (m->d_tetxyz) (void)hipFree(m->d_tetxyz);
  if (m->d_tetnbr) (void)hipFree(m->d_tetnbr);
  if (m->d_bvh) (void)hipFree(m->d_bvh);
  if (m->d_rstar) (void)hipFree(m->d_rstar);
  if (m->d_rstar_faces) (void)hipFree(m->d_rstar_faces);
  if (m->d_perm) (void)hipFree(m->d_perm);
  if (m->d_inv_perm) (void)hipFree(m->d_inv_perm);
  if (m->d_counters) (void)hipFree(m->d_counters);
  m->d_faces = nullptr;
  m->d_bfaces = nullptr;
  m->d_tetxyz = nullptr;
  m->d_tetnbr = nullptr;
  m->d_bvh = nullptr;
  m->d_rstar = nullptr;
  m->d_rstar_faces = nullptr;
  m->d_perm = m->d_inv_perm = nullptr;
  m->d_counters = nullptr;
}

// ---------------------------------------------------------------- geometry
// Circular cone-beam frames.  cos/sin in double, exact at quarter turns.
namespace {
void quarter_exact_cos_sin(double th, double* c, double* s) {
  const double half_pi = M_PI / 2.0;
  double k = std::nearbyint(th / half_pi);
  if (std::fabs(th - k * half_pi) < 1e-12) {
    long q = (long)k % 4;
    if (q < 0) q += 4;
    *c = (q == 0) ? 1.0 : (q == 2) ? -1.0 : 0.0;
    *s = (q == 1) ? 1.0 : (q == 3) ? -1.0 : 0.0;
  } else {
    *c = std::cos(th);
    *s = std::sin(th);
  }
}
}  // namespace

tct_status geom_build(const tct_cone* cone, const double* angles, int32_t na, int device, tct_geom** out) {
  *out = nullptr;
  if (!cone || !angles || na <= 0 || cone->nu <= 0 || cone->nv <= 0 || !(cone->dsd > cone->dso) ||
      !(cone->dso > 0)) {
    set_error("tct_geom_create: bad cone geometry");
    return TCT_E_ARG;
  }
  if ((int64_t)na * cone->nu * cone->nv >= ((int64_t)1 << 40)) {
    set_error("tct_geom_create: too many rays");
    return TCT_E_ARG;
  }
  tct_geom* g = new tct_geom();
  g->device = device;
  g->cone = *cone;
  g->na = na;
  g->angles.assign(angles, angles + na);
  g->frame.resize(12 * (size_t)na);
  for (int a = 0; a < na; ++a) {
    double c, s;
    quarter_exact_cos_sin(angles[a], &c, &s);
    float* f = &g->frame[12 * (size_t)a];
    f[0] = (float)(cone->dso * c);
    f[1] = (float)(cone->dso * s);
    f[2] = 0.f;
    f[3] = (float)(-(cone->dsd - cone->dso) * c);
    f[4] = (float)(-(cone->dsd - cone->dso) * s);
    f[5] = 0.f;
    f[6] = (float)(-s);
    f[7] = (float)c;
    f[8] = 0.f;
    f[9] = 0.f;
    f[10] = 0.f;
    f[11] = 1.f;
  }
  g->ut.resize(cone->nu);
  g->vt.resize(cone->nv);
  for (int i = 0; i < cone->nu; ++i) g->ut[i] = (float)((i - (cone->nu - 1) / 2.0) * cone->du + cone->off_u);
  for (int j = 0; j < cone->nv; ++j) g->vt[j] = (float)((j - (cone->nv - 1) / 2.0) * cone->dv + cone->off_v);
  if (hipSetDevice(device) != hipSuccess) {
    set_error("tct_geom_create: hipSetDevice failed");
    delete g;
    return TCT_E_HIP;
  }
  int64_t bytes = 0;
  tct_status st;
  if ((st = upload(g->frame, &g->d_frame, &bytes)) != TCT_OK || (st = upload(g->ut, &g->d_ut, &bytes)) != TCT_OK ||
      (st = upload(g->vt, &g->d_vt, &bytes)) != TCT_OK) {
    if (g->d_frame) (void)hipFree(g->d_frame);
    if (g->d_ut) (void)hipFree(g->d_ut);
    if (g->d_vt) (void)hipFree(g->d_vt);
    delete g;
    return st;
  }
  *out = g;
  return TCT_OK;
}

// The whole mesh must lie strictly between the source and the detector plane
// for every angle, so that t in (0, 1) along each ray covers it.  Checked on
// the eight corners of the node bounding box in double.
tct_status check_geometry(const tct_mesh* m, const tct_geom* g) {
  for (int a = 0; a < g->na; ++a) {
    const float* f = &g->frame[12 * (size_t)a];
    double w[3] = {(double)f[3] - f[0], (double)f[4] - f[1], (double)f[5] - f[2]};
    double dd = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    for (int c = 0; c < 8; ++c) {
      double p[3] = {(c & 1) ? m->hi[0] : m->lo[0], (c & 2) ? m->hi[1] : m->lo[1], (c & 4) ? m->hi[2] : m->lo[2]};
      double s = ((p[0] - f[0]) * w[0] + (p[1] - f[1]) * w[1] + (p[2] - f[2]) * w[2]) / dd;
      if (!(s > 1e-6 && s < 1.0 - 1e-6)) {
        set_error("the mesh is not strictly between the source and the detector at angle " + std::to_string(a));
        return TCT_E_GEOM;
      }
    }
  }
  return TCT_OK;
}

}  // namespace tct
