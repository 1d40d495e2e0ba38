// R*-tree over the boundary faces: the paper's entry-search structure
// (Section II-E), built on the host by one-by-one insertion with the R*
// rules of Beckmann et al. (least overlap enlargement when choosing among
// leaves, forced reinsertion of the 30% of entries farthest from a node's
// centre on its first overflow per level, and the margin-then-overlap split),
// with the paper's node capacity of 4 to 10 entries.
//
// The tree is flattened in depth-first preorder into the same node format as
// the boundary BVH (box, skip link, leaf field), so the device descends it
// without a stack: an interior node's first child is the next node, a
// missed box jumps to `skip`.  A leaf node's field is first * 16 + count
// with its face ids in a separate list.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "common.h"
#include "rstar.h"

namespace tct {

namespace {

struct Box {
  float lo[3], hi[3];
};

Box box_union(const Box& a, const Box& b) {
  Box r;
  for (int k = 0; k < 3; ++k) {
    r.lo[k] = std::min(a.lo[k], b.lo[k]);
    r.hi[k] = std::max(a.hi[k], b.hi[k]);
  }
  return r;
}

// Volumes and margins in double: padded face boxes are thin, and float
// products of three small extents lose the comparisons the rules rely on.
double volume(const Box& b) {
  double v = 1.0;
  for (int k = 0; k < 3; ++k) v *= std::max(0.0, (double)b.hi[k] - (double)b.lo[k]);
  return v;
}

double margin(const Box& b) {
  double s = 0.0;
  for (int k = 0; k < 3; ++k) s += (double)b.hi[k] - (double)b.lo[k];
  return s;
}

double overlap(const Box& a, const Box& b) {
  double v = 1.0;
  for (int k = 0; k < 3; ++k) {
    double lo = std::max(a.lo[k], b.lo[k]), hi = std::min(a.hi[k], b.hi[k]);
    if (hi <= lo) return 0.0;
    v *= hi - lo;
  }
  return v;
}

struct Node {
  int level;               // 0: entries are faces; L: entries are nodes of level L - 1
  std::vector<int> child;  // face ids or node ids
  Box box;
};

class Builder {
 public:
  Builder(const std::vector<Box>& faces, int max_entries, int min_entries)
      : faces_(faces), M_(max_entries), m_(min_entries) {
    nodes_.push_back(Node{0, {}, Box{{INFINITY, INFINITY, INFINITY}, {-INFINITY, -INFINITY, -INFINITY}}});
    root_ = 0;
  }

  void insert_face(int f) {
    reinserted_.assign(nodes_[root_].level + 2, false);
    pending_.clear();
    insert(f, 0);
    // Entries removed by forced reinsertion go back in, closest first; each
    // may trigger further overflows, handled the same way.
    while (!pending_.empty()) {
      auto e = pending_.back();
      pending_.pop_back();
      insert(e.first, e.second);
    }
  }

  int root() const { return root_; }
  const std::vector<Node>& nodes() const { return nodes_; }

 private:
  const Box& entry_box(int level, int id) const { return level == 0 ? faces_[id] : nodes_[id].box; }

  void recompute(int n) {
    Node& nd = nodes_[n];
    Box b{{INFINITY, INFINITY, INFINITY}, {-INFINITY, -INFINITY, -INFINITY}};
    for (int c : nd.child) b = box_union(b, entry_box(nd.level, c));
    nd.box = b;
  }

  // Entry `id` (a face when level == 0, else a node of level - 1) goes into
  // a node of level `level`.
  void insert(int id, int level) {
    if ((int)reinserted_.size() < nodes_[root_].level + 2) reinserted_.resize(nodes_[root_].level + 2, false);
    int split = insert_rec(root_, id, level);
    if (split >= 0) {
      Node r{nodes_[root_].level + 1, {root_, split}, Box{}};
      nodes_.push_back(r);
      root_ = (int)nodes_.size() - 1;
      recompute(root_);
      reinserted_.resize(nodes_[root_].level + 2, false);
    }
  }

  // Returns the id of a new sibling when `n` was split, else -1.
  int insert_rec(int n, int id, int level) {
    if (nodes_[n].level == level) {
      nodes_[n].child.push_back(id);
    } else {
      int c = choose_child(n, entry_box(level, id));
      int split = insert_rec(c, id, level);
      if (split >= 0) nodes_[n].child.push_back(split);
    }
    recompute(n);
    if ((int)nodes_[n].child.size() > M_) return overflow(n);
    return -1;
  }

  // ChooseSubtree: least overlap enlargement among leaf children, least
  // volume enlargement higher up; ties by volume enlargement, then volume.
  int choose_child(int n, const Box& b) const {
    const Node& nd = nodes_[n];
    const int cl = nd.level - 1;
    const bool leaves = cl == 0;
    int best = -1;
    double b0 = 0, b1 = 0, b2 = 0;
    for (size_t i = 0; i < nd.child.size(); ++i) {
      const Box& cb = entry_box(nd.level, nd.child[i]);
      const Box ub = box_union(cb, b);
      double k0 = 0.0;
      if (leaves) {
        for (size_t j = 0; j < nd.child.size(); ++j) {
          if (j == i) continue;
          const Box& ob = entry_box(nd.level, nd.child[j]);
          k0 += overlap(ub, ob) - overlap(cb, ob);
        }
      }
      const double v = volume(cb), k1 = volume(ub) - v, k2 = v;
      if (best < 0 || k0 < b0 || (k0 == b0 && (k1 < b1 || (k1 == b1 && k2 < b2)))) {
        best = (int)i;
        b0 = k0;
        b1 = k1;
        b2 = k2;
      }
    }
    (void)cl;
    return nd.child[best];
  }

  int overflow(int n) {
    const int level = nodes_[n].level;
    if (n != root_ && !reinserted_[level]) {
      reinserted_[level] = true;
      reinsert(n);
      return -1;
    }
    return split(n);
  }

  // Forced reinsertion: remove the p entries whose box centres are farthest
  // from the node's box centre and queue them, closest of them first.
  void reinsert(int n) {
    Node& nd = nodes_[n];
    const int p = std::max(1, (int)std::lround(0.3 * M_));
    double c[3];
    for (int k = 0; k < 3; ++k) c[k] = 0.5 * ((double)nd.box.lo[k] + nd.box.hi[k]);
    std::vector<std::pair<double, int>> d;
    for (int id : nd.child) {
      const Box& b = entry_box(nd.level, id);
      double s = 0.0;
      for (int k = 0; k < 3; ++k) {
        double x = 0.5 * ((double)b.lo[k] + b.hi[k]) - c[k];
        s += x * x;
      }
      d.push_back({s, id});
    }
    std::stable_sort(d.begin(), d.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
    nd.child.clear();
    for (size_t i = p; i < d.size(); ++i) nd.child.push_back(d[i].second);
    recompute(n);
    // pending_ is a stack: push the farthest first so the closest pops first.
    for (int i = 0; i < p; ++i) pending_.push_back({d[i].second, nd.level});
  }

  // Split of an overfull node: the axis with the least sum of margins over
  // all legal distributions, then on it the distribution with the least
  // overlap (ties: least total volume).  Returns the new node.
  int split(int n) {
    const int level = nodes_[n].level;
    std::vector<int> e = nodes_[n].child;
    const int count = (int)e.size();
    const int dists = count - 2 * m_ + 1;  // first group sizes m .. count - m
    auto sorted = [&](int axis, int by_hi) {
      std::vector<int> s = e;
      std::stable_sort(s.begin(), s.end(), [&](int a, int b) {
        const Box& A = entry_box(level, a);
        const Box& B = entry_box(level, b);
        float ka = by_hi ? A.hi[axis] : A.lo[axis], kb = by_hi ? B.hi[axis] : B.lo[axis];
        float ta = by_hi ? A.lo[axis] : A.hi[axis], tb = by_hi ? B.lo[axis] : B.hi[axis];
        if (ka != kb) return ka < kb;
        return ta < tb;
      });
      return s;
    };
    auto group_boxes = [&](const std::vector<int>& s, int k, Box& g1, Box& g2) {
      g1 = Box{{INFINITY, INFINITY, INFINITY}, {-INFINITY, -INFINITY, -INFINITY}};
      g2 = g1;
      for (int i = 0; i < count; ++i) {
        if (i < k)
          g1 = box_union(g1, entry_box(level, s[i]));
        else
          g2 = box_union(g2, entry_box(level, s[i]));
      }
    };
    int axis = 0;
    double best_margin = INFINITY;
    for (int a = 0; a < 3; ++a) {
      double S = 0.0;
      for (int h = 0; h < 2; ++h) {
        std::vector<int> s = sorted(a, h);
        for (int t = 0; t < dists; ++t) {
          Box g1, g2;
          group_boxes(s, m_ + t, g1, g2);
          S += margin(g1) + margin(g2);
        }
      }
      if (S < best_margin) {
        best_margin = S;
        axis = a;
      }
    }
    std::vector<int> best_s;
    int best_k = -1;
    double bo = 0, bv = 0;
    for (int h = 0; h < 2; ++h) {
      std::vector<int> s = sorted(axis, h);
      for (int t = 0; t < dists; ++t) {
        Box g1, g2;
        const int k = m_ + t;
        group_boxes(s, k, g1, g2);
        double o = overlap(g1, g2), v = volume(g1) + volume(g2);
        if (best_k < 0 || o < bo || (o == bo && v < bv)) {
          best_k = k;
          best_s = s;
          bo = o;
          bv = v;
        }
      }
    }
    Node nn{level, std::vector<int>(best_s.begin() + best_k, best_s.end()), Box{}};
    nodes_[n].child.assign(best_s.begin(), best_s.begin() + best_k);
    recompute(n);
    nodes_.push_back(nn);
    const int id = (int)nodes_.size() - 1;
    recompute(id);
    return id;
  }

  const std::vector<Box>& faces_;
  const int M_, m_;
  std::vector<Node> nodes_;
  int root_;
  std::vector<bool> reinserted_;
  std::vector<std::pair<int, int>> pending_;  // (entry, level of the node that takes it)
};

void emit(const std::vector<Node>& nodes, int n, std::vector<BvhNode>& out, std::vector<int32_t>& list) {
  const Node& nd = nodes[n];
  const int me = (int)out.size();
  out.push_back(BvhNode());
  for (int k = 0; k < 3; ++k) {
    out[me].lo[k] = nd.box.lo[k];
    out[me].hi[k] = nd.box.hi[k];
  }
  if (nd.level == 0) {
    out[me].leaf = (int)list.size() * 16 + (int)nd.child.size();
    for (int f : nd.child) list.push_back(f);
  } else {
    out[me].leaf = -1;
    for (int c : nd.child) emit(nodes, c, out, list);
  }
  out[me].skip = (int)out.size();
}

}  // namespace

void rstar_build(const float* face_lo, const float* face_hi, int nfaces, float pad, RstarTree& tree) {
  std::vector<Box> boxes(nfaces);
  for (int f = 0; f < nfaces; ++f)
    for (int k = 0; k < 3; ++k) {
      boxes[f].lo[k] = face_lo[3 * (size_t)f + k] - pad;
      boxes[f].hi[k] = face_hi[3 * (size_t)f + k] + pad;
    }
  Builder b(boxes, kRstarMaxEntries, kRstarMinEntries);
  for (int f = 0; f < nfaces; ++f) b.insert_face(f);
  tree.nodes.clear();
  tree.faces.clear();
  emit(b.nodes(), b.root(), tree.nodes, tree.faces);
  for (auto& nd : tree.nodes)
    if (nd.skip >= (int)tree.nodes.size()) nd.skip = -1;
  tree.height = b.nodes()[b.root()].level + 1;
}

}  // namespace tct
