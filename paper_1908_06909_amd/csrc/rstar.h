// R*-tree over boundary faces (host build), flattened into BvhNode preorder.
#pragma once

#include <cstdint>
#include <vector>

#include "common.h"

namespace tct {

// Node capacity chosen in Section II-E.
constexpr int kRstarMaxEntries = 10;
constexpr int kRstarMinEntries = 4;

struct RstarTree {
  std::vector<BvhNode> nodes;   // preorder; leaf field = first * 16 + count, -1 for interior nodes
  std::vector<int32_t> faces;   // face ids of the leaves, in leaf order
  int height = 0;               // levels, leaves included
};

// Boxes of nfaces faces ([nfaces][3] lo and hi), each padded by `pad`.
void rstar_build(const float* face_lo, const float* face_hi, int nfaces, float pad, RstarTree& tree);

}  // namespace tct
