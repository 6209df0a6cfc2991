// Host-side bounding volume hierarchy builder (binned surface-area
// heuristic), emitted as a threaded depth-first node array for stackless
// traversal on the device.
#pragma once
#include <vector>

#include "bvh_layout.h"

namespace ur {

struct PrimBounds {
    double lo[3], hi[3];
};

struct BvhResult {
    std::vector<BvhNode> nodes;   // depth-first preorder, skip indices set
    std::vector<int> order;       // BVH slot -> original primitive index
    int max_depth = 0;
};

// Builds over `prims`.  Leaves hold at most `leaf_max` (<= 15) primitives.
// Node boxes are the FP64 union of their primitives' boxes grown by
// `dilate` metres and rounded outward to FP32.
BvhResult build_bvh(const std::vector<PrimBounds> &prims, int leaf_max, double dilate);

// Collapses the binary tree of a threaded layout into four-wide nodes
// (greedily opening the largest-area inner child until four children or
// only leaves remain), in depth-first order with the root at 0.  Leaves and
// primitive order are unchanged.  Empty for an empty tree.
std::vector<Bvh4Node> collapse_bvh4(const std::vector<BvhNode> &nodes);

// Quantises four-wide nodes to the 64-byte layout (conservative decode).
std::vector<Bvh4NodeQ> quantize_bvh4(const std::vector<Bvh4Node> &nodes);

// FP32 decode of child k of a quantised node, as the device evaluates it.
void decode_bvh4q(const Bvh4NodeQ &n, int k, float lo[3], float hi[3]);

}  // namespace ur
