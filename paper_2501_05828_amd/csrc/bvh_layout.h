// BVH node layout shared by the host builder and the device traversal.
// Plain C++ (no HIP types) so the builder can also be compiled by a host
// compiler for self-checks.
#pragma once

namespace ur {

// Threaded (escape-index) BVH node in depth-first preorder, 32 bytes:
//   lo = (bmin.x, bmin.y, bmin.z, skip as int bits)
//   hi = (bmax.x, bmax.y, bmax.z, leaf as int bits)
// skip = index of the node after this subtree; leaf = -1 for an inner node,
// else (first << 4) | count.  The first child of an inner node is the next
// node.  Boxes are dilated and rounded outward so an FP32 slab test never
// rejects a primitive the FP64 test would accept.
struct alignas(16) BvhNode {
    float lo[4];
    float hi[4];
};

// Four-wide node (128 bytes, one cache line) for ordered closest-hit
// traversal: the boxes of up to four children, one axis per row, and the
// children: >= 0 an inner node index, -1 an empty slot (box set to a far
// point so the slab test fails), else ~((first << 4) | count) for a leaf.
// The child boxes are the binary tree's node boxes, so the same
// conservativeness holds.
struct alignas(16) Bvh4Node {
    float lo_x[4], hi_x[4], lo_y[4], hi_y[4], lo_z[4], hi_z[4];
    int child[4];
    int pad[4];
};

}  // namespace ur
