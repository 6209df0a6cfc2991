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

// The same node quantised to 64 bytes (half a cache line): child boxes are
// 8-bit offsets from the node origin in steps of a power of two per axis,
//   lo = origin + qlo * 2^(e - 127),  hi = origin + qhi * 2^(e - 127),
// rounded outward so that, evaluated in FP32 (the product is exact, the sum
// rounds once), every decoded box contains the FP32 box it replaces.
//   org = (origin.x, origin.y, origin.z, ex | ey << 8 | ez << 16 as int bits)
//   q[0..3] = qlo_x, q[4..7] = qlo_y, q[8..11] = qlo_z,
//   q[12..15] = qhi_x, q[16..19] = qhi_y, q[20..23] = qhi_z (child k at +k)
struct alignas(16) Bvh4NodeQ {
    float org[4];
    unsigned char q[32];
    int child[4];
};
static_assert(sizeof(Bvh4NodeQ) == 64, "quantised node layout");

}  // namespace ur
