// Closest-hit query of the trace kernels (UltraRay, arXiv 2501.05828,
// Sec. 2.2), shared by the forward trace and the adjoint's value pass: box
// exit, spheres and planes, then the four-wide BVH in nearest-first order
// with a per-lane LDS stack (the threaded binary walk as the exact fallback
// of an overflowing stack).  Every decision is FP64; FP32 only culls boxes,
// conservatively.  Included by one translation unit each; the definitions
// live in an unnamed namespace.
#pragma once
#include "trace_device.h"

namespace {
using namespace ur;
using namespace ur::dev;

// Per-lane event counters (compiled out unless COUNT).
struct Counters {
    uint32_t v[kNumStats];
};
enum {
    C_RAYS, C_SEGMENTS, C_REFLECT, C_TRANSMIT, C_TIR, C_SCAT_EVENTS, C_NEE_ZERO, C_NEE_CAST, C_NEE_BLOCKED,
    C_DIRECT, C_RECORDS, C_DROPPED, C_EDGE, C_TERM_BOX, C_TERM_BOUNCE, C_TERM_TIME, C_TERM_PATH, C_MISMATCH,
    C_TRI_NODES, C_TRI_TESTS, C_SCAT_CELLS, C_SCAT_TESTS, C_SHADOW_NODES, C_SHADOW_TRI_TESTS, C_TERM_ROUGH,
    C_SURF_EVENTS, C_SURF_ZERO
};

#define CNT(k)                  \
    do {                        \
        if constexpr (COUNT)    \
            ++cnt.v[k];         \
    } while (0)

// --------------------------------------------------------- closest hit query
struct Hit {
    double t;
    int64_t id;
    int face;      // box face 0..5 if id == id_box
    int local;     // triangle slot in BVH order, sphere or plane index
};

// During a tree walk a triangle hit carries this id and its slot in
// `local`; its original id (tri_id[local]) is looked up at ties and once the
// walk is done (resolve_hit), not at every closer hit.
constexpr int64_t kTriPending = -2;

__device__ __forceinline__ int64_t best_id(const TraceParams &P, const Hit &h) {
    return h.id == kTriPending ? (int64_t)P.tri_id[h.local] : h.id;
}

__device__ __forceinline__ void resolve_hit(const TraceParams &P, Hit &h) {
    if (h.id == kTriPending) h.id = P.tri_id[h.local];
}

// Per-lane traversal stack in LDS, entry-major (entry i of lane l at
// base[i * stride]) so lanes at the same depth touch consecutive words.
struct LdsStack {
    int2 *base;
    int stride;
};
#ifndef UR_STACK
#define UR_STACK 16
#endif
constexpr int kStack = UR_STACK;   // entries per lane
// Escape-index walk over the binary tree: complete, stackless, fixed order.
template <bool COUNT>
__device__ __forceinline__ void walk_threaded(const TraceParams &P, const double *o, const double *d, int64_t skip,
                                              const CullRay &cr, float &tmf, Hit &h, Counters &cnt) {
    int ni = 0;
    while (ni < P.n_tnodes) {
        const Node n = load_node(P.tnodes, ni);
        CNT(C_TRI_NODES);
        if (!slab(n, cr, tmf)) {
            ni = node_skip(n);
            continue;
        }
        const int leaf = node_leaf(n);
        if (leaf < 0) {
            ++ni;
            continue;
        }
        const int first = leaf >> 4, count = leaf & 15;
        for (int k = first; k < first + count; ++k) {
            if (k == skip) continue;
            CNT(C_TRI_TESTS);
            double t;
            if (tri_isect(P.tri + 9 * (int64_t)k, o, d, t) && t > kEpsT &&
                (t < h.t || (t == h.t && P.tri_id[k] < best_id(P, h)))) {
                h.t = t;
                h.id = kTriPending;
                h.local = k;
                tmf = cull_tmax(t);
            }
        }
        ni = node_skip(n);
    }
}

// Ordered walk over the four-wide tree.  A visit tests the four child boxes
// of node `cur` from one 64-byte quantised node (wide_decode), hands the hit
// leaf children back as a pending set, continues with the nearest hit inner
// child and stacks the others, farthest first (wide_next).  Popped entries
// whose entry distance exceeds the current best are dropped.  A push that
// finds the stack full sets `overflow` (the caller then re-walks the tree
// with the escape-index walk and the best hit so far).  The triangles of the
// pending leaves are tested by test_leaves: at once in walk_wide, and in the
// extend kernel once enough lanes of the wavefront hold some, so that the
// FP64 test runs on many lanes together.  A later test only leaves the
// culling distance longer for a while (more visits, never a missed hit), so
// the result is always the exact closest hit (nearest t, lower id on ties).
struct Pending {
    unsigned mask;   // hit leaf children still to test (bit k: child k)
    int c[4];        // the node's child words; a leaf is ~((first << 4) | count)
};

template <bool COUNT>
__device__ __forceinline__ void wide_decode(const TraceParams &P, const CullRay &cr, float tmf, int cur, float key[4],
                                            int val[4], Pending &pd, Counters &cnt) {
    const uint4 *q = reinterpret_cast<const uint4 *>(P.tnodes4 + cur);
    const uint4 org = q[0], w0 = q[1], w1 = q[2];
    const int4 ch = reinterpret_cast<const int4 *>(q)[3];
    CNT(C_TRI_NODES);
    // child box planes as t = q * (step * inv) + (origin - o) * inv per axis
    const float sx = __int_as_float((int)((org.w & 255u) << 23)), sy = __int_as_float((int)(((org.w >> 8) & 255u) << 23));
    const float sz = __int_as_float((int)(((org.w >> 16) & 255u) << 23));
    const float ax = sx * cr.ix, ay = sy * cr.iy, az = sz * cr.iz;
    const float bx = (__uint_as_float(org.x) - cr.ox) * cr.ix, by = (__uint_as_float(org.y) - cr.oy) * cr.iy;
    const float bz = (__uint_as_float(org.z) - cr.oz) * cr.iz;
    pd.c[0] = ch.x;
    pd.c[1] = ch.y;
    pd.c[2] = ch.z;
    pd.c[3] = ch.w;
    unsigned leaves = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float x0 = fmaf((float)((w0.x >> (8 * k)) & 255u), ax, bx);
        const float y0 = fmaf((float)((w0.y >> (8 * k)) & 255u), ay, by);
        const float z0 = fmaf((float)((w0.z >> (8 * k)) & 255u), az, bz);
        const float x1 = fmaf((float)((w0.w >> (8 * k)) & 255u), ax, bx);
        const float y1 = fmaf((float)((w1.x >> (8 * k)) & 255u), ay, by);
        const float z1 = fmaf((float)((w1.y >> (8 * k)) & 255u), az, bz);
        const float tn = fmaxf(fmaxf(fminf(x0, x1), fminf(y0, y1)), fmaxf(fminf(z0, z1), 0.0f));
        const float tf = fminf(fminf(fmaxf(x0, x1), fmaxf(y0, y1)), fminf(fmaxf(z0, z1), tmf));
        const bool hit = tn <= tf && pd.c[k] != -1;
        if (hit && pd.c[k] < -1) leaves |= 1u << k;
        key[k] = hit && pd.c[k] >= 0 ? tn : INFINITY;
        val[k] = pd.c[k];
    }
    pd.mask = leaves;
}

// The triangles of every pending leaf, in one loop, so that a wavefront runs
// the FP64 test once per triangle position rather than once per child slot.
// (A triangle's original id is loaded only at a tie; see kTriPending.)
template <bool COUNT>
__device__ __forceinline__ void test_leaves(const TraceParams &P, const double *o, const double *d, int64_t skip,
                                            float &tmf, Hit &h, const Pending &pd, Counters &cnt) {
    unsigned leaves = pd.mask;
    int j = 0, je = 0;
    while (true) {
        while (j >= je && leaves) {
            const int k = __builtin_ctz(leaves);
            leaves &= leaves - 1;
            const int w = ~(k == 0 ? pd.c[0] : (k == 1 ? pd.c[1] : (k == 2 ? pd.c[2] : pd.c[3])));
            j = w >> 4;
            je = j + (w & 15);
        }
        if (j >= je) break;
        if (j != skip) {
            CNT(C_TRI_TESTS);
            double t;
            if (tri_isect(P.tri + 9 * (int64_t)j, o, d, t) && t > kEpsT &&
                (t < h.t || (t == h.t && P.tri_id[j] < best_id(P, h)))) {
                h.t = t;
                h.id = kTriPending;
                h.local = j;
                tmf = cull_tmax(t);
            }
        }
        ++j;
    }
}

// Sorts the decoded children, stacks all but the nearest hit inner child and
// continues there, else pops.  Returns false when the walk is done.
__device__ __forceinline__ bool wide_next(float key[4], int val[4], float tmf, int &cur, int &sp, bool &overflow,
                                          LdsStack stk) {
    // sort the four (key, child) pairs ascending: 5 compare-exchanges
    auto cx = [&](int a, int b) {   // selects, not a branch per exchange
        const bool sw = key[b] < key[a];
        const float ka = key[a], kb = key[b];
        const int va = val[a], vb = val[b];
        key[a] = sw ? kb : ka;
        key[b] = sw ? ka : kb;
        val[a] = sw ? vb : va;
        val[b] = sw ? va : vb;
    };
    cx(0, 1);
    cx(2, 3);
    cx(0, 2);
    cx(1, 3);
    cx(1, 2);
#pragma unroll
    for (int k = 3; k >= 1; --k) {
        if (key[k] <= tmf) {
            if (sp < kStack) {
                stk.base[sp * stk.stride] = make_int2(val[k], __float_as_int(key[k]));
                ++sp;
            } else {
                overflow = true;
            }
        }
    }
    if (key[0] <= tmf) {
        cur = val[0];
        return true;
    }
    while (sp > 0) {
        --sp;
        const int2 e = stk.base[sp * stk.stride];
        if (__int_as_float(e.y) <= tmf) {
            cur = e.x;
            return true;
        }
    }
    return false;
}

// One visit with its leaves tested at once (the culling distance is then
// already the new best for the children stacked).
template <bool COUNT>
__device__ __forceinline__ bool wide_step(const TraceParams &P, const double *o, const double *d, int64_t skip,
                                          const CullRay &cr, float &tmf, Hit &h, int &cur, int &sp, bool &overflow,
                                          LdsStack stk, Counters &cnt) {
    float key[4];
    int val[4];
    Pending pd;
    wide_decode<COUNT>(P, cr, tmf, cur, key, val, pd, cnt);
    test_leaves<COUNT>(P, o, d, skip, tmf, h, pd, cnt);
    return wide_next(key, val, tmf, cur, sp, overflow, stk);
}

// Whether the segment [0, tmf] meets the box of every triangle (the binary
// tree's root box, tested as the escape-index walk tests it): if not, no
// node of either tree can hold a hit and the walk is skipped.
__device__ __forceinline__ bool meets_tree(const TraceParams &P, const CullRay &cr, float tmf) {
    const float ax = (P.tree_lo_f[0] - cr.ox) * cr.ix, bx = (P.tree_hi_f[0] - cr.ox) * cr.ix;
    const float ay = (P.tree_lo_f[1] - cr.oy) * cr.iy, by = (P.tree_hi_f[1] - cr.oy) * cr.iy;
    const float az = (P.tree_lo_f[2] - cr.oz) * cr.iz, bz = (P.tree_hi_f[2] - cr.oz) * cr.iz;
    const float tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), 0.0f));
    const float tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), tmf));
    return tn <= tf;
}

// Complete ordered walk; the result is always the exact closest hit
// (nearest t, lower id on ties): after a stack overflow the escape-index
// walk re-visits the whole tree with the best hit so far.
template <bool COUNT>
__device__ __forceinline__ void walk_wide(const TraceParams &P, const double *o, const double *d, int64_t skip,
                                          Hit &h, LdsStack stk, Counters &cnt) {
    const CullRay cr = make_cull(o, d);
    float tmf = cull_tmax(h.t);
    if (!meets_tree(P, cr, tmf)) return;
    int sp = 0, cur = 0;
    bool overflow = false;
    while (wide_step<COUNT>(P, o, d, skip, cr, tmf, h, cur, sp, overflow, stk, cnt)) {
    }
    if (overflow) walk_threaded<COUNT>(P, o, d, skip, cr, tmf, h, cnt);
}

// Face of a convex array: the cylinder of radius R about the y axis through
// (0, 0, -R), met from outside while moving towards the axis
// (b = (o_x, o_z + R).(d_x, d_z) < 0) at the nearer root
// t = c / (-b + sqrt(b^2 - a c)), a = d_x^2 + d_z^2, c = o_x^2 + o_z (o_z + 2R)
// (squared distance minus R^2 without cancellation).  +inf if missed.
__device__ __forceinline__ double probe_face(const TraceParams &P, const double *o, const double *d) {
    const double R = P.radius;
    const double aa = d[0] * d[0] + d[2] * d[2];
    const double b = o[0] * d[0] + (o[2] + R) * d[2];
    const double c = o[0] * o[0] + o[2] * (o[2] + 2.0 * R);
    const double disc = b * b - aa * c;
    if (!(b < 0.0) || aa == 0.0 || disc < 0.0) return INFINITY;
    const double t = c / (-b + sqrt(disc));
    return t > kEpsT ? t : INFINITY;
}

// Nearest exit through the box faces or, on a convex array, its face (face 6)
// (the starting candidate).  CONVEX = false: a kernel variant for linear arrays.
template <bool CONVEX = true>
__device__ __forceinline__ Hit box_exit(const TraceParams &P, const double *o, const double *d) {
    Hit h;
    h.t = INFINITY;
    h.face = -1;
    h.id = P.id_box;
    h.local = -1;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (d[i] == 0.0) continue;
        // face chosen first, one quotient per axis whatever the lane's sign
        const int fi = d[i] > 0.0 ? 3 + i : i;
        const double t = ((d[i] > 0.0 ? P.box[3 + i] : P.box[i]) - o[i]) / d[i];
        if (t < h.t) {
            h.t = t;
            h.face = fi;
        }
    }
    if (CONVEX && P.convex) {
        const double tp = probe_face(P, o, d);
        if (tp < h.t) {
            h.t = tp;
            h.face = 6;
        }
    }
    return h;
}

// Spheres and planes (tested before the triangles; the order does not
// matter: the nearest t wins, the lower id on ties).
__device__ __forceinline__ void analytic_hits(const TraceParams &P, const double *o, const double *d, int64_t skip,
                                              Hit &h) {
    for (int j = 0; j < P.n_sph; ++j) {
        double t0, t1;
        if (!sph_roots(P.sph + 4 * j, o, d, t0, t1)) continue;
        const double t = t0 > kEpsT ? t0 : t1;
        if (!(t > kEpsT)) continue;
        const int64_t id = P.id_sph0 + j;
        if (t < h.t || (t == h.t && id < h.id)) {
            h.t = t;
            h.id = id;
            h.local = j;
        }
    }
    for (int j = 0; j < P.n_pln; ++j) {
        const int64_t id = P.id_pln0 + j;
        if (id == skip) continue;
        double t;
        if (!pln_isect(P.pln + 4 * j, o, d, t) || !(t > kEpsT)) continue;
        if (t < h.t || (t == h.t && id < h.id)) {
            h.t = t;
            h.id = id;
            h.local = j;
        }
    }
}

// Nearest hit along (o, d), excluding the flat primitive `skip` (a
// triangle's slot in BVH order or a plane's id, -1 for none).
template <bool COUNT>
__device__ __forceinline__ Hit closest_hit(const TraceParams &P, const double *o, const double *d, int64_t skip,
                                           LdsStack stk, Counters &cnt) {
    Hit h = box_exit(P, o, d);
    // spheres and planes first: their nearest hit bounds the culling
    // distance of the tree walk from its first node (the result is the same
    // in any order: nearest t, lower id on ties)
    analytic_hits(P, o, d, skip, h);
    if (P.n_tnodes4 > 0) walk_wide<COUNT>(P, o, d, skip, h, stk, cnt);
    resolve_hit(P, h);
    return h;
}

}  // namespace
