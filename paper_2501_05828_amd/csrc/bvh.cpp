// Binned-SAH BVH builder producing a threaded (escape-index) layout.
#include "bvh.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace ur {
namespace {

constexpr int kBins = 16;

struct Box {
    double lo[3] = {INFINITY, INFINITY, INFINITY};
    double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    void grow(const double *l, const double *h) {
        for (int i = 0; i < 3; ++i) {
            lo[i] = std::min(lo[i], l[i]);
            hi[i] = std::max(hi[i], h[i]);
        }
    }
    void grow(const Box &b) { grow(b.lo, b.hi); }
    double area() const {
        if (lo[0] > hi[0]) return 0.0;
        const double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
        return 2.0 * (dx * dy + dy * dz + dz * dx);
    }
};

float round_down(double x) {
    float f = (float)x;
    if ((double)f > x) f = std::nextafter(f, -INFINITY);
    return std::nextafter(f, -INFINITY);
}

float round_up(double x) {
    float f = (float)x;
    if ((double)f < x) f = std::nextafter(f, INFINITY);
    return std::nextafter(f, INFINITY);
}

struct Builder {
    const std::vector<PrimBounds> &prims;
    std::vector<int> idx;
    std::vector<double> cen;   // 3 per primitive
    int leaf_max;
    double dilate;
    BvhResult res;

    Builder(const std::vector<PrimBounds> &p, int lm, double dl) : prims(p), leaf_max(lm), dilate(dl) {
        idx.resize(p.size());
        cen.resize(3 * p.size());
        for (size_t i = 0; i < p.size(); ++i) {
            idx[i] = (int)i;
            for (int k = 0; k < 3; ++k) cen[3 * i + k] = 0.5 * (p[i].lo[k] + p[i].hi[k]);
        }
    }

    void set_box(BvhNode &n, const Box &b) const {
        for (int k = 0; k < 3; ++k) {
            n.lo[k] = round_down(b.lo[k] - dilate);
            n.hi[k] = round_up(b.hi[k] + dilate);
        }
    }

    static void set_int(float &f, int v) { std::memcpy(&f, &v, sizeof(int)); }

    void make_leaf(int node, int begin, int end) {
        set_int(res.nodes[node].hi[3], (begin << 4) | (end - begin));
    }

    void emit(int begin, int end, int depth) {
        res.max_depth = std::max(res.max_depth, depth);
        const int node = (int)res.nodes.size();
        res.nodes.push_back(BvhNode{});
        Box b, cb;
        for (int i = begin; i < end; ++i) {
            b.grow(prims[idx[i]].lo, prims[idx[i]].hi);
            cb.grow(&cen[3 * idx[i]], &cen[3 * idx[i]]);
        }
        set_box(res.nodes[node], b);
        set_int(res.nodes[node].hi[3], -1);
        const int n = end - begin;
        int mid = -1;
        if (n > 1) {
            int axis = 0;
            for (int k = 1; k < 3; ++k)
                if (cb.hi[k] - cb.lo[k] > cb.hi[axis] - cb.lo[axis]) axis = k;
            const double ext = cb.hi[axis] - cb.lo[axis];
            if (ext > 0.0) {
                Box bins[kBins];
                int cnt[kBins] = {0};
                auto bin_of = [&](int p) {
                    int k = (int)((cen[3 * p + axis] - cb.lo[axis]) / ext * kBins);
                    return std::min(kBins - 1, std::max(0, k));
                };
                for (int i = begin; i < end; ++i) {
                    const int k = bin_of(idx[i]);
                    ++cnt[k];
                    bins[k].grow(prims[idx[i]].lo, prims[idx[i]].hi);
                }
                double best = INFINITY;
                int best_k = -1;
                Box left;
                int nl = 0;
                for (int k = 0; k < kBins - 1; ++k) {
                    left.grow(bins[k]);
                    nl += cnt[k];
                    Box right;
                    int nr = 0;
                    for (int j = k + 1; j < kBins; ++j) {
                        right.grow(bins[j]);
                        nr += cnt[j];
                    }
                    if (nl == 0 || nr == 0) continue;
                    const double c = left.area() * nl + right.area() * nr;
                    if (c < best) {
                        best = c;
                        best_k = k;
                    }
                }
                const double leaf_cost = b.area() * n;
                const double split_cost = b.area() * 1.0 + best;   // one traversal step per split
                if (best_k >= 0 && (n > leaf_max || split_cost < leaf_cost)) {
                    int *m = std::partition(idx.data() + begin, idx.data() + end,
                                            [&](int p) { return bin_of(p) <= best_k; });
                    mid = (int)(m - idx.data());
                }
            }
            if (mid < 0 && n > leaf_max) {   // coincident centroids: split by index
                mid = begin + n / 2;
                int axis2 = axis;
                std::nth_element(idx.data() + begin, idx.data() + mid, idx.data() + end,
                                 [&](int a, int c) { return cen[3 * a + axis2] < cen[3 * c + axis2]; });
            }
        }
        if (mid < 0) {
            make_leaf(node, begin, end);
        } else {
            emit(begin, mid, depth + 1);
            emit(mid, end, depth + 1);
        }
        set_int(res.nodes[node].lo[3], (int)res.nodes.size());
    }
};

}  // namespace

namespace {

int as_int(float f) {
    int v;
    std::memcpy(&v, &f, sizeof(int));
    return v;
}

struct Collapser {
    const std::vector<BvhNode> &n2;
    std::vector<Bvh4Node> out;

    bool leaf(int i) const { return as_int(n2[i].hi[3]) >= 0; }
    int second_child(int i) const { return as_int(n2[i + 1].lo[3]); }
    double area(int i) const {
        const double dx = (double)n2[i].hi[0] - n2[i].lo[0], dy = (double)n2[i].hi[1] - n2[i].lo[1],
                     dz = (double)n2[i].hi[2] - n2[i].lo[2];
        return dx * dy + dy * dz + dz * dx;
    }

    void set_child(int node, int k, int src, int child) {
        Bvh4Node &q = out[node];
        q.lo_x[k] = n2[src].lo[0];
        q.lo_y[k] = n2[src].lo[1];
        q.lo_z[k] = n2[src].lo[2];
        q.hi_x[k] = n2[src].hi[0];
        q.hi_y[k] = n2[src].hi[1];
        q.hi_z[k] = n2[src].hi[2];
        q.child[k] = child;
    }

    int make_node() {
        Bvh4Node q;
        for (int k = 0; k < 4; ++k) {
            q.lo_x[k] = q.hi_x[k] = q.lo_y[k] = q.hi_y[k] = q.lo_z[k] = q.hi_z[k] = 1e30f;
            q.child[k] = -1;
            q.pad[k] = 0;
        }
        out.push_back(q);
        return (int)out.size() - 1;
    }

    // r: inner node of the binary tree
    int build(int r) {
        const int node = make_node();
        std::vector<int> ch = {r + 1, second_child(r)};
        while (ch.size() < 4) {
            int best = -1;
            double ba = -1.0;
            for (size_t k = 0; k < ch.size(); ++k)
                if (!leaf(ch[k]) && area(ch[k]) > ba) {
                    ba = area(ch[k]);
                    best = (int)k;
                }
            if (best < 0) break;
            const int c = ch[best];
            ch.erase(ch.begin() + best);
            ch.push_back(c + 1);
            ch.push_back(second_child(c));
        }
        for (size_t k = 0; k < ch.size(); ++k) {
            if (leaf(ch[k])) {
                set_child(node, (int)k, ch[k], ~as_int(n2[ch[k]].hi[3]));
            } else {
                const int sub = build(ch[k]);
                set_child(node, (int)k, ch[k], sub);
            }
        }
        return node;
    }
};

}  // namespace

std::vector<Bvh4Node> collapse_bvh4(const std::vector<BvhNode> &nodes) {
    Collapser c{nodes, {}};
    if (nodes.empty()) return {};
    if (c.leaf(0)) {
        const int node = c.make_node();
        c.set_child(node, 0, 0, ~as_int(nodes[0].hi[3]));
    } else {
        c.build(0);
    }
    return std::move(c.out);
}

namespace {

// fl(o + q * 2^(e - 127)) in FP32: the product is exact, the sum rounds once
float decode1(float o, int q, int e) {
    volatile float prod = std::ldexp((float)q, e - 127);
    volatile float sum = o + prod;
    return sum;
}

}  // namespace

void decode_bvh4q(const Bvh4NodeQ &n, int k, float lo[3], float hi[3]) {
    int ebits;
    std::memcpy(&ebits, &n.org[3], sizeof(int));
    for (int a = 0; a < 3; ++a) {
        const int e = (ebits >> (8 * a)) & 255;
        lo[a] = decode1(n.org[a], n.q[4 * a + k], e);
        hi[a] = decode1(n.org[a], n.q[12 + 4 * a + k], e);
    }
}

std::vector<Bvh4NodeQ> quantize_bvh4(const std::vector<Bvh4Node> &nodes) {
    std::vector<Bvh4NodeQ> out(nodes.size());
    for (size_t i = 0; i < nodes.size(); ++i) {
        const Bvh4Node &n = nodes[i];
        Bvh4NodeQ &q = out[i];
        std::memset(&q, 0, sizeof(q));
        const float *L[3] = {n.lo_x, n.lo_y, n.lo_z}, *H[3] = {n.hi_x, n.hi_y, n.hi_z};
        int ebits = 0;
        for (int a = 0; a < 3; ++a) {
            float ulo = INFINITY, uhi = -INFINITY;
            for (int k = 0; k < 4; ++k)
                if (n.child[k] != -1) {
                    ulo = std::min(ulo, L[a][k]);
                    uhi = std::max(uhi, H[a][k]);
                }
            if (!(ulo <= uhi)) ulo = uhi = 0.0f;   // no children (never for a built tree)
            const float o = std::nextafter(ulo, -INFINITY);
            q.org[a] = o;
            // smallest step 2^(e-127) with 254 steps covering the extent (one
            // step of room for the outward rounding)
            int e = 1;
            while (e < 254 && (double)std::ldexp(1.0f, e - 127) * 254.0 < (double)uhi - (double)o) ++e;
            ebits |= e << (8 * a);
            for (int k = 0; k < 4; ++k) {
                if (n.child[k] == -1) {
                    q.q[4 * a + k] = 255;
                    q.q[12 + 4 * a + k] = 0;
                    continue;
                }
                const double s = std::ldexp(1.0, e - 127);
                int lo_q = (int)std::floor(((double)L[a][k] - (double)o) / s);
                int hi_q = (int)std::ceil(((double)H[a][k] - (double)o) / s);
                lo_q = std::max(0, std::min(255, lo_q));
                hi_q = std::max(0, std::min(255, hi_q));
                while (lo_q > 0 && decode1(o, lo_q, e) > L[a][k]) --lo_q;
                while (hi_q < 255 && decode1(o, hi_q, e) < H[a][k]) ++hi_q;
                q.q[4 * a + k] = (unsigned char)lo_q;
                q.q[12 + 4 * a + k] = (unsigned char)hi_q;
            }
        }
        std::memcpy(&q.org[3], &ebits, sizeof(int));
        for (int k = 0; k < 4; ++k) q.child[k] = n.child[k];
    }
    return out;
}

BvhResult build_bvh(const std::vector<PrimBounds> &prims, int leaf_max, double dilate) {
    Builder b(prims, std::min(15, std::max(1, leaf_max)), dilate);
    if (!prims.empty()) b.emit(0, (int)prims.size(), 0);
    b.res.order = b.idx;
    return std::move(b.res);
}

}  // namespace ur
