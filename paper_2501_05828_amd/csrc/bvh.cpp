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

BvhResult build_bvh(const std::vector<PrimBounds> &prims, int leaf_max, double dilate) {
    Builder b(prims, std::min(15, std::max(1, leaf_max)), dilate);
    if (!prims.empty()) b.emit(0, (int)prims.size(), 0);
    b.res.order = b.idx;
    return std::move(b.res);
}

}  // namespace ur
