// Host self-check of the BVH builder used by the HIP library: structure
// (skip indices, leaf ranges, containment) and conservative FP32 culling.
// The traversal loops mirror the device's stackless escape-index walk and
// its ordered four-wide walk with a bounded stack (falling back to the
// escape-index walk on overflow); the reference is brute-force FP64.
// usage: bvh_selfcheck <prims.bin> <n> <kind: tri|pt> <dilate> <radius> <n_rays> <seed>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "bvh.h"

using namespace ur;

static int as_int(float f) { int v; std::memcpy(&v, &f, 4); return v; }

static bool tri_isect(const double *v, const double *o, const double *d, double &t) {
    double e1[3], e2[3], p[3], tv[3], q[3];
    for (int i = 0; i < 3; ++i) { e1[i] = v[3 + i] - v[i]; e2[i] = v[6 + i] - v[i]; tv[i] = o[i] - v[i]; }
    p[0] = d[1] * e2[2] - d[2] * e2[1]; p[1] = d[2] * e2[0] - d[0] * e2[2]; p[2] = d[0] * e2[1] - d[1] * e2[0];
    double det = e1[0] * p[0] + e1[1] * p[1] + e1[2] * p[2];
    if (det == 0) return false;
    double inv = 1 / det, u = (tv[0] * p[0] + tv[1] * p[1] + tv[2] * p[2]) * inv;
    if (u < 0 || u > 1) return false;
    q[0] = tv[1] * e1[2] - tv[2] * e1[1]; q[1] = tv[2] * e1[0] - tv[0] * e1[2]; q[2] = tv[0] * e1[1] - tv[1] * e1[0];
    double vv = (d[0] * q[0] + d[1] * q[1] + d[2] * q[2]) * inv;
    if (vv < 0 || u + vv > 1) return false;
    t = (e2[0] * q[0] + e2[1] * q[1] + e2[2] * q[2]) * inv;
    return true;
}

static float safe_inv(double d) { double a = std::fabs(d) < 1e-20 ? std::copysign(1e-20, d) : d; return (float)(1.0 / a); }

static bool slab(const BvhNode &n, const float *o, const float *inv, float tmax) {
    float tn = 0.0f, tf = tmax;
    for (int k = 0; k < 3; ++k) {
        float a = (n.lo[k] - o[k]) * inv[k], b = (n.hi[k] - o[k]) * inv[k];
        tn = std::fmax(tn, std::fmin(a, b));
        tf = std::fmin(tf, std::fmax(a, b));
    }
    return tn <= tf;
}

int main(int argc, char **argv) {
    if (argc < 8) return 2;
    FILE *f = std::fopen(argv[1], "rb");
    long n = std::atol(argv[2]);
    bool tri = std::strcmp(argv[3], "tri") == 0;
    double dil = std::atof(argv[4]), rad = std::atof(argv[5]);
    long nrays = std::atol(argv[6]);
    int per = tri ? 9 : 4;
    std::vector<double> P(n * per);
    if (!f || std::fread(P.data(), 8, P.size(), f) != P.size()) { std::puts("read error"); return 2; }
    std::fclose(f);
    std::vector<PrimBounds> pb(n);
    for (long i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            if (tri) {
                pb[i].lo[k] = std::fmin(P[9 * i + k], std::fmin(P[9 * i + 3 + k], P[9 * i + 6 + k]));
                pb[i].hi[k] = std::fmax(P[9 * i + k], std::fmax(P[9 * i + 3 + k], P[9 * i + 6 + k]));
            } else {
                pb[i].lo[k] = P[4 * i + k] - rad;
                pb[i].hi[k] = P[4 * i + k] + rad;
            }
        }
    const int leaf_max = argc > 8 ? std::atoi(argv[8]) : (tri ? 1 : 8);
    BvhResult r = build_bvh(pb, leaf_max, dil);
    const int nn = (int)r.nodes.size();
    std::vector<int> seen(n, 0), slot_of(n, -1);
    for (long k = 0; k < n; ++k) slot_of[r.order[k]] = (int)k;
    // structure
    for (int i = 0; i < nn; ++i) {
        const BvhNode &b = r.nodes[i];
        int skip = as_int(b.lo[3]), leaf = as_int(b.hi[3]);
        if (skip <= i || skip > nn) { std::printf("bad skip %d at %d\n", skip, i); return 1; }
        for (int k = 0; k < 3; ++k) if (!(b.lo[k] <= b.hi[k])) { std::puts("empty box"); return 1; }
        if (leaf >= 0) {
            int first = leaf >> 4, cnt = leaf & 15;
            if (skip != i + 1 || cnt < 1 || first < 0 || first + cnt > n) { std::puts("bad leaf"); return 1; }
            for (int s = first; s < first + cnt; ++s) {
                seen[r.order[s]]++;
                for (int k = 0; k < 3; ++k)
                    if (!((double)b.lo[k] < pb[r.order[s]].lo[k] - 0.9 * dil && (double)b.hi[k] > pb[r.order[s]].hi[k] + 0.9 * dil)) {
                        std::puts("leaf box does not contain primitive"); return 1;
                    }
            }
        } else {
            // children: i+1 .. skip-1 ; every descendant box within this box
            for (int j = i + 1; j < skip; ++j)
                for (int k = 0; k < 3; ++k)
                    if (r.nodes[j].lo[k] < b.lo[k] || r.nodes[j].hi[k] > b.hi[k]) { std::puts("child outside parent"); return 1; }
            if (skip == i + 1) { std::puts("inner node without children"); return 1; }
        }
    }
    for (long i = 0; i < n; ++i) if (seen[i] != 1) { std::printf("prim %ld seen %d times\n", i, seen[i]); return 1; }
    if (nn && as_int(r.nodes[0].lo[3]) != nn) { std::puts("root skip != n_nodes"); return 1; }
    // culling vs brute force
    double lo[3] = {1e30, 1e30, 1e30}, hi[3] = {-1e30, -1e30, -1e30};
    for (long i = 0; i < n; ++i) for (int k = 0; k < 3; ++k) { lo[k] = std::fmin(lo[k], pb[i].lo[k]); hi[k] = std::fmax(hi[k], pb[i].hi[k]); }
    std::mt19937_64 g(std::atol(argv[7]));
    std::uniform_real_distribution<double> U(0, 1);
    std::normal_distribution<double> N(0, 1);
    long missed = 0, visits = 0;
    for (long q = 0; q < nrays; ++q) {
        double o[3], d[3];
        for (int k = 0; k < 3; ++k) o[k] = lo[k] + (hi[k] - lo[k]) * (1.4 * U(g) - 0.2);
        double l = 0; for (int k = 0; k < 3; ++k) { d[k] = N(g); l += d[k] * d[k]; }
        l = std::sqrt(l); for (int k = 0; k < 3; ++k) d[k] /= l;
        if (q % 7 == 0) { d[0] = 0.0; d[1] = 0.0; d[2] = 1.0; }
        double tmax = 0.05 + 0.1 * U(g);
        // brute force set of primitives the FP64 test accepts on [0, tmax)
        std::vector<int> want;
        for (long i = 0; i < n; ++i) {
            if (tri) { double t; if (tri_isect(&P[9 * i], o, d, t) && t > 1e-9 && t < tmax) want.push_back((int)i); }
            else {
                double p[3] = {P[4 * i] - o[0], P[4 * i + 1] - o[1], P[4 * i + 2] - o[2]};
                double s = p[0] * d[0] + p[1] * d[1] + p[2] * d[2];
                if (!(s >= 0 && s < tmax)) continue;
                double pp[3] = {p[0] - s * d[0], p[1] - s * d[1], p[2] - s * d[2]};
                if (pp[0] * pp[0] + pp[1] * pp[1] + pp[2] * pp[2] <= rad * rad) want.push_back((int)i);
            }
        }
        float of[3] = {(float)o[0], (float)o[1], (float)o[2]}, inv[3] = {safe_inv(d[0]), safe_inv(d[1]), safe_inv(d[2])};
        float tmf = (float)(tmax * (1.0 + 1e-6) + 1e-6);
        std::vector<char> reached(n, 0);
        int i = 0;
        while (i < nn) {
            const BvhNode &b = r.nodes[i];
            ++visits;
            if (!slab(b, of, inv, tmf)) { i = as_int(b.lo[3]); continue; }
            int leaf = as_int(b.hi[3]);
            if (leaf < 0) { ++i; continue; }
            for (int s = leaf >> 4; s < (leaf >> 4) + (leaf & 15); ++s) reached[r.order[s]] = 1;
            i = as_int(b.lo[3]);
        }
        for (int w : want) if (!reached[w]) ++missed;
    }
    std::printf("nodes %d depth %d visits/ray %.1f missed %ld\n", nn, r.max_depth, nrays ? (double)visits / nrays : 0.0, missed);
    if (missed) return 1;
    if (!tri) return 0;
    // ---- four-wide layout: structure
    std::vector<Bvh4Node> q4 = collapse_bvh4(r.nodes);
    std::vector<int> seen4(n, 0);
    std::vector<int> todo = {0};
    int n4 = 0;
    while (!todo.empty()) {
        const int i = todo.back();
        todo.pop_back();
        ++n4;
        const Bvh4Node &b = q4[i];
        for (int k = 0; k < 4; ++k) {
            const int c = b.child[k];
            if (c == -1) continue;
            if (c >= 0) {
                if (c <= i || c >= (int)q4.size()) { std::puts("bad bvh4 child"); return 1; }
                todo.push_back(c);
            } else {
                const int code = ~c, first = code >> 4, cnt = code & 15;
                if (cnt < 1 || first + cnt > n) { std::puts("bad bvh4 leaf"); return 1; }
                for (int s = first; s < first + cnt; ++s) {
                    seen4[r.order[s]]++;
                    const PrimBounds &p = pb[r.order[s]];
                    if (!(b.lo_x[k] <= p.lo[0] && b.lo_y[k] <= p.lo[1] && b.lo_z[k] <= p.lo[2] && b.hi_x[k] >= p.hi[0] &&
                          b.hi_y[k] >= p.hi[1] && b.hi_z[k] >= p.hi[2])) { std::puts("bvh4 leaf box"); return 1; }
                }
            }
        }
    }
    if (n4 != (int)q4.size()) { std::puts("unreachable bvh4 nodes"); return 1; }
    // quantised nodes: every decoded child box contains the FP32 box
    const std::vector<Bvh4NodeQ> qq = collapse_bvh4(r.nodes).empty() ? std::vector<Bvh4NodeQ>() : quantize_bvh4(q4);
    for (size_t i = 0; i < qq.size(); ++i)
        for (int k = 0; k < 4; ++k) {
            if (q4[i].child[k] == -1) continue;
            float dl[3], dh[3];
            decode_bvh4q(qq[i], k, dl, dh);
            const float bl[3] = {q4[i].lo_x[k], q4[i].lo_y[k], q4[i].lo_z[k]}, bh[3] = {q4[i].hi_x[k], q4[i].hi_y[k], q4[i].hi_z[k]};
            for (int a = 0; a < 3; ++a)
                if (!(dl[a] <= bl[a] && dh[a] >= bh[a]) || qq[i].child[k] != q4[i].child[k]) {
                    std::printf("quantised box %zu/%d axis %d does not contain the node box\n", i, k, a); return 1;
                }
            int ebits;
            std::memcpy(&ebits, &qq[i].org[3], sizeof(int));
            for (int a = 0; a < 3; ++a) {   // and stays within three steps of it
                const double step = std::ldexp(1.0, ((ebits >> (8 * a)) & 255) - 127);
                if ((double)dh[a] - dl[a] > (double)bh[a] - bl[a] + 3.0 * step) { std::puts("quantised box too loose"); return 1; }
            }
        }
    for (long i = 0; i < n; ++i) if (seen4[i] != 1) { std::printf("bvh4: prim %ld seen %d times\n", i, seen4[i]); return 1; }
    // ---- ordered closest hit with a 16-entry stack vs brute force
    std::mt19937_64 g2(std::atol(argv[7]) + 1);
    long wrong = 0, overflows = 0, v4 = 0;
    for (long q = 0; q < nrays; ++q) {
        double o[3], d[3];
        for (int k = 0; k < 3; ++k) o[k] = lo[k] + (hi[k] - lo[k]) * (1.4 * U(g2) - 0.2);
        double l = 0; for (int k = 0; k < 3; ++k) { d[k] = N(g2); l += d[k] * d[k]; }
        l = std::sqrt(l); for (int k = 0; k < 3; ++k) d[k] /= l;
        const double tmax = 0.05 + 0.1 * U(g2);
        double tb = tmax; int hb = -1;
        for (long i = 0; i < n; ++i) {
            double t;
            if (tri_isect(&P[9 * i], o, d, t) && t > 1e-9 && (t < tb || (t == tb && i < hb))) { tb = t; hb = (int)i; }
        }
        double tg = tmax; int hg = -1;
        auto test_leaf = [&](int code, float &tmf) {
            for (int s = code >> 4; s < (code >> 4) + (code & 15); ++s) {
                double t; const int id = r.order[s];
                if (tri_isect(&P[9 * id], o, d, t) && t > 1e-9 && (t < tg || (t == tg && id < hg))) {
                    tg = t; hg = id; tmf = (float)(t * (1.0 + 1e-6) + 1e-6);
                }
            }
        };
        float of[3] = {(float)o[0], (float)o[1], (float)o[2]}, inv[3] = {safe_inv(d[0]), safe_inv(d[1]), safe_inv(d[2])};
        float tmf = (float)(tmax * (1.0 + 1e-6) + 1e-6);
        int stk_n[16]; float stk_t[16]; int sp = 0, cur = 0; bool overflow = false;
        while (true) {
            const Bvh4Node &b = q4[cur];
            ++v4;
            float tn[4]; bool hit[4];
            for (int k = 0; k < 4; ++k) {
                float bl[3], bh[3];
                decode_bvh4q(qq[cur], k, bl, bh);
                float a0 = 0.0f, a1 = tmf;
                for (int j = 0; j < 3; ++j) {
                    const float x0 = (bl[j] - of[j]) * inv[j], x1 = (bh[j] - of[j]) * inv[j];
                    a0 = std::fmax(a0, std::fmin(x0, x1)); a1 = std::fmin(a1, std::fmax(x0, x1));
                }
                tn[k] = a0; hit[k] = a0 <= a1 && b.child[k] != -1;
            }
            for (int k = 0; k < 4; ++k) if (hit[k] && b.child[k] < -1) test_leaf(~b.child[k], tmf);
            int ord[4], m = 0;
            for (int k = 0; k < 4; ++k) if (hit[k] && b.child[k] >= 0 && tn[k] <= tmf) ord[m++] = k;
            for (int a = 1; a < m; ++a) for (int c = a; c > 0 && tn[ord[c]] < tn[ord[c - 1]]; --c) std::swap(ord[c], ord[c - 1]);
            if (m > 0) {
                for (int a = m - 1; a >= 1; --a) {
                    if (sp < 16) { stk_n[sp] = b.child[ord[a]]; stk_t[sp] = tn[ord[a]]; ++sp; }
                    else overflow = true;
                }
                cur = b.child[ord[0]];
                continue;
            }
            bool found = false;
            while (sp > 0) { --sp; if (stk_t[sp] <= tmf) { cur = stk_n[sp]; found = true; break; } }
            if (!found) break;
        }
        if (overflow) {
            ++overflows;
            int i = 0;
            while (i < nn) {
                const BvhNode &bb = r.nodes[i];
                if (!slab(bb, of, inv, tmf)) { i = as_int(bb.lo[3]); continue; }
                const int leaf = as_int(bb.hi[3]);
                if (leaf < 0) { ++i; continue; }
                test_leaf(leaf, tmf);
                i = as_int(bb.lo[3]);
            }
        }
        if (hg != hb || tg != tb) ++wrong;
    }
    std::printf("bvh4 nodes %zu visits/ray %.2f overflows %ld wrong %ld\n", q4.size(), nrays ? (double)v4 / nrays : 0.0,
                overflows, wrong);
    return wrong ? 1 : 0;
}
