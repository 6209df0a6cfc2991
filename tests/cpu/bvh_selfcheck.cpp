// Host self-check of the BVH builder used by the HIP library: structure
// (skip indices, leaf ranges, containment) and conservative FP32 culling.
// The traversal loop mirrors the device's stackless escape-index walk; the
// reference is a brute-force FP64 closest hit.
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
    BvhResult r = build_bvh(pb, tri ? 4 : 8, dil);
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
    return missed ? 1 : 0;
}
