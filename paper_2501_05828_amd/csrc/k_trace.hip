// Full-path Monte Carlo ultrasound ray tracing on gfx950 (UltraRay, arXiv
// 2501.05828, Sec. 2.2-2.3).
//
// One lane traces one primary ray through all of its segments.  Decisive
// state (origin, direction, weight, time, path length) is FP64, and every
// discrete decision -- closest hit and its tie-break, capsule inclusion of a
// scatterer, receiving element, reflect-or-transmit, receive cut-off, time
// bin -- is taken in FP64, so the device reproduces the FP64 reference
// estimator path by path.  FP32 is used only to cull bounding boxes, whose
// extents are dilated and rounded outward so culling never rejects a
// primitive the FP64 test would accept.
//
// Acceleration structures are threaded (escape-index) BVHs in depth-first
// order: traversal needs no stack, so the closest-hit query, the scatterer
// capsule query and the secondary-ray crossing query nest without any
// per-lane stack memory.
#include "ur_internal.h"
#include "../../include/ultraray.h"

namespace {
using namespace ur;

struct Counters {
    uint32_t v[kNumStats];
};
enum {
    C_RAYS, C_SEGMENTS, C_REFLECT, C_TRANSMIT, C_TIR, C_SCAT_EVENTS, C_NEE_ZERO, C_NEE_CAST, C_NEE_BLOCKED,
    C_DIRECT, C_RECORDS, C_DROPPED, C_EDGE, C_TERM_BOX, C_TERM_BOUNCE, C_TERM_TIME, C_TERM_PATH, C_MISMATCH,
    C_TRI_NODES, C_TRI_TESTS, C_SCAT_NODES, C_SCAT_TESTS, C_SHADOW_NODES, C_SHADOW_TRI_TESTS
};

#define CNT(k)                  \
    do {                        \
        if constexpr (COUNT)    \
            ++cnt.v[k];         \
    } while (0)

// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with the key bumped by the Weyl constants.
__device__ __forceinline__ void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                                       uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// counter = (ray, element | tx << 16, segment | purpose << 16, k)
__device__ __forceinline__ void draw(const TraceParams &P, uint32_t ray, int e, int tx, int seg, uint32_t purpose,
                                     uint32_t k, uint32_t out[4]) {
    philox(ray, (uint32_t)e | ((uint32_t)tx << 16), (uint32_t)seg | (purpose << 16), k, P.key0, P.key1, out);
}

__device__ __forceinline__ double u01(uint32_t x) { return ((double)x + 0.5) * 0x1p-32; }

__device__ __forceinline__ double dot3(const double *a, const double *b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// ------------------------------------------------------------- FP32 culling
struct CullRay {
    float ox, oy, oz, ix, iy, iz;
};

__device__ __forceinline__ float safe_inv(double d) {
    const double a = fabs(d) < 1e-20 ? copysign(1e-20, d) : d;
    return (float)(1.0 / a);
}

__device__ __forceinline__ CullRay make_cull(const double *o, const double *d) {
    CullRay c;
    c.ox = (float)o[0];
    c.oy = (float)o[1];
    c.oz = (float)o[2];
    c.ix = safe_inv(d[0]);
    c.iy = safe_inv(d[1]);
    c.iz = safe_inv(d[2]);
    return c;
}

// conservative upper bound of an FP64 ray parameter for the FP32 box test
__device__ __forceinline__ float cull_tmax(double t) { return (float)(t * (1.0 + 1e-6) + 1e-6); }

struct Node {
    float4 lo, hi;
};

__device__ __forceinline__ Node load_node(const BvhNode *nodes, int i) {
    const float4 *p = reinterpret_cast<const float4 *>(nodes + i);
    return Node{p[0], p[1]};
}

__device__ __forceinline__ bool slab(const Node &n, const CullRay &r, float tmax) {
    const float tx0 = (n.lo.x - r.ox) * r.ix, tx1 = (n.hi.x - r.ox) * r.ix;
    const float ty0 = (n.lo.y - r.oy) * r.iy, ty1 = (n.hi.y - r.oy) * r.iy;
    const float tz0 = (n.lo.z - r.oz) * r.iz, tz1 = (n.hi.z - r.oz) * r.iz;
    const float tn = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.0f));
    const float tf = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), tmax));
    return tn <= tf;
}

__device__ __forceinline__ int node_skip(const Node &n) { return __float_as_int(n.lo.w); }
__device__ __forceinline__ int node_leaf(const Node &n) { return __float_as_int(n.hi.w); }

// ---------------------------------------------------------- FP64 primitives
// Moller-Trumbore with precomputed edges e1 = v1 - v0, e2 = v2 - v0.
__device__ __forceinline__ bool tri_isect(const double *tr, const double *o, const double *d, double &t) {
    const double *v0 = tr, *e1 = tr + 3, *e2 = tr + 6;
    const double p0 = d[1] * e2[2] - d[2] * e2[1];
    const double p1 = d[2] * e2[0] - d[0] * e2[2];
    const double p2 = d[0] * e2[1] - d[1] * e2[0];
    const double det = e1[0] * p0 + e1[1] * p1 + e1[2] * p2;
    if (det == 0.0) return false;
    const double inv = 1.0 / det;
    const double t0 = o[0] - v0[0], t1 = o[1] - v0[1], t2 = o[2] - v0[2];
    const double u = (t0 * p0 + t1 * p1 + t2 * p2) * inv;
    if (u < 0.0 || u > 1.0) return false;
    const double q0 = t1 * e1[2] - t2 * e1[1];
    const double q1 = t2 * e1[0] - t0 * e1[2];
    const double q2 = t0 * e1[1] - t1 * e1[0];
    const double v = (d[0] * q0 + d[1] * q1 + d[2] * q2) * inv;
    if (v < 0.0 || u + v > 1.0) return false;
    t = (e2[0] * q0 + e2[1] * q1 + e2[2] * q2) * inv;
    return true;
}

__device__ __forceinline__ void tri_normal(const double *tr, double *n) {
    const double *e1 = tr + 3, *e2 = tr + 6;
    n[0] = e1[1] * e2[2] - e1[2] * e2[1];
    n[1] = e1[2] * e2[0] - e1[0] * e2[2];
    n[2] = e1[0] * e2[1] - e1[1] * e2[0];
    const double l = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    n[0] /= l;
    n[1] /= l;
    n[2] /= l;
}

__device__ __forceinline__ bool sph_roots(const double *s, const double *o, const double *d, double &t0,
                                          double &t1) {
    const double oc[3] = {o[0] - s[0], o[1] - s[1], o[2] - s[2]};
    const double b = dot3(oc, d);
    const double c = dot3(oc, oc) - s[3] * s[3];
    const double disc = b * b - c;
    if (disc < 0.0) return false;
    const double sq = sqrt(disc);
    t0 = -b - sq;
    t1 = -b + sq;
    return true;
}

__device__ __forceinline__ bool pln_isect(const double *p, const double *o, const double *d, double &t) {
    const double den = dot3(p, d);
    if (den == 0.0) return false;
    t = (p[3] - dot3(p, o)) / den;
    return true;
}

// Transmitted intensity fraction 1 - A_r^2 (Eqs. 8, 11) of a straight crossing.
__device__ __forceinline__ double transmit_fraction(double z1, double z2, double cos_r) {
    const double eta = z1 / z2;
    const double rad = 1.0 - eta * eta * (1.0 - cos_r * cos_r);
    if (rad < 0.0) return 0.0;
    const double cos_t = sqrt(rad);
    const double den = z1 * cos_r + z2 * cos_t;
    if (den == 0.0) return 0.0;
    const double A = (z1 * cos_r - z2 * cos_t) / den;
    return 1.0 - A * A;
}

// Receive directivity, Eq. 13.
__device__ __forceinline__ double directivity(double al, double am, double ac) {
    al = fabs(al);
    if (al > ac) return 0.0;
    if (al <= am) return 1.0;
    return (ac - al) / (ac - am);
}

// Equal-area square -> hemisphere map: Shirley-Chiu concentric disk, then
// the area-preserving lift z = 1 - r^2, xy scaled by sqrt(2 - r^2).
__device__ __forceinline__ void hemisphere(double a, double b, double *d) {
    const double sa = 2.0 * a - 1.0, sb = 2.0 * b - 1.0;
    if (sa == 0.0 && sb == 0.0) {
        d[0] = 0.0;
        d[1] = 0.0;
        d[2] = 1.0;
        return;
    }
    double r, phi;
    if (fabs(sa) > fabs(sb)) {
        r = sa;
        phi = (M_PI / 4.0) * (sb / sa);
    } else {
        r = sb;
        phi = M_PI / 2.0 - (M_PI / 4.0) * (sa / sb);
    }
    const double r2 = r * r, sc = sqrt(2.0 - r2);
    double sp, cp;
    sincos(phi, &sp, &cp);
    d[0] = r * cp * sc;
    d[1] = r * sp * sc;
    d[2] = 1.0 - r2;
}

// ------------------------------------------------------------------ records
template <bool LOG>
__device__ __forceinline__ void log_event(const EventLog &L, int kind, int tx, int elem, int seg, int64_t id,
                                          double t, double v, const double *p) {
    if constexpr (LOG) {
        const unsigned long long k = atomicAdd(L.count, 1ull);
        if ((int64_t)k < L.cap) {
            ur_event *E = (ur_event *)L.events + k;
            E->kind = kind;
            E->tx = tx;
            E->elem = elem;
            E->seg = seg;
            E->id = id;
            E->t = t;
            E->value = v;
            E->x = p[0];
            E->y = p[1];
            E->z = p[2];
        }
    }
}

// Bins one arriving contribution into ch_raw with device-scope float atomics.
template <bool COUNT, bool LOG>
__device__ __forceinline__ void record(const TraceParams &P, const EventLog &L, Counters &cnt, int kind, int tx,
                                       int e, int seg, int64_t id, double t, double v, const double *p) {
    log_event<LOG>(L, kind, tx, e, seg, id, t, v, p);
    if (!(t < P.t_max) || t < 0.0) {
        CNT(C_DROPPED);
        return;
    }
    CNT(C_RECORDS);
    const double x = t * P.fs;
    if constexpr (COUNT) {
        const double fr = x - floor(x);
        if (fr < 1e-5 || fr > 1.0 - 1e-5) ++cnt.v[C_EDGE];
    }
    float *ch = P.ch_raw + ((int64_t)tx * P.E + e) * P.S;
    if (P.binning == UR_BIN_NEAREST) {
        const int n = (int)floor(x);
        if (n >= 0 && n < P.S) unsafeAtomicAdd(ch + n, (float)v);
    } else {
        const double tau = x - 0.5;
        const double f0 = floor(tau);
        const int n0 = (int)f0;
        const double f = tau - f0;
        if (n0 >= 0 && n0 < P.S) unsafeAtomicAdd(ch + n0, (float)((1.0 - f) * v));
        if (n0 + 1 >= 0 && n0 + 1 < P.S) unsafeAtomicAdd(ch + n0 + 1, (float)(f * v));
    }
}

// --------------------------------------------------------- closest hit query
struct Hit {
    double t;
    int64_t id;
    int face;      // box face 0..5 if id == id_box
    int local;     // triangle slot in BVH order, sphere or plane index
};

template <bool COUNT>
__device__ __forceinline__ Hit closest_hit(const TraceParams &P, const double *o, const double *d, int64_t skip,
                                           Counters &cnt) {
    Hit h;
    h.t = INFINITY;
    h.face = -1;
    h.id = P.id_box;
    h.local = -1;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double t;
        int fi;
        if (d[i] > 0.0) {
            t = (P.box[3 + i] - o[i]) / d[i];
            fi = 3 + i;
        } else if (d[i] < 0.0) {
            t = (P.box[i] - o[i]) / d[i];
            fi = i;
        } else {
            continue;
        }
        if (t < h.t) {
            h.t = t;
            h.face = fi;
        }
    }
    if (P.n_tnodes > 0) {
        const CullRay cr = make_cull(o, d);
        float tmf = cull_tmax(h.t);
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
                const int id = P.tri_id[k];
                if (id == skip) continue;
                CNT(C_TRI_TESTS);
                double t;
                if (tri_isect(P.tri + 9 * (int64_t)k, o, d, t) && t > kEpsT &&
                    (t < h.t || (t == h.t && id < h.id))) {
                    h.t = t;
                    h.id = id;
                    h.local = k;
                    tmf = cull_tmax(t);
                }
            }
            ni = node_skip(n);
        }
    }
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
    return h;
}

// ----------------------------------------------- secondary ray (transducer sampling)
// Straight ray from q toward a chosen element centre: product of transmitted
// fractions and order-free sums of the attenuation and slowness changes at
// every crossing in (eps, dist - eps).  Returns false if blocked (T = 0).
template <bool COUNT>
__device__ __forceinline__ bool shadow(const TraceParams &P, const double *q, const double *vh, double dist,
                                       double &T, double &sum_a, double &sum_c, Counters &cnt) {
    T = 1.0;
    sum_a = 0.0;
    sum_c = 0.0;
    const double lo = kEpsT, hi = dist - kEpsT;
    auto cross_at = [&](double t, const double *ng, int mf, int mb) {
        const double dn = dot3(vh, ng);
        const int before = dn < 0.0 ? mf : mb, after = dn < 0.0 ? mb : mf;
        const Material A = P.mat[before], Bm = P.mat[after];
        T *= transmit_fraction(A.Z, Bm.Z, fabs(dn));
        sum_a += (Bm.ka - A.ka) * (dist - t);
        sum_c += (Bm.inv_c - A.inv_c) * (dist - t);
    };
    if (P.n_tnodes > 0) {
        const CullRay cr = make_cull(q, vh);
        const float tmf = cull_tmax(dist);
        int ni = 0;
        while (ni < P.n_tnodes) {
            const Node n = load_node(P.tnodes, ni);
            CNT(C_SHADOW_NODES);
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
                CNT(C_SHADOW_TRI_TESTS);
                double t;
                const double *tr = P.tri + 9 * (int64_t)k;
                if (tri_isect(tr, q, vh, t) && t > lo && t < hi) {
                    double ng[3];
                    tri_normal(tr, ng);
                    cross_at(t, ng, P.tri_mat[2 * k], P.tri_mat[2 * k + 1]);
                    if (T == 0.0) return false;
                }
            }
            ni = node_skip(n);
        }
    }
    for (int j = 0; j < P.n_sph; ++j) {
        const double *sp = P.sph + 4 * j;
        double t0, t1;
        if (!sph_roots(sp, q, vh, t0, t1)) continue;
        const double tr[2] = {t0, t1};
        for (int r = 0; r < 2; ++r) {
            if (tr[r] > lo && tr[r] < hi) {
                double ng[3];
                for (int i = 0; i < 3; ++i) ng[i] = (q[i] + tr[r] * vh[i] - sp[i]) / sp[3];
                cross_at(tr[r], ng, P.sph_mat[2 * j], P.sph_mat[2 * j + 1]);
            }
        }
    }
    for (int j = 0; j < P.n_pln; ++j) {
        double t;
        if (pln_isect(P.pln + 4 * j, q, vh, t) && t > lo && t < hi)
            cross_at(t, P.pln + 4 * j, P.pln_mat[2 * j], P.pln_mat[2 * j + 1]);
    }
    return T != 0.0;
}

// Scatterer k captured at distance s along the segment: re-radiation toward a
// uniformly chosen element centre (Sec. 2.3 "Transducer Sampling", Eq. 13).
template <bool COUNT, bool LOG>
__device__ __noinline__ void scatter_nee(const TraceParams &P, const EventLog &L, Counters &cnt, int tx, int e,
                                         uint32_t ray, int seg, int k, double amp, const double *o, const double *d,
                                         double w, double t, int med, double s) {
    const Material M = P.mat[med];
    const double q[3] = {o[0] + s * d[0], o[1] + s * d[1], o[2] + s * d[2]};
    const double wq = w * exp(-M.ka * s);
    const double tq = t + s * M.inv_c;
    uint32_t x[4];
    draw(P, ray, e, tx, seg, 2, (uint32_t)k, x);
    const int er = (int)(((uint64_t)x[0] * (uint64_t)P.E) >> 32);
    const double v[3] = {P.xe[er] - q[0], 0.0 - q[1], 0.0 - q[2]};
    const double dist = sqrt(dot3(v, v));
    const double vh[3] = {v[0] / dist, v[1] / dist, v[2] / dist};
    const double cos_a = -vh[2];
    const double ca = fmin(1.0, fmax(-1.0, cos_a));
    const double fdir = directivity(acos(ca), P.alpha_m, P.alpha_c);
    CNT(C_SCAT_EVENTS);
    if (fdir <= 0.0) {
        CNT(C_NEE_ZERO);
        return;
    }
    CNT(C_NEE_CAST);
    double T, sum_a, sum_c;
    if (!shadow<COUNT>(P, q, vh, dist, T, sum_a, sum_c, cnt)) {
        CNT(C_NEE_BLOCKED);
        return;
    }
    const double att = exp(-(M.ka * dist + sum_a));
    const double tc = tq + dist * M.inv_c + sum_c;
    const double c = wq * amp * (double)P.E * P.area_e * cos_a * fdir / (4.0 * M_PI * dist * dist) * T * att;
    record<COUNT, LOG>(P, L, cnt, 1, tx, er, seg, k, tc, c, q);
}

template <bool COUNT, bool LOG>
__device__ __forceinline__ void scatter_events(const TraceParams &P, const EventLog &L, Counters &cnt, int tx, int e,
                                               uint32_t ray, int seg, const double *o, const double *d, double w,
                                               double t, int med, double t_seg) {
    if (P.n_snodes == 0) return;
    const CullRay cr = make_cull(o, d);
    const float tmf = cull_tmax(t_seg);
    int ni = 0;
    while (ni < P.n_snodes) {
        const Node n = load_node(P.snodes, ni);
        CNT(C_SCAT_NODES);
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
        for (int j = first; j < first + count; ++j) {
            CNT(C_SCAT_TESTS);
            const double4 sk = P.scat[j];
            const double p[3] = {sk.x - o[0], sk.y - o[1], sk.z - o[2]};
            const double s = dot3(p, d);
            if (!(s >= 0.0 && s < t_seg)) continue;
            const double pp[3] = {p[0] - s * d[0], p[1] - s * d[1], p[2] - s * d[2]};
            if (dot3(pp, pp) > P.r_s2) continue;
            scatter_nee<COUNT, LOG>(P, L, cnt, tx, e, ray, seg, P.scat_id[j], sk.w, o, d, w, t, med, s);
        }
        ni = node_skip(n);
    }
}

// ------------------------------------------------------------------ one path
template <bool COUNT, bool LOG>
__device__ void trace_path(const TraceParams &P, const EventLog &L, Counters &cnt, int tx, int e, uint32_t ray,
                           double *o, double *d, double w, double t, int med) {
    double len = 0.0;
    int64_t last = -1;
    CNT(C_RAYS);
    for (int b = 0; b <= P.B; ++b) {
        CNT(C_SEGMENTS);
        const Hit h = closest_hit<COUNT>(P, o, d, last, cnt);
        double t_seg = h.t;
        bool clipped = false;
        if (len + t_seg > P.max_path) {
            t_seg = P.max_path - len;
            clipped = true;
        }
        scatter_events<COUNT, LOG>(P, L, cnt, tx, e, ray, b, o, d, w, t, med, t_seg);
        const Material M = P.mat[med];
        w *= exp(-M.ka * t_seg);
        t += t_seg * M.inv_c;
        len += t_seg;
        o[0] += t_seg * d[0];
        o[1] += t_seg * d[1];
        o[2] += t_seg * d[2];
        if (clipped) {
            CNT(C_TERM_PATH);
            log_event<LOG>(L, 4, tx, e, b, -3, t, w, o);
            return;
        }
        if (t >= P.t_max) {
            CNT(C_TERM_TIME);
            log_event<LOG>(L, 4, tx, e, b, -2, t, w, o);
            return;
        }
        if (h.id == P.id_box) {
            if (h.face == 2 && fabs(o[0]) <= P.half_ap && fabs(o[1]) <= 0.5 * P.elev) {
                int er = (int)floor((o[0] + P.half_ap) / P.pitch);
                er = er < 0 ? 0 : (er > P.E - 1 ? P.E - 1 : er);
                const double ca = fmin(1.0, fmax(-1.0, -d[2]));
                const double fdir = directivity(acos(ca), P.alpha_m, P.alpha_c);
                if (fdir > 0.0) {
                    CNT(C_DIRECT);
                    record<COUNT, LOG>(P, L, cnt, 0, tx, er, b, -1, t, w * fdir, o);
                }
            }
            CNT(C_TERM_BOX);
            log_event<LOG>(L, 4, tx, e, b, -1, t, w, o);
            return;
        }
        if (b == P.B) {
            CNT(C_TERM_BOUNCE);
            log_event<LOG>(L, 4, tx, e, b, -4, t, w, o);
            return;
        }
        // impedance boundary: geometric normal and the two materials
        double ng[3];
        int mf, mb;
        if (h.id < P.id_sph0) {
            tri_normal(P.tri + 9 * (int64_t)h.local, ng);
            mf = P.tri_mat[2 * h.local];
            mb = P.tri_mat[2 * h.local + 1];
        } else if (h.id < P.id_pln0) {
            const double *sp = P.sph + 4 * h.local;
            for (int i = 0; i < 3; ++i) ng[i] = (o[i] - sp[i]) / sp[3];
            mf = P.sph_mat[2 * h.local];
            mb = P.sph_mat[2 * h.local + 1];
        } else {
            const double *pp = P.pln + 4 * h.local;
            ng[0] = pp[0];
            ng[1] = pp[1];
            ng[2] = pp[2];
            mf = P.pln_mat[2 * h.local];
            mb = P.pln_mat[2 * h.local + 1];
        }
        // Eqs. 7-11 with eta = Z_before / Z_after and the reflect-or-transmit draw
        int before, after;
        if (dot3(d, ng) < 0.0) {
            before = mf;
            after = mb;
        } else {
            before = mb;
            after = mf;
            ng[0] = -ng[0];
            ng[1] = -ng[1];
            ng[2] = -ng[2];
        }
        if (before != med) CNT(C_MISMATCH);
        const double z1 = P.mat[before].Z, z2 = P.mat[after].Z;
        const double cos_r = -dot3(d, ng);
        const double eta = z1 / z2;
        const double rad = 1.0 - eta * eta * (1.0 - cos_r * cos_r);
        double R, cos_t = 0.0;
        if (rad < 0.0) {
            R = 1.0;
        } else {
            cos_t = sqrt(rad);
            const double den = z1 * cos_r + z2 * cos_t;
            if (den == 0.0) {
                R = 1.0;
            } else {
                const double A = (z1 * cos_r - z2 * cos_t) / den;
                R = A * A;
            }
        }
        uint32_t x[4];
        draw(P, ray, e, tx, b, 1, 0, x);
        const double y = u01(x[0]);
        double nd[3];
        const bool refl = y < R;
        if (refl) {
            for (int i = 0; i < 3; ++i) nd[i] = d[i] + 2.0 * cos_r * ng[i];
            if (R >= 1.0) CNT(C_TIR);
            else CNT(C_REFLECT);
            med = before;
        } else {
            const double f = eta * cos_r - cos_t;
            for (int i = 0; i < 3; ++i) nd[i] = eta * d[i] + f * ng[i];
            CNT(C_TRANSMIT);
            med = after;
        }
        const double l = sqrt(dot3(nd, nd));
        d[0] = nd[0] / l;
        d[1] = nd[1] / l;
        d[2] = nd[2] / l;
        log_event<LOG>(L, refl ? 2 : 3, tx, e, b, h.id, t, w, o);
        last = (h.id < P.id_sph0 || h.id >= P.id_pln0) ? h.id : -1;
    }
}

// Emission (Eqs. 4 and 6): origin uniform on the element face, direction from
// the uniform or tabulated proposal on the equal-area map, weight
// cos(theta) / (rays per transmit * pdf).
__device__ __forceinline__ void emit(const TraceParams &P, int tx, int e, uint32_t ray, double *o, double *d,
                                     double &w) {
    uint32_t x[4];
    draw(P, ray, e, tx, 0, 0, 0, x);
    const double u0 = u01(x[0]), u1 = u01(x[1]), u2 = u01(x[2]), u3 = u01(x[3]);
    o[0] = P.xe[e] + (u0 - 0.5) * P.pitch;
    o[1] = (u1 - 0.5) * P.elev;
    o[2] = 0.0;
    double ca, cb, pdf;
    if (!P.proposal) {
        ca = u2;
        cb = u3;
        pdf = 1.0 / (2.0 * M_PI);
    } else {
        uint32_t y[4];
        draw(P, ray, e, tx, 0, 3, 0, y);
        const double uc = u01(y[0]);
        const int64_t row = ((int64_t)tx * P.E + e) * kCells;
        const float *cdf = P.cdf + row;
        int lo = 0, hi = kCells;                 // first cell with uc <= cdf[cell]
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (uc <= (double)cdf[mid]) hi = mid;
            else lo = mid + 1;
        }
        const int cell = lo < kCells ? lo : kCells - 1;
        ca = ((double)(cell % 32) + u2) / 32.0;
        cb = ((double)(cell / 32) + u3) / 32.0;
        pdf = (double)P.pdf[row + cell] * (double)kCells / (2.0 * M_PI);
    }
    hemisphere(ca, cb, d);
    w = d[2] / (P.n_per_tx * pdf);
}

template <bool COUNT>
__device__ __forceinline__ void flush_counters(const TraceParams &P, Counters &cnt) {
    if constexpr (COUNT) {
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int k = 0; k < kNumStats; ++k) {
            uint32_t v = cnt.v[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0 && v) atomicAdd(P.stats + k, (unsigned long long)v);
        }
    }
}

template <bool COUNT>
__global__ __launch_bounds__(256) void k_trace(TraceParams P) {
    Counters cnt;
    if constexpr (COUNT) {
#pragma unroll
        for (int k = 0; k < kNumStats; ++k) cnt.v[k] = 0;
    }
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P.n_work) {
        const int64_t q = i / P.per_el;
        const uint32_t ray = (uint32_t)((i - q * P.per_el) * P.stride + P.offset);
        const int e = (int)(q % P.E);
        const int tx = (int)(q / P.E);
        double o[3], d[3], w;
        emit(P, tx, e, ray, o, d, w);
        EventLog L{};
        trace_path<COUNT, false>(P, L, cnt, tx, e, ray, o, d, w, P.tau[(int64_t)tx * P.E + e], P.top_medium);
    }
    flush_counters<COUNT>(P, cnt);
}

__global__ __launch_bounds__(64) void k_trace_rays(TraceParams P, const ur_ray *rays, int64_t n, EventLog L) {
    Counters cnt;
#pragma unroll
    for (int k = 0; k < kNumStats; ++k) cnt.v[k] = 0;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const ur_ray r = rays[i];
        double o[3] = {r.o[0], r.o[1], r.o[2]}, d[3] = {r.d[0], r.d[1], r.d[2]};
        trace_path<true, true>(P, L, cnt, (int)r.tx, (int)r.elem, (uint32_t)r.ray, o, d, r.w, r.t, (int)r.medium);
    }
    flush_counters<true>(P, cnt);
}

__global__ void k_philox(const uint32_t *ctr, uint32_t *out, int64_t n, uint32_t k0, uint32_t k1) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t r[4];
    philox(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1, r);
    for (int j = 0; j < 4; ++j) out[4 * i + j] = r[j];
}

}  // namespace

hipError_t ur_launch_trace(const ur::TraceParams &p, bool count, hipStream_t s) {
    if (p.n_work <= 0) return hipSuccess;
    const int64_t blocks = (p.n_work + 255) / 256;
    if (count) hipLaunchKernelGGL(k_trace<true>, dim3((unsigned)blocks), dim3(256), 0, s, p);
    else hipLaunchKernelGGL(k_trace<false>, dim3((unsigned)blocks), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t ur_launch_trace_rays(const ur::TraceParams &p, const void *rays_dev, int64_t n, ur::EventLog log,
                                hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 63) / 64;
    hipLaunchKernelGGL(k_trace_rays, dim3((unsigned)blocks), dim3(64), 0, s, p, (const ur_ray *)rays_dev, n, log);
    return hipGetLastError();
}

hipError_t ur_launch_philox(const uint32_t *ctr, uint32_t *out, int64_t n, uint32_t k0, uint32_t k1, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ctr, out, n, k0, k1);
    return hipGetLastError();
}
