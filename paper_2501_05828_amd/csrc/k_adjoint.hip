// Path-replay adjoint of the channel-data estimator on gfx950.
//
// Every path of a trace is regenerated from its Philox counters at the
// current parameters theta0 and followed with the same decisions (closest
// primitive, reflect-or-transmit, captures, receiving elements, crossings).
// Along the path each quantity is carried as a dual number (a value and its
// tangents along the pass's parameter directions, two per tangent pass); at
// every contribution c with arrival time t
// the gradient of J = sum_records g(t) c receives g(t) dc + c g'(t) dt, where
// g is the adjoint of the binned channel data (g' is non-zero only for the
// linear binning filter).
//
// The reflect-or-transmit choice keeps its probability attached: the weight
// is multiplied by R / value(R) after a reflection and (1 - R) / value(1 - R)
// after a transmission, so that the tangent carries the derivative of the
// choice probability and the gradient is that of the expectation for the
// sampled decisions.  The value pass (no tangent) also accumulates the
// gradients with respect to every scatterer amplitude (dc/da_k = c / a_k) and
// every attenuation coefficient (d log c / d alpha_m = -kappa x path length in
// material m).
//
// Every decision is taken on values, so it is the same in every pass.  The
// value pass records, for a range of paths, each segment's closest primitive
// and the captures that reach a contribution; the tangent passes over the
// same range read them instead of walking the tree and the scatterer grid
// again (a path with more captures than the record holds walks the grid).
#include "closest_hit.h"
#include "trace_device.h"
#include "ultraray.h"

namespace {
using namespace ur;
using namespace ur::dev;

constexpr int kAdjMat = kAdjMaxMat;

// Dual numbers: a value and its derivatives along K parameter directions.
template <int K>
struct DK {
    double v, t[K];
};
template <int K>
__device__ __forceinline__ DK<K> operator+(DK<K> a, const DK<K> &b) {
    a.v += b.v;
#pragma unroll
    for (int k = 0; k < K; ++k) a.t[k] += b.t[k];
    return a;
}
template <int K>
__device__ __forceinline__ DK<K> operator-(DK<K> a, const DK<K> &b) {
    a.v -= b.v;
#pragma unroll
    for (int k = 0; k < K; ++k) a.t[k] -= b.t[k];
    return a;
}
template <int K>
__device__ __forceinline__ DK<K> operator-(DK<K> a) {
    a.v = -a.v;
#pragma unroll
    for (int k = 0; k < K; ++k) a.t[k] = -a.t[k];
    return a;
}
template <int K>
__device__ __forceinline__ DK<K> operator*(const DK<K> &a, const DK<K> &b) {
    DK<K> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.t[k] = a.t[k] * b.v + a.v * b.t[k];
    return r;
}
template <int K>
__device__ __forceinline__ DK<K> operator*(double s, DK<K> a) {
    a.v = s * a.v;
#pragma unroll
    for (int k = 0; k < K; ++k) a.t[k] = s * a.t[k];
    return a;
}
template <int K>
__device__ __forceinline__ DK<K> operator/(const DK<K> &a, const DK<K> &b) {
    DK<K> r;
    r.v = a.v / b.v;
    const double b2 = b.v * b.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.t[k] = (a.t[k] * b.v - a.v * b.t[k]) / b2;
    return r;
}
// f(a) with f' given: value f(a.v), tangents f'(a.v) a.t
template <int K>
__device__ __forceinline__ DK<K> dchain(const DK<K> &a, double f, double df) {
    DK<K> r;
    r.v = f;
#pragma unroll
    for (int k = 0; k < K; ++k) r.t[k] = a.t[k] * df;
    return r;
}
template <int K>
__device__ __forceinline__ DK<K> dsqrt(const DK<K> &a) {
    const double r = sqrt(a.v);
    DK<K> o;
    o.v = r;
#pragma unroll
    for (int k = 0; k < K; ++k) o.t[k] = a.t[k] / (2.0 * r);
    return o;
}
template <int K>
__device__ __forceinline__ DK<K> dexp(const DK<K> &a) {
    const double e = exp(a.v);
    return dchain(a, e, e);
}
template <int K>
__device__ __forceinline__ DK<K> dacos(const DK<K> &a) {
    const double x = fmin(1.0, fmax(-1.0, a.v));
    const double s = sqrt(fmax(1.0 - x * x, 1e-300));
    DK<K> o;
    o.v = acos(x);
#pragma unroll
    for (int k = 0; k < K; ++k) o.t[k] = -a.t[k] / s;
    return o;
}
template <int K>
__device__ __forceinline__ DK<K> ddot(const DK<K> *a, const DK<K> *b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
template <int K>
__device__ __forceinline__ DK<K> ddot(const DK<K> *a, const double *b) {
    return b[0] * a[0] + b[1] * a[1] + b[2] * a[2];
}

// Tangent passes carry up to kAdjTan parameter directions at once (the
// value pass none): the record reads, the secondary rays' tree walks and the
// emission are shared by them.  Two is fastest (all gradients of the large
// scene at every 4th ray: 1.89 s with one, 1.22 s with two, 1.26 s with
// three, 1.36 s with four: more directions spill more registers).
#ifndef UR_ADJ_TAN
#define UR_ADJ_TAN 2
#endif
constexpr int kAdjTan = UR_ADJ_TAN;

struct AdjParams {
    TraceParams P;
    int n_tan;                  // parameter directions of this pass (0: value pass)
    AdjTangent tan[kAdjTan];    // kind 1: impedance of material index; 2: coordinate coord of sphere index
    const float *g;          // [T][E][S] adjoint of the binned channel data
    float *grad_amp;         // [n_scat] or null (value pass)
    double *grad_alpha;      // [n_mat] or null (value pass)
    double *value_out;       // [1] sum of g(t) c over the replayed contributions, or null
    double kappa;            // d ka / d alpha [Np/m per dB/(cm MHz)]
    int attach_choice;       // 1: keep R / value(R) on the path weight
    AdjRecord rec;           // decisions kept from the value pass (the tangent passes replay them)
};

// Adjoint of the binned data at arrival time t and its slope in t.
__device__ __forceinline__ bool adj_at(const AdjParams &A, int tx, int e, double t, double &g, double &gs) {
    const TraceParams &P = A.P;
    if (!(t < P.t_max) || t < 0.0) return false;
    const float *ch = A.g + ((int64_t)tx * P.E + e) * P.S;
    const double x = t * P.fs;
    if (P.binning == UR_BIN_NEAREST) {
        const int n = (int)floor(x);
        g = (n >= 0 && n < P.S) ? (double)ch[n] : 0.0;
        gs = 0.0;
    } else {
        const double tau = x - 0.5, f0 = floor(tau), f = tau - f0;
        const int n0 = (int)f0;
        const double g0 = (n0 >= 0 && n0 < P.S) ? (double)ch[n0] : 0.0;
        const double g1 = (n0 + 1 >= 0 && n0 + 1 < P.S) ? (double)ch[n0 + 1] : 0.0;
        g = (1.0 - f) * g0 + f * g1;
        gs = (g1 - g0) * P.fs;
    }
    return true;
}

struct Acc {
    double val;               // sum of g(t) c
    double tan[kAdjTan];      // tangent-pass accumulators
    double alpha[kAdjMat];    // value pass: dJ/d alpha_m
};

// The replay's arithmetic on K-direction dual numbers (K = 1 for the value
// pass, whose tangents are zero; kAdjTan for the tangent passes).
template <int K>
struct Rep {
    using D = DK<K>;
    static __device__ __forceinline__ D dd(double v) {
        D r;
        r.v = v;
#pragma unroll
        for (int k = 0; k < K; ++k) r.t[k] = 0.0;
        return r;
    }

    static __device__ __forceinline__ D mat_Z(const AdjParams &A, int m) {
        D z;
        z.v = A.P.mat[m].Z;
#pragma unroll
        for (int k = 0; k < K; ++k) z.t[k] = (k < A.n_tan && A.tan[k].kind == 1 && A.tan[k].index == m) ? 1.0 : 0.0;
        return z;
    }

    static __device__ __forceinline__ void sph_center(const AdjParams &A, int j, D *c, double *r) {
        const double *s = A.P.sph + 4 * j;
        for (int i = 0; i < 3; ++i) {
            c[i].v = s[i];
#pragma unroll
            for (int k = 0; k < K; ++k)
                c[i].t[k] = (k < A.n_tan && A.tan[k].kind == 2 && A.tan[k].index == j && A.tan[k].coord == i) ? 1.0 : 0.0;
        }
        *r = s[3];
    }

    // Smith masking G1 of the GGX distribution at a dual cos(theta_v) (as ggx_g1).
    static __device__ __forceinline__ D dggx_g1(double alpha, D cv) {
        const D c2 = cv * cv;
        const D tan2 = (dd(1.0) - c2) / c2;
        return dd(2.0) / (dd(1.0) + dsqrt(dd(1.0) + (alpha * alpha) * tan2));
    }

    // Microfacet normal of ggx_sample about a dual unit normal n: the random
    // numbers fix its polar and azimuthal angles about n; the basis (onb) follows n.
    static __device__ __forceinline__ void dggx_sample(const D *n, double alpha, double xi1, double xi2, D *h) {
        const double sg = copysign(1.0, n[2].v);
        const D a = dd(-1.0) / (dd(sg) + n[2]);
        const D c = n[0] * n[1] * a;
        const D t[3] = {dd(1.0) + sg * n[0] * n[0] * a, sg * c, -sg * n[0]};
        const D b[3] = {c, dd(sg) + n[1] * n[1] * a, -n[1]};
        const double q = 1.0 - xi1 + alpha * alpha * xi1;
        const double ct = sqrt((1.0 - xi1) / q), st = alpha * sqrt(xi1 / q);
        double sp, cp;
        sincos(2.0 * M_PI * xi2, &sp, &cp);
        for (int i = 0; i < 3; ++i) h[i] = (st * cp) * t[i] + (st * sp) * b[i] + ct * n[i];
    }

    // Dual-number transmitted fraction 1 - A_r^2 of a straight crossing.
    static __device__ __forceinline__ D transmit_fraction_d(D z1, D z2, D cos_r) {
        const D eta = z1 / z2;
        const D rad = dd(1.0) - eta * eta * (dd(1.0) - cos_r * cos_r);
        if (rad.v < 0.0) return dd(0.0);
        const D cos_t = dsqrt(rad);
        const D den = z1 * cos_r + z2 * cos_t;
        if (den.v == 0.0) return dd(0.0);
        const D Ar = (z1 * cos_r - z2 * cos_t) / den;
        return dd(1.0) - Ar * Ar;
    }

    // Crossings of the secondary ray q + s vh, s in (eps, dist - eps): product of
    // transmitted fractions, order-free attenuation and slowness sums, and (value
    // pass) the length spent in each material.
    static __device__ bool shadow_d(const AdjParams &A, const D *q, const D *vh, D dist, int med, D &T, D &sum_a, D &sum_c,
                             double *len_m) {
        const TraceParams &P = A.P;
        T = dd(1.0);
        sum_a = dd(0.0);
        sum_c = dd(0.0);
        const double lo = kEpsT, hi = dist.v - kEpsT;
        if (len_m) {
            for (int m = 0; m < kAdjMat; ++m) len_m[m] = 0.0;
            for (int m = 0; m < kAdjMat; ++m)
                if (m == med) len_m[m] = dist.v;
        }
        auto cross_at = [&](D t, const D *ng, int mf, int mb) {
            const D dn = ddot(vh, ng);
            const bool front = dn.v < 0.0;
            const int before = front ? mf : mb, after = front ? mb : mf;
            const D adn = front ? -dn : dn;
            T = T * transmit_fraction_d(mat_Z(A, before), mat_Z(A, after), adn);
            const D rem = dist - t;
            sum_a = sum_a + (P.mat[after].ka - P.mat[before].ka) * rem;
            sum_c = sum_c + (P.mat[after].inv_c - P.mat[before].inv_c) * rem;
            if (len_m)
                for (int m = 0; m < kAdjMat; ++m) len_m[m] += ((m == after) - (m == before)) * rem.v;
        };
        const double qv[3] = {q[0].v, q[1].v, q[2].v}, vv[3] = {vh[0].v, vh[1].v, vh[2].v};
        if (P.n_tnodes > 0) {
            const CullRay cr = make_cull(qv, vv);
            const float tmf = cull_tmax(dist.v);
            int ni = 0;
            while (ni < P.n_tnodes) {
                const Node n = load_node(P.tnodes, ni);
                if (!slab(n, cr, tmf)) {
                    ni = node_skip(n);
                    continue;
                }
                const int leaf = node_leaf(n);
                if (leaf < 0) {
                    ++ni;
                    continue;
                }
                for (int k = leaf >> 4; k < (leaf >> 4) + (leaf & 15); ++k) {
                    const double *tr = P.tri + 9 * (int64_t)k;
                    double tv;
                    if (!tri_isect(tr, qv, vv, tv) || !(tv > lo && tv < hi)) continue;
                    // t = e2.(tv x e1) / e1.(d x e2) with tv = q - v0
                    const double *v0 = tr, *e1 = tr + 3, *e2 = tr + 6;
                    const D tq[3] = {q[0] - dd(v0[0]), q[1] - dd(v0[1]), q[2] - dd(v0[2])};
                    const D pv[3] = {vh[1] * dd(e2[2]) - vh[2] * dd(e2[1]), vh[2] * dd(e2[0]) - vh[0] * dd(e2[2]),
                                     vh[0] * dd(e2[1]) - vh[1] * dd(e2[0])};
                    const D det = ddot(pv, e1);
                    const D qq[3] = {tq[1] * dd(e1[2]) - tq[2] * dd(e1[1]), tq[2] * dd(e1[0]) - tq[0] * dd(e1[2]),
                                     tq[0] * dd(e1[1]) - tq[1] * dd(e1[0])};
                    const D t = ddot(qq, e2) / det;
                    double nv[3];
                    tri_normal(P, k, nv);
                    const D ng[3] = {dd(nv[0]), dd(nv[1]), dd(nv[2])};
                    cross_at(t, ng, P.tri_mat[2 * k], P.tri_mat[2 * k + 1]);
                    if (T.v == 0.0) return false;
                }
                ni = node_skip(n);
            }
        }
        for (int j = 0; j < P.n_sph; ++j) {
            D c[3];
            double r;
            sph_center(A, j, c, &r);
            const D oc[3] = {q[0] - c[0], q[1] - c[1], q[2] - c[2]};
            const D b = ddot(oc, vh);
            const D cc = ddot(oc, oc) - dd(r * r);
            const D disc = b * b - cc;
            if (disc.v < 0.0) continue;
            const D sq = dsqrt(disc);
            const D roots[2] = {-b - sq, -b + sq};
            for (int k = 0; k < 2; ++k) {
                if (!(roots[k].v > lo && roots[k].v < hi)) continue;
                const D ng[3] = {(q[0] + roots[k] * vh[0] - c[0]) / dd(r), (q[1] + roots[k] * vh[1] - c[1]) / dd(r),
                                 (q[2] + roots[k] * vh[2] - c[2]) / dd(r)};
                cross_at(roots[k], ng, P.sph_mat[2 * j], P.sph_mat[2 * j + 1]);
            }
        }
        for (int j = 0; j < P.n_pln; ++j) {
            const double *pl = P.pln + 4 * j;
            const D den = ddot(vh, pl);
            if (den.v == 0.0) continue;
            const D t = (dd(pl[3]) - ddot(q, pl)) / den;
            if (!(t.v > lo && t.v < hi)) continue;
            const D ng[3] = {dd(pl[0]), dd(pl[1]), dd(pl[2])};
            cross_at(t, ng, P.pln_mat[2 * j], P.pln_mat[2 * j + 1]);
        }
        return T.v != 0.0;
    }

    // Accumulates the gradient of one contribution c arriving at time t.
    // c_unit is the contribution per unit amplitude of scatterer k (k < 0: none).
    static __device__ __forceinline__ void contribute(const AdjParams &A, Acc &acc, int tx, int er, D c, D t, int k,
                                               double c_unit, const double *len_path, const double *len_sh) {
        double g, gs;
        if (!adj_at(A, tx, er, t.v, g, gs)) return;
        acc.val += g * c.v;
        if (A.n_tan > 0) {
#pragma unroll
            for (int j = 0; j < K; ++j) acc.tan[j] += g * c.t[j] + gs * c.v * t.t[j];
            return;
        }
        if (A.grad_amp && k >= 0) atomicAdd(A.grad_amp + k, (float)(g * c_unit));
        if (A.grad_alpha)
            for (int m = 0; m < kAdjMat; ++m) {
                const double L = len_path[m] + (len_sh ? len_sh[m] : 0.0);
                // d/d alpha_m of g(t) c: the amplitude factor exp(-kappa alpha L)
                acc.alpha[m] += g * c.v * (-A.kappa * L);
            }
    }

    // LEN: the value pass with attenuation gradients, which tracks the length
    // each path and secondary ray spends in every material.
    template <bool LEN>
    static __device__ void replay_paths(const AdjParams &A, Acc &acc, LdsStack stk) {
        const TraceParams &P = A.P;
        const bool record = A.rec.mode == 1, replay = A.rec.mode == 2;
        const int lane = threadIdx.x & 63;
        // Persistent lanes: a lane whose path has ended takes the next one of the
        // range (one atomic per wavefront and refill), so that a wavefront does
        // not wait for its longest path; every iteration is one segment.
        int tx = 0, e = 0;
        uint32_t ray = 0;
        int64_t slot = 0;
        AdjSeg *segs = nullptr;
        AdjCap *caps = nullptr;
        int ncap = 0;
        bool walk_grid = true;
        D o[3], d[3], w, t, len;
        double len_m[LEN ? kAdjMat : 1];
        int med = 0, b = 0;
        int64_t last = -1;
        bool live = false, done = false;
        for (;;) {
            const unsigned long long need = __ballot(!live && !done);
            if (need) {
                const int first = __ffsll((long long)need) - 1;
                unsigned long long base = 0;
                if (lane == first) base = atomicAdd(A.rec.next, (unsigned long long)__popcll(need));
                base = __shfl(base, first, 64);
                if (!live && !done) {
                    const int64_t i = A.rec.begin + (int64_t)base + __popcll(need & ((1ull << lane) - 1ull));
                    if (i < A.rec.end) {
                        slot = i - A.rec.begin;
                        const int64_t q = i / P.per_el;
                        ray = (uint32_t)((i - q * P.per_el) * P.stride + P.offset);
                        tx = P.sa ? (int)q : (int)(q / P.E);
                        e = P.sa ? (int)q : (int)(q % P.E);
                        segs = A.rec.mode ? A.rec.seg + slot * (P.B + 1) : nullptr;
                        caps = A.rec.mode ? A.rec.cap + slot * kAdjCapRec : nullptr;
                        ncap = 0;
                        walk_grid = true;
                        if (record) A.rec.ncap[slot] = 0;
                        if (replay && A.rec.ncap[slot] != kAdjCapOverflow) {
                            ncap = A.rec.ncap[slot];
                            walk_grid = false;
                        }
                        double o0[3], d0[3], w0;
                        int cell;
                        emit(P, tx, e, ray, o0, d0, w0, cell);
                        for (int k = 0; k < 3; ++k) {
                            o[k] = dd(o0[k]);
                            d[k] = dd(d0[k]);
                        }
                        w = dd(w0);
                        t = dd(P.tau[(int64_t)tx * P.E + e]);
                        len = dd(0.0);
                        for (int m = 0; m < (LEN ? kAdjMat : 1); ++m) len_m[m] = 0.0;
                        med = P.top_medium;
                        last = -1;
                        b = 0;
                        live = true;
                    } else {
                        done = true;
                    }
                }
            }
            if (!__any(live)) break;
            if (!live) continue;
            // closest primitive by value (or as the value pass recorded it)
            const double ov[3] = {o[0].v, o[1].v, o[2].v}, dv[3] = {d[0].v, d[1].v, d[2].v};
            double tbest = INFINITY;
            int face = -1;
            int64_t hid = P.id_box;
            int hloc = -1;
            if (replay) {
                const AdjSeg r = segs[b];
                tbest = r.t;
                hid = r.hid;
                if (hid == P.id_box) face = r.aux;
                else hloc = r.aux;
            } else {
                // the trace's own query: box exit, spheres, planes, four-wide tree
                Counters cnt;
                const Hit h = closest_hit<false>(P, ov, dv, last, stk, cnt);
                tbest = h.t;
                hid = h.id;
                face = h.face;
                hloc = h.local;
                if (record) segs[b] = AdjSeg{tbest, (int)hid, hid == P.id_box ? face : hloc};
            }
            // dual distance to the chosen primitive
            D th;
            D sc[3];
            double srad = 0.0;
            if (hid == P.id_box && face == 6) {
                const D R = dd(P.radius);
                const D aa = d[0] * d[0] + d[2] * d[2], bq = o[0] * d[0] + (o[2] + R) * d[2];
                const D cq = o[0] * o[0] + o[2] * (o[2] + dd(2.0) * R);
                th = cq / (-bq + dsqrt(bq * bq - aa * cq));
            } else if (hid == P.id_box) {
                const int ax = face % 3;
                th = (dd(P.box[face]) - o[ax]) / d[ax];
            } else if (hid < P.id_sph0) {
                const double *tr = P.tri + 9 * (int64_t)hloc, *v0 = tr, *e1 = tr + 3, *e2 = tr + 6;
                const D tq[3] = {o[0] - dd(v0[0]), o[1] - dd(v0[1]), o[2] - dd(v0[2])};
                const D pv[3] = {d[1] * dd(e2[2]) - d[2] * dd(e2[1]), d[2] * dd(e2[0]) - d[0] * dd(e2[2]),
                                 d[0] * dd(e2[1]) - d[1] * dd(e2[0])};
                const D qq[3] = {tq[1] * dd(e1[2]) - tq[2] * dd(e1[1]), tq[2] * dd(e1[0]) - tq[0] * dd(e1[2]),
                                 tq[0] * dd(e1[1]) - tq[1] * dd(e1[0])};
                th = ddot(qq, e2) / ddot(pv, e1);
            } else if (hid < P.id_pln0) {
                sph_center(A, hloc, sc, &srad);
                const D oc[3] = {o[0] - sc[0], o[1] - sc[1], o[2] - sc[2]};
                const D bb = ddot(oc, d), cc = ddot(oc, oc) - dd(srad * srad);
                const D sq = dsqrt(bb * bb - cc);
                const D r0 = -bb - sq;
                th = r0.v > kEpsT ? r0 : -bb + sq;
            } else {
                const double *pl = P.pln + 4 * hloc;
                th = (dd(pl[3]) - ddot(o, pl)) / ddot(d, pl);
            }
            th.v = tbest;   // the value follows the forward query exactly
            D tseg = th;
            bool clipped = false;
            if (len.v + tseg.v > P.max_path) {
                tseg = dd(P.max_path) - len;
                clipped = true;
            }
            // captures on [0, tseg) and their secondary rays
            if (P.n_scat > 0) {
                const Material M = P.mat[med];
                // one capture of item j whose secondary ray goes to element er of
                // the n_e that could be drawn; recorded if it reaches a contribution
                auto capture = [&](int j, int er, int n_e) {
                    const double4 sk = P.items[j];
                    const int k = P.item_id[j];
                    const D pd[3] = {dd(sk.x) - o[0], dd(sk.y) - o[1], dd(sk.z) - o[2]};
                    const D sd = ddot(pd, d);
                    const D q[3] = {o[0] + sd * d[0], o[1] + sd * d[1], o[2] + sd * d[2]};
                    const double4 g = P.convex ? P.elem[er] : make_double4(P.xe[er], 0.0, 0.0, 1.0);
                    const D v[3] = {dd(g.x) - q[0], -q[1], dd(g.y) - q[2]};
                    const D dist = dsqrt(ddot(v, v));
                    const D vh[3] = {v[0] / dist, v[1] / dist, v[2] / dist};
                    const D cos_a = P.convex ? -(vh[0] * dd(g.z) + vh[2] * dd(g.w)) : -vh[2];
                    const D al = dacos(cos_a);
                    D f;
                    if (al.v > P.alpha_c) return;
                    if (al.v <= P.alpha_m) f = dd(1.0);
                    else f = (dd(P.alpha_c) - al) / dd(P.alpha_c - P.alpha_m);
                    D T, sa, sc2;
                    double lsh[LEN ? kAdjMat : 1];
                    if (!shadow_d(A, q, vh, dist, med, T, sa, sc2, LEN ? lsh : nullptr)) return;
                    if (record) {
                        if (ncap < kAdjCapRec) {
                            caps[ncap] = AdjCap{j, (unsigned short)er, (unsigned short)b};
                            A.rec.ncap[slot] = (unsigned char)++ncap;
                        } else {
                            A.rec.ncap[slot] = kAdjCapOverflow;
                        }
                    }
                    const D wq = w * dexp(-(M.ka * sd));
                    const D tq = t + M.inv_c * sd;
                    const D att = dexp(-(M.ka * dist + sa));
                    const D tc = tq + M.inv_c * dist + sc2;
                    const D cu = wq * dd((double)n_e * P.area_e / (4.0 * M_PI)) * cos_a * f / (dist * dist) * T * att;
                    const D cval = sk.w * cu;
                    if constexpr (LEN) {
                        double lp[kAdjMat];
                        for (int m = 0; m < kAdjMat; ++m) lp[m] = len_m[m] + (m == med ? sd.v : 0.0);
                        contribute(A, acc, tx, er, cval, tc, k, cu.v, lp, lsh);
                    } else {
                        contribute(A, acc, tx, er, cval, tc, k, cu.v, nullptr, nullptr);
                    }
                };
                if (walk_grid) {
                    dda_walk(P.grid, ov, dv, tseg.v, [&](int gcell, double ta, double tb) {
                        const int j1 = P.cell_start[gcell + 1];
                        for (int j = P.cell_start[gcell]; j < j1; ++j) {
                            const double4 sk = P.items[j];
                            const double p[3] = {sk.x - ov[0], sk.y - ov[1], sk.z - ov[2]};
                            const double s = dot3(p, dv);
                            if (!(s >= ta && s < tb)) continue;
                            const double pp[3] = {p[0] - s * dv[0], p[1] - s * dv[1], p[2] - s * dv[2]};
                            if (dot3(pp, pp) > P.r_s2) continue;
                            const int k = P.item_id[j];
                            const D pd[3] = {dd(sk.x) - o[0], dd(sk.y) - o[1], dd(sk.z) - o[2]};
                            const D sd = ddot(pd, d);
                            int e_lo, n_e;
                            if (!elem_range(P, o[0].v + sd.v * d[0].v, o[1].v + sd.v * d[1].v, o[2].v + sd.v * d[2].v,
                                            e_lo, n_e))
                                continue;
                            uint32_t x[4];
                            draw(P, ray, e, tx, b, 2, (uint32_t)k, x);
                            capture(j, e_lo + (int)(((uint64_t)x[0] * (uint64_t)n_e) >> 32), n_e);
                        }
                        return true;
                    });
                } else {
                    for (int c = 0; c < ncap; ++c) {
                        const AdjCap r = caps[c];
                        if (r.seg != b) continue;
                        const double4 sk = P.items[r.item];
                        const D pd[3] = {dd(sk.x) - o[0], dd(sk.y) - o[1], dd(sk.z) - o[2]};
                        const D sd = ddot(pd, d);
                        int e_lo, n_e;
                        elem_range(P, o[0].v + sd.v * d[0].v, o[1].v + sd.v * d[1].v, o[2].v + sd.v * d[2].v, e_lo, n_e);
                        capture(r.item, r.er, n_e);
                    }
                }
            }
            // transport
            const Material M = P.mat[med];
            w = w * dexp(-(M.ka * tseg));
            t = t + M.inv_c * tseg;
            len = len + tseg;
            if constexpr (LEN)
                for (int m = 0; m < kAdjMat; ++m)
                    if (m == med) len_m[m] += tseg.v;
            for (int i = 0; i < 3; ++i) o[i] = o[i] + tseg * d[i];
            if (clipped || t.v >= P.t_max) {
                live = false;
                continue;
            }
            if (hid == P.id_box) {
                if (P.convex) {
                    if (face == 6 && fabs(o[1].v) <= 0.5 * P.elev) {
                        const double ph = atan2(o[0].v, o[2].v + P.radius);
                        if (fabs(ph) <= P.half_arc) {
                            int er = (int)floor(ph / P.dphi + 0.5 * (double)P.E);
                            er = er < 0 ? 0 : (er > P.E - 1 ? P.E - 1 : er);
                            const double4 g = P.elem[er];
                            const D al = dacos(-(d[0] * dd(g.z) + d[2] * dd(g.w)));
                            if (al.v <= P.alpha_c) {
                                const D f = al.v <= P.alpha_m ? dd(1.0) : (dd(P.alpha_c) - al) / dd(P.alpha_c - P.alpha_m);
                                contribute(A, acc, tx, er, w * f, t, -1, 0.0, LEN ? len_m : nullptr, nullptr);
                            }
                        }
                    }
                    live = false;
                    continue;
                }
                if (face == 2 && fabs(o[0].v) <= P.half_ap && fabs(o[1].v) <= 0.5 * P.elev) {
                    int er = (int)floor((o[0].v + P.half_ap) / P.pitch);
                    er = er < 0 ? 0 : (er > P.E - 1 ? P.E - 1 : er);
                    const D al = dacos(-d[2]);
                    if (al.v <= P.alpha_c) {
                        const D f = al.v <= P.alpha_m ? dd(1.0) : (dd(P.alpha_c) - al) / dd(P.alpha_c - P.alpha_m);
                        contribute(A, acc, tx, er, w * f, t, -1, 0.0, LEN ? len_m : nullptr, nullptr);
                    }
                }
                live = false;
                continue;
            }
            if (b == P.B) {
                live = false;
                continue;
            }
            // interface: dual normal, Eqs. 7-11, attached choice probability
            D ng[3];
            int mf, mb;
            if (hid < P.id_sph0) {
                double nv[3];
                tri_normal(P, hloc, nv);
                for (int i = 0; i < 3; ++i) ng[i] = dd(nv[i]);
                mf = P.tri_mat[2 * hloc];
                mb = P.tri_mat[2 * hloc + 1];
            } else if (hid < P.id_pln0) {
                for (int i = 0; i < 3; ++i) ng[i] = (o[i] - sc[i]) / dd(srad);
                mf = P.sph_mat[2 * hloc];
                mb = P.sph_mat[2 * hloc + 1];
            } else {
                const double *pl = P.pln + 4 * hloc;
                for (int i = 0; i < 3; ++i) ng[i] = dd(pl[i]);
                mf = P.pln_mat[2 * hloc];
                mb = P.pln_mat[2 * hloc + 1];
            }
            int before, after;
            if (ddot(d, ng).v < 0.0) {
                before = mf;
                after = mb;
            } else {
                before = mb;
                after = mf;
                for (int i = 0; i < 3; ++i) ng[i] = -ng[i];
            }
            const D z1 = mat_Z(A, before), z2 = mat_Z(A, after);
            uint32_t x[4];
            draw(P, ray, e, tx, b, 1, 0, x);
            const double y = u01(x[0]);
            // a rough boundary (Eq. 12; its echoes by direct hits only): Eqs. 7-11
            // about the microfacet normal drawn from the second and third words
            const double alpha = fmax(P.mat[mf].rough, P.mat[mb].rough);
            D mn[3] = {ng[0], ng[1], ng[2]}, cn = dd(1.0);
            if (alpha > 0.0) {
                dggx_sample(ng, alpha, u01(x[1]), u01(x[2]), mn);
                cn = -ddot(d, ng);
                if (!(-ddot(d, mn).v > 0.0)) {
                    live = false;
                    continue;
                }
            }
            const D cos_r = -ddot(d, mn);
            const D eta = z1 / z2;
            const D rad = dd(1.0) - eta * eta * (dd(1.0) - cos_r * cos_r);
            D R = dd(1.0), cos_t = dd(0.0);
            if (rad.v >= 0.0) {
                cos_t = dsqrt(rad);
                const D den = z1 * cos_r + z2 * cos_t;
                if (den.v != 0.0) {
                    const D Ar = (z1 * cos_r - z2 * cos_t) / den;
                    R = Ar * Ar;
                }
            }
            D nd[3];
            const bool refl = y < R.v;
            if (refl) {
                for (int i = 0; i < 3; ++i) nd[i] = d[i] + dd(2.0) * cos_r * mn[i];
            } else {
                const D f = eta * cos_r - cos_t;
                for (int i = 0; i < 3; ++i) nd[i] = eta * d[i] + f * mn[i];
            }
            const D l = dsqrt(ddot(nd, nd));
            for (int i = 0; i < 3; ++i) nd[i] = nd[i] / l;
            if (alpha > 0.0) {
                // a new direction on the wrong side of the surface is absorbed;
                // else the weight factor |i.mn| G1(i) G1(o) / (|i.n| |mn.n|)
                const D co = ddot(nd, ng);
                if (refl ? !(co.v > 0.0) : !(co.v < 0.0)) {
                    live = false;
                    continue;
                }
                w = w * (cos_r * dggx_g1(alpha, cn) * dggx_g1(alpha, co.v < 0.0 ? -co : co) / (cn * ddot(mn, ng)));
            }
            if (refl) {
                if (A.attach_choice) w = w * (R / dd(R.v));
                med = before;
            } else {
                const D Tr = dd(1.0) - R;
                if (A.attach_choice) w = w * (Tr / dd(Tr.v));
                med = after;
            }
            for (int i = 0; i < 3; ++i) d[i] = nd[i];
            // the flat primitive just left: a triangle by its slot, a plane by id
            last = hid < P.id_sph0 ? hloc : (hid >= P.id_pln0 ? hid : -1);
            ++b;
        }
    }
};

// Waves per SIMD the register allocation is held to: the dual-number state
// needs about 300 registers a lane, so one wave fits without spilling; two
// waves (256 registers and some spills to scratch) hide more latency and are
// faster (measured: one 3.18 s, two 2.08 s, three 2.89 s for all gradients of
// the large scene at every 4th ray).
#ifndef UR_REPLAY_WAVES
#define UR_REPLAY_WAVES 2
#endif
template <bool LEN, int K>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(UR_REPLAY_WAVES, UR_REPLAY_WAVES))) void k_replay(
    AdjParams A) {
    Acc acc;
    acc.val = 0.0;
    for (int j = 0; j < kAdjTan; ++j) acc.tan[j] = 0.0;
    for (int m = 0; m < kAdjMat; ++m) acc.alpha[m] = 0.0;
    const TraceParams &P = A.P;
    __shared__ int2 s_stack[kStack * 256];
    const LdsStack stk{s_stack + threadIdx.x, 256};
    Rep<K>::template replay_paths<LEN>(A, acc, stk);
    // wavefront sums, one atomic per wavefront and output
    const int lane = threadIdx.x & 63;
    if (A.value_out) {
        double v = acc.val;
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0 && v != 0.0) atomicAdd(A.value_out, v);
    }
    if (A.n_tan > 0) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (j >= A.n_tan || !A.tan[j].out) continue;
            double v = acc.tan[j];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0 && v != 0.0) atomicAdd(A.tan[j].out, v);
        }
    } else if (LEN && A.grad_alpha) {
        for (int m = 0; m < kAdjMat && m < P.n_mat; ++m) {
            double v = acc.alpha[m];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0 && v != 0.0) atomicAdd(A.grad_alpha + m, v);
        }
    }
}

__global__ void k_zero_f64(double *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

}  // namespace

hipError_t ur_launch_zero_f64(double *p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

namespace {
// Blocks of 256 that stay resident at once (the persistent grid).
template <class K>
hipError_t replay_blocks(K kernel, int64_t needed, unsigned &blocks) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0);
    if (e != hipSuccess) return e;
    const int64_t resident = (int64_t)cus * (per_cu > 0 ? per_cu : 1);
    blocks = (unsigned)(needed < resident ? (needed > 0 ? needed : 1) : resident);
    return hipSuccess;
}

__global__ void k_zero_u64(unsigned long long *p) {
    if (threadIdx.x == 0) *p = 0ull;
}
}  // namespace

hipError_t ur_launch_replay(const ur::TraceParams &p, int n_tan, const AdjTangent *tans, const float *g,
                            float *grad_amp, double *grad_alpha, double *value_out, double kappa, int attach_choice,
                            const AdjRecord &rec, hipStream_t s) {
    const int64_t n = rec.end - rec.begin;
    if (n <= 0) return hipGetLastError();
    if (!rec.next || n_tan < 0 || (n_tan > 0 && !tans)) return hipErrorInvalidValue;
    AdjParams A;
    A.P = p;
    A.g = g;
    A.kappa = kappa;
    A.attach_choice = attach_choice;
    A.rec = rec;
    const int64_t needed = (n + 255) / 256;
    unsigned blocks = 1;
    hipError_t e;
    if (n_tan == 0) {
        // the value pass
        A.n_tan = 0;
        A.grad_amp = grad_amp;
        A.grad_alpha = grad_alpha;
        A.value_out = value_out;
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, rec.next);
        if (grad_alpha) {
            if ((e = replay_blocks(k_replay<true, 1>, needed, blocks)) != hipSuccess) return e;
            hipLaunchKernelGGL((k_replay<true, 1>), dim3(blocks), dim3(256), 0, s, A);
        } else {
            if ((e = replay_blocks(k_replay<false, 1>, needed, blocks)) != hipSuccess) return e;
            hipLaunchKernelGGL((k_replay<false, 1>), dim3(blocks), dim3(256), 0, s, A);
        }
        return hipGetLastError();
    }
    // tangent passes, kAdjTan parameter directions each
    A.grad_amp = nullptr;
    A.grad_alpha = nullptr;
    A.value_out = nullptr;
    if ((e = replay_blocks(k_replay<false, kAdjTan>, needed, blocks)) != hipSuccess) return e;
    for (int j0 = 0; j0 < n_tan; j0 += kAdjTan) {
        A.n_tan = n_tan - j0 < kAdjTan ? n_tan - j0 : kAdjTan;
        for (int j = 0; j < kAdjTan; ++j) A.tan[j] = j < A.n_tan ? tans[j0 + j] : AdjTangent{0, 0, 0, nullptr};
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, rec.next);
        hipLaunchKernelGGL((k_replay<false, kAdjTan>), dim3(blocks), dim3(256), 0, s, A);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------- direct-hit edge terms
// A direct hit is binned into the element whose face holds its landing
// point, so its contribution jumps where the landing point crosses an
// element edge, an end of the aperture or an elevation edge; a geometry
// parameter moves those crossings.  The term is integrated exactly along the
// emission origin's lateral coordinate u0 (Eq. 4) of every path family, the
// direction, elevation coordinate and choices held fixed: by the Leibniz rule
// each crossing at u0* adds [F] dx_n/dtheta / |dx_n/du0|, F = c g(t) and [F]
// its jump across the edge in the direction of increasing x_n.  The family is
// evaluated at n_scan + 1 evenly spaced u0; an interval whose ends follow
// different sequences of primitives and choices is halved (down to 1e-12 or
// 48 levels), and inside an interval that follows one sequence every edge
// between its landings is located by safeguarded Newton steps.  On a
// convex array the origin moves along the element's arc and the direction
// turns with it, the landing coordinate across the elements is the arc
// angle, and each element receives against its own normal.  Plane-wave
// transmits, smooth boundaries, uniform emission, choice attached.  Dual
// numbers carry two tangents: u0 and one parameter direction; the scan and
// the crossings are found once per family, and each crossing is replayed
// once per parameter for its derivative.
namespace {
using E2 = Rep<2>;
using D2 = DK<2>;
static_assert(kAdjTan >= 2, "the edge pass carries two directions: u0 and one parameter");

struct EdgeHit {
    bool inside;             // the landing point lies on an element
    int er;                  // that element
    D2 x[2];                 // landing coordinates: across the elements (x, or the arc angle), y
    D2 c, t;                 // weight x receive directivity of element er, arrival time
    double w, d[3];          // the weight and the arrival direction (values)
    unsigned long long sig;  // the sequence of primitives and choices
};

// Weight x receive directivity (Eq. 13) of the landing h into element er,
// against that element's normal.
__device__ __forceinline__ double edge_c(const TraceParams &P, const EdgeHit &h, int er) {
    double ca;
    if (P.convex) {
        const double4 g = P.elem[er];
        ca = -(h.d[0] * g.z + h.d[2] * g.w);
    } else {
        ca = -h.d[2];
    }
    const double al = acos(fmin(1.0, fmax(-1.0, ca)));
    if (!(al <= P.alpha_c)) return 0.0;
    return h.w * (al <= P.alpha_m ? 1.0 : (P.alpha_c - al) / (P.alpha_c - P.alpha_m));
}

// The family's path at origin coordinate u0 (tangent 0: u0; tangent 1: the
// parameter direction dir, kind 0 for none); true if it ends on the array's
// plane within the bounce, time and length limits.
__device__ bool edge_path(const AdjParams &A, const AdjTangent &dir, int tx, int e, uint32_t ray, double u0,
                          LdsStack stk, EdgeHit &out) {
    const TraceParams &P = A.P;
    uint32_t x[4];
    draw(P, ray, e, tx, 0, 0, 0, x);
    double dv0[3];
    hemisphere(u01(x[2]), u01(x[3]), dv0);
    D2 o[3], d[3];
    o[1] = E2::dd((u01(x[1]) - 0.5) * P.elev);
    if (P.convex) {
        // on the element's arc; the direction turns with the local normal
        const double ph = ((double)e - 0.5 * (double)(P.E - 1) + (u0 - 0.5)) * P.dphi;
        double sp, cp;
        sincos(ph, &sp, &cp);
        const double h = sin(0.5 * ph);
        o[0] = E2::dd(P.radius * sp);
        o[0].t[0] = P.radius * cp * P.dphi;
        o[2] = E2::dd(-2.0 * P.radius * h * h);
        o[2].t[0] = -2.0 * P.radius * h * cos(0.5 * ph) * P.dphi;
        d[0] = E2::dd(dv0[0] * cp + dv0[2] * sp);
        d[0].t[0] = (-dv0[0] * sp + dv0[2] * cp) * P.dphi;
        d[1] = E2::dd(dv0[1]);
        d[2] = E2::dd(dv0[2] * cp - dv0[0] * sp);
        d[2].t[0] = (-dv0[2] * sp - dv0[0] * cp) * P.dphi;
    } else {
        o[0] = E2::dd(P.xe[e] + (u0 - 0.5) * P.pitch);
        o[0].t[0] = P.pitch;
        o[2] = E2::dd(0.0);
        for (int i = 0; i < 3; ++i) d[i] = E2::dd(dv0[i]);
    }
    D2 w = E2::dd(dv0[2] / (P.n_per_tx * (1.0 / (2.0 * M_PI)))), t = E2::dd(P.tau[(int64_t)tx * P.E + e]);
    D2 len = E2::dd(0.0);
    int med = P.top_medium;
    int64_t last = -1;
    unsigned long long sig = 1469598103934665603ull;
    for (int b = 0; b <= P.B; ++b) {
        const double ov[3] = {o[0].v, o[1].v, o[2].v}, dv[3] = {d[0].v, d[1].v, d[2].v};
        Counters cnt;
        const Hit h = closest_hit<false>(P, ov, dv, last, stk, cnt);
        const int64_t hid = h.id;
        const int hloc = h.local, face = h.face;
        D2 th, sc[3];
        double srad = 0.0;
        if (hid == P.id_box && face == 6) {
            const D2 R = E2::dd(P.radius);
            const D2 aa = d[0] * d[0] + d[2] * d[2], bq = o[0] * d[0] + (o[2] + R) * d[2];
            const D2 cq = o[0] * o[0] + o[2] * (o[2] + E2::dd(2.0) * R);
            th = cq / (-bq + dsqrt(bq * bq - aa * cq));
        } else if (hid == P.id_box) {
            const int ax = face % 3;
            th = (E2::dd(P.box[face]) - o[ax]) / d[ax];
        } else if (hid < P.id_sph0) {
            const double *tr = P.tri + 9 * (int64_t)hloc, *v0 = tr, *e1 = tr + 3, *e2 = tr + 6;
            const D2 tq[3] = {o[0] - E2::dd(v0[0]), o[1] - E2::dd(v0[1]), o[2] - E2::dd(v0[2])};
            const D2 pv[3] = {d[1] * E2::dd(e2[2]) - d[2] * E2::dd(e2[1]), d[2] * E2::dd(e2[0]) - d[0] * E2::dd(e2[2]),
                              d[0] * E2::dd(e2[1]) - d[1] * E2::dd(e2[0])};
            const D2 qq[3] = {tq[1] * E2::dd(e1[2]) - tq[2] * E2::dd(e1[1]),
                              tq[2] * E2::dd(e1[0]) - tq[0] * E2::dd(e1[2]),
                              tq[0] * E2::dd(e1[1]) - tq[1] * E2::dd(e1[0])};
            th = ddot(qq, e2) / ddot(pv, e1);
        } else if (hid < P.id_pln0) {
            const double *sp = P.sph + 4 * hloc;
            for (int i = 0; i < 3; ++i) {
                sc[i] = E2::dd(sp[i]);
                sc[i].t[1] = (dir.kind == 2 && dir.index == hloc && dir.coord == i) ? 1.0 : 0.0;
            }
            srad = sp[3];
            const D2 oc[3] = {o[0] - sc[0], o[1] - sc[1], o[2] - sc[2]};
            const D2 bb = ddot(oc, d), cc = ddot(oc, oc) - E2::dd(srad * srad);
            const D2 sq = dsqrt(bb * bb - cc);
            const D2 r0 = -bb - sq;
            th = r0.v > kEpsT ? r0 : -bb + sq;
        } else {
            const double *pl = P.pln + 4 * hloc;
            th = (E2::dd(pl[3]) - ddot(o, pl)) / ddot(d, pl);
        }
        th.v = h.t;
        D2 tseg = th;
        bool clipped = false;
        if (len.v + tseg.v > P.max_path) {
            tseg = E2::dd(P.max_path) - len;
            clipped = true;
        }
        const Material M = P.mat[med];
        w = w * dexp(-(M.ka * tseg));
        t = t + M.inv_c * tseg;
        len = len + tseg;
        for (int i = 0; i < 3; ++i) o[i] = o[i] + tseg * d[i];
        if (clipped || t.v >= P.t_max) return false;
        sig = (sig ^ (unsigned long long)(8 * (hid + 1) + face + 1)) * 1099511628211ull;
        if (hid == P.id_box) {
            int er;
            D2 ca;
            if (P.convex) {
                // the arc angle atan2(x, z + R) of the landing point
                if (face != 6) return false;
                const D2 zc = o[2] + E2::dd(P.radius);
                const double r2 = o[0].v * o[0].v + zc.v * zc.v;
                D2 ph = E2::dd(atan2(o[0].v, zc.v));
                for (int k = 0; k < 2; ++k) ph.t[k] = (zc.v * o[0].t[k] - o[0].v * zc.t[k]) / r2;
                out.x[0] = ph;
                out.inside = fabs(ph.v) <= P.half_arc && fabs(o[1].v) <= 0.5 * P.elev;
                er = (int)floor(ph.v / P.dphi + 0.5 * (double)P.E);
                er = er < 0 ? 0 : (er > P.E - 1 ? P.E - 1 : er);
                const double4 g = P.elem[er];
                ca = -(d[0] * E2::dd(g.z) + d[2] * E2::dd(g.w));
            } else {
                if (face != 2) return false;
                out.x[0] = o[0];
                out.inside = fabs(o[0].v) <= P.half_ap && fabs(o[1].v) <= 0.5 * P.elev;
                er = (int)floor((o[0].v + P.half_ap) / P.pitch);
                er = er < 0 ? 0 : (er > P.E - 1 ? P.E - 1 : er);
                ca = -d[2];
            }
            out.x[1] = o[1];
            out.er = er;
            out.w = w.v;
            for (int i = 0; i < 3; ++i) out.d[i] = d[i].v;
            const D2 al = dacos(ca);
            out.c = al.v <= P.alpha_c
                        ? w * (al.v <= P.alpha_m ? E2::dd(1.0) : (E2::dd(P.alpha_c) - al) / E2::dd(P.alpha_c - P.alpha_m))
                        : E2::dd(0.0);
            out.t = t;
            out.sig = sig;
            return true;
        }
        if (b == P.B) return false;
        D2 ng[3];
        int mf, mb;
        if (hid < P.id_sph0) {
            double nv[3];
            tri_normal(P, hloc, nv);
            for (int i = 0; i < 3; ++i) ng[i] = E2::dd(nv[i]);
            mf = P.tri_mat[2 * hloc];
            mb = P.tri_mat[2 * hloc + 1];
        } else if (hid < P.id_pln0) {
            for (int i = 0; i < 3; ++i) ng[i] = (o[i] - sc[i]) / E2::dd(srad);
            mf = P.sph_mat[2 * hloc];
            mb = P.sph_mat[2 * hloc + 1];
        } else {
            const double *pl = P.pln + 4 * hloc;
            for (int i = 0; i < 3; ++i) ng[i] = E2::dd(pl[i]);
            mf = P.pln_mat[2 * hloc];
            mb = P.pln_mat[2 * hloc + 1];
        }
        int before, after;
        if (ddot(d, ng).v < 0.0) {
            before = mf;
            after = mb;
        } else {
            before = mb;
            after = mf;
            for (int i = 0; i < 3; ++i) ng[i] = -ng[i];
        }
        D2 z1 = E2::dd(P.mat[before].Z), z2 = E2::dd(P.mat[after].Z);
        z1.t[1] = (dir.kind == 1 && dir.index == before) ? 1.0 : 0.0;
        z2.t[1] = (dir.kind == 1 && dir.index == after) ? 1.0 : 0.0;
        draw(P, ray, e, tx, b, 1, 0, x);
        const double y = u01(x[0]);
        const D2 cos_r = -ddot(d, ng);
        const D2 eta = z1 / z2;
        const D2 rad = E2::dd(1.0) - eta * eta * (E2::dd(1.0) - cos_r * cos_r);
        D2 R = E2::dd(1.0), cos_t = E2::dd(0.0);
        if (rad.v >= 0.0) {
            cos_t = dsqrt(rad);
            const D2 den = z1 * cos_r + z2 * cos_t;
            if (den.v != 0.0) {
                const D2 Ar = (z1 * cos_r - z2 * cos_t) / den;
                R = Ar * Ar;
            }
        }
        D2 nd[3];
        const bool refl = y < R.v;
        if (refl) {
            for (int i = 0; i < 3; ++i) nd[i] = d[i] + E2::dd(2.0) * cos_r * ng[i];
            w = w * (R / E2::dd(R.v));
            med = before;
        } else {
            const D2 f = eta * cos_r - cos_t;
            for (int i = 0; i < 3; ++i) nd[i] = eta * d[i] + f * ng[i];
            const D2 Tr = E2::dd(1.0) - R;
            w = w * (Tr / E2::dd(Tr.v));
            med = after;
        }
        const D2 l = dsqrt(ddot(nd, nd));
        for (int i = 0; i < 3; ++i) d[i] = nd[i] / l;
        sig = (sig ^ (unsigned long long)(2 + (refl ? 1 : 0))) * 1099511628211ull;
        last = hid < P.id_sph0 ? hloc : (hid >= P.id_pln0 ? hid : -1);
    }
    return false;
}

// One end of a scanned interval.
struct EdgeEnd {
    double u, x, y;
    unsigned long long sig;
    bool have;
};

constexpr AdjTangent kNoDirection{0, 0, 0, nullptr};

__device__ __forceinline__ EdgeEnd edge_end(const AdjParams &A, int tx, int e, uint32_t ray, double u, LdsStack stk) {
    EdgeHit h;
    EdgeEnd r;
    r.u = u;
    r.have = edge_path(A, kNoDirection, tx, e, ray, u, stk, h);
    r.x = r.have ? h.x[0].v : 0.0;
    r.y = r.have ? h.x[1].v : 0.0;
    r.sig = r.have ? h.sig : 0ull;
    return r;
}

// The u0 in (ua, ub) where landing coordinate k crosses X (Newton steps kept
// inside the bracket, bisection when a step leaves it), on paths with the
// sequence sig; false if the sequence changes on the way.
__device__ bool edge_root(const AdjParams &A, int tx, int e, uint32_t ray, double ua, double ub, double fa, int k,
                          double X, unsigned long long sig, LdsStack stk, double &root) {
    double u = 0.5 * (ua + ub);
    EdgeHit out;
    for (int it = 0; it < 100; ++it) {
        root = u;
        if (!edge_path(A, kNoDirection, tx, e, ray, u, stk, out) || out.sig != sig) return false;
        const double f = out.x[k].v - X, df = out.x[k].t[0];
        if (f == 0.0 || ub - ua < 1e-15) return true;
        if ((f < 0.0) == (fa < 0.0)) {
            ua = u;
            fa = f;
        } else {
            ub = u;
        }
        double un = df != 0.0 ? u - f / df : 0.5 * (ua + ub);
        if (!(un > ua && un < ub)) un = 0.5 * (ua + ub);
        if (un == u) return true;
        u = un;
    }
    return true;
}

// Parameter p of the edge pass: impedances first, then sphere coordinates.
__device__ __forceinline__ AdjTangent edge_direction(const TraceParams &P, int p) {
    return p < P.n_mat ? AdjTangent{1, p, 0, nullptr} : AdjTangent{2, (p - P.n_mat) / 3, (p - P.n_mat) % 3, nullptr};
}

// Adds the jump term of a crossing of landing coordinate k at u0 = root, with
// jump(hit) the jump of F there, for every parameter to acc.
template <class J>
__device__ void edge_terms(const AdjParams &A, int tx, int e, uint32_t ray, double root, int k, LdsStack stk,
                           J jump, double *acc) {
    const TraceParams &P = A.P;
    const int np = P.n_mat + 3 * P.n_sph;
    for (int p = 0; p < np; ++p) {
        EdgeHit at;
        if (!edge_path(A, edge_direction(P, p), tx, e, ray, root, stk, at)) return;
        const double du = fabs(at.x[k].t[0]);
        if (!(du > 0.0)) return;
        const double jf = jump(at);
        if (jf == 0.0) return;
        acc[p] += jf * at.x[k].t[1] / du;
    }
}

// The edge crossings of one interval that follows one sequence (ends a, b).
__device__ void edge_crossings(const AdjParams &A, int tx, int e, uint32_t ray, const EdgeEnd &a, const EdgeEnd &b,
                               LdsStack stk, double *acc) {
    const TraceParams &P = A.P;
    const double half_el = 0.5 * P.elev;
    double root;
    const double lo = fmin(a.x, b.x), hi = fmax(a.x, b.x);
    // element edges and aperture ends (the edge k lies between elements k-1
    // and k), in x or in the arc angle
    const double x0 = P.convex ? -0.5 * (double)P.E * P.dphi : -P.half_ap, step = P.convex ? P.dphi : P.pitch;
    const int k0 = (int)ceil((lo - x0) / step) - 1, k1 = (int)floor((hi - x0) / step) + 1;
    for (int k = k0 < 0 ? 0 : k0; k <= (k1 > P.E ? P.E : k1); ++k) {
        const double X = P.convex ? ((double)k - 0.5 * (double)P.E) * P.dphi : -P.half_ap + (double)k * P.pitch;
        if (!(X > lo && X < hi)) continue;
        if (!edge_root(A, tx, e, ray, a.u, b.u, a.x - X, 0, X, a.sig, stk, root)) continue;
        edge_terms(A, tx, e, ray, root, 0, stk, [&](const EdgeHit &at) {
            if (!(fabs(at.x[1].v) <= half_el)) return 0.0;
            double gv, gs;
            const double fr = k < P.E && adj_at(A, tx, k, at.t.v, gv, gs) ? edge_c(P, at, k) * gv : 0.0;
            const double fl = k > 0 && adj_at(A, tx, k - 1, at.t.v, gv, gs) ? edge_c(P, at, k - 1) * gv : 0.0;
            return fr - fl;
        }, acc);
    }
    // elevation edges: inside below the edge in |y|
    for (int sgn = -1; sgn <= 1; sgn += 2) {
        const double Y = sgn * half_el;
        if (!((a.y - Y) * (b.y - Y) < 0.0)) continue;
        if (!edge_root(A, tx, e, ray, a.u, b.u, a.y - Y, 1, Y, a.sig, stk, root)) continue;
        edge_terms(A, tx, e, ray, root, 1, stk, [&](const EdgeHit &at) {
            if (!(fabs(at.x[0].v) <= (P.convex ? P.half_arc : P.half_ap))) return 0.0;
            double gv, gs;
            const double fin = adj_at(A, tx, at.er, at.t.v, gv, gs) ? at.c.v * gv : 0.0;
            return sgn > 0 ? -fin : fin;
        }, acc);
    }
}

// The family's edge term: the scan, the halving of intervals whose ends
// follow different sequences (a depth-first stack of intervals, the lower
// half first), and the crossings of the rest.
constexpr int kEdgeDepth = 48;
__device__ void edge_family(const AdjParams &A, int tx, int e, uint32_t ray, int n_scan, LdsStack stk, double *acc) {
    struct Item {
        EdgeEnd a, b;
        int depth;
    };
    Item st[kEdgeDepth + 2];
    EdgeEnd prev = edge_end(A, tx, e, ray, 0.0, stk);
    for (int j = 1; j <= n_scan; ++j) {
        const EdgeEnd cur = edge_end(A, tx, e, ray, (double)j / n_scan, stk);
        int sp = 0;
        st[sp++] = Item{prev, cur, 0};
        while (sp > 0) {
            const Item it = st[--sp];
            if (!it.a.have && !it.b.have) continue;
            if (!it.a.have || !it.b.have || it.a.sig != it.b.sig) {
                if (it.depth >= kEdgeDepth || it.b.u - it.a.u < 1e-12) continue;
                const EdgeEnd m = edge_end(A, tx, e, ray, 0.5 * (it.a.u + it.b.u), stk);
                st[sp++] = Item{m, it.b, it.depth + 1};   // (at most one entry per level stays pending)
                st[sp++] = Item{it.a, m, it.depth + 1};
                continue;
            }
            edge_crossings(A, tx, e, ray, it.a, it.b, stk, acc);
        }
        prev = cur;
    }
}

constexpr int kEdgeMaxParams = 32;
__global__ __launch_bounds__(256) void k_edges(AdjParams A, int n_scan, double *out_z, double *out_sph) {
    __shared__ int2 s_stack[kStack * 256];
    const LdsStack stk{s_stack + threadIdx.x, 256};
    const TraceParams &P = A.P;
    const int np = P.n_mat + 3 * P.n_sph;
    double acc[kEdgeMaxParams];
    for (int p = 0; p < kEdgeMaxParams; ++p) acc[p] = 0.0;
    const int64_t i = A.rec.begin + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < A.rec.end) {
        const int64_t q = i / P.per_el;
        const uint32_t ray = (uint32_t)((i - q * P.per_el) * P.stride + P.offset);
        edge_family(A, (int)(q / P.E), (int)(q % P.E), ray, n_scan, stk, acc);
    }
    for (int p = 0; p < np; ++p) {
        double v = acc[p];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        double *o = p < P.n_mat ? out_z + p : (out_sph ? out_sph + (p - P.n_mat) : nullptr);
        if (p < P.n_mat && !out_z) o = nullptr;
        if ((threadIdx.x & 63) == 0 && v != 0.0 && o) atomicAdd(o, v);
    }
}
}  // namespace

hipError_t ur_launch_edges(const ur::TraceParams &p, double *out_z, double *out_sph, const float *g, int n_scan,
                           hipStream_t s) {
    if (n_scan < 1 || (!out_z && !out_sph) || p.n_mat + 3 * p.n_sph > kEdgeMaxParams) return hipErrorInvalidValue;
    if (p.n_work <= 0) return hipSuccess;
    AdjParams A;
    A.P = p;
    A.n_tan = 0;
    A.g = g;
    A.grad_amp = nullptr;
    A.grad_alpha = nullptr;
    A.value_out = nullptr;
    A.kappa = 0.0;
    A.attach_choice = 1;
    A.rec = AdjRecord{0, 0, p.n_work, nullptr, nullptr, nullptr, nullptr};
    hipLaunchKernelGGL(k_edges, dim3((unsigned)((p.n_work + 255) / 256)), dim3(256), 0, s, A, n_scan, out_z, out_sph);
    return hipGetLastError();
}
