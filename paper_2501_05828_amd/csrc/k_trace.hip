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
// A closest-hit query first takes the box exit, the planes and the spheres
// (so its culling distance is tight from the first node), skips the tree if
// the segment misses the box of every triangle, and otherwise walks a
// four-wide BVH (64-byte quantised nodes, one triangle per leaf) in
// nearest-first order with a per-lane stack in LDS; the secondary rays'
// crossing queries and the exact fallback of an overflowing stack walk the
// same tree in its threaded (escape-index) binary layout, which needs no
// stack.  Scatterer captures come from a uniform grid walked by a 3D DDA
// whose cell intervals partition the segment, so every capture is reported
// once.
//
// The trace runs as two persistent kernels joined by a segment queue:
// k_extend advances each lane's closest-hit query by one or two node visits
// per step, tests the triangles of entered leaves in batches, shades
// finished queries in batches (interfaces, direct hits, termination) and
// queues the segments that can reach the scatterer grid;
// k_scatter walks the queued segments through the grid and queues the
// transducer-sampling candidates, whose secondary rays k_nee casts.  Lanes
// refill independently from chunks of work that a wavefront takes by guided
// self-scheduling (one atomic per chunk), so lanes do not idle behind long
// paths.  k_trace is the single-loop form of the same arithmetic, used to
// re-trace a range whose sampling queue overflowed; k_trace_rays (compiled in
// k_trace_rays.hip) runs it for explicit rays with an event log.
#include "closest_hit.h"
#include "trace_device.h"
#include "ultraray.h"

namespace {
using namespace ur;
using namespace ur::dev;

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

// Bins one arriving contribution into ch_raw with device-scope float atomics
// (or, in the deterministic mode, stages it for k_bin.hip).
template <bool COUNT, bool LOG>
__device__ __forceinline__ void record(const TraceParams &P, const EventLog &L, Counters &cnt, int kind, int tx,
                                       int e, int seg, int64_t id, double t, double v, const double *p, int e_emit,
                                       int cell) {
    log_event<LOG>(L, kind, tx, e, seg, id, t, v, p);
    if (!(t < P.t_max) || t < 0.0) {
        CNT(C_DROPPED);
        return;
    }
    CNT(C_RECORDS);
    if (P.rec && cell >= 0) {
        const unsigned long long slot = atomicAdd(P.rec_count, 1ull);
        if ((int64_t)slot < P.rec_cap)
            P.rec[slot] = RecordEntry{(uint32_t)(((int64_t)tx * P.E + e_emit) * kCells + cell), (float)fabs(v)};
    }
    const double x = t * P.fs;
    if constexpr (COUNT) {
        const double fr = x - floor(x);
        if (fr < 1e-5 || fr > 1.0 - 1e-5) ++cnt.v[C_EDGE];
    }
    if (P.det) {
        // deterministic binning: staged, binned after the trace in a fixed order
        const unsigned long long slot = atomicAdd(P.det_count, 1ull);
        if ((int64_t)slot < P.det_cap) P.det[slot] = DetRecord{x, v, (int64_t)tx * P.E + e};
        return;
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

constexpr int kChunk = kRayChunk;   // work items a wave takes from the range at a time (largest chunk)

// Guided self-scheduling: a wavefront takes about 1/8 of its share of the
// work still left (seen at its last grab), between 64 and kChunk items, so
// the end of a range is shared out in small pieces.
__device__ __forceinline__ unsigned long long guided_chunk(unsigned long long left) {
    const unsigned long long waves = (unsigned long long)gridDim.x * (blockDim.x >> 6);
    const unsigned long long c = left / (8ull * waves);
    return c < 64ull ? 64ull : (c > (unsigned long long)kChunk ? (unsigned long long)kChunk : c);
}
// lanes that must be waiting before a wavefront shades finished queries and
// starts new rays (extend), or refills segments (scatter): batching the
// divergent shading / refill code amortises it over many lanes
#ifndef UR_BATCH_EXTEND
#define UR_BATCH_EXTEND 24
#endif
#ifndef UR_BATCH_SCATTER
#define UR_BATCH_SCATTER 32
#endif
// lanes that must hold pending leaves before a wavefront of the extend
// kernel tests their triangles (or no lane can visit a node without first
// testing its pending leaves)
#ifndef UR_BATCH_LEAF
#define UR_BATCH_LEAF 12
#endif
// a second node visit in the same loop pass when this many lanes can take
// one (fewer passes through the batch tests)
#ifndef UR_SECOND_STEP
#define UR_SECOND_STEP 16
#endif
constexpr int kBatchExtend = UR_BATCH_EXTEND;
constexpr int kSecondStep = UR_SECOND_STEP;
constexpr int kBatchScatter = UR_BATCH_SCATTER;
constexpr int kBatchLeaf = UR_BATCH_LEAF;

// ----------------------------------------------- secondary ray (transducer sampling)
// Straight ray from q toward a chosen element centre: product of transmitted
// fractions and order-free sums of the attenuation and slowness changes at
// every crossing in (eps, dist - eps).  Returns false if blocked (T = 0).
template <bool COUNT>
__device__ __forceinline__ bool shadow(const TraceParams &P, const double *q, const double *vh, double dist,
                                       double &T, double &sum_a, double &sum_c, int &n_cross, Counters &cnt) {
    T = 1.0;
    sum_a = 0.0;
    sum_c = 0.0;
    n_cross = 0;
    const double lo = kEpsT, hi = dist - kEpsT;
    auto cross_at = [&](double t, const double *ng, int mf, int mb) {
        const double dn = dot3(vh, ng);
        const int before = dn < 0.0 ? mf : mb, after = dn < 0.0 ? mb : mf;
        const Material A = P.mat[before], Bm = P.mat[after];
        T *= transmit_fraction(A.Z, Bm.Z, fabs(dn));
        ++n_cross;
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
                    tri_normal(P, k, ng);
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

// Scatterer k captured at distance s along the segment (Sec. 2.3
// "Transducer Sampling"): the capture re-radiates toward a uniformly chosen
// element centre.  In two steps.  nee_point places the capture point q and
// returns false (a zero-valued capture) when no element at all can accept it:
// the cut-off test of nee_candidate only gets easier to meet as the lateral
// offset vx^2 to the drawn element grows, so if it holds already at vx = 0
// (with a relative margin far above the rounding of either side) it holds for
// every element, and the element draw is skipped.
template <bool COUNT>
__device__ __forceinline__ bool nee_point(const TraceParams &P, Counters &cnt, const double *o, const double *d,
                                          double s, NeeEntry &c) {
    c.q[0] = o[0] + s * d[0];
    c.q[1] = o[1] + s * d[1];
    c.q[2] = o[2] + s * d[2];
    const double cc = P.cos_alpha_c;
    if (cc >= 0.0 && !P.convex) {
        const double vy = c.q[1], mvz = c.q[2];
        if (mvz < 0.0 || mvz * mvz < cc * cc * (vy * vy + mvz * mvz) * (1.0 - 1e-9)) {
            CNT(C_SCAT_EVENTS);
            CNT(C_NEE_ZERO);
            return false;
        }
    }
    return true;
}

// The element draw and the receive directivity (Eq. 13) for a capture point
// placed by nee_point.  Fills the candidate and returns true if the
// directivity of the drawn element is non-zero.
// CONE_CONVEX = false: a variant without the convex array's cone-restricted
// element range (linear arrays, or the uniform choice)
template <bool COUNT, bool CONE_CONVEX = true>
__device__ __forceinline__ bool nee_candidate(const TraceParams &P, Counters &cnt, int tx, int e, uint32_t ray,
                                              int seg, int k, double amp, double w, double t, int med, double s,
                                              int cell, NeeEntry &c) {
    const double cc = P.cos_alpha_c;
    int e_lo, n_e;
    if (!elem_range<CONE_CONVEX>(P, c.q[0], c.q[1], c.q[2], e_lo, n_e)) {
        CNT(C_SCAT_EVENTS);
        CNT(C_NEE_ZERO);
        return false;
    }
    uint32_t x[4];
    draw(P, ray, e, tx, seg, 2, (uint32_t)k, x);
    const int er = e_lo + (int)(((uint64_t)x[0] * (uint64_t)n_e) >> 32);
    // cut-off of Eq. 13 without acos or sqrt: with v = element - q and n the
    // element normal, alpha > alpha_c  <=>  cos(alpha) = -v.n / |v| < cos(alpha_c)
    // (n = +z on a linear array: -v.n = q_z)
    const double vy = c.q[1];
    double mvz, r2;
    if (P.convex) {
        const double4 g = P.elem[er];
        const double vx = g.x - c.q[0], vz = g.y - c.q[2];
        mvz = -(vx * g.z + vz * g.w);
        r2 = vx * vx + vy * vy + vz * vz;
    } else {
        const double vx = P.xe[er] - c.q[0];
        mvz = c.q[2];
        r2 = vx * vx + vy * vy + mvz * mvz;
    }
    const double lhs = mvz * mvz, rhs = cc * cc * r2;
    const bool cut = cc >= 0.0 ? (mvz < 0.0 || lhs < rhs) : (mvz < 0.0 && lhs > rhs);
    CNT(C_SCAT_EVENTS);
    if (cut) {
        CNT(C_NEE_ZERO);
        return false;
    }
    const Material M = P.mat[med];
    c.wq = w * atten(-M.ka * s) * amp;
    c.tq = t + s * M.inv_c;
    c.tx = tx;
    c.er = er;
    c.med = med;
    c.seg = seg;
    c.k = k;
    c.e = e;
    c.ray = ray;
    c.cell = cell;
    c.ne = n_e;
    c.mis = -1.0f;
    return true;
}

// Casts the secondary ray of a candidate: straight toward the element centre,
// multiplied by the transmitted fraction of every boundary it crosses and by
// the attenuation and delay of the media along it; the element subtends
// area * cos(alpha) / r^2 of the 4 pi re-radiation, divided by the 1/E
// choice probability.
template <bool COUNT, bool LOG>
__device__ __forceinline__ void nee_cast(const TraceParams &P, const EventLog &L, Counters &cnt, const NeeEntry &c) {
    const Material M = P.mat[c.med];
    const double4 g = P.convex ? P.elem[c.er] : make_double4(P.xe[c.er], 0.0, 0.0, 1.0);
    const double v[3] = {g.x - c.q[0], 0.0 - c.q[1], g.y - c.q[2]};
    const double dist = sqrt(dot3(v, v));
    const double vh[3] = {v[0] / dist, v[1] / dist, v[2] / dist};
    const double cos_a = P.convex ? -(vh[0] * g.z + vh[2] * g.w) : -vh[2];
    const double fdir = directivity(acos(fmin(1.0, fmax(-1.0, cos_a))), P.alpha_m, P.alpha_c);
    if (fdir <= 0.0) return;   // exactly at the cut-off
    CNT(C_NEE_CAST);
    double T, sum_a, sum_c;
    int n_cross;
    if (!shadow<COUNT>(P, c.q, vh, dist, T, sum_a, sum_c, n_cross, cnt)) {
        CNT(C_NEE_BLOCKED);
        return;
    }
    // a rough boundary's secondary ray shares its path with the direct hits
    // of the primary ray's next segment (balance-heuristic weight); if its
    // straight path crosses a boundary, the primary ray would interact there
    // instead, and the echo through that boundary reaches the element only as
    // the primary ray's own continuation, already counted: it records nothing
    if (c.mis >= 0.0f && n_cross > 0) {
        CNT(C_NEE_BLOCKED);
        return;
    }
    const double att = atten(-(M.ka * dist + sum_a));
    const double tc = c.tq + dist * M.inv_c + sum_c;
    double val = c.wq * (double)c.ne * P.area_e * cos_a * fdir / (4.0 * M_PI * dist * dist) * T * att;
    if (c.mis >= 0.0f) val *= (double)c.mis;
    record<COUNT, LOG>(P, L, cnt, c.mis >= 0.0f ? 5 : 1, c.tx, c.er, c.seg, c.k, tc, val, c.q, c.e, c.cell);
}

// Transducer sampling at a rough boundary (Sec. 2.3: at a boundary the
// primary ray first sends a secondary ray, then the boundary draws its own
// continuation).  The target is drawn as for scatterers (purpose 4 of the
// counters); the entry carries the boundary's scattering toward it
// (rough_fcos), times 4 pi so that nee_cast's isotropic 1/(4 pi) cancels,
// starts in the medium on the target's side, and carries the balance
// heuristic p_nee / (p_nee + p) with p_nee = r^2 / (K A cos(alpha)) the
// density, per solid angle, of drawing a point of the element's face and p
// the boundary sampler's density of the same direction.  n is the normal on
// the incident side, m_in and m_out the materials on its two sides.
template <bool COUNT, bool LOG, int MODE, bool CONVEX = true>
__device__ void surface_nee(const TraceParams &P, const EventLog &L, Counters &cnt, int tx, int e, uint32_t ray,
                            int cell, int seg, int id, const double *x, const double *d, const double *n, int m_in,
                            int m_out, double alpha, double w, double t) {
    CNT(C_SURF_EVENTS);
    // (a linear array hears x only if its nearest element centre in x does:
    // the same conservative test as for scatterer captures, no draw needed)
    const double cc = P.cos_alpha_c;
    if (cc >= 0.0 && !P.convex &&
        (x[2] < 0.0 || x[2] * x[2] < cc * cc * (x[1] * x[1] + x[2] * x[2]) * (1.0 - 1e-9))) {
        CNT(C_SURF_ZERO);
        return;
    }
    int e_lo, n_e;
    if (!elem_range<CONVEX>(P, x[0], x[1], x[2], e_lo, n_e)) {
        CNT(C_SURF_ZERO);
        return;
    }
    uint32_t xr[4];
    draw(P, ray, e, tx, seg, 4, 0, xr);
    const int er = e_lo + (int)(((uint64_t)xr[0] * (uint64_t)n_e) >> 32);
    const double4 g = P.convex ? P.elem[er] : make_double4(P.xe[er], 0.0, 0.0, 1.0);
    const double v[3] = {g.x - x[0], 0.0 - x[1], g.y - x[2]};
    const double dist = sqrt(dot3(v, v));
    const double od[3] = {v[0] / dist, v[1] / dist, v[2] / dist};
    const double cos_a = P.convex ? -(od[0] * g.z + od[2] * g.w) : -od[2];
    const double fdir = directivity(acos(fmin(1.0, fmax(-1.0, cos_a))), P.alpha_m, P.alpha_c);
    const double wi[3] = {-d[0], -d[1], -d[2]};
    double pdf = 0.0;
    const double fc = fdir > 0.0 ? rough_fcos(wi, n, P.mat[m_in].Z, P.mat[m_out].Z, alpha, od, pdf) : 0.0;
    if (!(fc > 0.0)) {
        CNT(C_SURF_ZERO);
        return;
    }
    const double p_nee = dist * dist / ((double)n_e * P.area_e * cos_a);
    NeeEntry c;
    c.q[0] = x[0];
    c.q[1] = x[1];
    c.q[2] = x[2];
    c.wq = w * fc * (4.0 * M_PI);
    c.tq = t;
    c.tx = tx;
    c.er = er;
    c.med = dot3(od, n) > 0.0 ? m_in : m_out;
    c.seg = seg;
    c.k = id;
    c.e = e;
    c.ray = ray;
    c.cell = cell;
    c.ne = n_e;
    c.mis = (float)(p_nee / (p_nee + pdf));
    if constexpr (LOG || MODE == kInlineNeeOnly) {
        nee_cast<COUNT, LOG>(P, L, cnt, c);
    } else {
        const unsigned long long slot = atomicAdd(P.nee_count, 1ull);
        if ((int64_t)slot < P.nee_cap) P.nee[slot] = c;
    }
}

// Captures on the segment [0, t_seg) from the scatterer grid.  Candidates are
// cast inline (explicit-ray logging and the overflow re-trace) or appended to
// the transducer-sampling queue.
template <bool COUNT, bool LOG, int MODE>
__device__ __forceinline__ void scatter_events(const TraceParams &P, const EventLog &L, Counters &cnt, int tx, int e,
                                               uint32_t ray, int seg, const double *o, const double *d, double w,
                                               double t, int med, double t_seg, int cell) {
    if (P.n_scat == 0) return;
    // FP32 prefilter on 16-byte items: the rounding of positions, direction
    // and products stays below ~6e-7 x the largest coordinate, well inside
    // the widening pre_m of the interval and the radius, so every capture of
    // the exact FP64 test below passes it
    const float of[3] = {(float)o[0], (float)o[1], (float)o[2]};
    const float df[3] = {(float)d[0], (float)d[1], (float)d[2]};
    dda_walk(P.grid, o, d, t_seg, [&](int gcell, double ta, double tb) {
        CNT(C_SCAT_CELLS);
        const int j1 = P.cell_start[gcell + 1];
        const float taf = (float)ta - P.pre_m, tbf = (float)tb + P.pre_m;
        for (int jb = P.cell_start[gcell]; jb < j1; jb += 4) {
            // four independent loads in flight, then the four prefilter tests
            float4 f[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                f[k] = jb + k < j1 ? P.items_f[jb + k] : make_float4(1e30f, 1e30f, 1e30f, 0.0f);
            unsigned pass = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float pf[3] = {f[k].x - of[0], f[k].y - of[1], f[k].z - of[2]};
                const float sf = pf[0] * df[0] + pf[1] * df[1] + pf[2] * df[2];
                const float qf[3] = {pf[0] - sf * df[0], pf[1] - sf * df[1], pf[2] - sf * df[2]};
                if (sf >= taf && sf <= tbf && qf[0] * qf[0] + qf[1] * qf[1] + qf[2] * qf[2] <= P.pre_r2)
                    pass |= 1u << k;
            }
            if constexpr (COUNT) cnt.v[C_SCAT_TESTS] += (uint32_t)min(4, j1 - jb);
            while (pass) {
                const int j = jb + __builtin_ctz(pass);
                pass &= pass - 1;
                const double4 sk = P.items[j];
                const double p[3] = {sk.x - o[0], sk.y - o[1], sk.z - o[2]};
                const double s = dot3(p, d);
                if (!(s >= ta && s < tb)) continue;
                const double pp[3] = {p[0] - s * d[0], p[1] - s * d[1], p[2] - s * d[2]};
                if (dot3(pp, pp) > P.r_s2) continue;
                NeeEntry c;
                if (!nee_point<COUNT>(P, cnt, o, d, s, c) ||
                    !nee_candidate<COUNT>(P, cnt, tx, e, ray, seg, P.item_id[j], sk.w, w, t, med, s, cell, c))
                    continue;
                if constexpr (LOG || MODE == kInlineNeeOnly) {
                    nee_cast<COUNT, LOG>(P, L, cnt, c);
                } else {
                    const unsigned long long slot = atomicAdd(P.nee_count, 1ull);
                    if ((int64_t)slot < P.nee_cap) P.nee[slot] = c;
                }
            }
        }
        return true;
    });
}

// ------------------------------------------------------------------ one path
struct RayState {
    double o[3], d[3], w, t, len;
    int64_t last;      // flat primitive just left (excluded from the next hit): a triangle's
                       // slot in BVH order, a plane's id; -1 if none
    int med, seg, tx, e;
    uint32_t ray;
    int cell;          // emission direction cell (32 x 32 grid), -1 for explicit rays
    // after a rough boundary with transducer sampling: the sampler's density of
    // the direction taken and the element range of its secondary ray (ne_prev
    // = 0 otherwise), for the balance heuristic of a direct hit that follows
    double pdf_prev = 0.0;
    int lo_prev = 0, ne_prev = 0;
};

// Appends the segment [0, t_seg) of R to the segment queue.  Called by the
// lanes of a wavefront that finish a closest-hit query in the same step: the
// first of them hands out the rest of the wavefront's current chunk of slots
// and, if that runs short, takes a new chunk of kSegChunk with one atomic for
// the remaining lanes; each lane writes its entry.  No slot is skipped except
// at the end of a wavefront's last chunk (marked unused by the kernel).
// Whether the segment o + t d, t in [0, t_end], can pass through the part of
// the scatterer grid box inside its acceptance wedge: FP32 slab and
// half-space tests (the segment's culling origin and reciprocals) against the
// box grown by 10 um and the wedge grown by 50 um.  The FP32 rounding moves
// the clip parameters by well under 1 um over the scene, so a segment that
// can capture a scatterer some element hears is never dropped; a zero
// direction component has a reciprocal of +-1e20, which keeps the slab test
// exact in sign.
__device__ __forceinline__ bool meets_grid(const TraceParams &P, const CullRay &cr, const double *d, double t_end) {
    const float ax = (P.grid_lo_f[0] - cr.ox) * cr.ix, bx = (P.grid_hi_f[0] - cr.ox) * cr.ix;
    const float ay = (P.grid_lo_f[1] - cr.oy) * cr.iy, by = (P.grid_hi_f[1] - cr.oy) * cr.iy;
    const float az = (P.grid_lo_f[2] - cr.oz) * cr.iz, bz = (P.grid_hi_f[2] - cr.oz) * cr.iz;
    float t0 = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), 0.0f));
    float t1 = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), cull_tmax(t_end) + 1e-5f));
    if (P.grid_wb_f >= 0.0f) {
        const float dy = (float)d[1], dz = (float)d[2];
#pragma unroll
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            const float c0 = (float)sgn * cr.oy - P.grid_wb_f * cr.oz - P.grid_wa_f;
            const float c1 = (float)sgn * dy - P.grid_wb_f * dz;
            const float tb = -c0 * __builtin_amdgcn_rcpf(c1);
            t1 = c1 > 0.0f ? fminf(t1, tb) : t1;
            t0 = c1 < 0.0f ? fmaxf(t0, tb) : t0;
            if (c1 == 0.0f && c0 > 0.0f) t1 = -1.0f;
        }
    }
    return t0 <= t1;
}

__device__ __forceinline__ void push_segment(const TraceParams &P, const RayState &R, double t_seg,
                                             volatile unsigned long long *chunk) {
    const unsigned long long mask = __ballot(1);
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)mask) - 1;
    const int n = __popcll(mask);
    unsigned long long beg = 0, fresh = 0, rem = 0;
    if (lane == leader) {
        beg = chunk[0];
        const unsigned long long end = chunk[1];
        rem = end - beg;
        if (rem < (unsigned long long)n) {
            fresh = atomicAdd(P.seg_count, (unsigned long long)kSegChunk);
            chunk[0] = fresh + (n - rem);
            chunk[1] = fresh + kSegChunk;
        } else {
            chunk[0] = beg + n;
        }
    }
    auto bcast = [&](unsigned long long v) {
        const uint32_t lo = __shfl((uint32_t)v, leader), hi = __shfl((uint32_t)(v >> 32), leader);
        return ((unsigned long long)hi << 32) | lo;
    };
    beg = bcast(beg);
    fresh = bcast(fresh);
    rem = bcast(rem);
    const unsigned long long rank = __popcll(mask & ((1ull << lane) - 1ull));
    const unsigned long long slot = rank < rem ? beg + rank : fresh + (rank - rem);
    if ((int64_t)slot >= P.seg_cap) {
        atomicAdd(P.seg_lost, 1ull);
        return;
    }
    // streaming (non-temporal) stores: the queue is read once, by another
    // kernel, and should not displace the tree and grid from the L2
    SegHot &E = P.segq[slot];
    for (int k = 0; k < 3; ++k) {
        __builtin_nontemporal_store(R.o[k], &E.o[k]);
        __builtin_nontemporal_store(R.d[k], &E.d[k]);
    }
    __builtin_nontemporal_store(t_seg, &E.t_seg);
    __builtin_nontemporal_store(R.ray, &E.ray);
    __builtin_nontemporal_store(((uint32_t)R.tx << 16) | (uint32_t)R.e, &E.txe);
    SegCold &C = P.segc[slot];
    __builtin_nontemporal_store(R.w, &C.w);
    __builtin_nontemporal_store(R.t, &C.t);
    __builtin_nontemporal_store(R.med, &C.med);
    __builtin_nontemporal_store(R.seg, &C.seg);
    __builtin_nontemporal_store(R.cell, &C.cell);
}

// The rest of a segment once its closest hit h is known: scatterer captures
// on [0, t_seg) (inline, or queued for the scatter kernel when SPLIT), then
// transport and the hit itself (see advance).  Returns false when the ray
// has ended.
// Balance-heuristic weight of a direct hit into element er at distance r
// (the segment just traced) and receive cosine ca, when the segment started
// at a rough boundary whose secondary ray could have drawn er: p / (p +
// p_nee) with p the boundary sampler's density of the direction taken and
// p_nee = r^2 / (K A ca).  1 otherwise.
template <bool ROUGH>
__device__ __forceinline__ double direct_mis(const TraceParams &P, const RayState &R, int er, double r, double ca) {
    if (!ROUGH || R.ne_prev == 0 || er < R.lo_prev || er >= R.lo_prev + R.ne_prev) return 1.0;
    const double p_nee = r * r / ((double)R.ne_prev * P.area_e * ca);
    return R.pdf_prev / (R.pdf_prev + p_nee);
}

template <bool COUNT, bool LOG, int MODE, bool SPLIT, bool ROUGH = true, bool CONVEX = true>
__device__ __forceinline__ bool after_hit(const TraceParams &P, const EventLog &L, Counters &cnt, RayState &R,
                                          const Hit &h, volatile unsigned long long *chunk, bool near_grid = true) {
    const int b = R.seg;
    double *o = R.o, *d = R.d;
    double t_seg = h.t;
    bool clipped = false;
    if (R.len + t_seg > P.max_path) {
        t_seg = P.max_path - R.len;
        clipped = true;
    }
    if constexpr (SPLIT) {
        if (near_grid && t_seg > 0.0) push_segment(P, R, t_seg, chunk);
    } else {
        scatter_events<COUNT, LOG, MODE>(P, L, cnt, R.tx, R.e, R.ray, b, o, d, R.w, R.t, R.med, t_seg, R.cell);
    }
    const Material M = P.mat[R.med];
    R.w *= atten(-M.ka * t_seg);
    R.t += t_seg * M.inv_c;
    R.len += t_seg;
    o[0] += t_seg * d[0];
    o[1] += t_seg * d[1];
    o[2] += t_seg * d[2];
    if (clipped) {
        CNT(C_TERM_PATH);
        log_event<LOG>(L, 4, R.tx, R.e, b, -3, R.t, R.w, o);
        return false;
    }
    if (R.t >= P.t_max) {
        CNT(C_TERM_TIME);
        log_event<LOG>(L, 4, R.tx, R.e, b, -2, R.t, R.w, o);
        return false;
    }
    if (h.id == P.id_box) {
        // (the acos is skipped where the cosine is clearly below cos alpha_c:
        // Eq. 13 is zero there, and the margin is far above acos's rounding)
        if (CONVEX && P.convex) {
            // the element whose arc holds the landing point; the receive
            // angle is taken to that element's normal
            if (h.face == 6 && fabs(o[1]) <= 0.5 * P.elev) {
                const double ph = atan2(o[0], o[2] + P.radius);
                if (fabs(ph) <= P.half_arc) {
                    int er = (int)floor(ph / P.dphi + 0.5 * (double)P.E);
                    er = er < 0 ? 0 : (er > P.E - 1 ? P.E - 1 : er);
                    const double4 g = P.elem[er];
                    const double ca = fmin(1.0, fmax(-1.0, -(d[0] * g.z + d[2] * g.w)));
                    const double fdir = directivity(acos(ca), P.alpha_m, P.alpha_c);
                    if (MODE != kInlineNeeOnly && fdir > 0.0) {
                        CNT(C_DIRECT);
                        record<COUNT, LOG>(P, L, cnt, 0, R.tx, er, b, -1, R.t,
                                           R.w * fdir * direct_mis<ROUGH>(P, R, er, t_seg, ca), o, R.e, R.cell);
                    }
                }
            }
        } else if (h.face == 2 && fabs(o[0]) <= P.half_ap && fabs(o[1]) <= 0.5 * P.elev &&
                   -d[2] >= P.cos_alpha_c - 1e-9) {
            int er = (int)floor((o[0] + P.half_ap) / P.pitch);
            er = er < 0 ? 0 : (er > P.E - 1 ? P.E - 1 : er);
            const double ca = fmin(1.0, fmax(-1.0, -d[2]));
            const double fdir = directivity(acos(ca), P.alpha_m, P.alpha_c);
            if (MODE != kInlineNeeOnly && fdir > 0.0) {
                CNT(C_DIRECT);
                record<COUNT, LOG>(P, L, cnt, 0, R.tx, er, b, -1, R.t,
                                   R.w * fdir * direct_mis<ROUGH>(P, R, er, t_seg, ca), o, R.e, R.cell);
            }
        }
        CNT(C_TERM_BOX);
        log_event<LOG>(L, 4, R.tx, R.e, b, -1, R.t, R.w, o);
        return false;
    }
    if (b == P.B) {
        CNT(C_TERM_BOUNCE);
        log_event<LOG>(L, 4, R.tx, R.e, b, -4, R.t, R.w, o);
        return false;
    }
    // impedance boundary: geometric normal and the two materials
    double ng[3];
    int mf, mb;
    if (h.id < P.id_sph0) {
        tri_normal(P, h.local, ng);
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
    // (first word).  A boundary as rough as the rougher of its materials
    // (Eq. 12) acts about a microfacet normal mn drawn from the second and
    // third words, with weight factor |i.mn| G1(i) G1(o) / (|i.n| |mn.n|)
    // (Walter et al. 2007, Eq. 41); a microfacet facing away, or a new
    // direction on the wrong side of the surface, absorbs the ray.
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
    uint32_t x[4];
    draw(P, R.ray, R.e, R.tx, b, 1, 0, x);
    // (ROUGH = false: a kernel variant for scenes without rough materials)
    const double alpha = ROUGH ? fmax(P.mat[mf].rough, P.mat[mb].rough) : 0.0;
    double mn[3] = {ng[0], ng[1], ng[2]};
    if (ROUGH && alpha > 0.0) {
        // transducer sampling first, then the boundary's own draw
        if (P.rough_nee)
            surface_nee<COUNT, LOG, MODE, CONVEX>(P, L, cnt, R.tx, R.e, R.ray, R.cell, b, (int)h.id, o, d, ng, before, after,
                                          alpha, R.w, R.t);
        ggx_sample(ng, alpha, u01(x[1]), u01(x[2]), mn);
        if (!(-dot3(d, mn) > 0.0)) {
            CNT(C_TERM_ROUGH);
            log_event<LOG>(L, 4, R.tx, R.e, b, -5, R.t, R.w, o);
            return false;
        }
    }
    const double z1 = P.mat[before].Z, z2 = P.mat[after].Z;
    const double cos_r = -dot3(d, mn);
    const double eta = z1 / z2;
    const double rad = 1.0 - eta * eta * (1.0 - cos_r * cos_r);
    double R2, cos_t = 0.0;
    if (rad < 0.0) {
        R2 = 1.0;
    } else {
        cos_t = sqrt(rad);
        const double den = z1 * cos_r + z2 * cos_t;
        if (den == 0.0) {
            R2 = 1.0;
        } else {
            const double A = (z1 * cos_r - z2 * cos_t) / den;
            R2 = A * A;
        }
    }
    const double y = u01(x[0]);
    double nd[3];
    const bool refl = y < R2;
    if (refl) {
        for (int i = 0; i < 3; ++i) nd[i] = d[i] + 2.0 * cos_r * mn[i];
    } else {
        const double f = eta * cos_r - cos_t;
        for (int i = 0; i < 3; ++i) nd[i] = eta * d[i] + f * mn[i];
    }
    const double l = sqrt(dot3(nd, nd));
    nd[0] = nd[0] / l;
    nd[1] = nd[1] / l;
    nd[2] = nd[2] / l;
    if (ROUGH && alpha > 0.0) {
        const double co = dot3(nd, ng), cn = -dot3(d, ng);
        if (refl ? !(co > 0.0) : !(co < 0.0)) {
            CNT(C_TERM_ROUGH);
            log_event<LOG>(L, 4, R.tx, R.e, b, -5, R.t, R.w, o);
            return false;
        }
        R.w *= cos_r * ggx_g1(alpha, cn) * ggx_g1(alpha, fabs(co)) / (cn * dot3(mn, ng));
        if (P.rough_nee) {
            const double wi[3] = {-d[0], -d[1], -d[2]};
            rough_fcos(wi, ng, z1, z2, alpha, nd, R.pdf_prev);
            if (!elem_range<CONVEX>(P, o[0], o[1], o[2], R.lo_prev, R.ne_prev)) R.ne_prev = 0;
        } else {
            R.ne_prev = 0;
        }
    } else {
        R.ne_prev = 0;
    }
    if (before != R.med) CNT(C_MISMATCH);
    if (refl) {
        if (R2 >= 1.0) CNT(C_TIR);
        else CNT(C_REFLECT);
        R.med = before;
    } else {
        CNT(C_TRANSMIT);
        R.med = after;
    }
    d[0] = nd[0];
    d[1] = nd[1];
    d[2] = nd[2];
    log_event<LOG>(L, refl ? 2 : 3, R.tx, R.e, b, h.id, R.t, R.w, o);
    R.last = h.id < P.id_sph0 ? (int64_t)h.local : (h.id >= P.id_pln0 ? h.id : -1);
    R.seg = b + 1;
    return true;
}

// Advances a primary ray by one segment (Sec. 2.3 "Ray Traversal"): closest
// hit; scatterer captures on the segment; transport (attenuation
// exp(-alpha f d), delay d/c, path length); then the hit: leaving the box
// through the transducer aperture records weight x directivity into the
// element hit, any other box exit absorbs, an impedance boundary draws
// reflect-or-transmit (Eqs. 7-11) unless the interaction limit is reached.
// The ray also ends past max_path (segment clipped there) or when its time
// leaves the record window.  Returns false when the ray has ended.
template <bool COUNT, bool LOG, int MODE>
__device__ bool advance(const TraceParams &P, const EventLog &L, Counters &cnt, RayState &R, LdsStack stk) {
    CNT(C_SEGMENTS);
    const Hit h = closest_hit<COUNT>(P, R.o, R.d, R.last, stk, cnt);
    return after_hit<COUNT, LOG, MODE, false>(P, L, cnt, R, h, nullptr);
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

// Persistent trace kernel: wavefronts refill finished lanes with the next
// rays of the launch's work range (work item i -> transmit, element, ray with
// the ray index fastest) until the range is exhausted; each wave takes the
// range in chunks of kChunk items, so the shared counter sees one atomic per
// chunk instead of one per refill.  In the overflow
// re-trace mode the kernel does nothing unless the deferred run of the same
// range overflowed the transducer-sampling queue.  The register budget is
// capped at four wavefronts per SIMD: the loop is bound by the latency of
// dependent BVH-node and grid-cell loads, and measured on the bone phantom
// 4 waves/SIMD (128 VGPRs, a few spills) beats 2 (190 VGPRs, no spills) by
// 1.6x and 5-6 waves (heavier spilling) by 8-20%.
template <bool COUNT, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_trace(TraceParams P) {
    if (MODE == kInlineNeeOnly && (int64_t)*P.nee_count <= P.nee_cap) return;
    Counters cnt;
    if constexpr (COUNT) {
#pragma unroll
        for (int k = 0; k < kNumStats; ++k) cnt.v[k] = 0;
    }
    const EventLog L{};
    __shared__ int2 s_stack[kStack * 256];
    const LdsStack stk{s_stack + threadIdx.x, 256};
    const int lane = threadIdx.x & 63;
    const unsigned long long n_range = (unsigned long long)(P.work_end - P.work_begin);
    RayState R;
    bool active = false, exhausted = false;
    // wave-private chunk [cbeg, cend) of the range, refilled with one atomic
    // per kChunk work items (identical in every lane of the wave)
    unsigned long long cbeg = 0, cend = 0;
    while (true) {
        if (!exhausted) {
            const unsigned long long need = __ballot(!active);
            if (need) {
                if (cbeg >= cend) {
                    unsigned long long base = 0;
                    if (lane == 0) base = atomicAdd(P.work_next, (unsigned long long)kChunk);
                    const uint32_t lo = __shfl((uint32_t)base, 0), hi = __shfl((uint32_t)(base >> 32), 0);
                    base = ((unsigned long long)hi << 32) | lo;
                    if (base >= n_range) {
                        exhausted = true;
                    } else {
                        cbeg = base;
                        cend = base + kChunk < n_range ? base + kChunk : n_range;
                    }
                }
                if (!exhausted) {
                    const unsigned long long r = cbeg + __popcll(need & ((1ull << lane) - 1ull));
                    if (!active && r < cend) {
                        const int64_t i = P.work_begin + (int64_t)r;
                        const int64_t q = i / P.per_el;
                        R.ray = (uint32_t)((i - q * P.per_el) * P.stride + P.offset);
                        R.e = P.sa ? (int)q : (int)(q % P.E);   // synthetic aperture: transmit q is element q
                        R.tx = P.sa ? (int)q : (int)(q / P.E);
                        emit(P, R.tx, R.e, R.ray, R.o, R.d, R.w, R.cell);
                        R.t = P.tau[(int64_t)R.tx * P.E + R.e];
                        R.len = 0.0;
                        R.last = -1;
                        R.ne_prev = 0;
                        R.lo_prev = 0;
                        R.pdf_prev = 0.0;
                        R.med = P.top_medium;
                        R.seg = 0;
                        active = true;
                        CNT(C_RAYS);
                    }
                    const unsigned long long served = cbeg + __popcll(need);
                    cbeg = served < cend ? served : cend;
                }
            }
        }
        if (__ballot(active) == 0ull) break;
        if (active) active = advance<COUNT, false, MODE>(P, L, cnt, R, stk);
    }
    flush_counters<COUNT>(P, cnt);
}

// Extend kernel: the primary-ray side of a launch range.  Lanes refill
// independently (wave-private chunks of the range) and each step performs
// one four-wide node visit of the lane's current closest-hit query; a lane
// whose query completed shades the hit in the same step (Eqs. 7-11, direct
// hits, termination), queues the finished segment for the scatter kernel and
// starts its next query.  So no lane waits for the longest traversal of its
// wavefront, and the scatterer walk runs elsewhere with its own balance.
template <bool COUNT, bool ROUGH, bool CONVEX>
#ifndef UR_EXTEND_WAVES
#define UR_EXTEND_WAVES 4
#endif
#ifndef UR_EXTEND_WAVES_ROUGH
#define UR_EXTEND_WAVES_ROUGH 4
#endif
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ROUGH ? UR_EXTEND_WAVES_ROUGH : UR_EXTEND_WAVES))) void k_extend(TraceParams P) {
    Counters cnt;
    if constexpr (COUNT) {
#pragma unroll
        for (int k = 0; k < kNumStats; ++k) cnt.v[k] = 0;
    }
    const EventLog L{};
    __shared__ int2 s_stack[kStack * 256];
    __shared__ unsigned long long s_chunk[8];
    if (threadIdx.x < 8) s_chunk[threadIdx.x] = 0ull;
    __syncthreads();
    volatile unsigned long long *chunk = s_chunk + 2 * (threadIdx.x >> 6);
    const LdsStack stk{s_stack + threadIdx.x, 256};
    const int lane = threadIdx.x & 63;
    const unsigned long long n_range = (unsigned long long)(P.work_end - P.work_begin);
    RayState R;
    Hit h;
    CullRay cr;
    Pending pd;
    pd.mask = 0u;
    float tmf = 0.0f;
    int cur = 0, sp = 0, visits = 0;
    int npush = 0, ret = 0;   // segments this lane's ray may have queued; budget to hand back
    bool active = false, trav = false, overflow = false, exhausted = false, near_grid = false;
    unsigned long long cbeg = 0, cend = 0;
    auto start_segment = [&]() {
        CNT(C_SEGMENTS);
        // the box exit, then spheres and planes: their nearest hit bounds the
        // culling distance of the tree walk from its first node, and the
        // segment's length for the grid test (no triangle can make it longer)
        h = box_exit<CONVEX>(P, R.o, R.d);
        analytic_hits(P, R.o, R.d, R.last, h);
        cr = make_cull(R.o, R.d);
        tmf = cull_tmax(h.t);
        near_grid = P.n_scat > 0 && meets_grid(P, cr, R.d, h.t);
        cur = 0;
        sp = 0;
        overflow = false;
        trav = P.n_tnodes4 > 0 && meets_tree(P, cr, tmf);
    };
    while (true) {
        const unsigned long long busy = __ballot(active && (trav || pd.mask != 0u));
        if (!exhausted) {
            const unsigned long long need = __ballot(!active);
            if (need && (__popcll(need) >= kBatchExtend || busy == 0ull)) {
                if (cbeg >= cend) {
                    const unsigned long long want = guided_chunk(n_range > cend ? n_range - cend : 0ull);
                    bool admit = true;
                    if (P.seg_commit) {
                        // admission: the worst case of the new chunk, less what
                        // the rays finished since the last take did not queue
                        int back = ret;
                        for (int off = 32; off > 0; off >>= 1) back += __shfl_xor(back, off, 64);
                        ret = 0;
                        int ok = 0;
                        if (lane == 0) {
                            const unsigned long long add = want * (unsigned long long)(P.B + 1);
                            const unsigned long long delta = add - (unsigned long long)(long long)back;
                            const unsigned long long old = atomicAdd(P.seg_commit, delta);
                            ok = old + delta <= P.seg_limit;
                            // the first refusal closes the launch to every
                            // wavefront (the counter stays beyond any limit),
                            // so it drains at once as at the end of its range
                            if (!ok) atomicMax(P.seg_commit, ~0ull >> 2);
                        }
                        admit = __shfl(ok, 0) != 0;
                    }
                    unsigned long long base = n_range;
                    if (admit && lane == 0) base = atomicAdd(P.work_next, want);
                    const uint32_t lo = __shfl((uint32_t)base, 0), hi = __shfl((uint32_t)(base >> 32), 0);
                    base = ((unsigned long long)hi << 32) | lo;
                    if (base >= n_range) {
                        exhausted = true;
                    } else {
                        cbeg = base;
                        cend = base + want < n_range ? base + want : n_range;
                    }
                }
                if (!exhausted) {
                    const unsigned long long r = cbeg + __popcll(need & ((1ull << lane) - 1ull));
                    if (!active && r < cend) {
                        const int64_t i = P.work_begin + (int64_t)r;
                        const int64_t q = i / P.per_el;
                        R.ray = (uint32_t)((i - q * P.per_el) * P.stride + P.offset);
                        R.e = P.sa ? (int)q : (int)(q % P.E);   // synthetic aperture: transmit q is element q
                        R.tx = P.sa ? (int)q : (int)(q / P.E);
                        emit<CONVEX>(P, R.tx, R.e, R.ray, R.o, R.d, R.w, R.cell);
                        R.t = P.tau[(int64_t)R.tx * P.E + R.e];
                        R.len = 0.0;
                        R.last = -1;
                        R.ne_prev = 0;
                        R.lo_prev = 0;
                        R.pdf_prev = 0.0;
                        R.med = P.top_medium;
                        R.seg = 0;
                        active = true;
                        visits = 0;
                        npush = 0;
                        CNT(C_RAYS);
                        start_segment();
                    }
                    const unsigned long long served = cbeg + __popcll(need);
                    cbeg = served < cend ? served : cend;
                }
            }
        }
        if (__ballot(active) == 0ull) break;
        // a lane whose last visit entered leaves waits with them until enough
        // lanes (or every lane that could go on) do: then their triangles
        // are tested together
        const unsigned long long pend = __ballot(active && pd.mask != 0u);
        if (pend && (__popcll(pend) >= kBatchLeaf || __ballot(active && trav && pd.mask == 0u) == 0ull)) {
            if (active && pd.mask != 0u) {
                test_leaves<COUNT>(P, R.o, R.d, R.last, tmf, h, pd, cnt);
                pd.mask = 0u;
            }
        }
        auto visit = [&]() {
            float key[4];
            int val[4];
            wide_decode<COUNT>(P, cr, tmf, cur, key, val, pd, cnt);
            trav = wide_next(key, val, tmf, cur, sp, overflow, stk);
            ++visits;
        };
        if (active && trav && pd.mask == 0u) visit();
        if (__popcll(__ballot(active && trav && pd.mask == 0u)) >= kSecondStep) {
            if (active && trav && pd.mask == 0u) visit();
        }
        const unsigned long long done = __ballot(active && !trav && pd.mask == 0u);
        if (__popcll(done) < kBatchExtend && __ballot(active && (trav || pd.mask != 0u)) != 0ull) continue;
        if (active && !trav && pd.mask == 0u) {
            if (overflow) walk_threaded<COUNT>(P, R.o, R.d, R.last, cr, tmf, h, cnt);
            resolve_hit(P, h);
            npush += near_grid;   // after_hit queues the segment only if it meets the grid
            active = after_hit<COUNT, false, kDeferNee, true, ROUGH, CONVEX>(P, L, cnt, R, h, chunk, near_grid);
            if (!active) ret += P.B + 1 - npush;
            if (active) {
                start_segment();
            } else if (P.cost && R.cell >= 0) {
                // cost model of one path for a cost-aware proposal: node
                // visits + 2 per segment + 1.5 per grid cell of path length
                float c = (float)visits + 2.0f * (float)(R.seg + 1);
                if (P.n_scat > 0) c += 1.5f * (float)(R.len * P.grid.inv_h);
                atomicAdd(P.cost + ((int64_t)R.tx * P.E + R.e) * kCells + R.cell, c);
            }
        }
    }
    // the unused tail of this wavefront's last chunk of the segment queue
    const unsigned long long beg = chunk[0], end = chunk[1];
    for (unsigned long long k = beg + lane; k < end; k += 64)
        if ((int64_t)k < P.seg_cap) __builtin_nontemporal_store(kSegUnused, &P.segq[k].txe);
    flush_counters<COUNT>(P, cnt);
}

// Scatter kernel: captures on the queued segments (Sec. 2.3 "Transducer
// Sampling" candidates).  Lanes refill independently from the queue; each
// step either moves a lane's grid walk to its next cell or tests the next
// four items of its current cell (FP32 prefilter, then the exact FP64 test),
// with the same cell intervals as the inline walk, so each capture is found
// exactly once.  Candidates go to the transducer-sampling queue.
template <bool COUNT, bool CONE_CONVEX>
#ifndef UR_SCATTER_WAVES
#define UR_SCATTER_WAVES 4
#endif
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(UR_SCATTER_WAVES))) void k_scatter(TraceParams P) {
    Counters cnt;
    if constexpr (COUNT) {
#pragma unroll
        for (int k = 0; k < kNumStats; ++k) cnt.v[k] = 0;
    }
    const int lane = threadIdx.x & 63;
    const unsigned long long reserved = *P.seg_count;
    const unsigned long long n_seg = reserved < (unsigned long long)P.seg_cap ? reserved : (unsigned long long)P.seg_cap;
    const int limit = P.grid.n[0] + P.grid.n[1] + P.grid.n[2] + 3;
    double o[3], d[3], t_seg = 0.0, tb = 0.0;
    float of[3], df[3], taf = 0.0f, tbf = 0.0f;
    int j = 0, j1 = 0, visited = 0;
    uint32_t ray = 0, txe = 0;
    unsigned long long qslot = 0;
    DdaIter it;
    bool has = false, exhausted = false;
    unsigned long long cbeg = 0, cend = 0;
    auto enter_cell = [&]() {
        if (tb > it.ta) {
            CNT(C_SCAT_CELLS);
            j = P.cell_start[it.cell];
            j1 = P.cell_start[it.cell + 1];
            taf = (float)it.ta - P.pre_m;
            tbf = (float)tb + P.pre_m;
        } else {
            j = j1 = 0;
        }
    };
    while (true) {
        if (!exhausted) {
            const unsigned long long need = __ballot(!has);
            if (need && (__popcll(need) >= kBatchScatter || need == ~0ull)) {
                if (cbeg >= cend) {
                    const unsigned long long want = guided_chunk(n_seg > cend ? n_seg - cend : 0ull);
                    unsigned long long base = 0;
                    if (lane == 0) base = atomicAdd(P.seg_next, want);
                    const uint32_t lo = __shfl((uint32_t)base, 0), hi = __shfl((uint32_t)(base >> 32), 0);
                    base = ((unsigned long long)hi << 32) | lo;
                    if (base >= n_seg) {
                        exhausted = true;
                    } else {
                        cbeg = base;
                        cend = base + want < n_seg ? base + want : n_seg;
                    }
                }
                if (!exhausted) {
                    const unsigned long long r = cbeg + __popcll(need & ((1ull << lane) - 1ull));
                    if (!has && r < cend) {
                        const SegHot &E = P.segq[r];
                        txe = __builtin_nontemporal_load(&E.txe);
                        if (txe != kSegUnused) {
                            for (int k = 0; k < 3; ++k) {
                                o[k] = __builtin_nontemporal_load(&E.o[k]);
                                d[k] = __builtin_nontemporal_load(&E.d[k]);
                                of[k] = (float)o[k];
                                df[k] = (float)d[k];
                            }
                            t_seg = __builtin_nontemporal_load(&E.t_seg);
                            ray = __builtin_nontemporal_load(&E.ray);
                            qslot = r;
                            // the walk covers the part of the segment inside
                            // the grid box; t_seg becomes the end of that part
                            if (it.init(P.grid, o, d, t_seg, t_seg)) {
                                tb = it.bound(t_seg);
                                visited = 1;
                                enter_cell();
                                has = true;
                            }
                        }
                    }
                    const unsigned long long served = cbeg + __popcll(need);
                    cbeg = served < cend ? served : cend;
                }
            }
        }
        if (__ballot(has) == 0ull) break;
        if (!has) continue;
        // the next four items of the current cell, then (once the cell is
        // exhausted) the move to the next cell, in the same step
        if (j < j1) {
            float4 f[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                f[k] = j + k < j1 ? P.items_f[j + k] : make_float4(1e30f, 1e30f, 1e30f, 0.0f);
            unsigned pass = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float pf[3] = {f[k].x - of[0], f[k].y - of[1], f[k].z - of[2]};
                const float sf = pf[0] * df[0] + pf[1] * df[1] + pf[2] * df[2];
                const float qf[3] = {pf[0] - sf * df[0], pf[1] - sf * df[1], pf[2] - sf * df[2]};
                if (sf >= taf && sf <= tbf && qf[0] * qf[0] + qf[1] * qf[1] + qf[2] * qf[2] <= P.pre_r2)
                    pass |= 1u << k;
            }
            if constexpr (COUNT) cnt.v[C_SCAT_TESTS] += (uint32_t)min(4, j1 - j);
            while (pass) {
                const int jj = j + __builtin_ctz(pass);
                pass &= pass - 1;
                const double4 sk = P.items[jj];
                const double p[3] = {sk.x - o[0], sk.y - o[1], sk.z - o[2]};
                const double s = dot3(p, d);
                if (!(s >= it.ta && s < tb)) continue;
                const double pp[3] = {p[0] - s * d[0], p[1] - s * d[1], p[2] - s * d[2]};
                if (dot3(pp, pp) > P.r_s2) continue;
                NeeEntry c;
                if (!nee_point<COUNT>(P, cnt, o, d, s, c)) continue;
                // the capture-only part of the segment, read only here
                const SegCold &C = P.segc[qslot];
                if (!nee_candidate<COUNT, CONE_CONVEX>(P, cnt, (int)(txe >> 16), (int)(txe & 0xffffu), ray, C.seg, P.item_id[jj],
                                          sk.w, C.w, C.t, C.med, s, C.cell, c))
                    continue;
                const unsigned long long slot = atomicAdd(P.nee_count, 1ull);
                if ((int64_t)slot < P.nee_cap) P.nee[slot] = c;
            }
            j += 4;
        }
        if (j >= j1) {
            if (tb >= t_seg || visited >= limit || !it.step(P.grid, o, tb)) {
                has = false;
            } else {
                tb = it.bound(t_seg);
                ++visited;
                enter_cell();
            }
        }
    }
    flush_counters<COUNT>(P, cnt);
}

// Casts the queued secondary rays (one lane per candidate).  Skipped when the
// queue overflowed: the range is then re-traced with inline sampling.
template <bool COUNT>
__global__ __launch_bounds__(256) void k_nee(TraceParams P) {
    const unsigned long long n = *P.nee_count;
    if ((int64_t)n > P.nee_cap) return;
    Counters cnt;
    if constexpr (COUNT) {
#pragma unroll
        for (int k = 0; k < kNumStats; ++k) cnt.v[k] = 0;
    }
    const EventLog L{};
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * blockDim.x)
        nee_cast<COUNT, false>(P, L, cnt, P.nee[i]);
    flush_counters<COUNT>(P, cnt);
}

// (k_trace_rays is compiled only in k_trace_rays.hip, with its own flags.)
#ifdef UR_TRACE_RAYS_ONLY
__global__ __launch_bounds__(64) void k_trace_rays(TraceParams P, const ur_ray *rays, int64_t n, EventLog L) {
    __shared__ int2 s_stack[kStack * 64];
    const LdsStack stk{s_stack + threadIdx.x, 64};
    Counters cnt;
#pragma unroll
    for (int k = 0; k < kNumStats; ++k) cnt.v[k] = 0;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const ur_ray r = rays[i];
        RayState R;
        for (int k = 0; k < 3; ++k) {
            R.o[k] = r.o[k];
            R.d[k] = r.d[k];
        }
        R.w = r.w;
        R.t = r.t;
        R.len = 0.0;
        R.last = -1;
        R.ne_prev = 0;
        R.lo_prev = 0;
        R.pdf_prev = 0.0;
        R.med = (int)r.medium;
        R.seg = 0;
        R.tx = (int)r.tx;
        R.e = (int)r.elem;
        R.ray = (uint32_t)r.ray;
        R.cell = -1;
        ++cnt.v[C_RAYS];
        while (advance<true, true, kDeferNee>(P, L, cnt, R, stk)) {
        }
    }
    flush_counters<true>(P, cnt);
}
#else

__global__ void k_philox(const uint32_t *ctr, uint32_t *out, int64_t n, uint32_t k0, uint32_t k1) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t r[4];
    philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1, r);
    for (int j = 0; j < 4; ++j) out[4 * i + j] = r[j];
}
#endif  // UR_TRACE_RAYS_ONLY

}  // namespace

#ifndef UR_TRACE_RAYS_ONLY
namespace {
template <class K>
hipError_t resident_blocks(K kernel, int64_t needed, unsigned &blocks) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0);
    if (e != hipSuccess) return e;
    const int64_t resident = (int64_t)cus * (per_cu > 0 ? per_cu : 1);
    blocks = (unsigned)(needed < resident ? (needed > 0 ? needed : 1) : resident);
    return hipSuccess;
}
}  // namespace

hipError_t ur_launch_trace(const ur::TraceParams &p, bool count, int mode, hipStream_t s) {
    const int64_t needed = (p.work_end - p.work_begin + 255) / 256;
    if (needed <= 0) return hipSuccess;
    unsigned blocks = 0;
    hipError_t e;
#define UR_LAUNCH(C, M)                                                                  \
    do {                                                                                 \
        if ((e = resident_blocks(k_trace<C, M>, needed, blocks)) != hipSuccess) return e; \
        hipLaunchKernelGGL((k_trace<C, M>), dim3(blocks), dim3(256), 0, s, p);           \
    } while (0)
    if (mode == ur::kDeferNee) {
        if (count) UR_LAUNCH(true, ur::kDeferNee);
        else UR_LAUNCH(false, ur::kDeferNee);
    } else {
        if (count) UR_LAUNCH(true, ur::kInlineNeeOnly);
        else UR_LAUNCH(false, ur::kInlineNeeOnly);
    }
#undef UR_LAUNCH
    return hipGetLastError();
}

hipError_t ur_launch_extend(const ur::TraceParams &p, bool count, hipStream_t s) {
    const int64_t needed = (p.work_end - p.work_begin + 255) / 256;
    if (needed <= 0) return hipSuccess;
    unsigned blocks = 0;
    hipError_t e;
#define UR_EXTEND(C, RG, CV)                                                   \
    do {                                                                       \
        e = resident_blocks(k_extend<C, RG, CV>, needed, blocks);              \
        if (e != hipSuccess) return e;                                         \
        hipLaunchKernelGGL((k_extend<C, RG, CV>), dim3(blocks), dim3(256), 0, s, p); \
    } while (0)
#define UR_EXTEND_CV(C, RG)                  \
    do {                                     \
        if (p.convex) UR_EXTEND(C, RG, true); \
        else UR_EXTEND(C, RG, false);        \
    } while (0)
    if (count) {
        if (p.any_rough) UR_EXTEND_CV(true, true);
        else UR_EXTEND_CV(true, false);
    } else {
        if (p.any_rough) UR_EXTEND_CV(false, true);
        else UR_EXTEND_CV(false, false);
    }
#undef UR_EXTEND_CV
#undef UR_EXTEND
    return hipGetLastError();
}

int64_t ur_extend_max_waves() {
    unsigned most = 0;
    const void *variants[] = {(const void *)k_extend<true, true, true>,   (const void *)k_extend<true, true, false>,
                              (const void *)k_extend<true, false, true>,  (const void *)k_extend<true, false, false>,
                              (const void *)k_extend<false, true, true>,  (const void *)k_extend<false, true, false>,
                              (const void *)k_extend<false, false, true>, (const void *)k_extend<false, false, false>};
    for (const void *k : variants) {
        unsigned b = 0;
        if (resident_blocks(k, int64_t(1) << 40, b) != hipSuccess) return -1;
        most = b > most ? b : most;
    }
    return 4 * (int64_t)most;
}

hipError_t ur_launch_scatter(const ur::TraceParams &p, bool count, hipStream_t s) {
    unsigned blocks = 0;
    const int64_t needed = (p.seg_cap + 255) / 256;
    // (CONE_CONVEX = false: a variant without the convex array's cone-restricted
    // element range, whose registers slow the walk by a sixth)
#define UR_SCATTER(C, CV)                                                        \
    do {                                                                         \
        hipError_t e = resident_blocks(k_scatter<C, CV>, needed, blocks);        \
        if (e != hipSuccess) return e;                                           \
        hipLaunchKernelGGL((k_scatter<C, CV>), dim3(blocks), dim3(256), 0, s, p); \
    } while (0)
    const bool cc = p.convex && p.elem_choice == UR_ELEMENT_CONE;
    if (count) {
        if (cc) UR_SCATTER(true, true);
        else UR_SCATTER(true, false);
    } else {
        if (cc) UR_SCATTER(false, true);
        else UR_SCATTER(false, false);
    }
#undef UR_SCATTER
    return hipGetLastError();
}

hipError_t ur_launch_nee(const ur::TraceParams &p, bool count, hipStream_t s) {
    unsigned blocks = 0;
    hipError_t e = count ? resident_blocks(k_nee<true>, (p.nee_cap + 255) / 256, blocks)
                         : resident_blocks(k_nee<false>, (p.nee_cap + 255) / 256, blocks);
    if (e != hipSuccess) return e;
    if (count) hipLaunchKernelGGL(k_nee<true>, dim3(blocks), dim3(256), 0, s, p);
    else hipLaunchKernelGGL(k_nee<false>, dim3(blocks), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t ur_launch_philox(const uint32_t *ctr, uint32_t *out, int64_t n, uint32_t k0, uint32_t k1, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ctr, out, n, k0, k1);
    return hipGetLastError();
}
#endif  // UR_TRACE_RAYS_ONLY

#ifdef UR_TRACE_RAYS_ONLY
hipError_t ur_launch_trace_rays(const ur::TraceParams &p, const void *rays_dev, int64_t n, ur::EventLog log,
                                hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 63) / 64;
    hipLaunchKernelGGL(k_trace_rays, dim3((unsigned)blocks), dim3(64), 0, s, p, (const ur_ray *)rays_dev, n, log);
    return hipGetLastError();
}
#endif
