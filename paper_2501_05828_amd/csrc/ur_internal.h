// Internal data layouts shared by the host runtime (ur_host.cpp) and the
// gfx950 kernels (*.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bvh_layout.h"
#include "scatter_grid.h"
#include "ultraray.h"

namespace ur {

constexpr int kAdjMaxMat = 8;   // materials with attenuation gradients
constexpr int kMaxMat = 16;
constexpr int kMaxSph = 64;
constexpr int kMaxPln = 64;
constexpr int kCells = 1024;          // 32 x 32 emission-direction cells
constexpr double kEpsT = 1e-9;        // self-intersection guard along a ray [m]
constexpr int kNumStats = 27;
constexpr int kSegChunk = 256;   // segment-queue slots a wavefront reserves at a time
constexpr int kRayChunk = 1024;  // most work items a wavefront takes from a range at a time
constexpr int64_t kSplitRays = int64_t(1) << 29;   // most rays per launch range

// Per-material constants, FP64: impedance, amplitude attenuation [Np/m] at
// the centre frequency, slowness [s/m].
struct Material {
    double Z, ka, inv_c, rough;   // rough: GGX alpha of Eq. 12, 0 = smooth
};

// Transducer-sampling candidate: a scatterer capture whose chosen element
// passes the receive cut-off; the secondary ray is cast by a later kernel.
// One primary-ray segment waiting for its scatterer walk, in two arrays: the
// part every walk reads (64 bytes: start, direction, length, ray and
// transmit/element) and the part only a capture that some element may hear
// reads (32 bytes: weight, time, medium, segment index, emission cell).
// txe = transmit << 16 | element; kSegUnused marks an unused slot.
struct SegHot {
    double o[3], d[3];
    double t_seg;
    uint32_t ray, txe;
};
struct SegCold {
    double w, t;
    int med, seg, cell, pad;
};
constexpr uint32_t kSegUnused = 0xffffffffu;

static_assert(sizeof(SegHot) == 64 && sizeof(SegCold) == 32, "segment entry layout");

struct NeeEntry {
    double q[3];       // capture point on the primary segment (or the rough boundary's hit point)
    double wq;         // primary weight at q times the scatterer amplitude (rough boundary: times
                       // its scattering toward the element, times 4 pi)
    double tq;         // arrival time at q
    int tx, er, med, seg;
    int k, e;          // scatterer (original index) or boundary id, and emitting element
    uint32_t ray;
    int cell;          // emission direction cell of the primary ray
    int ne;            // elements the target was drawn from (weight of the choice)
    float mis;         // < 0: a scatterer's entry; else a rough boundary's, with its balance-heuristic
                       // weight (applied when the straight path crosses no boundary)
};

// Recorded contribution for training the emission proposal:
// bin = (tx * E + emitting element) * 1024 + emission cell, value = |c|.
struct RecordEntry {
    uint32_t bin;
    float value;
};

// Trace-kernel modes.
enum TraceMode {
    kDeferNee = 0,     // direct hits recorded, transducer sampling queued
    kInlineNeeOnly = 1 // transducer sampling cast inline, direct hits not recorded
};

struct TraceParams {
    // acquisition
    int E, T, S, binning;
    uint32_t n_el;                    // rays per element per transmit
    int B;                            // max interface interactions
    int proposal;                     // 0 uniform, 1 table
    uint32_t key0, key1;
    int64_t stride, offset, per_el, n_work;
    double pitch, elev, fs, t_max, max_path, alpha_m, alpha_c, r_s2, n_per_tx, half_ap, area_e;
    double cos_alpha_c;               // cosine of the receive cut-off angle
    double tan_alpha_c;               // its tangent (element choice restricted to the cone)
    double sin_alpha_c;               // and its sine (the same on a convex array)
    int elem_choice;                  // UR_ELEMENT_UNIFORM or UR_ELEMENT_CONE
    int sa;                           // synthetic aperture: transmit t = element t, counters of transmit 0
    int convex;                       // elements on an arc of radius `radius` (else a line on z = 0)
    int rough_nee;                    // transducer sampling at rough boundaries (with the balance heuristic)
    double radius, dphi, half_arc;    // convex: radius, angle per element (pitch / radius), E dphi / 2
    const double4 *elem;              // convex: [E] centre x, centre z, sin and cos of the normal's angle
    const double *xe;                 // [E]
    const double *tau;                // [T][E]
    const float *pdf, *cdf;           // [T][E][1024] or null
    // scene
    int n_mat, n_sph, n_pln, top_medium;
    int64_t id_sph0, id_pln0, id_box;
    double box[6];
    const Material *mat;              // [n_mat]
    const double *sph;                // [n_sph][4]
    const int *sph_mat;               // [n_sph][2]
    const double *pln;                // [n_pln][4]
    const int *pln_mat;               // [n_pln][2]
    // triangles in BVH leaf order: v0, e1 = v1 - v0, e2 = v2 - v0
    const double *tri;                // [n_tri][9]
    const double4 *tri_n;             // [n_tri] unit geometric normal (e1 x e2) / |e1 x e2|, .w unused
    const int *tri_mat;               // [n_tri][2]
    const int *tri_id;                // original index (tie-break, exclusion)
    const BvhNode *tnodes;            // threaded binary tree (any-hit walks, fallback)
    const Bvh4NodeQ *tnodes4;         // four-wide tree, quantised (closest hit)
    int n_tri, n_tnodes, n_tnodes4;
    float tree_lo_f[3], tree_hi_f[3]; // box of the binary tree's root (every triangle, dilated, FP32)
    // scatterers: uniform grid, items grouped by cell (copies of position +
    // amplitude, and the original index that keys the RNG counter)
    GridInfo grid;
    float grid_lo_f[3], grid_hi_f[3]; // grid box grown by 10 um, rounded outward to FP32 (segment cull)
    float grid_wa_f, grid_wb_f;       // the grid's acceptance wedge grown by 50 um, FP32 (wb < 0: none)
    const int *cell_start;            // [cells + 1]
    const double4 *items;             // [n_items]
    const float4 *items_f;            // [n_items] positions rounded to FP32, for the conservative prefilter
    float pre_m;                      // prefilter widening [m]: 1 um + 4e-6 x the largest box coordinate
    float pre_r2;                     // prefilter capture radius^2, (r_s + pre_m)^2 rounded up
    const int *item_id;               // [n_items]
    int n_scat;
    int any_rough;                    // some material has a GGX roughness > 0
    // outputs and work distribution
    float *ch_raw;                    // [T][E][S]
    unsigned long long *stats;        // [kNumStats] or null
    unsigned long long *work_next;    // persistent-kernel work counter (zeroed before launch)
    int64_t work_begin, work_end;     // work items [begin, end) of this launch
    float *cost;                      // [T*E][1024] per-emission-cell path cost, or null
    SegHot *segq;                     // segment queue between the extend and scatter kernels
    SegCold *segc;                    // its capture-only part, same slots
    unsigned long long *seg_count;    // slots reserved (chunks of kSegChunk)
    unsigned long long *seg_next;     // scatter-kernel work counter
    unsigned long long *seg_lost;     // segments that found no slot (must stay 0)
    int64_t seg_cap;
    // Admission to the segment queue when it cannot hold the worst case of a
    // whole range: a wavefront takes a chunk of c rays only by adding c (B + 1)
    // to seg_commit without passing seg_limit, and hands back (B + 1) less the
    // segments each finished ray queued at its next take; the first refusal
    // closes the launch, which then ends when its rays finish (null: every
    // ray of the range is taken).
    unsigned long long *seg_commit = nullptr;
    unsigned long long seg_limit = 0;
    NeeEntry *nee;                    // transducer-sampling queue
    unsigned long long *nee_count;    // entries written (may exceed capacity)
    int64_t nee_cap;
    RecordEntry *rec;                 // contribution records, or null
    unsigned long long *rec_count;    // records offered (may exceed capacity)
    int64_t rec_cap;
    // deterministic binning: records staged here instead of float atomics
    struct DetRecord *det = nullptr;
    unsigned long long *det_count = nullptr;   // records offered (may exceed det_cap)
    int64_t det_cap = 0;
};

// One record staged for deterministic binning: its fractional sample
// position x = t fs, its value and its channel tx * E + e.
struct DetRecord {
    double x, v;
    int64_t ch;
};

// Explicit-ray logging (test path).
struct EventLog {
    void *events;                     // ur_event [cap]
    unsigned long long *count;
    int64_t cap;
};

struct DasParams {
    int E, T, S, nx, nz;
    int sector;                       // pixel (ix, iz) at angle x0 + ix dx, depth z0 + iz dz (convex arrays)
    double x0, dx, z0, dz, fs_over_c0, fs;
    double radius;                    // centre of curvature (0, 0, -radius) of sector grids
    const double *xe;                 // [E]
    const double *ze;                 // [E] element depths (convex arrays) or null (all on z = 0)
    const float *apod;                // [E]
    const double4 *txc;               // [T]: (sin*fs/c0, cos*fs/c0, -xref*sin*fs/c0 - 1/2, 0)
    const float2 *rf;                 // [T][E][S]
    float2 *iq;                       // [nx][nz] or null
    float *env;                       // [nx][nz]
};

}  // namespace ur

// kernel launchers (defined in the .hip files)
hipError_t ur_launch_trace(const ur::TraceParams &p, bool count, int mode, hipStream_t s);
hipError_t ur_launch_nee(const ur::TraceParams &p, bool count, hipStream_t s);
hipError_t ur_launch_extend(const ur::TraceParams &p, bool count, hipStream_t s);
hipError_t ur_launch_scatter(const ur::TraceParams &p, bool count, hipStream_t s);
int64_t ur_extend_max_waves();   // wavefronts of a full extend launch (bounds the queue's chunk slack)
hipError_t ur_launch_trace_rays(const ur::TraceParams &p, const void *rays_dev, int64_t n, ur::EventLog log,
                                hipStream_t s);
hipError_t ur_launch_scan_convert(double radius, int np, int nr, double p0, double p1, double r0, double r1,
                                  const float *img, int nx, int nz, double x0, double x1, double z0, double z1,
                                  float fill, float *out, hipStream_t s);
hipError_t ur_launch_synth_angles(const float *sa, const double *angles, int n_ang, int E, int S,
                                  const double *xe_host, const double *ze_host, const double *xe_dev,
                                  const double *ze_dev, double c0, double fs, float *out, hipStream_t s);
hipError_t ur_launch_pulse(const float *raw, float2 *rf, const float2 *taps, int K, int64_t n_ch, int S,
                           hipStream_t s);
hipError_t ur_launch_das(const ur::DasParams &p, hipStream_t s);
hipError_t ur_launch_bmode(const float *env, float *bmode, int64_t n, float dr_db, unsigned int *max_bits,
                           hipStream_t s);
hipError_t ur_mlp_gemm(const float *A, int64_t sar, int64_t sac, const float *B, int64_t sbr, int64_t sbc, float *C,
                       int M, int N, int K, const float *bias, const float *mask, int relu, hipStream_t s);
hipError_t ur_mlp_features(const double *xe, const double *angles, int E, int T, double half_ap, double amax,
                           const float *rff, float *X, hipStream_t s);
hipError_t ur_mlp_softmax_ce(const float *Z, const float *H, const float *tot, float *Q, float *dZ, float *loss,
                             int R, hipStream_t s);
hipError_t ur_mlp_colsum(const float *X, int R, int N, float *out, hipStream_t s);
hipError_t ur_mlp_sum(const float *x, int64_t n, float *out, hipStream_t s);
hipError_t ur_mlp_fill(float *p, int64_t n, float v, hipStream_t s);
hipError_t ur_mlp_adam(float *w, float *m, float *v, const float *g, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2, hipStream_t s);
hipError_t ur_mlp_tables(const float *Q, int R, float eps, float *pdf, float *cdf, hipStream_t s);
hipError_t ur_mlp_record_reweight(ur::RecordEntry *rec, int64_t n_rec, const float *cost, double rays_per_row,
                                  float *s2, int64_t n_bins, hipStream_t s);
hipError_t ur_mlp_record_hist(const ur::RecordEntry *rec, int64_t n_rec, int64_t batch, uint64_t seed, uint32_t step,
                              int64_t n_bins, float *hist, hipStream_t s);
hipError_t ur_launch_env_adj(const float2 *iq, const float *g_env, float2 *g_iq, int64_t n, hipStream_t s);
hipError_t ur_launch_das_adj(const ur::DasParams &p, const float2 *g_iq, float *g_rf, hipStream_t s);
hipError_t ur_launch_pulse_adj(const float2 *g_rf, float *g_raw, const float2 *taps, int K, int64_t n_ch, int S,
                               hipStream_t s);
hipError_t ur_launch_zero_f64(double *p, int n, hipStream_t s);
// The decisions of the adjoint's value pass over a range of paths, kept for
// its tangent passes: per path and segment the closest primitive and its
// distance, and per path up to kAdjCapRec captures that reach a contribution.
struct AdjSeg {
    double t;       // distance to the closest primitive
    int hid;        // its id
    int aux;        // its triangle slot, sphere or plane index, or the box face
};
struct AdjCap {
    int item;               // scatterer item (grid order)
    unsigned short er;      // receiving element drawn
    unsigned short seg;     // segment of the path
};
constexpr int kAdjCapRec = 8;
constexpr unsigned char kAdjCapOverflow = 255;   // more captures than kAdjCapRec: walk the grid again
struct AdjRecord {
    int mode;               // 0 none, 1 record, 2 replay from the record
    int64_t begin, end;     // work items of the range
    AdjSeg *seg;            // [end - begin][B + 1]
    AdjCap *cap;            // [end - begin][kAdjCapRec]
    unsigned char *ncap;    // [end - begin]
    unsigned long long *next;   // work counter of the persistent lanes (zeroed by the launcher)
};
// One parameter direction of a tangent pass and where its derivative is added.
struct AdjTangent {
    int kind;       // 1: impedance of material index; 2: coordinate coord of sphere index
    int index, coord;
    double *out;    // [1] device accumulator
};
// n_tan = 0: the value pass (amplitudes into grad_amp, attenuations into
// grad_alpha, J into value_out; each nullable); else the tangent passes of
// the n_tan directions in tans (host array), a few per launch.
hipError_t ur_launch_replay(const ur::TraceParams &p, int n_tan, const AdjTangent *tans, const float *g,
                            float *grad_amp, double *grad_alpha, double *value_out, double kappa, int attach_choice,
                            const AdjRecord &rec, hipStream_t s);
// The direct-hit edge terms of every impedance (added to out_z [n_mat]) and
// sphere coordinate (out_sph [n_sph][3]), each nullable, over the work items
// of p (n_scan + 1 origins per family; at most 32 parameters).
hipError_t ur_launch_edges(const ur::TraceParams &p, double *out_z, double *out_sph, const float *g, int n_scan,
                           hipStream_t s);
// Deterministic binning of the staged records into ch_raw [n_ch][S] (every
// sample written): ctr[0] the records offered, ctr[1] scratch for their
// largest |value| (cleared by the caller), bins [n_ch][S] int64 scratch
// (cleared by the caller).
hipError_t ur_launch_det_bin(const ur::DetRecord *rec, int64_t cap, unsigned long long *ctr, long long *bins,
                             float *ch_raw, int64_t n_ch, int S, int binning, hipStream_t s);
hipError_t ur_launch_philox(const uint32_t *ctr, uint32_t *out, int64_t n, uint32_t k0, uint32_t k1,
                            hipStream_t s);
