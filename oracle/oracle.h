/*
 * FP64 CPU oracle for the full-path ultrasound Monte Carlo tracer
 * (UltraRay, arXiv 2501.05828) and its plane-wave beamformer.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP library: every formula here is written out independently from
 * the paper (and from the readings listed where the paper is silent).
 *
 * All arithmetic is IEEE double precision.  Intersections are brute force
 * over every primitive (no acceleration structure), so the result is the
 * plain definition of "closest hit" / "every crossing".
 *
 * Units: metres, seconds, m/s; Z in MRayl; alpha in dB/(cm MHz).
 * Frame: x lateral, y elevation, z depth; a linear transducer face lies on
 * z = 0 facing +z, a convex one on a cylinder about the y axis touching z = 0.
 */
#ifndef UR_ORACLE_H
#define UR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Every field is 8 bytes wide so the layout is identical for ctypes. */
typedef struct {
    int64_t n_elements, n_tx, n_samples, rays_per_element, max_bounces, binning;
    double pitch, elevation, f_c, f_s, c0, n_cycles, r_s, max_path, alpha_m, alpha_c;
    uint64_t seed;
    const double *angles;      /* [n_tx] steering angles, rad                         */
    const float *pdf;          /* [n_tx][n_elements][1024] mixed proposal q', or NULL */
    const float *cdf;          /* [n_tx][n_elements][1024] inclusive CDF of q', or NULL */
    int64_t element_choice;    /* transducer sampling: 0 uniform over all elements, 1 uniform over the
                                * elements whose centre the capture point's cone can reach */
    int64_t scheme;            /* 0 steered plane waves; 1 synthetic aperture: n_tx = n_elements,
                                * transmit t fires element t alone without delay, its rays drawn
                                * with the counters of transmit 0 */
    double radius;             /* 0: linear array on z = 0; > 0: convex array of this radius, centre of
                                * curvature (0, 0, -radius), pitch = arc length; the box top must lie
                                * at or above the array's ends */
    int64_t rough_direct_only; /* 0: transducer sampling at rough boundaries, balanced with the direct hits
                                * that follow them; 1: direct hits only */
} or_acq;

typedef struct {
    int64_t n_mat, n_tri, n_sph, n_pln, n_scat, top_medium;
    const double *mat;         /* [n_mat][3]: Z, alpha, c        */
    const double *box;         /* [6]: min xyz, max xyz          */
    const double *tri;         /* [n_tri][9]: v0 v1 v2           */
    const int32_t *tri_mat;    /* [n_tri][2]: front, back        */
    const double *sph;         /* [n_sph][4]: centre, radius     */
    const int32_t *sph_mat;    /* [n_sph][2]: outside, inside    */
    const double *pln;         /* [n_pln][4]: n, d with n.x = d  */
    const int32_t *pln_mat;    /* [n_pln][2]: front, back        */
    const double *scat;        /* [n_scat][4]: position, amplitude */
    const double *rough;       /* [n_mat]: GGX roughness alpha (Eq. 12), 0 = smooth; NULL: all smooth */
} or_scene;

typedef struct {
    int64_t rays, segments, reflect, transmit, tir, scatter_events, nee_zero, nee_cast,
            nee_blocked, direct_hits, records, dropped, edge_band, term_box, term_bounce,
            term_time, term_path, media_mismatch, term_rough, surface_events, surface_zero;
} or_stats;

/* One entry of a path log (explicit-ray tracing). */
typedef struct {
    int64_t kind;   /* 0 direct-hit record, 1 scatter (NEE) record, 2 reflect, 3 transmit, 4 end,
                     * 5 rough-boundary (NEE) record */
    int64_t tx, elem, seg, id;  /* elem: receiving element for records; id: scatterer or primitive */
    double t, value, x, y, z;   /* t: arrival / event time; value: contribution or weight */
} or_event;

/* Explicit ray: origin, unit direction, weight, start time, ids for the RNG. */
typedef struct {
    double o[3], d[3], w, t;
    int64_t tx, elem, ray, medium;
} or_ray;

/* Global primitive ids: triangles, then spheres, then planes, then the box. */

int or_trace(const or_acq *a, const or_scene *s, int n_threads, double *ch_raw, or_stats *st);
int or_trace_rays(const or_acq *a, const or_scene *s, const or_ray *rays, int64_t n,
                  or_event *ev, int64_t cap, int64_t *n_ev, double *ch_raw, or_stats *st);
/* rec_hist (nullable) [n_tx][n_elements][1024] receives the summed |c| of
 * binned contributions by emitting element and emission direction cell. */
int or_trace_subset(const or_acq *a, const or_scene *s, int n_threads, int64_t ray_stride,
                    double *ch_raw, double *rec_hist, or_stats *st);

/* Forward-mode gradient of J = sum over records of g(t) c (g [n_tx][E][S]
 * the adjoint of the binned channel data) along the same paths as
 * or_trace_subset: grad_z, grad_alpha [n_mat], grad_sph [n_sph][3],
 * grad_amp [n_scat] (each nullable), J the value.  attach_choice 0 freezes
 * the reflect-or-transmit choice; 1 adds the derivative of its probability.
 * Returns -3 for rough boundaries, -1 for bad arguments. */
int or_trace_grad(const or_acq *a, const or_scene *s, int n_threads, int64_t ray_stride, const double *g,
                  int attach_choice, double *J, double *grad_z, double *grad_alpha, double *grad_sph,
                  double *grad_amp);

/* The same for explicit rays (as or_trace_rays). */
int or_trace_rays_grad(const or_acq *a, const or_scene *s, const or_ray *rays, int64_t n, const double *g,
                       int attach_choice, double *J, double *grad_z, double *grad_alpha, double *grad_sph,
                       double *grad_amp);
/* Element-edge terms of the direct hits that or_trace_grad's interior
 * derivative leaves out (element edges, aperture ends, elevation edges),
 * integrated exactly along the emission origin's lateral coordinate: for
 * every path family of or_trace_subset's paths, the crossings of the landing
 * point over n_scan + 1 evenly spaced origins (choice attached).  corr_z
 * [n_mat], corr_sph [n_sph][3] (each nullable).  Linear and convex arrays,
 * plane-wave transmits, uniform emission; -3 for rough boundaries, -1 for
 * bad arguments. */
int or_trace_grad_edges(const or_acq *a, const or_scene *s, int n_threads, int64_t ray_stride, const double *g,
                        int n_scan, double *corr_z, double *corr_sph);
/* One path family of or_trace_grad_edges (transmit tx, element e, ray):
 * at the n origin coordinates u0, F = c g(t) (0 off the elements or without
 * a landing), its interior derivative dF [n][n_mat + 3 n_sph], the landing
 * point X [n][2] (NaN if none) and the sequence of primitives and choices
 * sig [n] (0 if none); B [n_mat + 3 n_sph] the family's edge term from an
 * n_scan scan.  attach 0 freezes the reflect-or-transmit choice. */
int or_edge_family(const or_acq *a, const or_scene *s, const double *g, int64_t tx, int64_t e, int64_t ray, int attach,
                   int64_t n, const double *u0, double *F, double *dF, double *X, uint64_t *sig, int n_scan, double *B);
int or_pulse_taps(const or_acq *a, double *taps, int64_t cap);   /* returns K, taps [2K+1][2] */
int or_pulse(const or_acq *a, int64_t n_channels, const double *ch_raw, double *ch_rf);
/* Plane waves synthesised from synthetic-aperture data ch_sa [E][E][S]:
 * out[k][er][s] = sum over e of ch_sa[e][er] at s - tau_k(e) fs (linear
 * interpolation, zero outside), tau_k the delays of angle k (or_delay). */
int or_synthesize(const or_acq *a, const double *ch_sa, const double *angles, int64_t n_ang, double *out);
int or_das(const or_acq *a, int64_t nx, int64_t nz, double x0, double x1, double z0, double z1,
           const double *ch_rf, int n_threads, double *iq);
int or_das_points(const or_acq *a, const double *xz, int64_t n, const double *ch_rf, double *iq);
int or_envelope(int64_t n, const double *iq, double dr_db, double *env, double *bmode);

/* Building blocks exposed for the pins. */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void or_hemisphere(double a, double b, double d[3]);
double or_directivity(double alpha, double alpha_m, double alpha_c);
int or_interface(const double d[3], const double n[3], double z_front, double z_back, double y,
                 double out_d[3], double *R);
/* Rough boundary (Eq. 12): returns 1 reflect, 0 transmit, -1 absorbed; *wf the weight factor. */
int or_interface_rough(const double d[3], const double n[3], double z_front, double z_back, double alpha,
                       double y, double xi1, double xi2, double out_d[3], double *R, double *wf);
void or_onb(const double n[3], double t[3], double b[3]);
void or_ggx_sample(const double n[3], double alpha, double xi1, double xi2, double h[3]);
double or_ggx_d(double alpha, double cos_h);
double or_ggx_g1(double alpha, double cos_v);
/* f(wi, o) |n.o| of a rough boundary and the sampler's density of o. */
double or_rough_fcos(const double wi[3], const double n[3], double z1, double z2, double alpha, const double o[3],
                     double *pdf);
double or_delay(const or_acq *a, int64_t tx, int64_t e);
/* Elements a capture point can hear (cone-restricted choice); 0 if none. */
int or_cone_elements(const or_acq *a, const double q[3], int64_t *e_lo, int64_t *n_e);
/* Element e's centre x, z and the sine, cosine of its normal's angle from +z. */
void or_element_geometry(const or_acq *a, int64_t e, double out[4]);
/* Sector grid [np][nr] pixel positions (x, z) about the centre of curvature. */
int or_sector_points(double radius, int64_t np, int64_t nr, double p0, double p1, double r0, double r1,
                     double *xz);
/* Bilinear scan conversion of a sector image [np][nr] onto a Cartesian grid [nx][nz]. */
int or_scan_convert(double radius, int64_t np, int64_t nr, double p0, double p1, double r0, double r1,
                    const double *img, int64_t nx, int64_t nz, double x0, double x1, double z0, double z1,
                    double fill, double *out);
int64_t or_closest_hit(const or_scene *s, const double o[3], const double d[3], int64_t skip,
                       double *t_hit);
int64_t or_crossings(const or_scene *s, const double o[3], const double d[3], double t_max,
                     double *ts, int64_t cap);

#ifdef __cplusplus
}
#endif
#endif
