/*
 * FP64 CPU oracle: full-path ultrasound Monte Carlo tracer, pulse shaping,
 * plane-wave delay-and-sum and envelope (UltraRay, arXiv 2501.05828).
 *
 * TEST INFRASTRUCTURE ONLY -- loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no
 * code, header, table or constant generator with the HIP library.
 *
 * Structure follows the paper's pipeline (Fig. 2): emission (Sec. 2.3 "Ray
 * Emission", Eqs. 4 and 6), traversal with Snell/Fresnel interface events and
 * the reflect-or-transmit choice (Sec. 2.3 "Ray Traversal", Eqs. 7-11), the
 * transducer sampling of secondary rays with the receive directivity
 * (Sec. 2.3 "Transducer Sampling", Eq. 13), recording into the time-pressure
 * signal, the Gaussian-windowed sinusoidal pulse (Eq. 14) and classic
 * plane-wave delay-and-sum with demodulation and log compression
 * (Sec. 2.3 "Phase Calculation and Signal Processing").  Point scatterers and
 * attenuation, which the paper lists as future work (Sec. 5), follow the
 * readings documented with each function below.
 *
 * Intersections are brute force over all primitives.  Random numbers come
 * from Philox4x32-10 (Salmon et al., SC'11) with the counter layout
 *   (ray, element | tx << 16, segment | purpose << 16, k)
 * and purposes 0 emission, 1 reflect/transmit choice, 2 receiving-element
 * choice for scatterer k, 3 proposal cell.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846
#define EPS_T 1e-9          /* self-intersection guard along a ray [m]      */
#define NCELL 1024          /* 32 x 32 emission-direction cells             */

/* ------------------------------------------------------------------ vectors */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static void sub3(const double *a, const double *b, double *c) { c[0] = a[0] - b[0]; c[1] = a[1] - b[1]; c[2] = a[2] - b[2]; }
static void normalize3(double *a)
{
    double l = sqrt(dot3(a, a));
    a[0] /= l; a[1] /= l; a[2] /= l;
}

/* ------------------------------------------------------------------- Philox */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* uniform in (0,1), exact in double: (x + 1/2) / 2^32 */
static double unif(uint32_t x) { return ((double)x + 0.5) * (1.0 / 4294967296.0); }

/* ------------------------------------------------------------------ context */
typedef struct {
    const or_acq *a;
    const or_scene *s;
    double *ka;      /* amplitude attenuation per material [Np/m] at f_c */
    double *inv_c;   /* 1/c per material [s/m]                           */
    double *xe;      /* element centres along x [m]                      */
    double *ze;      /* element centres along z [m] (0 for a linear array) */
    double *sne;     /* sin of the element's normal angle (0 linear)      */
    double *cne;     /* cos of the element's normal angle (1 linear)      */
    double *tau;     /* [tx][e] transmit delays [s]                      */
    double area_e, n_per_tx, t_max, half_ap, dphi, half_arc;
    int64_t id_sph0, id_pln0, id_box;
} octx;

typedef struct {
    double *hist;      /* [tx][e][n] or NULL */
    double *rhist;     /* [tx][e_emit][cell]: summed |c| of binned contributions, or NULL */
    or_event *ev;
    int64_t cap, n;
    or_stats st;
} sink;

/* Element e's centre (x, z) and the sine and cosine of the angle of its
 * outward normal from +z (Sec. 2.3 "Ray Emission": lateral elements on a
 * circle of the given radius; infinite radius = linear array).  A convex
 * array of radius R has its centre of curvature at (0, 0, -R); the pitch is
 * the arc length between neighbouring centres, so element e sits at angle
 * phi_e = (e - (E-1)/2) pitch / R, at R (sin phi_e, 0, cos phi_e) from the
 * centre; the middle of the array touches z = 0.  z = R cos phi - R is
 * evaluated as -2 R sin^2(phi/2). */
void or_element_geometry(const or_acq *a, int64_t e, double out[4])
{
    double off = (double)e - 0.5 * (double)(a->n_elements - 1);
    if (a->radius > 0.0) {
        double ph = off * a->pitch / a->radius, h = sin(0.5 * ph);
        out[0] = a->radius * sin(ph);
        out[1] = -2.0 * a->radius * h * h;
        out[2] = sin(ph);
        out[3] = cos(ph);
    } else {
        out[0] = off * a->pitch;
        out[1] = 0.0;
        out[2] = 0.0;
        out[3] = 1.0;
    }
}

double or_delay(const or_acq *a, int64_t tx, int64_t e)
{
    /* Plane-wave steering (Sec. 2.3 "Ray Emission", Fig. 3): each element
     * fires when the steered plane front k = (sin theta, 0, cos theta)
     * passes its centre, k.c_e / c0, referenced to the element that fires
     * first so that all delays are non-negative.  On a linear array this is
     * x_e sin(theta) / c0 up to the reference. */
    if (a->radius > 0.0) {
        double st = sin(a->angles[tx]), ct = cos(a->angles[tx]), g[4], ref = INFINITY;
        for (int64_t j = 0; j < a->n_elements; ++j) {
            or_element_geometry(a, j, g);
            double v = g[0] * st + g[1] * ct;
            if (v < ref) ref = v;
        }
        or_element_geometry(a, e, g);
        return (g[0] * st + g[1] * ct - ref) / a->c0;
    }
    double xe = ((double)e - 0.5 * (double)(a->n_elements - 1)) * a->pitch;
    double x0 = (0.0 - 0.5 * (double)(a->n_elements - 1)) * a->pitch;
    double xl = ((double)(a->n_elements - 1) - 0.5 * (double)(a->n_elements - 1)) * a->pitch;
    double st = sin(a->angles[tx]);
    double xref = st >= 0 ? x0 : xl;
    return (xe - xref) * st / a->c0;
}

static int ctx_init(octx *C, const or_acq *a, const or_scene *s)
{
    memset(C, 0, sizeof(*C));
    C->a = a;
    C->s = s;
    C->ka = (double *)malloc(sizeof(double) * (size_t)(s->n_mat > 0 ? s->n_mat : 1));
    C->inv_c = (double *)malloc(sizeof(double) * (size_t)(s->n_mat > 0 ? s->n_mat : 1));
    C->xe = (double *)malloc(sizeof(double) * (size_t)a->n_elements);
    C->ze = (double *)malloc(sizeof(double) * (size_t)a->n_elements);
    C->sne = (double *)malloc(sizeof(double) * (size_t)a->n_elements);
    C->cne = (double *)malloc(sizeof(double) * (size_t)a->n_elements);
    C->tau = (double *)malloc(sizeof(double) * (size_t)(a->n_elements * a->n_tx));
    if (!C->ka || !C->inv_c || !C->xe || !C->ze || !C->sne || !C->cne || !C->tau) return -2;
    /* a convex array: its face must lie inside the box (which absorbs at its
     * top face), and the cone-restricted element choice is for linear arrays */
    if (a->radius < 0.0) return -1;
    if (a->radius > 0.0) {
        double hp = 0.5 * (double)a->n_elements * a->pitch / a->radius, h = sin(0.5 * hp);
        if (hp >= 0.5 * PI || s->box[2] > -2.0 * a->radius * h * h) return -1;
    }
    for (int64_t m = 0; m < s->n_mat; ++m) {
        /* alpha [dB/(cm MHz)] * f [MHz] * 100 cm/m * ln(10)/20 Np/dB */
        C->ka[m] = s->mat[3 * m + 1] * (a->f_c * 1e-6) * 100.0 * log(10.0) / 20.0;
        C->inv_c[m] = 1.0 / s->mat[3 * m + 2];
    }
    for (int64_t e = 0; e < a->n_elements; ++e) {
        double g[4];
        or_element_geometry(a, e, g);
        C->xe[e] = g[0];
        C->ze[e] = g[1];
        C->sne[e] = g[2];
        C->cne[e] = g[3];
    }
    for (int64_t tx = 0; tx < a->n_tx; ++tx)
        for (int64_t e = 0; e < a->n_elements; ++e)
            C->tau[tx * a->n_elements + e] = a->scheme == 1 ? 0.0 : or_delay(a, tx, e);
    C->area_e = a->pitch * a->elevation;
    C->n_per_tx = (double)a->n_elements * (double)a->rays_per_element;
    C->t_max = (double)a->n_samples / a->f_s;
    C->half_ap = 0.5 * (double)a->n_elements * a->pitch;
    C->dphi = a->radius > 0.0 ? a->pitch / a->radius : 0.0;
    C->half_arc = 0.5 * (double)a->n_elements * C->dphi;
    C->id_sph0 = s->n_tri;
    C->id_pln0 = s->n_tri + s->n_sph;
    C->id_box = s->n_tri + s->n_sph + s->n_pln;
    return 0;
}

static void ctx_free(octx *C)
{
    free(C->ka); free(C->inv_c); free(C->xe); free(C->ze); free(C->sne); free(C->cne); free(C->tau);
}

static void draw(const octx *C, uint32_t ray, int64_t e, int64_t tx, int64_t seg, uint32_t purpose,
                 uint32_t k, uint32_t out[4])
{
    /* synthetic aperture: every transmit draws as transmit 0 (one element each) */
    uint32_t txr = C->a->scheme == 1 ? 0u : (uint32_t)tx;
    uint32_t ctr[4] = {ray, (uint32_t)e | (txr << 16), (uint32_t)seg | (purpose << 16), k};
    uint32_t key[2] = {(uint32_t)C->a->seed, (uint32_t)(C->a->seed >> 32)};
    or_philox(ctr, key, out);
}

/* --------------------------------------------------------- emission (Eq. 4, 6) */
/* Equal-area map of the unit square onto the +z hemisphere: Shirley-Chiu
 * concentric square-to-disk map followed by the area-preserving lift
 * z = 1 - r^2, (x, y) scaled by sqrt(2 - r^2).  Uniform (a, b) give uniform
 * directions (pdf 1/(2 pi) per steradian); each of 32x32 square cells maps to
 * 2 pi / 1024 sr. */
void or_hemisphere(double a, double b, double d[3])
{
    double sa = 2.0 * a - 1.0, sb = 2.0 * b - 1.0, r, phi;
    if (sa == 0.0 && sb == 0.0) {
        d[0] = 0.0; d[1] = 0.0; d[2] = 1.0;
        return;
    }
    if (fabs(sa) > fabs(sb)) {
        r = sa;
        phi = (PI / 4.0) * (sb / sa);
    } else {
        r = sb;
        phi = PI / 2.0 - (PI / 4.0) * (sa / sb);
    }
    double r2 = r * r, sc = sqrt(2.0 - r2);
    d[0] = r * cos(phi) * sc;
    d[1] = r * sin(phi) * sc;
    d[2] = 1.0 - r2;
}

/* Ray emission: origin uniform on the element face, direction from the
 * proposal, Monte Carlo weight = emission directivity (cosine, Eq. 6) over
 * (number of rays per transmit x direction pdf) as in Eq. 4. */
static void emit(const octx *C, int64_t tx, int64_t e, uint32_t ray, double o[3], double d[3], double *w,
                 int64_t *cell_out)
{
    const or_acq *a = C->a;
    uint32_t x[4];
    draw(C, ray, e, tx, 0, 0, 0, x);
    double u0 = unif(x[0]), u1 = unif(x[1]), u2 = unif(x[2]), u3 = unif(x[3]);
    /* on a convex array the origin lies on the element's arc and the
     * direction is drawn about the outward normal there */
    double sp = 0.0, cp = 1.0;
    if (a->radius > 0.0) {
        double ph = ((double)e - 0.5 * (double)(a->n_elements - 1) + (u0 - 0.5)) * C->dphi, h = sin(0.5 * ph);
        sp = sin(ph);
        cp = cos(ph);
        o[0] = a->radius * sp;
        o[2] = -2.0 * a->radius * h * h;
    } else {
        o[0] = C->xe[e] + (u0 - 0.5) * a->pitch;
        o[2] = 0.0;
    }
    o[1] = (u1 - 0.5) * a->elevation;
    double ca, cb, pdf;
    if (a->cdf == NULL) {
        ca = u2;
        cb = u3;
        pdf = 1.0 / (2.0 * PI);
        *cell_out = (int64_t)floor(32.0 * u3) * 32 + (int64_t)floor(32.0 * u2);
    } else {
        uint32_t y[4];
        draw(C, ray, e, tx, 0, 3, 0, y);
        double uc = unif(y[0]);
        const float *cdf = a->cdf + (tx * a->n_elements + e) * NCELL;
        int cell = NCELL - 1;
        for (int c = 0; c < NCELL; ++c) {
            if (uc <= (double)cdf[c]) {
                cell = c;
                break;
            }
        }
        *cell_out = cell;
        ca = ((double)(cell % 32) + u2) / 32.0;
        cb = ((double)(cell / 32) + u3) / 32.0;
        pdf = (double)a->pdf[(tx * a->n_elements + e) * NCELL + cell] * (double)NCELL / (2.0 * PI);
    }
    double hl[3];
    or_hemisphere(ca, cb, hl);
    /* local frame: tangent (cos phi, 0, -sin phi), y, normal (sin phi, 0, cos phi) */
    if (a->radius > 0.0) {
        d[0] = hl[0] * cp + hl[2] * sp;
        d[1] = hl[1];
        d[2] = hl[2] * cp - hl[0] * sp;
    } else {
        d[0] = hl[0]; d[1] = hl[1]; d[2] = hl[2];
    }
    *w = hl[2] / (C->n_per_tx * pdf);
}

/* ------------------------------------------------------ directivity (Eq. 13) */
double or_directivity(double alpha, double alpha_m, double alpha_c)
{
    double al = fabs(alpha);
    if (al > alpha_c) return 0.0;
    if (al <= alpha_m) return 1.0;
    return (alpha_c - al) / (alpha_c - alpha_m);
}

/* ------------------------------------------------ interface (Eqs. 7-11) */
/* Reflect-or-transmit at an impedance boundary.  ng is the geometric normal
 * (pointing to the front side); the side the ray comes from fixes which
 * material is "before" (Z1) and "after" (Z2), eta = Z1/Z2.  Reflection iff
 * y < A_r^2; a negative radicand in Eq. 8 (total internal reflection) gives
 * A_r^2 = 1.  Returns 1 for reflection. */
static int fresnel_step(const double d[3], const double ng[3], double z_front, double z_back, double y,
                        double od[3], double *R_out, int *from_front)
{
    double n[3] = {ng[0], ng[1], ng[2]};
    double z1, z2;
    if (dot3(d, n) < 0.0) {
        z1 = z_front; z2 = z_back; *from_front = 1;
    } else {
        z1 = z_back; z2 = z_front; *from_front = 0;
        n[0] = -n[0]; n[1] = -n[1]; n[2] = -n[2];
    }
    double cos_r = -dot3(d, n);                       /* Eq. 7 */
    double eta = z1 / z2;
    double rad = 1.0 - eta * eta * (1.0 - cos_r * cos_r);
    double R, cos_t = 0.0;
    if (rad < 0.0) {
        R = 1.0;
    } else {
        cos_t = sqrt(rad);                            /* Eq. 8 */
        double den = z1 * cos_r + z2 * cos_t;
        if (den == 0.0) {
            R = 1.0;
        } else {
            double A = (z1 * cos_r - z2 * cos_t) / den;  /* Eq. 11 */
            R = A * A;
        }
    }
    *R_out = R;
    if (y < R) {                                      /* Eq. 9 */
        od[0] = d[0] + 2.0 * cos_r * n[0];
        od[1] = d[1] + 2.0 * cos_r * n[1];
        od[2] = d[2] + 2.0 * cos_r * n[2];
        normalize3(od);
        return 1;
    }
    double f = eta * cos_r - cos_t;                   /* Eq. 10 */
    od[0] = eta * d[0] + f * n[0];
    od[1] = eta * d[1] + f * n[1];
    od[2] = eta * d[2] + f * n[2];
    normalize3(od);
    return 0;
}

int or_interface(const double d[3], const double n[3], double z_front, double z_back, double y,
                 double out_d[3], double *R)
{
    int ff;
    return fresnel_step(d, n, z_front, z_back, y, out_d, R, &ff);
}

/* ------------------------------------------ rough interfaces (Eq. 12, GGX) */
/* A boundary between two materials is as rough as the rougher of them.  At a
 * rough boundary a microfacet normal h is drawn around the macro normal n
 * (facing the incoming ray) with density D(h) (n.h), D the GGX distribution
 * of Eq. 12 (Walter et al. 2007, Eqs. 33, 35, 36); Eqs. 7-11 then act with h
 * in place of n.  The weight factor is Walter et al.'s Eq. 41 with the
 * separable Smith masking of Eq. 34: |i.h| G1(i) G1(o) / (|i.n| |h.n|).  A
 * microfacet facing away from the ray, or a new direction on the wrong side
 * of the macro surface, absorbs the ray. */

/* Orthonormal basis (t, b) completing a unit n: the branch-free
 * construction of Duff et al., "Building an Orthonormal Basis, Revisited"
 * (JCGT 6(1), 2017). */
void or_onb(const double n[3], double t[3], double b[3])
{
    double sg = copysign(1.0, n[2]);
    double a = -1.0 / (sg + n[2]);
    double c = n[0] * n[1] * a;
    t[0] = 1.0 + sg * n[0] * n[0] * a;
    t[1] = sg * c;
    t[2] = -sg * n[0];
    b[0] = c;
    b[1] = sg + n[1] * n[1] * a;
    b[2] = -n[1];
}

/* Eq. 12 as printed, in terms of cos(theta_h) = n.h */
double or_ggx_d(double alpha, double cos_h)
{
    double a2 = alpha * alpha;
    double q = cos_h * cos_h * (a2 - 1.0) + 1.0;
    return a2 / (PI * q * q);
}

/* h with density D(h) (n.h): tan^2(theta) = alpha^2 xi1 / (1 - xi1), phi = 2 pi xi2 */
void or_ggx_sample(const double n[3], double alpha, double xi1, double xi2, double h[3])
{
    double t[3], b[3];
    or_onb(n, t, b);
    double q = 1.0 - xi1 + alpha * alpha * xi1;
    double ct = sqrt((1.0 - xi1) / q), st = alpha * sqrt(xi1 / q);
    double ph = 2.0 * PI * xi2;
    double cp = cos(ph), sp = sin(ph);
    for (int i = 0; i < 3; ++i) h[i] = st * cp * t[i] + st * sp * b[i] + ct * n[i];
}

/* Smith masking for GGX (Walter et al. Eq. 34) at cos(theta_v) = v.n > 0 */
double or_ggx_g1(double alpha, double cos_v)
{
    double tan2 = (1.0 - cos_v * cos_v) / (cos_v * cos_v);
    return 2.0 / (1.0 + sqrt(1.0 + alpha * alpha * tan2));
}

static int rough_step(const double d[3], const double ng[3], double z_front, double z_back, double alpha,
                      double y, double xi1, double xi2, double od[3], double *R_out, int *from_front,
                      double *wf)
{
    double n[3] = {ng[0], ng[1], ng[2]};
    double z1, z2;
    if (dot3(d, n) < 0.0) {
        z1 = z_front; z2 = z_back; *from_front = 1;
    } else {
        z1 = z_back; z2 = z_front; *from_front = 0;
        n[0] = -n[0]; n[1] = -n[1]; n[2] = -n[2];
    }
    *wf = 0.0;
    *R_out = 0.0;
    double h[3];
    or_ggx_sample(n, alpha, xi1, xi2, h);
    double ci = -dot3(d, h), cn = -dot3(d, n);
    if (!(ci > 0.0)) return -1;                 /* the microfacet faces away */
    int dummy;
    int refl = fresnel_step(d, h, z1, z2, y, od, R_out, &dummy);   /* Eqs. 7-11 about h */
    double co = dot3(od, n);
    if (refl ? !(co > 0.0) : !(co < 0.0)) return -1;               /* wrong side of the surface */
    *wf = ci * or_ggx_g1(alpha, cn) * or_ggx_g1(alpha, fabs(co)) / (cn * dot3(h, n));
    return refl;
}

int or_interface_rough(const double d[3], const double n[3], double z_front, double z_back, double alpha,
                       double y, double xi1, double xi2, double out_d[3], double *R, double *wf)
{
    int ff;
    return rough_step(d, n, z_front, z_back, alpha, y, xi1, xi2, out_d, R, &ff, wf);
}

/* The rough boundary's scattering toward a given direction o, as implied by
 * the sampler of rough_step.  wi = -d is the reversed incident
 * direction and n the normal on its side, z1 (incident side) and z2 the
 * impedances, eta = z1/z2 the refraction ratio of Eq. 9.  The microfacet
 * normal that sends wi to o is h = wi + o when o lies on the incident side
 * (reflection) and +-(eta wi + o) otherwise (refraction, Eq. 9 about h),
 * normalised with n.h > 0.  The sampler draws h with density D(h) (n.h),
 * reflects with the Fresnel probability R_h of Eq. 11 about h and maps h to o
 * with |dh/do| = 1/(4 |o.h|) (reflection) or |o.h| / (eta wi.h + o.h)^2
 * (refraction, Walter et al. 2007); so the direction density is
 * p(o) = D (n.h) P J with P = R_h or 1 - R_h.  Its weight (rough_step)
 * times p(o) is the returned f(wi, o) |n.o| = (wi.h) G1(wi) G1(o) D P J / (n.wi).
 * Returns 0 (and *pdf = 0) for directions the sampler cannot produce. */
double or_rough_fcos(const double wi[3], const double n[3], double z1, double z2, double alpha, const double o[3],
                     double *pdf)
{
    *pdf = 0.0;
    double cni = dot3(wi, n), cno = dot3(o, n), eta = z1 / z2, h[3];
    if (!(cni > 0.0) || cno == 0.0) return 0.0;
    int refl = cno > 0.0;
    for (int k = 0; k < 3; ++k) h[k] = refl ? wi[k] + o[k] : eta * wi[k] + o[k];
    double hl = sqrt(dot3(h, h));
    if (!(hl > 0.0)) return 0.0;
    double sg = dot3(h, n) < 0.0 ? -1.0 : 1.0;
    for (int k = 0; k < 3; ++k) h[k] *= sg / hl;
    double ci = dot3(wi, h), co = dot3(o, h), chn = dot3(h, n);
    if (!(ci > 0.0) || !(chn > 0.0)) return 0.0;
    if (refl ? !(co > 0.0) : !(co < 0.0)) return 0.0;
    /* Fresnel reflectance about h (Eqs. 8, 11; total internal reflection: 1) */
    double rad = 1.0 - eta * eta * (1.0 - ci * ci), Rh = 1.0;
    if (rad >= 0.0) {
        double ct = sqrt(rad), den = z1 * ci + z2 * ct;
        if (den != 0.0) {
            double A = (z1 * ci - z2 * ct) / den;
            Rh = A * A;
        }
    }
    double P = refl ? Rh : 1.0 - Rh;
    double J;
    if (refl) {
        J = 1.0 / (4.0 * co);
    } else {
        double den = eta * ci + co;
        if (den == 0.0) return 0.0;
        J = -co / (den * den);
    }
    double D = or_ggx_d(alpha, chn);
    *pdf = D * chn * P * J;
    return ci * or_ggx_g1(alpha, cni) * or_ggx_g1(alpha, fabs(cno)) * D * P * J / cni;
}

/* Transmitted intensity fraction 1 - A_r^2 for a straight (unbent) crossing. */
static double transmit_fraction(double z1, double z2, double cos_r)
{
    double eta = z1 / z2;
    double rad = 1.0 - eta * eta * (1.0 - cos_r * cos_r);
    if (rad < 0.0) return 0.0;
    double cos_t = sqrt(rad);
    double den = z1 * cos_r + z2 * cos_t;
    if (den == 0.0) return 0.0;
    double A = (z1 * cos_r - z2 * cos_t) / den;
    return 1.0 - A * A;
}

/* ------------------------------------------------------------ intersections */
/* Moller-Trumbore ray/triangle test; returns 1 and the ray parameter on a hit. */
static int tri_isect(const double *v, const double o[3], const double d[3], double *t_out)
{
    double e1[3], e2[3], p[3], tv[3], q[3];
    sub3(v + 3, v, e1);
    sub3(v + 6, v, e2);
    cross3(d, e2, p);
    double det = dot3(e1, p);
    if (det == 0.0) return 0;
    double inv = 1.0 / det;
    sub3(o, v, tv);
    double u = dot3(tv, p) * inv;
    if (u < 0.0 || u > 1.0) return 0;
    cross3(tv, e1, q);
    double vv = dot3(d, q) * inv;
    if (vv < 0.0 || u + vv > 1.0) return 0;
    *t_out = dot3(e2, q) * inv;
    return 1;
}

static void tri_normal(const double *v, double n[3])
{
    double e1[3], e2[3];
    sub3(v + 3, v, e1);
    sub3(v + 6, v, e2);
    cross3(e1, e2, n);
    normalize3(n);
}

static int sph_roots(const double *s, const double o[3], const double d[3], double *t0, double *t1)
{
    double oc[3];
    sub3(o, s, oc);
    double b = dot3(oc, d);
    double c = dot3(oc, oc) - s[3] * s[3];
    double disc = b * b - c;
    if (disc < 0.0) return 0;
    double sq = sqrt(disc);
    *t0 = -b - sq;
    *t1 = -b + sq;
    return 1;
}

static int pln_isect(const double *p, const double o[3], const double d[3], double *t)
{
    double den = dot3(p, d);
    if (den == 0.0) return 0;
    *t = (p[3] - dot3(p, o)) / den;
    return 1;
}

/* Exit through the absorbing box; face 0..2 = min x,y,z, 3..5 = max x,y,z. */
static double box_exit(const double *box, const double o[3], const double d[3], int *face)
{
    double best = INFINITY;
    int f = -1;
    for (int i = 0; i < 3; ++i) {
        double t;
        int fi;
        if (d[i] > 0.0) {
            t = (box[3 + i] - o[i]) / d[i];
            fi = 3 + i;
        } else if (d[i] < 0.0) {
            t = (box[i] - o[i]) / d[i];
            fi = i;
        } else {
            continue;
        }
        if (t < best) {
            best = t;
            f = fi;
        }
    }
    *face = f;
    return best;
}

typedef struct {
    double t;
    int64_t id;
    int face;
} hit;

static void consider(hit *h, double t, int64_t id)
{
    if (t < h->t || (t == h->t && id < h->id)) {
        h->t = t;
        h->id = id;
    }
}

/* Closest hit over every primitive with t > EPS_T.  The flat primitive the
 * ray has just left (skip) is excluded; the box exit always exists and loses
 * ties because its id is the largest. */
/* The face of a convex array is the cylinder of radius R about the y axis
 * through (0, 0, -R); it absorbs like the box faces (face 6).  A ray from
 * outside meets it where |(o_x, o_z + R) + t (d_x, d_z)| = R: with
 * b = (o_x, o_z + R).(d_x, d_z) < 0 (moving towards the axis), the nearer
 * root t = c / (-b + sqrt(b^2 - a c)), a = d_x^2 + d_z^2,
 * c = o_x^2 + o_z (o_z + 2R) (the squared distance minus R^2, written
 * without cancellation). */
static double probe_face(const or_acq *a, const double o[3], const double d[3])
{
    double R = a->radius;
    double aa = d[0] * d[0] + d[2] * d[2];
    double b = o[0] * d[0] + (o[2] + R) * d[2];
    double c = o[0] * o[0] + o[2] * (o[2] + 2.0 * R);
    if (!(b < 0.0) || aa == 0.0) return INFINITY;
    double disc = b * b - aa * c;
    if (disc < 0.0) return INFINITY;
    double t = c / (-b + sqrt(disc));
    return t > EPS_T ? t : INFINITY;
}

static hit closest(const octx *C, const double o[3], const double d[3], int64_t skip)
{
    const or_scene *s = C->s;
    hit h;
    h.t = box_exit(s->box, o, d, &h.face);
    h.id = C->id_box;
    if (C->a && C->a->radius > 0.0) {
        double tp = probe_face(C->a, o, d);
        if (tp < h.t) {
            h.t = tp;
            h.face = 6;
        }
    }
    for (int64_t i = 0; i < s->n_tri; ++i) {
        double t;
        if (i == skip) continue;
        if (tri_isect(s->tri + 9 * i, o, d, &t) && t > EPS_T) consider(&h, t, i);
    }
    for (int64_t j = 0; j < s->n_sph; ++j) {
        double t0, t1;
        if (!sph_roots(s->sph + 4 * j, o, d, &t0, &t1)) continue;
        if (t0 > EPS_T) consider(&h, t0, C->id_sph0 + j);
        else if (t1 > EPS_T) consider(&h, t1, C->id_sph0 + j);
    }
    for (int64_t p = 0; p < s->n_pln; ++p) {
        double t;
        if (C->id_pln0 + p == skip) continue;
        if (pln_isect(s->pln + 4 * p, o, d, &t) && t > EPS_T) consider(&h, t, C->id_pln0 + p);
    }
    return h;
}

int64_t or_closest_hit(const or_scene *s, const double o[3], const double d[3], int64_t skip, double *t_hit)
{
    octx C;
    memset(&C, 0, sizeof(C));
    C.s = s;
    C.id_sph0 = s->n_tri;
    C.id_pln0 = s->n_tri + s->n_sph;
    C.id_box = s->n_tri + s->n_sph + s->n_pln;
    hit h = closest(&C, o, d, skip);
    *t_hit = h.t;
    return h.id;
}

/* Every crossing of the open segment (EPS_T, t_max - EPS_T); returns the
 * count and, if ts != NULL, up to cap crossing distances (unsorted). */
int64_t or_crossings(const or_scene *s, const double o[3], const double d[3], double t_max, double *ts,
                     int64_t cap)
{
    int64_t n = 0;
    double lo = EPS_T, hi = t_max - EPS_T;
    for (int64_t i = 0; i < s->n_tri; ++i) {
        double t;
        if (tri_isect(s->tri + 9 * i, o, d, &t) && t > lo && t < hi) {
            if (ts && n < cap) ts[n] = t;
            ++n;
        }
    }
    for (int64_t j = 0; j < s->n_sph; ++j) {
        double t0, t1;
        if (!sph_roots(s->sph + 4 * j, o, d, &t0, &t1)) continue;
        if (t0 > lo && t0 < hi) { if (ts && n < cap) ts[n] = t0; ++n; }
        if (t1 > lo && t1 < hi) { if (ts && n < cap) ts[n] = t1; ++n; }
    }
    for (int64_t p = 0; p < s->n_pln; ++p) {
        double t;
        if (pln_isect(s->pln + 4 * p, o, d, &t) && t > lo && t < hi) {
            if (ts && n < cap) ts[n] = t;
            ++n;
        }
    }
    return n;
}

/* ------------------------------------------------------------------ records */
static void log_event(sink *K, int64_t kind, int64_t tx, int64_t elem, int64_t seg, int64_t id, double t,
                      double v, const double p[3])
{
    if (!K->ev) return;
    if (K->n < K->cap) {
        or_event *E = &K->ev[K->n];
        E->kind = kind; E->tx = tx; E->elem = elem; E->seg = seg; E->id = id;
        E->t = t; E->value = v;
        E->x = p ? p[0] : 0.0; E->y = p ? p[1] : 0.0; E->z = p ? p[2] : 0.0;
    }
    K->n++;
}

/* Record an arriving contribution into the element's time-pressure signal
 * (Sec. 2.3 "Phase Calculation").  Sample n holds arrivals in
 * [n/fs, (n+1)/fs) (nearest / box filter); the linear (tent) filter splits a
 * record between the two samples whose centres (n + 1/2)/fs bracket it.
 * Arrivals at or after S/fs fall outside the record window. */
static void record(const octx *C, sink *K, int64_t kind, int64_t tx, int64_t e, int64_t seg, int64_t id,
                   double t, double v, const double p[3], int64_t e_emit, int64_t cell)
{
    const or_acq *a = C->a;
    log_event(K, kind, tx, e, seg, id, t, v, p);
    if (!(t < C->t_max) || t < 0.0) {
        K->st.dropped++;
        return;
    }
    K->st.records++;
    if (K->rhist && cell >= 0) K->rhist[(tx * a->n_elements + e_emit) * NCELL + cell] += fabs(v);
    double x = t * a->f_s;
    double fr = x - floor(x);
    if (fr < 1e-5 || fr > 1.0 - 1e-5) K->st.edge_band++;
    if (!K->hist) return;
    double *h = K->hist + (tx * a->n_elements + e) * a->n_samples;
    if (a->binning == 0) {
        int64_t n = (int64_t)floor(x);
        if (n >= 0 && n < a->n_samples) h[n] += v;
    } else {
        double tau = x - 0.5;
        double f0 = floor(tau);
        int64_t n0 = (int64_t)f0;
        double f = tau - f0;
        if (n0 >= 0 && n0 < a->n_samples) h[n0] += (1.0 - f) * v;
        if (n0 + 1 >= 0 && n0 + 1 < a->n_samples) h[n0 + 1] += f * v;
    }
}

/* Every crossing of a straight secondary ray from q along vh over the open
 * interval (EPS_T, dist - EPS_T), in any order: the product T of transmitted
 * fractions (zero on total internal reflection) and the changes of
 * attenuation and slowness it picks up (R6).  Returns the number of
 * crossings. */
static int64_t shadow_cast(const octx *C, const double q[3], const double vh[3], double dist, double *T_out,
                           double *sa_out, double *sc_out)
{
    const or_scene *sc = C->s;
    double T = 1.0, sum_a = 0.0, sum_c = 0.0;
    int64_t n_cross = 0;
    double lo = EPS_T, hi = dist - EPS_T;
    for (int64_t pid = 0; pid < sc->n_tri + sc->n_sph + sc->n_pln; ++pid) {
        double ts[2];
        int nt = 0;
        double ng[2][3];
        int64_t mf, mb;
        if (pid < sc->n_tri) {
            double tt;
            if (tri_isect(sc->tri + 9 * pid, q, vh, &tt) && tt > lo && tt < hi) {
                ts[nt] = tt;
                tri_normal(sc->tri + 9 * pid, ng[nt]);
                ++nt;
            }
            mf = sc->tri_mat[2 * pid];
            mb = sc->tri_mat[2 * pid + 1];
        } else if (pid < sc->n_tri + sc->n_sph) {
            int64_t j = pid - sc->n_tri;
            const double *sp = sc->sph + 4 * j;
            double t0, t1;
            if (sph_roots(sp, q, vh, &t0, &t1)) {
                double tr[2] = {t0, t1};
                for (int r = 0; r < 2; ++r) {
                    if (tr[r] > lo && tr[r] < hi) {
                        ts[nt] = tr[r];
                        for (int i = 0; i < 3; ++i) ng[nt][i] = (q[i] + tr[r] * vh[i] - sp[i]) / sp[3];
                        ++nt;
                    }
                }
            }
            mf = sc->sph_mat[2 * j];
            mb = sc->sph_mat[2 * j + 1];
        } else {
            int64_t p = pid - sc->n_tri - sc->n_sph;
            double tt;
            if (pln_isect(sc->pln + 4 * p, q, vh, &tt) && tt > lo && tt < hi) {
                ts[nt] = tt;
                for (int i = 0; i < 3; ++i) ng[nt][i] = sc->pln[4 * p + i];
                ++nt;
            }
            mf = sc->pln_mat[2 * p];
            mb = sc->pln_mat[2 * p + 1];
        }
        for (int c = 0; c < nt; ++c) {
            double dn = dot3(vh, ng[c]);
            int64_t before = dn < 0.0 ? mf : mb, after = dn < 0.0 ? mb : mf;
            T *= transmit_fraction(sc->mat[3 * before], sc->mat[3 * after], fabs(dn));
            ++n_cross;
            sum_a += (C->ka[after] - C->ka[before]) * (dist - ts[c]);
            sum_c += (C->inv_c[after] - C->inv_c[before]) * (dist - ts[c]);
        }
    }
    *T_out = T;
    *sa_out = sum_a;
    *sc_out = sum_c;
    return n_cross;
}

/* Element choice for transducer sampling (Sec. 2.3).  Uniform over all E
 * element centres, or, with element_choice = 1, uniform over the K elements
 * whose centre can lie inside the acceptance cone of q (Eq. 13 is zero for
 * the others); the contribution carries 1/p = E or K.  Sets [*e_lo,
 * *e_lo + *n_e) and returns 0 when no element can hear q.
 * Linear array: |x_e - q_x| <= rho with rho^2 = q_z^2 tan^2(alpha_c) - q_y^2.
 * Convex array: with q at distance s > R from the centre of curvature, angle
 * psi about it and elevation y, the cosine of the angle between q - c(phi)
 * and the normal at phi grows with c = cos(psi - phi) (for c >= R/s), and
 * reaches cos(alpha_c) at
 * c* = (R sin^2 alpha_c + cos alpha_c sqrt(s^2 + y^2 - R^2 sin^2 alpha_c)) / s,
 * the larger root of (s c - R)^2 = cos^2(alpha_c) |q - c(phi)|^2: the
 * elements with |phi_e - psi| <= acos(c*), none if c* > 1.
 * Both intervals are widened by a relative 1e-9 so that rounding never drops
 * an element. */
int or_cone_elements(const or_acq *a, const double q[3], int64_t *e_lo, int64_t *n_e)
{
    *e_lo = 0;
    *n_e = a->n_elements;
    if (a->element_choice != 1 || !(a->alpha_c < 0.5 * PI)) return 1;
    double half = 0.5 * (double)(a->n_elements - 1), lo_f = 0.0, hi_f = -1.0;
    if (a->radius > 0.0) {
        double R = a->radius, zc = q[2] + R;
        double sq = sqrt(q[0] * q[0] + zc * zc), sa = sin(a->alpha_c), ca = cos(a->alpha_c);
        if (sq > R) {
            double cs = (R * sa * sa + ca * sqrt(sq * sq + q[1] * q[1] - R * R * sa * sa)) / sq;
            if (cs <= 1.0) {
                double dl = acos(cs) * (1.0 + 1e-9) + 1e-12, psi = atan2(q[0], zc), dphi = a->pitch / R;
                lo_f = ceil((psi - dl) / dphi + half);
                hi_f = floor((psi + dl) / dphi + half);
            }
        }
    } else {
        double tc = tan(a->alpha_c);
        double rho2 = q[2] * q[2] * tc * tc - q[1] * q[1];
        if (q[2] > 0.0 && rho2 >= 0.0) {
            double rho = sqrt(rho2) * (1.0 + 1e-9) + 1e-12;
            lo_f = ceil((q[0] - rho) / a->pitch + half);
            hi_f = floor((q[0] + rho) / a->pitch + half);
        }
    }
    if (lo_f < 0.0) lo_f = 0.0;
    if (hi_f > (double)(a->n_elements - 1)) hi_f = (double)(a->n_elements - 1);
    if (hi_f < lo_f) return 0;
    *e_lo = (int64_t)lo_f;
    *n_e = (int64_t)hi_f - *e_lo + 1;
    return 1;
}

/* ------------------------------------------ transducer sampling at scatterers */
/* A point scatterer k whose capture capsule (radius r_s) contains the primary
 * segment re-radiates isotropically with signed albedo a_k.  A secondary ray
 * is cast from the projection point q to the centre of a uniformly chosen
 * element e' (Sec. 2.3 "Transducer Sampling").  It keeps its straight
 * direction and is multiplied by the transmitted fraction 1 - A_r^2 at every
 * boundary it crosses (zero on total internal reflection), and by the
 * attenuation and delay of each medium along it.  The receive directivity
 * (Eq. 13) uses the angle between the reversed arrival direction and the
 * element normal.  The element subtends area*cos(alpha)/r^2 of the 4 pi
 * re-radiation, divided by the 1/E choice probability. */
static void scatter_nee(const octx *C, sink *K, int64_t tx, int64_t e, uint32_t ray, int64_t seg, int64_t k,
                        const double o[3], const double d[3], double w, double t, int64_t med, double s, int64_t cell)
{
    const or_acq *a = C->a;
    const or_scene *sc = C->s;
    double q[3] = {o[0] + s * d[0], o[1] + s * d[1], o[2] + s * d[2]};
    double wq = w * exp(-C->ka[med] * s);
    double tq = t + s * C->inv_c[med];
    int64_t e_lo = 0, n_e = a->n_elements;
    if (a->element_choice == 1 && !or_cone_elements(a, q, &e_lo, &n_e)) {
        K->st.scatter_events++;
        K->st.nee_zero++;
        return;
    }
    uint32_t x[4];
    draw(C, ray, e, tx, seg, 2, (uint32_t)k, x);
    int64_t er = e_lo + (int64_t)(((uint64_t)x[0] * (uint64_t)n_e) >> 32);
    double v[3] = {C->xe[er] - q[0], 0.0 - q[1], C->ze[er] - q[2]};
    double dist = sqrt(dot3(v, v));
    double vh[3] = {v[0] / dist, v[1] / dist, v[2] / dist};
    double cos_a = a->radius > 0.0 ? -(vh[0] * C->sne[er] + vh[2] * C->cne[er]) : -vh[2];
    double ca = cos_a > 1.0 ? 1.0 : (cos_a < -1.0 ? -1.0 : cos_a);
    double fdir = or_directivity(acos(ca), a->alpha_m, a->alpha_c);
    K->st.scatter_events++;
    if (fdir <= 0.0) {
        K->st.nee_zero++;
        return;
    }
    K->st.nee_cast++;
    double T, sum_a, sum_c;
    shadow_cast(C, q, vh, dist, &T, &sum_a, &sum_c);
    if (T == 0.0) {
        K->st.nee_blocked++;
        return;
    }
    double att = exp(-(C->ka[med] * dist + sum_a));
    double tc = tq + dist * C->inv_c[med] + sum_c;
    double amp = sc->scat[4 * k + 3];
    double c = wq * amp * (double)n_e * C->area_e * cos_a * fdir / (4.0 * PI * dist * dist) * T * att;
    record(C, K, 1, tx, er, seg, k, tc, c, q, e, cell);
}

/* Transducer sampling at a rough boundary: when a primary ray meets a
 * rough boundary it first sends a secondary ray from the hit point x to the
 * centre of an element drawn as for scatterers (purpose 4 of the counters),
 * weighted by the boundary's scattering toward that direction,
 * f(wi, o) |n.o| (or_rough_fcos), by the element's solid angle
 * A cos(alpha) / r^2 and Eq. 13, by 1/p of the element choice, and, like the
 * scatterers' secondary rays, by the transmitted fractions, attenuation and
 * delays along the straight path (R6).  It starts in the medium on o's side.
 * The same arrival can also be found by the continuing primary ray as a
 * direct hit on the next segment: both are weighted by the balance
 * heuristic, this one by p_nee / (p_nee + p(o)) with
 * p_nee = r^2 / (K A cos(alpha)) the density, per solid angle, of drawing a
 * point of the element's face.  A secondary ray whose straight path crosses
 * a boundary records nothing (counted as blocked): the primary ray would
 * interact at that boundary, so its only route to the element through it is
 * the primary ray's own continuation, which the direct hits already count
 * with full weight; a straight, transmission-weighted connection would count
 * that echo a second time. */
static void surface_nee(const octx *C, sink *K, int64_t tx, int64_t e, uint32_t ray, int64_t seg, int64_t id,
                        const double x[3], const double d[3], const double n[3], int64_t m_in, int64_t m_out,
                        double alpha, double w, double t, int64_t cell)
{
    const or_acq *a = C->a;
    const or_scene *sc = C->s;
    int64_t e_lo = 0, n_e = a->n_elements;
    K->st.surface_events++;
    if (!or_cone_elements(a, x, &e_lo, &n_e)) {
        K->st.surface_zero++;
        return;
    }
    uint32_t xr[4];
    draw(C, ray, e, tx, seg, 4, 0, xr);
    int64_t er = e_lo + (int64_t)(((uint64_t)xr[0] * (uint64_t)n_e) >> 32);
    double v[3] = {C->xe[er] - x[0], 0.0 - x[1], C->ze[er] - x[2]};
    double dist = sqrt(dot3(v, v));
    double o[3] = {v[0] / dist, v[1] / dist, v[2] / dist};
    double cos_a = a->radius > 0.0 ? -(o[0] * C->sne[er] + o[2] * C->cne[er]) : -o[2];
    double ca = cos_a > 1.0 ? 1.0 : (cos_a < -1.0 ? -1.0 : cos_a);
    double fdir = or_directivity(acos(ca), a->alpha_m, a->alpha_c);
    double wi[3] = {-d[0], -d[1], -d[2]}, pdf;
    double fc = fdir > 0.0 ? or_rough_fcos(wi, n, sc->mat[3 * m_in], sc->mat[3 * m_out], alpha, o, &pdf) : 0.0;
    if (!(fc > 0.0)) {
        K->st.surface_zero++;
        return;
    }
    K->st.nee_cast++;
    int64_t med = dot3(o, n) > 0.0 ? m_in : m_out;
    double T, sum_a, sum_c;
    int64_t nc = shadow_cast(C, x, o, dist, &T, &sum_a, &sum_c);
    if (nc > 0 || T == 0.0) {
        K->st.nee_blocked++;
        return;
    }
    double area = C->area_e * cos_a;
    double p_nee = dist * dist / ((double)n_e * area);
    double mis = p_nee / (p_nee + pdf);
    double att = exp(-(C->ka[med] * dist + sum_a));
    double tc = t + dist * C->inv_c[med] + sum_c;
    double c = w * fc * area / (dist * dist) * fdir * (double)n_e * mis * T * att;
    record(C, K, 5, tx, er, seg, id, tc, c, x, e, cell);
}

/* All scatterers whose capture capsule the segment [0, t_seg) passes:
 * projection s = (p_k - o).d in [0, t_seg) and perpendicular distance <= r_s. */
static void scatter_events(const octx *C, sink *K, int64_t tx, int64_t e, uint32_t ray, int64_t seg,
                           const double o[3], const double d[3], double w, double t, int64_t med, double t_seg,
                           int64_t cell)
{
    const or_scene *sc = C->s;
    double r2 = C->a->r_s * C->a->r_s;
    for (int64_t k = 0; k < sc->n_scat; ++k) {
        double p[3];
        sub3(sc->scat + 4 * k, o, p);
        double s = dot3(p, d);
        if (!(s >= 0.0 && s < t_seg)) continue;
        double perp[3] = {p[0] - s * d[0], p[1] - s * d[1], p[2] - s * d[2]};
        if (dot3(perp, perp) > r2) continue;
        scatter_nee(C, K, tx, e, ray, seg, k, o, d, w, t, med, s, cell);
    }
}

/* ------------------------------------------------------------- path tracing */
/* Follows one primary ray (Sec. 2.3 "Ray Traversal") for segments
 * 0..max_bounces.  Each segment: closest hit; scatterer events on the
 * segment; transport (attenuation exp(-alpha f d), delay d/c, path length);
 * then the hit: the box exit through the transducer aperture records
 * weight x directivity into the element it lands on, any other box exit
 * absorbs, an impedance boundary draws reflect-or-transmit unless the
 * interaction limit is reached.  The ray also ends when its path exceeds
 * max_path (the segment is clipped there) or its time leaves the window. */
static void trace_path(const octx *C, sink *K, int64_t tx, int64_t e, uint32_t ray, const double o_in[3],
                       const double d_in[3], double w, double t, int64_t med, int64_t cell)
{
    const or_acq *a = C->a;
    const or_scene *sc = C->s;
    double o[3] = {o_in[0], o_in[1], o_in[2]}, d[3] = {d_in[0], d_in[1], d_in[2]};
    double len = 0.0;
    int64_t last = -1;
    /* the last interaction, if rough: the density of the direction the ray
     * left it in and its element range, for the balance heuristic of a direct
     * hit on the next segment */
    int prev_rough = 0;
    double prev_pdf = 0.0;
    int64_t prev_lo = 0, prev_n = 0;
    K->st.rays++;
    for (int64_t b = 0; b <= a->max_bounces; ++b) {
        K->st.segments++;
        hit h = closest(C, o, d, last);
        double t_seg = h.t;
        int clipped = 0;
        if (len + t_seg > a->max_path) {
            t_seg = a->max_path - len;
            clipped = 1;
        }
        scatter_events(C, K, tx, e, ray, b, o, d, w, t, med, t_seg, cell);
        w *= exp(-C->ka[med] * t_seg);
        t += t_seg * C->inv_c[med];
        len += t_seg;
        for (int i = 0; i < 3; ++i) o[i] += t_seg * d[i];
        if (clipped) {
            K->st.term_path++;
            log_event(K, 4, tx, e, b, -3, t, w, o);
            return;
        }
        if (t >= C->t_max) {
            K->st.term_time++;
            log_event(K, 4, tx, e, b, -2, t, w, o);
            return;
        }
        if (h.id == C->id_box) {
            if (h.face == 6 && fabs(o[1]) <= 0.5 * a->elevation) {
                /* convex array: the element whose arc holds the landing point;
                 * the receive angle is taken to that element's normal */
                double ph = atan2(o[0], o[2] + a->radius);
                if (fabs(ph) <= C->half_arc) {
                    int64_t er = (int64_t)floor(ph / C->dphi + 0.5 * (double)a->n_elements);
                    if (er < 0) er = 0;
                    if (er > a->n_elements - 1) er = a->n_elements - 1;
                    double ca = -(d[0] * C->sne[er] + d[2] * C->cne[er]);
                    ca = ca > 1.0 ? 1.0 : (ca < -1.0 ? -1.0 : ca);
                    double fdir = or_directivity(acos(ca), a->alpha_m, a->alpha_c);
                    if (fdir > 0.0) {
                        double mis = 1.0;
                        if (prev_rough && er >= prev_lo && er < prev_lo + prev_n) {
                            double p_nee = t_seg * t_seg / ((double)prev_n * C->area_e * ca);
                            mis = prev_pdf / (prev_pdf + p_nee);
                        }
                        K->st.direct_hits++;
                        record(C, K, 0, tx, er, b, -1, t, w * fdir * mis, o, e, cell);
                    }
                }
            }
            if (a->radius == 0.0 && h.face == 2 && fabs(o[0]) <= C->half_ap && fabs(o[1]) <= 0.5 * a->elevation) {
                int64_t er = (int64_t)floor((o[0] + C->half_ap) / a->pitch);
                if (er < 0) er = 0;
                if (er > a->n_elements - 1) er = a->n_elements - 1;
                double ca = -d[2];
                ca = ca > 1.0 ? 1.0 : (ca < -1.0 ? -1.0 : ca);
                double fdir = or_directivity(acos(ca), a->alpha_m, a->alpha_c);
                if (fdir > 0.0) {
                    double mis = 1.0;
                    if (prev_rough && er >= prev_lo && er < prev_lo + prev_n) {
                        double p_nee = t_seg * t_seg / ((double)prev_n * C->area_e * ca);
                        mis = prev_pdf / (prev_pdf + p_nee);
                    }
                    K->st.direct_hits++;
                    record(C, K, 0, tx, er, b, -1, t, w * fdir * mis, o, e, cell);
                }
            }
            K->st.term_box++;
            log_event(K, 4, tx, e, b, -1, t, w, o);
            return;
        }
        if (b == a->max_bounces) {
            K->st.term_bounce++;
            log_event(K, 4, tx, e, b, -4, t, w, o);
            return;
        }
        /* impedance boundary */
        double ng[3];
        int64_t mf, mb;
        if (h.id < C->id_sph0) {
            tri_normal(sc->tri + 9 * h.id, ng);
            mf = sc->tri_mat[2 * h.id];
            mb = sc->tri_mat[2 * h.id + 1];
        } else if (h.id < C->id_pln0) {
            const double *sp = sc->sph + 4 * (h.id - C->id_sph0);
            for (int i = 0; i < 3; ++i) ng[i] = (o[i] - sp[i]) / sp[3];
            mf = sc->sph_mat[2 * (h.id - C->id_sph0)];
            mb = sc->sph_mat[2 * (h.id - C->id_sph0) + 1];
        } else {
            const double *pp = sc->pln + 4 * (h.id - C->id_pln0);
            for (int i = 0; i < 3; ++i) ng[i] = pp[i];
            mf = sc->pln_mat[2 * (h.id - C->id_pln0)];
            mb = sc->pln_mat[2 * (h.id - C->id_pln0) + 1];
        }
        uint32_t x[4];
        draw(C, ray, e, tx, b, 1, 0, x);
        double y = unif(x[0]), R, nd[3];
        int from_front, refl;
        double alpha = 0.0;
        if (sc->rough) alpha = sc->rough[mf] > sc->rough[mb] ? sc->rough[mf] : sc->rough[mb];
        if (alpha > 0.0) {
            /* transducer sampling first, then the boundary's own draw */
            int fr = dot3(d, ng) < 0.0;
            double nn[3] = {fr ? ng[0] : -ng[0], fr ? ng[1] : -ng[1], fr ? ng[2] : -ng[2]};
            int64_t m_in = fr ? mf : mb, m_out = fr ? mb : mf;
            if (!a->rough_direct_only) surface_nee(C, K, tx, e, ray, b, h.id, o, d, nn, m_in, m_out, alpha, w, t, cell);
            double wf;
            refl = rough_step(d, ng, sc->mat[3 * mf], sc->mat[3 * mb], alpha, y, unif(x[1]), unif(x[2]), nd, &R,
                              &from_front, &wf);
            if (refl < 0) {
                K->st.term_rough++;
                log_event(K, 4, tx, e, b, -5, t, w, o);
                return;
            }
            w *= wf;
            double wi[3] = {-d[0], -d[1], -d[2]};
            or_rough_fcos(wi, nn, sc->mat[3 * m_in], sc->mat[3 * m_out], alpha, nd, &prev_pdf);
            prev_rough = !a->rough_direct_only;
            if (!or_cone_elements(a, o, &prev_lo, &prev_n)) prev_n = 0;
        } else {
            refl = fresnel_step(d, ng, sc->mat[3 * mf], sc->mat[3 * mb], y, nd, &R, &from_front);
            prev_rough = 0;
        }
        int64_t before = from_front ? mf : mb, after = from_front ? mb : mf;
        if (before != med) K->st.media_mismatch++;
        if (refl) {
            if (R >= 1.0) K->st.tir++;
            else K->st.reflect++;
            med = before;
        } else {
            K->st.transmit++;
            med = after;
        }
        log_event(K, refl ? 2 : 3, tx, e, b, h.id, t, w, o);
        d[0] = nd[0]; d[1] = nd[1]; d[2] = nd[2];
        last = (h.id < C->id_sph0 || h.id >= C->id_pln0) ? h.id : -1;
    }
}

static void stats_add(or_stats *a, const or_stats *b)
{
    const int64_t *pb = (const int64_t *)b;
    int64_t *pa = (int64_t *)a;
    for (size_t i = 0; i < sizeof(or_stats) / sizeof(int64_t); ++i) pa[i] += pb[i];
}

static int trace_impl(const or_acq *a, const or_scene *s, int n_threads, int64_t stride, double *ch_raw,
                      double *rec_hist, or_stats *st_out)
{
    if (a->n_elements <= 0 || a->n_elements > 65535 || a->n_tx <= 0 || a->n_tx > 65535 || a->n_samples <= 0 ||
        a->rays_per_element < 0 || a->max_bounces < 0 || a->max_bounces > 65535 || stride <= 0 ||
        (a->scheme == 1 && a->n_tx != a->n_elements))
        return -1;
    octx C;
    int rc_init = ctx_init(&C, a, s);
    if (rc_init) {
        ctx_free(&C);
        return rc_init;
    }
    int nt = n_threads;
#ifdef _OPENMP
    if (nt <= 0) nt = omp_get_max_threads();
#else
    nt = 1;
#endif
    if (nt < 1) nt = 1;
    size_t nh = (size_t)(a->n_tx * a->n_elements * a->n_samples);
    sink *sinks = (sink *)calloc((size_t)nt, sizeof(sink));
    if (!sinks) return -2;
    size_t nr = (size_t)(a->n_tx * a->n_elements * NCELL);
    for (int i = 0; i < nt; ++i) {
        sinks[i].hist = (double *)calloc(nh, sizeof(double));
        if (!sinks[i].hist) return -2;
        if (rec_hist) {
            sinks[i].rhist = (double *)calloc(nr, sizeof(double));
            if (!sinks[i].rhist) return -2;
        }
    }
    int64_t per_el = (a->rays_per_element + stride - 1) / stride;
    /* synthetic aperture: transmit t is element t alone */
    int64_t n_work = (a->scheme == 1 ? 1 : a->n_tx) * a->n_elements * per_el;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nt)
#endif
    for (int64_t i = 0; i < n_work; ++i) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        int64_t rr = (i % per_el) * stride;
        int64_t e = (i / per_el) % a->n_elements;
        int64_t tx = a->scheme == 1 ? e : i / (per_el * a->n_elements);
        double o[3], d[3], w;
        int64_t cell = -1;
        emit(&C, tx, e, (uint32_t)rr, o, d, &w, &cell);
        trace_path(&C, &sinks[tid], tx, e, (uint32_t)rr, o, d, w, C.tau[tx * a->n_elements + e],
                   s->top_medium, cell);
    }
    memset(ch_raw, 0, nh * sizeof(double));
    or_stats st;
    memset(&st, 0, sizeof(st));
    if (rec_hist) memset(rec_hist, 0, nr * sizeof(double));
    for (int i = 0; i < nt; ++i) {
        for (size_t j = 0; j < nh; ++j) ch_raw[j] += sinks[i].hist[j];
        if (rec_hist)
            for (size_t j = 0; j < nr; ++j) rec_hist[j] += sinks[i].rhist[j];
        stats_add(&st, &sinks[i].st);
        free(sinks[i].hist);
        free(sinks[i].rhist);
    }
    free(sinks);
    if (st_out) *st_out = st;
    ctx_free(&C);
    return 0;
}

int or_trace(const or_acq *a, const or_scene *s, int n_threads, double *ch_raw, or_stats *st)
{
    return trace_impl(a, s, n_threads, 1, ch_raw, NULL, st);
}

int or_trace_subset(const or_acq *a, const or_scene *s, int n_threads, int64_t ray_stride, double *ch_raw,
                    double *rec_hist, or_stats *st)
{
    return trace_impl(a, s, n_threads, ray_stride, ch_raw, rec_hist, st);
}

/* Explicit rays (origin, direction, weight, time, ids) traced one by one;
 * logs every record and interface event. */
int or_trace_rays(const or_acq *a, const or_scene *s, const or_ray *rays, int64_t n, or_event *ev, int64_t cap,
                  int64_t *n_ev, double *ch_raw, or_stats *st_out)
{
    octx C;
    int rc_init = ctx_init(&C, a, s);
    if (rc_init) {
        ctx_free(&C);
        return rc_init;
    }
    sink K;
    memset(&K, 0, sizeof(K));
    K.ev = ev;
    K.cap = cap;
    K.hist = ch_raw;
    if (ch_raw) memset(ch_raw, 0, sizeof(double) * (size_t)(a->n_tx * a->n_elements * a->n_samples));
    for (int64_t i = 0; i < n; ++i) {
        const or_ray *r = &rays[i];
        trace_path(&C, &K, r->tx, r->elem, (uint32_t)r->ray, r->o, r->d, r->w, r->t, r->medium, -1);
    }
    if (n_ev) *n_ev = K.n;
    if (st_out) *st_out = K.st;
    ctx_free(&C);
    return 0;
}

/* ================================================ gradient (forward mode) */
/* Derivatives of the functional J = sum over records of g(t) c, where g is
 * a given adjoint of the binned channel data, with respect to the scene's
 * impedances Z_m, attenuation coefficients alpha_m, sphere centres and
 * scatterer amplitudes a_k.  Every path of or_trace is replayed with the
 * same decisions (closest primitive, captures, receiving elements,
 * crossings, reflect or transmit, taken on the FP64 values exactly as in
 * trace_path), and every continuous quantity along it -- position,
 * direction, distance, weight, time, path length -- is carried as a dual
 * number: a value and its partial derivatives along every parameter
 * (forward-mode differentiation of the estimator's formulas).  A record of
 * value c at time t adds g(t) dc + c g'(t) dt, with g'(t) the slope of g
 * between the sample centres under linear binning and 0 under nearest
 * binning.  dJ/da_k = sum over the captures of k of g(t) c / a_k.
 *
 * The reflect-or-transmit choice: with attach_choice = 0 the choice is
 * frozen (the derivative of the fixed-seed estimator); with 1 the weight is
 * multiplied after the choice by R / value(R) (reflection) or
 * (1 - R) / value(1 - R) (transmission), which leaves its value unchanged
 * and adds the derivative of the choice probability (a score term), so the
 * result estimates the derivative of the expected data.  Geometry enters
 * through interior derivatives only: a capture, an element or an aperture
 * edge that appears or disappears under a change contributes no term.
 * Rough boundaries (Eq. 12) are replayed with the estimator that receives
 * their echoes by direct hits only (rough_direct_only = 1): the microfacet
 * normal follows the dual macro normal for the same random numbers, and the
 * weight factor is differentiated with it.  With transducer sampling at
 * rough boundaries the call returns -3. */
#define GRAD_MAX 64

static int g_nt;   /* number of active tangent directions (set before a replay) */

typedef struct {
    double v;
    double t[GRAD_MAX];
} dnum;

static dnum dn_c(double v)
{
    dnum r;
    r.v = v;
    for (int i = 0; i < g_nt; ++i) r.t[i] = 0.0;
    return r;
}
static dnum dn_add(dnum a, dnum b)
{
    a.v = a.v + b.v;
    for (int i = 0; i < g_nt; ++i) a.t[i] += b.t[i];
    return a;
}
static dnum dn_sub(dnum a, dnum b)
{
    a.v = a.v - b.v;
    for (int i = 0; i < g_nt; ++i) a.t[i] -= b.t[i];
    return a;
}
static dnum dn_neg(dnum a)
{
    a.v = -a.v;
    for (int i = 0; i < g_nt; ++i) a.t[i] = -a.t[i];
    return a;
}
static dnum dn_mul(dnum a, dnum b)
{
    dnum r;
    r.v = a.v * b.v;
    for (int i = 0; i < g_nt; ++i) r.t[i] = a.t[i] * b.v + a.v * b.t[i];
    return r;
}
/* a * s and s * a for a constant s */
static dnum dn_mulc(dnum a, double s)
{
    a.v = a.v * s;
    for (int i = 0; i < g_nt; ++i) a.t[i] *= s;
    return a;
}
/* a / s for a constant s */
static dnum dn_divc(dnum a, double s)
{
    a.v = a.v / s;
    for (int i = 0; i < g_nt; ++i) a.t[i] /= s;
    return a;
}
static dnum dn_div(dnum a, dnum b)
{
    dnum r;
    r.v = a.v / b.v;
    for (int i = 0; i < g_nt; ++i) r.t[i] = (a.t[i] * b.v - a.v * b.t[i]) / (b.v * b.v);
    return r;
}
static dnum dn_sqrt(dnum a)
{
    dnum r;
    r.v = sqrt(a.v);
    for (int i = 0; i < g_nt; ++i) r.t[i] = a.t[i] / (2.0 * r.v);
    return r;
}
static dnum dn_exp(dnum a)
{
    dnum r;
    r.v = exp(a.v);
    for (int i = 0; i < g_nt; ++i) r.t[i] = a.t[i] * r.v;
    return r;
}
/* acos of a value clamped to [-1, 1] (as the forward clamps the cosine) */
static dnum dn_acos(dnum a)
{
    dnum r;
    double x = a.v > 1.0 ? 1.0 : (a.v < -1.0 ? -1.0 : a.v);
    double s = sqrt(fmax(1.0 - x * x, 1e-300));
    r.v = acos(x);
    for (int i = 0; i < g_nt; ++i) r.t[i] = -a.t[i] / s;
    return r;
}
static dnum dn_dot(const dnum *a, const dnum *b)
{
    return dn_add(dn_add(dn_mul(a[0], b[0]), dn_mul(a[1], b[1])), dn_mul(a[2], b[2]));
}
/* p . a for a constant vector p (in the order p0 a0 + p1 a1 + p2 a2) */
static dnum dn_dotc(const double *p, const dnum *a)
{
    return dn_add(dn_add(dn_mulc(a[0], p[0]), dn_mulc(a[1], p[1])), dn_mulc(a[2], p[2]));
}

/* Receive directivity (Eq. 13) of a dual angle: 1 up to alpha_m, the linear
 * ramp to zero at alpha_c (the caller has checked alpha <= alpha_c). */
static dnum dn_directivity(dnum al, double alpha_m, double alpha_c)
{
    if (al.v <= alpha_m) return dn_c(1.0);
    return dn_divc(dn_sub(dn_c(alpha_c), al), alpha_c - alpha_m);
}

typedef struct {
    const octx *C;
    const double *g;      /* [tx][e][n] adjoint of the binned channel data */
    int attach;
    int n_mat;
    dnum *Z;              /* [n_mat] impedances (tangent m)                       */
    dnum *ka;             /* [n_mat] attenuation in Np/m (tangent n_mat + m)      */
    dnum *cen;            /* [n_sph][3] sphere centres (tangent 2 n_mat + 3 j + k) */
} gctx;

typedef struct {
    double J;
    double grad[GRAD_MAX];
    double *amp;          /* [n_scat] */
} gacc;

/* One record of dual value c at dual time t into element er of transmit tx;
 * c_unit (>= 0 index k) is its value per unit amplitude of scatterer k. */
static void grad_record(const gctx *G, gacc *A, int64_t tx, int64_t er, dnum c, dnum t, int64_t k, double c_unit)
{
    const octx *C = G->C;
    const or_acq *a = C->a;
    if (!(t.v < C->t_max) || t.v < 0.0) return;
    const double *ch = G->g + (tx * a->n_elements + er) * a->n_samples;
    double x = t.v * a->f_s, gv, gs;
    if (a->binning == 0) {
        int64_t n = (int64_t)floor(x);
        gv = (n >= 0 && n < a->n_samples) ? ch[n] : 0.0;
        gs = 0.0;
    } else {
        double tau = x - 0.5, f0 = floor(tau), f = tau - f0;
        int64_t n0 = (int64_t)f0;
        double g0 = (n0 >= 0 && n0 < a->n_samples) ? ch[n0] : 0.0;
        double g1 = (n0 + 1 >= 0 && n0 + 1 < a->n_samples) ? ch[n0 + 1] : 0.0;
        gv = (1.0 - f) * g0 + f * g1;
        gs = (g1 - g0) * a->f_s;
    }
    A->J += gv * c.v;
    for (int i = 0; i < g_nt; ++i) A->grad[i] += gv * c.t[i] + gs * c.v * t.t[i];
    if (k >= 0) A->amp[k] += gv * c_unit;
}

/* Transmitted fraction 1 - A_r^2 of a straight crossing, in duals. */
static dnum dn_transmit_fraction(dnum z1, dnum z2, dnum cos_r)
{
    dnum eta = dn_div(z1, z2);
    dnum rad = dn_sub(dn_c(1.0), dn_mul(dn_mul(eta, eta), dn_sub(dn_c(1.0), dn_mul(cos_r, cos_r))));
    if (rad.v < 0.0) return dn_c(0.0);
    dnum cos_t = dn_sqrt(rad);
    dnum den = dn_add(dn_mul(z1, cos_r), dn_mul(z2, cos_t));
    if (den.v == 0.0) return dn_c(0.0);
    dnum A = dn_div(dn_sub(dn_mul(z1, cos_r), dn_mul(z2, cos_t)), den);
    return dn_sub(dn_c(1.0), dn_mul(A, A));
}

/* Moller-Trumbore distance along (o, d) to triangle v, in duals (the
 * triangle is fixed); the caller has found the hit by value. */
static dnum dn_tri_t(const double *v, const dnum *o, const dnum *d)
{
    double e1[3], e2[3];
    sub3(v + 3, v, e1);
    sub3(v + 6, v, e2);
    dnum p[3] = {dn_sub(dn_mulc(d[1], e2[2]), dn_mulc(d[2], e2[1])),
                 dn_sub(dn_mulc(d[2], e2[0]), dn_mulc(d[0], e2[2])),
                 dn_sub(dn_mulc(d[0], e2[1]), dn_mulc(d[1], e2[0]))};
    dnum det = dn_add(dn_add(dn_mulc(p[0], e1[0]), dn_mulc(p[1], e1[1])), dn_mulc(p[2], e1[2]));
    dnum tv[3] = {dn_sub(o[0], dn_c(v[0])), dn_sub(o[1], dn_c(v[1])), dn_sub(o[2], dn_c(v[2]))};
    dnum q[3] = {dn_sub(dn_mulc(tv[1], e1[2]), dn_mulc(tv[2], e1[1])),
                 dn_sub(dn_mulc(tv[2], e1[0]), dn_mulc(tv[0], e1[2])),
                 dn_sub(dn_mulc(tv[0], e1[1]), dn_mulc(tv[1], e1[0]))};
    return dn_div(dn_dotc(e2, q), det);
}

/* Secondary ray from q along vh over (EPS_T, dist - EPS_T), as shadow_cast,
 * in duals: the crossings are found on the values in the same order; each
 * crossing's distance and normal carry their derivatives.  Returns 0 if a
 * crossing reflects totally (T = 0). */
static int grad_shadow(const gctx *G, const dnum *q, const dnum *vh, dnum dist, dnum *T_out, dnum *sa_out,
                       dnum *sc_out)
{
    const octx *C = G->C;
    const or_scene *sc = C->s;
    dnum T = dn_c(1.0), sum_a = dn_c(0.0), sum_c = dn_c(0.0);
    double qv[3] = {q[0].v, q[1].v, q[2].v}, vv[3] = {vh[0].v, vh[1].v, vh[2].v};
    double lo = EPS_T, hi = dist.v - EPS_T;
    for (int64_t pid = 0; pid < sc->n_tri + sc->n_sph + sc->n_pln; ++pid) {
        dnum ts[2], ng[2][3];
        int nt = 0;
        int64_t mf, mb;
        if (pid < sc->n_tri) {
            double tt;
            if (tri_isect(sc->tri + 9 * pid, qv, vv, &tt) && tt > lo && tt < hi) {
                ts[nt] = dn_tri_t(sc->tri + 9 * pid, q, vh);
                ts[nt].v = tt;
                double n[3];
                tri_normal(sc->tri + 9 * pid, n);
                for (int i = 0; i < 3; ++i) ng[nt][i] = dn_c(n[i]);
                ++nt;
            }
            mf = sc->tri_mat[2 * pid];
            mb = sc->tri_mat[2 * pid + 1];
        } else if (pid < sc->n_tri + sc->n_sph) {
            int64_t j = pid - sc->n_tri;
            const dnum *c = G->cen + 3 * j;
            double r = sc->sph[4 * j + 3];
            dnum oc[3] = {dn_sub(q[0], c[0]), dn_sub(q[1], c[1]), dn_sub(q[2], c[2])};
            dnum b = dn_dot(oc, vh);
            dnum cc = dn_sub(dn_dot(oc, oc), dn_c(r * r));
            dnum disc = dn_sub(dn_mul(b, b), cc);
            if (disc.v >= 0.0) {
                dnum sq = dn_sqrt(disc);
                dnum tr[2] = {dn_sub(dn_neg(b), sq), dn_add(dn_neg(b), sq)};
                for (int k = 0; k < 2; ++k) {
                    if (tr[k].v > lo && tr[k].v < hi) {
                        ts[nt] = tr[k];
                        for (int i = 0; i < 3; ++i)
                            ng[nt][i] = dn_divc(dn_sub(dn_add(q[i], dn_mul(tr[k], vh[i])), c[i]), r);
                        ++nt;
                    }
                }
            }
            mf = sc->sph_mat[2 * j];
            mb = sc->sph_mat[2 * j + 1];
        } else {
            int64_t p = pid - sc->n_tri - sc->n_sph;
            const double *pl = sc->pln + 4 * p;
            double tt;
            if (pln_isect(pl, qv, vv, &tt) && tt > lo && tt < hi) {
                ts[nt] = dn_div(dn_sub(dn_c(pl[3]), dn_dotc(pl, q)), dn_dotc(pl, vh));
                ts[nt].v = tt;
                for (int i = 0; i < 3; ++i) ng[nt][i] = dn_c(pl[i]);
                ++nt;
            }
            mf = sc->pln_mat[2 * p];
            mb = sc->pln_mat[2 * p + 1];
        }
        for (int c = 0; c < nt; ++c) {
            dnum dn = dn_dot(vh, ng[c]);
            int front = dn.v < 0.0;
            int64_t before = front ? mf : mb, after = front ? mb : mf;
            T = dn_mul(T, dn_transmit_fraction(G->Z[before], G->Z[after], front ? dn_neg(dn) : dn));
            dnum rem = dn_sub(dist, ts[c]);
            sum_a = dn_add(sum_a, dn_mul(dn_sub(G->ka[after], G->ka[before]), rem));
            sum_c = dn_add(sum_c, dn_mulc(rem, C->inv_c[after] - C->inv_c[before]));
        }
    }
    *T_out = T;
    *sa_out = sum_a;
    *sc_out = sum_c;
    return T.v != 0.0;
}

/* Capture of scatterer k at dual parameter s along the segment, as
 * scatter_nee. */
static void grad_capture(const gctx *G, gacc *A, int64_t tx, int64_t e, uint32_t ray, int64_t seg, int64_t k,
                         const dnum *o, const dnum *d, dnum w, dnum t, int64_t med)
{
    const octx *C = G->C;
    const or_acq *a = C->a;
    const double *sk = C->s->scat + 4 * k;
    dnum p[3] = {dn_sub(dn_c(sk[0]), o[0]), dn_sub(dn_c(sk[1]), o[1]), dn_sub(dn_c(sk[2]), o[2])};
    dnum s = dn_dot(p, d);
    dnum q[3] = {dn_add(o[0], dn_mul(s, d[0])), dn_add(o[1], dn_mul(s, d[1])), dn_add(o[2], dn_mul(s, d[2]))};
    dnum wq = dn_mul(w, dn_exp(dn_neg(dn_mul(G->ka[med], s))));
    dnum tq = dn_add(t, dn_mulc(s, C->inv_c[med]));
    double qv[3] = {q[0].v, q[1].v, q[2].v};
    int64_t e_lo = 0, n_e = a->n_elements;
    if (a->element_choice == 1 && !or_cone_elements(a, qv, &e_lo, &n_e)) return;
    uint32_t x[4];
    draw(C, ray, e, tx, seg, 2, (uint32_t)k, x);
    int64_t er = e_lo + (int64_t)(((uint64_t)x[0] * (uint64_t)n_e) >> 32);
    dnum v[3] = {dn_sub(dn_c(C->xe[er]), q[0]), dn_sub(dn_c(0.0), q[1]), dn_sub(dn_c(C->ze[er]), q[2])};
    dnum dist = dn_sqrt(dn_dot(v, v));
    dnum vh[3] = {dn_div(v[0], dist), dn_div(v[1], dist), dn_div(v[2], dist)};
    dnum cos_a = a->radius > 0.0 ? dn_neg(dn_add(dn_mulc(vh[0], C->sne[er]), dn_mulc(vh[2], C->cne[er])))
                                 : dn_neg(vh[2]);
    dnum al = dn_acos(cos_a);
    if (!(or_directivity(al.v, a->alpha_m, a->alpha_c) > 0.0)) return;
    dnum fdir = dn_directivity(al, a->alpha_m, a->alpha_c);
    dnum T, sum_a, sum_c;
    if (!grad_shadow(G, q, vh, dist, &T, &sum_a, &sum_c)) return;
    dnum att = dn_exp(dn_neg(dn_add(dn_mul(G->ka[med], dist), sum_a)));
    dnum tc = dn_add(dn_add(tq, dn_mulc(dist, C->inv_c[med])), sum_c);
    double amp = sk[3];
    /* the same product as scatter_nee, factor by factor */
    dnum geo = dn_mul(dn_mulc(dist, 4.0 * PI), dist);
    dnum cu = dn_mulc(dn_mulc(wq, (double)n_e), C->area_e);
    cu = dn_mul(dn_div(dn_mul(dn_mul(cu, cos_a), fdir), geo), T);
    cu = dn_mul(cu, att);
    dnum c = dn_mulc(dn_mulc(dn_mulc(wq, amp), (double)n_e), C->area_e);
    c = dn_mul(dn_mul(dn_div(dn_mul(dn_mul(c, cos_a), fdir), geo), T), att);
    grad_record(G, A, tx, er, c, tc, k, cu.v);
}

/* Dual distance along (o, d) to the primitive the value query chose (its
 * value is set to the query's). */
static dnum grad_distance(const gctx *G, const hit *h, const dnum *o, const dnum *d)
{
    const octx *C = G->C;
    const or_scene *s = C->s;
    dnum th;
    if (h->id == C->id_box && h->face == 6) {
        double R = C->a->radius;
        dnum aa = dn_add(dn_mul(d[0], d[0]), dn_mul(d[2], d[2]));
        dnum b = dn_add(dn_mul(o[0], d[0]), dn_mul(dn_add(o[2], dn_c(R)), d[2]));
        dnum c = dn_add(dn_mul(o[0], o[0]), dn_mul(o[2], dn_add(o[2], dn_c(2.0 * R))));
        th = dn_div(c, dn_add(dn_neg(b), dn_sqrt(dn_sub(dn_mul(b, b), dn_mul(aa, c)))));
    } else if (h->id == C->id_box) {
        int ax = h->face % 3;
        th = dn_div(dn_sub(dn_c(s->box[h->face]), o[ax]), d[ax]);
    } else if (h->id < C->id_sph0) {
        th = dn_tri_t(s->tri + 9 * h->id, o, d);
    } else if (h->id < C->id_pln0) {
        int64_t j = h->id - C->id_sph0;
        const dnum *c = G->cen + 3 * j;
        double r = s->sph[4 * j + 3];
        dnum oc[3] = {dn_sub(o[0], c[0]), dn_sub(o[1], c[1]), dn_sub(o[2], c[2])};
        dnum b = dn_dot(oc, d);
        dnum sq = dn_sqrt(dn_sub(dn_mul(b, b), dn_sub(dn_dot(oc, oc), dn_c(r * r))));
        dnum t0 = dn_sub(dn_neg(b), sq);
        th = t0.v > EPS_T ? t0 : dn_add(dn_neg(b), sq);
    } else {
        const double *pl = s->pln + 4 * (h->id - C->id_pln0);
        th = dn_div(dn_sub(dn_c(pl[3]), dn_dotc(pl, o)), dn_dotc(pl, d));
    }
    th.v = h->t;
    return th;
}

/* Smith masking G1 of the GGX distribution at a dual cos(theta_v) (as
 * or_ggx_g1). */
static dnum dn_ggx_g1(double alpha, dnum cv)
{
    dnum c2 = dn_mul(cv, cv);
    dnum tan2 = dn_div(dn_sub(dn_c(1.0), c2), c2);
    return dn_div(dn_c(2.0), dn_add(dn_c(1.0), dn_sqrt(dn_add(dn_c(1.0), dn_mulc(tan2, alpha * alpha)))));
}

/* Microfacet normal of or_ggx_sample about a dual unit normal n: the
 * random numbers fix the polar and azimuthal angles about n, the basis
 * (or_onb) follows n. */
static void dn_ggx_sample(const dnum *n, double alpha, double xi1, double xi2, dnum *h)
{
    double sg = copysign(1.0, n[2].v);
    dnum a = dn_div(dn_c(-1.0), dn_add(dn_c(sg), n[2]));
    dnum c = dn_mul(dn_mul(n[0], n[1]), a);
    dnum t[3] = {dn_add(dn_c(1.0), dn_mul(dn_mul(dn_mulc(n[0], sg), n[0]), a)), dn_mulc(c, sg), dn_mulc(n[0], -sg)};
    dnum b[3] = {c, dn_add(dn_c(sg), dn_mul(dn_mul(n[1], n[1]), a)), dn_neg(n[1])};
    double q = 1.0 - xi1 + alpha * alpha * xi1;
    double ct = sqrt((1.0 - xi1) / q), st = alpha * sqrt(xi1 / q);
    double ph = 2.0 * PI * xi2;
    double cp = cos(ph), sp = sin(ph);
    for (int i = 0; i < 3; ++i)
        h[i] = dn_add(dn_add(dn_mulc(t[i], st * cp), dn_mulc(b[i], st * sp)), dn_mulc(n[i], ct));
}

/* Replays one path of trace_path with dual numbers (smooth boundaries, and
 * rough ones without their secondary rays). */
static void grad_path(const gctx *G, gacc *A, int64_t tx, int64_t e, uint32_t ray, const double o_in[3],
                      const double d_in[3], double w0, double t0, int64_t med)
{
    const octx *C = G->C;
    const or_acq *a = C->a;
    const or_scene *sc = C->s;
    dnum o[3], d[3];
    for (int i = 0; i < 3; ++i) {
        o[i] = dn_c(o_in[i]);
        d[i] = dn_c(d_in[i]);
    }
    dnum w = dn_c(w0), t = dn_c(t0), len = dn_c(0.0);
    int64_t last = -1;
    double r2 = a->r_s * a->r_s;
    for (int64_t b = 0; b <= a->max_bounces; ++b) {
        double ov[3] = {o[0].v, o[1].v, o[2].v}, dv[3] = {d[0].v, d[1].v, d[2].v};
        hit h = closest(C, ov, dv, last);
        dnum tseg = grad_distance(G, &h, o, d);
        int clipped = 0;
        if (len.v + tseg.v > a->max_path) {
            tseg = dn_sub(dn_c(a->max_path), len);
            clipped = 1;
        }
        /* captures on [0, tseg), decided on the values as scatter_events */
        for (int64_t k = 0; k < sc->n_scat; ++k) {
            double p[3];
            sub3(sc->scat + 4 * k, ov, p);
            double sv = dot3(p, dv);
            if (!(sv >= 0.0 && sv < tseg.v)) continue;
            double perp[3] = {p[0] - sv * dv[0], p[1] - sv * dv[1], p[2] - sv * dv[2]};
            if (dot3(perp, perp) > r2) continue;
            grad_capture(G, A, tx, e, ray, b, k, o, d, w, t, med);
        }
        w = dn_mul(w, dn_exp(dn_neg(dn_mul(G->ka[med], tseg))));
        t = dn_add(t, dn_mulc(tseg, C->inv_c[med]));
        len = dn_add(len, tseg);
        for (int i = 0; i < 3; ++i) o[i] = dn_add(o[i], dn_mul(tseg, d[i]));
        if (clipped || t.v >= C->t_max) return;
        if (h.id == C->id_box) {
            int64_t er = -1;
            dnum ca;
            if (h.face == 6 && fabs(o[1].v) <= 0.5 * a->elevation) {
                double ph = atan2(o[0].v, o[2].v + a->radius);
                if (fabs(ph) <= C->half_arc) {
                    er = (int64_t)floor(ph / C->dphi + 0.5 * (double)a->n_elements);
                    if (er < 0) er = 0;
                    if (er > a->n_elements - 1) er = a->n_elements - 1;
                    ca = dn_neg(dn_add(dn_mulc(d[0], C->sne[er]), dn_mulc(d[2], C->cne[er])));
                }
            }
            if (a->radius == 0.0 && h.face == 2 && fabs(o[0].v) <= C->half_ap &&
                fabs(o[1].v) <= 0.5 * a->elevation) {
                er = (int64_t)floor((o[0].v + C->half_ap) / a->pitch);
                if (er < 0) er = 0;
                if (er > a->n_elements - 1) er = a->n_elements - 1;
                ca = dn_neg(d[2]);
            }
            if (er >= 0) {
                dnum al = dn_acos(ca);
                if (or_directivity(al.v, a->alpha_m, a->alpha_c) > 0.0)
                    grad_record(G, A, tx, er, dn_mul(w, dn_directivity(al, a->alpha_m, a->alpha_c)), t, -1, 0.0);
            }
            return;
        }
        if (b == a->max_bounces) return;
        /* impedance boundary, Eqs. 7-11 as fresnel_step */
        dnum ng[3];
        int64_t mf, mb;
        if (h.id < C->id_sph0) {
            double n[3];
            tri_normal(sc->tri + 9 * h.id, n);
            for (int i = 0; i < 3; ++i) ng[i] = dn_c(n[i]);
            mf = sc->tri_mat[2 * h.id];
            mb = sc->tri_mat[2 * h.id + 1];
        } else if (h.id < C->id_pln0) {
            int64_t j = h.id - C->id_sph0;
            for (int i = 0; i < 3; ++i) ng[i] = dn_divc(dn_sub(o[i], G->cen[3 * j + i]), sc->sph[4 * j + 3]);
            mf = sc->sph_mat[2 * j];
            mb = sc->sph_mat[2 * j + 1];
        } else {
            const double *pl = sc->pln + 4 * (h.id - C->id_pln0);
            for (int i = 0; i < 3; ++i) ng[i] = dn_c(pl[i]);
            mf = sc->pln_mat[2 * (h.id - C->id_pln0)];
            mb = sc->pln_mat[2 * (h.id - C->id_pln0) + 1];
        }
        int64_t before, after;
        if (dn_dot(d, ng).v < 0.0) {
            before = mf;
            after = mb;
        } else {
            before = mb;
            after = mf;
            for (int i = 0; i < 3; ++i) ng[i] = dn_neg(ng[i]);
        }
        dnum z1 = G->Z[before], z2 = G->Z[after];
        uint32_t x[4];
        draw(C, ray, e, tx, b, 1, 0, x);
        double y = unif(x[0]);
        double alpha = 0.0;
        if (sc->rough) alpha = sc->rough[mf] > sc->rough[mb] ? sc->rough[mf] : sc->rough[mb];
        dnum mn[3] = {ng[0], ng[1], ng[2]}, cn = dn_c(1.0);
        if (alpha > 0.0) {
            /* rough boundary (as rough_step): Eqs. 7-11 about the microfacet
             * normal drawn with the second and third words */
            dn_ggx_sample(ng, alpha, unif(x[1]), unif(x[2]), mn);
            dnum ci = dn_neg(dn_dot(d, mn));
            cn = dn_neg(dn_dot(d, ng));
            if (!(ci.v > 0.0)) return;
        }
        dnum cos_r = dn_neg(dn_dot(d, mn));
        dnum eta = dn_div(z1, z2);
        dnum rad = dn_sub(dn_c(1.0), dn_mul(dn_mul(eta, eta), dn_sub(dn_c(1.0), dn_mul(cos_r, cos_r))));
        dnum R = dn_c(1.0), cos_t = dn_c(0.0);
        if (rad.v >= 0.0) {
            cos_t = dn_sqrt(rad);
            dnum den = dn_add(dn_mul(z1, cos_r), dn_mul(z2, cos_t));
            if (den.v != 0.0) {
                dnum Ar = dn_div(dn_sub(dn_mul(z1, cos_r), dn_mul(z2, cos_t)), den);
                R = dn_mul(Ar, Ar);
            }
        }
        dnum nd[3];
        int refl = y < R.v;
        if (refl) {
            for (int i = 0; i < 3; ++i) nd[i] = dn_add(d[i], dn_mul(dn_mulc(cos_r, 2.0), mn[i]));
        } else {
            dnum f = dn_sub(dn_mul(eta, cos_r), cos_t);
            for (int i = 0; i < 3; ++i) nd[i] = dn_add(dn_mul(eta, d[i]), dn_mul(f, mn[i]));
        }
        dnum l = dn_sqrt(dn_dot(nd, nd));
        for (int i = 0; i < 3; ++i) nd[i] = dn_div(nd[i], l);
        if (alpha > 0.0) {
            /* wrong side of the macro surface: absorbed; else the weight
             * factor ci G1(i) G1(o) / (cn (mn.n)) */
            dnum co = dn_dot(nd, ng);
            if (refl ? !(co.v > 0.0) : !(co.v < 0.0)) return;
            dnum wf = dn_mul(dn_mul(cos_r, dn_ggx_g1(alpha, cn)), dn_ggx_g1(alpha, co.v < 0.0 ? dn_neg(co) : co));
            w = dn_mul(w, dn_div(wf, dn_mul(cn, dn_dot(mn, ng))));
        }
        if (refl) {
            if (G->attach) w = dn_mul(w, dn_divc(R, R.v));
            med = before;
        } else {
            dnum Tr = dn_sub(dn_c(1.0), R);
            if (G->attach) w = dn_mul(w, dn_divc(Tr, Tr.v));
            med = after;
        }
        for (int i = 0; i < 3; ++i) d[i] = nd[i];
        last = (h.id < C->id_sph0 || h.id >= C->id_pln0) ? h.id : -1;
    }
}

/* Emitted rays (every ray_stride-th of each row, rays == NULL) or the n_rays
 * explicit rays. */
static int grad_impl(const or_acq *a, const or_scene *s, int n_threads, int64_t ray_stride, const or_ray *rays,
                     int64_t n_rays, const double *g, int attach_choice, double *J, double *grad_z,
                     double *grad_alpha, double *grad_sph, double *grad_amp)
{
    if (a->n_elements <= 0 || a->n_elements > 65535 || a->n_tx <= 0 || a->n_tx > 65535 || a->n_samples <= 0 ||
        a->rays_per_element < 0 || a->max_bounces < 0 || ray_stride <= 0 || !g || a->cdf != NULL ||
        (a->scheme == 1 && a->n_tx != a->n_elements))
        return -1;
    if (2 * s->n_mat + 3 * s->n_sph > GRAD_MAX) return -1;
    if (s->rough && !a->rough_direct_only)
        for (int64_t m = 0; m < s->n_mat; ++m)
            if (s->rough[m] > 0.0) return -3;
    octx C;
    int rc_init = ctx_init(&C, a, s);
    if (rc_init) {
        ctx_free(&C);
        return rc_init;
    }
    g_nt = (int)(2 * s->n_mat + 3 * s->n_sph);
    gctx G;
    G.C = &C;
    G.g = g;
    G.attach = attach_choice;
    G.n_mat = (int)s->n_mat;
    G.Z = (dnum *)malloc(sizeof(dnum) * (size_t)(s->n_mat > 0 ? s->n_mat : 1));
    G.ka = (dnum *)malloc(sizeof(dnum) * (size_t)(s->n_mat > 0 ? s->n_mat : 1));
    G.cen = (dnum *)malloc(sizeof(dnum) * (size_t)(3 * s->n_sph + 1));
    double kappa = (a->f_c * 1e-6) * 100.0 * log(10.0) / 20.0;   /* d ka / d alpha */
    for (int64_t m = 0; m < s->n_mat; ++m) {
        G.Z[m] = dn_c(s->mat[3 * m]);
        G.Z[m].t[m] = 1.0;
        G.ka[m] = dn_c(C.ka[m]);
        G.ka[m].t[s->n_mat + m] = kappa;
    }
    for (int64_t j = 0; j < s->n_sph; ++j)
        for (int k = 0; k < 3; ++k) {
            G.cen[3 * j + k] = dn_c(s->sph[4 * j + k]);
            G.cen[3 * j + k].t[2 * s->n_mat + 3 * j + k] = 1.0;
        }
    int nt = n_threads;
#ifdef _OPENMP
    if (nt <= 0) nt = omp_get_max_threads();
#else
    nt = 1;
#endif
    if (nt < 1) nt = 1;
    gacc *acc = (gacc *)calloc((size_t)nt, sizeof(gacc));
    for (int i = 0; i < nt; ++i) acc[i].amp = (double *)calloc((size_t)(s->n_scat > 0 ? s->n_scat : 1), sizeof(double));
    int64_t per_el = (a->rays_per_element + ray_stride - 1) / ray_stride;
    int64_t n_work = rays ? n_rays : (a->scheme == 1 ? 1 : a->n_tx) * a->n_elements * per_el;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt)
#endif
    for (int64_t i = 0; i < n_work; ++i) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        if (rays) {
            const or_ray *r = &rays[i];
            grad_path(&G, &acc[tid], r->tx, r->elem, (uint32_t)r->ray, r->o, r->d, r->w, r->t, r->medium);
            continue;
        }
        int64_t rr = (i % per_el) * ray_stride;
        int64_t e = (i / per_el) % a->n_elements;
        int64_t tx = a->scheme == 1 ? e : i / (per_el * a->n_elements);
        double o[3], d[3], w;
        int64_t cell = -1;
        emit(&C, tx, e, (uint32_t)rr, o, d, &w, &cell);
        grad_path(&G, &acc[tid], tx, e, (uint32_t)rr, o, d, w, C.tau[tx * a->n_elements + e], s->top_medium);
    }
    /* fixed-order merge */
    double Jt = 0.0, gt[GRAD_MAX];
    memset(gt, 0, sizeof(gt));
    if (grad_amp) memset(grad_amp, 0, sizeof(double) * (size_t)s->n_scat);
    for (int i = 0; i < nt; ++i) {
        Jt += acc[i].J;
        for (int k = 0; k < g_nt; ++k) gt[k] += acc[i].grad[k];
        if (grad_amp)
            for (int64_t k = 0; k < s->n_scat; ++k) grad_amp[k] += acc[i].amp[k];
        free(acc[i].amp);
    }
    free(acc);
    if (J) *J = Jt;
    for (int64_t m = 0; m < s->n_mat; ++m) {
        if (grad_z) grad_z[m] = gt[m];
        if (grad_alpha) grad_alpha[m] = gt[s->n_mat + m];
    }
    if (grad_sph)
        for (int64_t j = 0; j < 3 * s->n_sph; ++j) grad_sph[j] = gt[2 * s->n_mat + j];
    free(G.Z);
    free(G.ka);
    free(G.cen);
    ctx_free(&C);
    return 0;
}

int or_trace_grad(const or_acq *a, const or_scene *s, int n_threads, int64_t ray_stride, const double *g,
                  int attach_choice, double *J, double *grad_z, double *grad_alpha, double *grad_sph,
                  double *grad_amp)
{
    return grad_impl(a, s, n_threads, ray_stride, NULL, 0, g, attach_choice, J, grad_z, grad_alpha, grad_sph,
                     grad_amp);
}

int or_trace_rays_grad(const or_acq *a, const or_scene *s, const or_ray *rays, int64_t n, const double *g,
                       int attach_choice, double *J, double *grad_z, double *grad_alpha, double *grad_sph,
                       double *grad_amp)
{
    if (n < 0 || (n > 0 && !rays)) return -1;
    return grad_impl(a, s, 1, 1, rays, n, g, attach_choice, J, grad_z, grad_alpha, grad_sph, grad_amp);
}

/* ----------------------------------------- element-edge terms of direct hits */
/* A direct hit is recorded into the element whose face holds its landing
 * point on the array's plane, so its contribution jumps where the landing
 * point crosses an element edge, an end of the aperture or an elevation
 * edge, and a geometry parameter theta that moves landing points moves these
 * jumps: or_trace_grad's interior derivative leaves their terms out.  Here
 * they are integrated exactly along one random number: the emission origin's
 * lateral coordinate u0 on the element face (Eq. 4), the direction, the
 * elevation coordinate and every choice held fixed.  For such a family of
 * paths F(u0) = c(u0) h(u0) (c the recorded value, h the adjoint g(t) of
 * the element holding the landing point x, 0 outside the aperture) and, by
 * the Leibniz rule on [0, 1], d/dtheta of its integral is the interior term
 * plus, at every u0* where x crosses an edge,
 *     [F] dx_n/dtheta / |dx_n/du0|,
 * [F] the jump of F across the edge in the direction of increasing x_n (x_n
 * the landing coordinate normal to the edge).  The crossings are found by
 * evaluating the family at n_scan + 1 evenly spaced u0 and halving every
 * interval whose ends follow different sequences of primitives and choices
 * (down to 1e-12), then by safeguarded Newton steps inside each interval
 * that follows one sequence.  The derivatives at u0* come from dual
 * numbers with u0 and every parameter as tangents.  On a convex array the
 * origin moves along the element's arc and the direction turns with it, the
 * landing coordinate across the elements is the arc angle, and each element
 * receives against its own normal, so F jumps in c as well as in g.  Smooth
 * boundaries, uniform emission; the reflect-or-transmit choice is attached,
 * as the result estimates the derivative of the expected data. */
typedef struct {
    int inside;      /* the landing point lies on an element */
    int64_t er;      /* that element */
    dnum x[2];       /* landing coordinates: across the elements (x, or the arc angle of a convex array), y */
    dnum c, t;       /* weight x receive directivity of element er (whether inside or not), arrival time */
    double w, d[3];  /* the weight and the arrival direction (values) */
    uint64_t sig;    /* the sequence of primitives and choices */
} ed_out;

/* Weight x receive directivity (Eq. 13) of a landing with weight w and
 * direction d into element er, against that element's normal. */
static double ed_c(const octx *C, const ed_out *o, int64_t er)
{
    const or_acq *a = C->a;
    double ca = a->radius > 0.0 ? -(o->d[0] * C->sne[er] + o->d[2] * C->cne[er]) : -o->d[2];
    double al = acos(ca > 1.0 ? 1.0 : (ca < -1.0 ? -1.0 : ca));
    return o->w * or_directivity(al, a->alpha_m, a->alpha_c);
}

/* sin and cos of a dual */
static void dn_sincos(dnum a, dnum *sn, dnum *cs)
{
    double s = sin(a.v), c = cos(a.v);
    *sn = dn_mulc(a, c);
    sn->v = s;
    *cs = dn_mulc(a, -s);
    cs->v = c;
}

/* Replays the family's path at origin coordinate u0 (tangent 0: u0; the
 * parameters' tangents come with G's Z and cen).  Returns 1 if it ends on
 * the array's plane within the bounce, time and length limits. */
static int ed_path(const gctx *G, int64_t tx, int64_t e, uint32_t ray, double u0, ed_out *out)
{
    const octx *C = G->C;
    const or_acq *a = C->a;
    const or_scene *sc = C->s;
    uint32_t x[4];
    draw(C, ray, e, tx, 0, 0, 0, x);
    double hl[3];
    or_hemisphere(unif(x[2]), unif(x[3]), hl);
    dnum o[3], d[3];
    o[1] = dn_c((unif(x[1]) - 0.5) * a->elevation);
    if (a->radius > 0.0) {
        /* on the element's arc; the direction turns with the local normal */
        dnum ph = dn_c(((double)e - 0.5 * (double)(a->n_elements - 1) + (u0 - 0.5)) * C->dphi);
        ph.t[0] = C->dphi;
        dnum sp, cp, sh, chh;
        dn_sincos(ph, &sp, &cp);
        dn_sincos(dn_mulc(ph, 0.5), &sh, &chh);
        o[0] = dn_mulc(sp, a->radius);
        o[2] = dn_mul(dn_mulc(sh, -2.0 * a->radius), sh);
        d[0] = dn_add(dn_mulc(cp, hl[0]), dn_mulc(sp, hl[2]));
        d[1] = dn_c(hl[1]);
        d[2] = dn_sub(dn_mulc(cp, hl[2]), dn_mulc(sp, hl[0]));
    } else {
        o[0] = dn_c(C->xe[e] + (u0 - 0.5) * a->pitch);
        o[0].t[0] = a->pitch;
        o[2] = dn_c(0.0);
        for (int i = 0; i < 3; ++i) d[i] = dn_c(hl[i]);
    }
    const double pdf = 1.0 / (2.0 * PI);
    dnum w = dn_c(hl[2] / (C->n_per_tx * pdf)), t = dn_c(C->tau[tx * a->n_elements + e]), len = dn_c(0.0);
    int64_t med = sc->top_medium, last = -1;
    uint64_t sig = 1469598103934665603ull;
    for (int64_t b = 0; b <= a->max_bounces; ++b) {
        double ov[3] = {o[0].v, o[1].v, o[2].v}, dv[3] = {d[0].v, d[1].v, d[2].v};
        hit h = closest(C, ov, dv, last);
        dnum tseg = grad_distance(G, &h, o, d);
        int clipped = 0;
        if (len.v + tseg.v > a->max_path) {
            tseg = dn_sub(dn_c(a->max_path), len);
            clipped = 1;
        }
        w = dn_mul(w, dn_exp(dn_neg(dn_mul(G->ka[med], tseg))));
        t = dn_add(t, dn_mulc(tseg, C->inv_c[med]));
        len = dn_add(len, tseg);
        for (int i = 0; i < 3; ++i) o[i] = dn_add(o[i], dn_mul(tseg, d[i]));
        if (clipped || t.v >= C->t_max) return 0;
        sig = (sig ^ (uint64_t)(8 * (h.id + 1) + h.face + 1)) * 1099511628211ull;
        if (h.id == C->id_box) {
            int64_t er;
            dnum ca;
            if (a->radius > 0.0) {
                /* the arc angle atan2(x, z + R) of the landing point */
                if (h.face != 6) return 0;
                dnum zc = dn_add(o[2], dn_c(a->radius));
                double r2 = o[0].v * o[0].v + zc.v * zc.v;
                dnum ph = dn_c(atan2(o[0].v, zc.v));
                for (int i = 0; i < g_nt; ++i) ph.t[i] = (zc.v * o[0].t[i] - o[0].v * zc.t[i]) / r2;
                out->x[0] = ph;
                out->inside = fabs(ph.v) <= C->half_arc && fabs(o[1].v) <= 0.5 * a->elevation;
                er = (int64_t)floor(ph.v / C->dphi + 0.5 * (double)a->n_elements);
                er = er < 0 ? 0 : (er > a->n_elements - 1 ? a->n_elements - 1 : er);
                ca = dn_neg(dn_add(dn_mulc(d[0], C->sne[er]), dn_mulc(d[2], C->cne[er])));
            } else {
                if (h.face != 2) return 0;
                out->x[0] = o[0];
                out->inside = fabs(o[0].v) <= C->half_ap && fabs(o[1].v) <= 0.5 * a->elevation;
                er = (int64_t)floor((o[0].v + C->half_ap) / a->pitch);
                er = er < 0 ? 0 : (er > a->n_elements - 1 ? a->n_elements - 1 : er);
                ca = dn_neg(d[2]);
            }
            out->x[1] = o[1];
            out->er = er;
            out->w = w.v;
            for (int i = 0; i < 3; ++i) out->d[i] = d[i].v;
            dnum al = dn_acos(ca);
            out->c = or_directivity(al.v, a->alpha_m, a->alpha_c) > 0.0
                         ? dn_mul(w, dn_directivity(al, a->alpha_m, a->alpha_c)) : dn_c(0.0);
            out->t = t;
            out->sig = sig;
            return 1;
        }
        if (b == a->max_bounces) return 0;
        dnum ng[3];
        int64_t mf, mb;
        if (h.id < C->id_sph0) {
            double n[3];
            tri_normal(sc->tri + 9 * h.id, n);
            for (int i = 0; i < 3; ++i) ng[i] = dn_c(n[i]);
            mf = sc->tri_mat[2 * h.id];
            mb = sc->tri_mat[2 * h.id + 1];
        } else if (h.id < C->id_pln0) {
            int64_t j = h.id - C->id_sph0;
            for (int i = 0; i < 3; ++i) ng[i] = dn_divc(dn_sub(o[i], G->cen[3 * j + i]), sc->sph[4 * j + 3]);
            mf = sc->sph_mat[2 * j];
            mb = sc->sph_mat[2 * j + 1];
        } else {
            const double *pl = sc->pln + 4 * (h.id - C->id_pln0);
            for (int i = 0; i < 3; ++i) ng[i] = dn_c(pl[i]);
            mf = sc->pln_mat[2 * (h.id - C->id_pln0)];
            mb = sc->pln_mat[2 * (h.id - C->id_pln0) + 1];
        }
        int64_t before, after;
        if (dn_dot(d, ng).v < 0.0) {
            before = mf;
            after = mb;
        } else {
            before = mb;
            after = mf;
            for (int i = 0; i < 3; ++i) ng[i] = dn_neg(ng[i]);
        }
        dnum z1 = G->Z[before], z2 = G->Z[after];
        draw(C, ray, e, tx, b, 1, 0, x);
        double y = unif(x[0]);
        dnum cos_r = dn_neg(dn_dot(d, ng));
        dnum eta = dn_div(z1, z2);
        dnum rad = dn_sub(dn_c(1.0), dn_mul(dn_mul(eta, eta), dn_sub(dn_c(1.0), dn_mul(cos_r, cos_r))));
        dnum R = dn_c(1.0), cos_t = dn_c(0.0);
        if (rad.v >= 0.0) {
            cos_t = dn_sqrt(rad);
            dnum den = dn_add(dn_mul(z1, cos_r), dn_mul(z2, cos_t));
            if (den.v != 0.0) {
                dnum Ar = dn_div(dn_sub(dn_mul(z1, cos_r), dn_mul(z2, cos_t)), den);
                R = dn_mul(Ar, Ar);
            }
        }
        dnum nd[3];
        int refl = y < R.v;
        if (refl) {
            for (int i = 0; i < 3; ++i) nd[i] = dn_add(d[i], dn_mul(dn_mulc(cos_r, 2.0), ng[i]));
            if (G->attach) w = dn_mul(w, dn_divc(R, R.v));
            med = before;
        } else {
            dnum f = dn_sub(dn_mul(eta, cos_r), cos_t);
            for (int i = 0; i < 3; ++i) nd[i] = dn_add(dn_mul(eta, d[i]), dn_mul(f, ng[i]));
            dnum Tr = dn_sub(dn_c(1.0), R);
            if (G->attach) w = dn_mul(w, dn_divc(Tr, Tr.v));
            med = after;
        }
        dnum l = dn_sqrt(dn_dot(nd, nd));
        for (int i = 0; i < 3; ++i) d[i] = dn_div(nd[i], l);
        sig = (sig ^ (uint64_t)(2 + refl)) * 1099511628211ull;
        last = (h.id < C->id_sph0 || h.id >= C->id_pln0) ? h.id : -1;
    }
    return 0;
}

/* The adjoint g of element er at time t (as grad_record); 0 outside the
 * recorded window. */
static double ed_adj(const octx *C, const double *g, int64_t tx, int64_t er, double t)
{
    const or_acq *a = C->a;
    if (!(t < C->t_max) || t < 0.0) return 0.0;
    const double *ch = g + (tx * a->n_elements + er) * a->n_samples;
    double x = t * a->f_s;
    if (a->binning == 0) {
        int64_t n = (int64_t)floor(x);
        return (n >= 0 && n < a->n_samples) ? ch[n] : 0.0;
    }
    double tau = x - 0.5, f0 = floor(tau), f = tau - f0;
    int64_t n0 = (int64_t)f0;
    double g0 = (n0 >= 0 && n0 < a->n_samples) ? ch[n0] : 0.0;
    double g1 = (n0 + 1 >= 0 && n0 + 1 < a->n_samples) ? ch[n0 + 1] : 0.0;
    return (1.0 - f) * g0 + f * g1;
}

/* The u0 in (ua, ub) where landing coordinate k crosses X, by Newton steps
 * kept inside the bracket (bisection when a step leaves it), on paths with
 * the sequence sig.  Returns 1 with the path there, 0 if the sequence
 * changes on the way. */
static int ed_root(const gctx *G, int64_t tx, int64_t e, uint32_t ray, double ua, double ub, double fa, int k,
                   double X, uint64_t sig, ed_out *out)
{
    double u = 0.5 * (ua + ub);
    for (int it = 0; it < 100; ++it) {
        if (!ed_path(G, tx, e, ray, u, out) || out->sig != sig) return 0;
        double f = out->x[k].v - X, df = out->x[k].t[0];
        if (f == 0.0 || ub - ua < 1e-15) return 1;
        if ((f < 0.0) == (fa < 0.0)) {
            ua = u;
            fa = f;
        } else {
            ub = u;
        }
        double un = df != 0.0 ? u - f / df : 0.5 * (ua + ub);
        if (!(un > ua && un < ub)) un = 0.5 * (ua + ub);
        if (un == u) return 1;
        u = un;
    }
    return 1;
}

/* The edge crossings of the family on [ua, ub] (landings A at ua and B at
 * ub, if any), added to acc: an interval whose ends follow different
 * sequences is halved until each part follows one (parts narrower than
 * 1e-12 are dropped). */
static void ed_interval(const gctx *G, const double *g, int64_t tx, int64_t e, uint32_t ray, double ua, int ha,
                        const ed_out *A, double ub, int hb, const ed_out *B, int depth, double *acc, int np)
{
    const octx *C = G->C;
    const or_acq *a = C->a;
    if (!ha && !hb) return;
    if (!ha || !hb || A->sig != B->sig) {
        if (depth >= 48 || ub - ua < 1e-12) return;
        const double um = 0.5 * (ua + ub);
        ed_out M;
        const int hm = ed_path(G, tx, e, ray, um, &M);
        ed_interval(G, g, tx, e, ray, ua, ha, A, um, hm, &M, depth + 1, acc, np);
        ed_interval(G, g, tx, e, ray, um, hm, &M, ub, hb, B, depth + 1, acc, np);
        return;
    }
    ed_out at;
    const double half_el = 0.5 * a->elevation;
    /* element edges and aperture ends crossed (in x, or in the arc angle of
     * a convex array, whose elements each have their own normal) */
    const int convex = a->radius > 0.0;
    const double xa = A->x[0].v, xb = B->x[0].v;
    const double lo = xa < xb ? xa : xb, hi = xa < xb ? xb : xa;
    for (int64_t k = 0; k <= a->n_elements; ++k) {
        const double X = convex ? ((double)k - 0.5 * (double)a->n_elements) * C->dphi
                                : -C->half_ap + (double)k * a->pitch;
        if (!(X > lo && X < hi)) continue;
        if (!ed_root(G, tx, e, ray, ua, ub, xa - X, 0, X, A->sig, &at)) continue;
        if (!(fabs(at.x[1].v) <= half_el)) continue;
        const double fr = k < a->n_elements ? ed_c(C, &at, k) * ed_adj(C, g, tx, k, at.t.v) : 0.0;
        const double fl = k > 0 ? ed_c(C, &at, k - 1) * ed_adj(C, g, tx, k - 1, at.t.v) : 0.0;
        const double jump = fr - fl, du = fabs(at.x[0].t[0]);
        if (!(du > 0.0)) continue;
        for (int p = 0; p < np; ++p) acc[p] += jump * at.x[0].t[1 + p] / du;
    }
    /* elevation edges crossed in y: inside below the edge in |y|, so F
     * jumps by -F_in across +Y and by +F_in across -Y */
    const double ya = A->x[1].v, yb = B->x[1].v;
    for (int sgn = -1; sgn <= 1; sgn += 2) {
        const double Y = sgn * half_el;
        if (!((ya - Y) * (yb - Y) < 0.0)) continue;
        if (!ed_root(G, tx, e, ray, ua, ub, ya - Y, 1, Y, A->sig, &at)) continue;
        if (!(fabs(at.x[0].v) <= (convex ? C->half_arc : C->half_ap))) continue;
        const double fin = at.c.v * ed_adj(C, g, tx, at.er, at.t.v);
        const double jump = sgn > 0 ? -fin : fin, du = fabs(at.x[1].t[0]);
        if (!(du > 0.0)) continue;
        for (int p = 0; p < np; ++p) acc[p] += jump * at.x[1].t[1 + p] / du;
    }
}

/* Parameters of the edge replays: impedances (tangents 1 ..), then sphere
 * centres; tangent 0 is the origin coordinate u0. */
static int ed_setup(const or_acq *a, const or_scene *s, int attach, octx *C, gctx *G)
{
    if (a->n_elements <= 0 || a->n_elements > 65535 || a->n_tx <= 0 || a->n_tx > 65535 || a->n_samples <= 0 ||
        a->rays_per_element < 0 || a->max_bounces < 0 || a->cdf != NULL || a->scheme == 1)
        return -1;
    if (1 + s->n_mat + 3 * s->n_sph > GRAD_MAX) return -1;
    if (s->rough)
        for (int64_t m = 0; m < s->n_mat; ++m)
            if (s->rough[m] > 0.0) return -3;
    int rc = ctx_init(C, a, s);
    if (rc) {
        ctx_free(C);
        return rc;
    }
    g_nt = (int)(1 + s->n_mat + 3 * s->n_sph);
    G->C = C;
    G->g = NULL;
    G->attach = attach;
    G->n_mat = (int)s->n_mat;
    G->Z = (dnum *)malloc(sizeof(dnum) * (size_t)(s->n_mat > 0 ? s->n_mat : 1));
    G->ka = (dnum *)malloc(sizeof(dnum) * (size_t)(s->n_mat > 0 ? s->n_mat : 1));
    G->cen = (dnum *)malloc(sizeof(dnum) * (size_t)(3 * s->n_sph + 1));
    for (int64_t m = 0; m < s->n_mat; ++m) {
        G->Z[m] = dn_c(s->mat[3 * m]);
        G->Z[m].t[1 + m] = 1.0;
        G->ka[m] = dn_c(C->ka[m]);
    }
    for (int64_t j = 0; j < 3 * s->n_sph; ++j) {
        G->cen[j] = dn_c(s->sph[4 * (j / 3) + j % 3]);
        G->cen[j].t[1 + s->n_mat + j] = 1.0;
    }
    return 0;
}

static void ed_free(octx *C, gctx *G)
{
    free(G->Z);
    free(G->ka);
    free(G->cen);
    ctx_free(C);
}

/* The edge term of one family, added to acc [np]. */
static void ed_family(const gctx *G, const double *g, int64_t tx, int64_t e, uint32_t ray, int n_scan, double *acc,
                      int np)
{
    ed_out prev, cur;
    int have_prev = ed_path(G, tx, e, ray, 0.0, &prev);
    for (int j = 1; j <= n_scan; ++j) {
        const double ua = (double)(j - 1) / n_scan, ub = (double)j / n_scan;
        int have = ed_path(G, tx, e, ray, ub, &cur);
        ed_interval(G, g, tx, e, ray, ua, have_prev, &prev, ub, have, &cur, 0, acc, np);
        prev = cur;
        have_prev = have;
    }
}

int or_trace_grad_edges(const or_acq *a, const or_scene *s, int n_threads, int64_t ray_stride, const double *g,
                        int n_scan, double *corr_z, double *corr_sph)
{
    if (ray_stride <= 0 || !g || n_scan < 1) return -1;
    octx C;
    gctx G;
    int rc = ed_setup(a, s, 1, &C, &G);
    if (rc) return rc;
    G.g = g;
    const int np = (int)(s->n_mat + 3 * s->n_sph);
    int nt = n_threads;
#ifdef _OPENMP
    if (nt <= 0) nt = omp_get_max_threads();
#else
    nt = 1;
#endif
    if (nt < 1) nt = 1;
    double *acc = (double *)calloc((size_t)nt * (size_t)(np > 0 ? np : 1), sizeof(double));
    int64_t per_el = (a->rays_per_element + ray_stride - 1) / ray_stride;
    int64_t n_work = a->n_tx * a->n_elements * per_el;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt)
#endif
    for (int64_t i = 0; i < n_work; ++i) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        int64_t rr = (i % per_el) * ray_stride;
        int64_t e = (i / per_el) % a->n_elements;
        int64_t tx = i / (per_el * a->n_elements);
        ed_family(&G, g, tx, e, (uint32_t)rr, n_scan, acc + (size_t)tid * np, np);
    }
    for (int p = 0; p < np; ++p) {
        double v = 0.0;
        for (int i = 0; i < nt; ++i) v += acc[(size_t)i * np + p];
        if (p < s->n_mat) {
            if (corr_z) corr_z[p] = v;
        } else if (corr_sph) {
            corr_sph[p - s->n_mat] = v;
        }
    }
    free(acc);
    ed_free(&C, &G);
    return 0;
}

/* One family (transmit tx, element e, ray) at the n origin coordinates u0:
 * F = c g(t) (0 if the landing is off the elements or the path does not
 * land), its interior derivative along every parameter dF [n][np]
 * (g(t) dc + c g'(t) dt), the landing point X [n][2] (NaN if none) and the
 * sequence sig [n] (0 if none); and the family's edge term B [np] from an
 * n_scan scan.  attach 0 freezes the reflect-or-transmit choice. */
int or_edge_family(const or_acq *a, const or_scene *s, const double *g, int64_t tx, int64_t e, int64_t ray, int attach,
                   int64_t n, const double *u0, double *F, double *dF, double *X, uint64_t *sig, int n_scan, double *B)
{
    if (!g || n < 0 || (n > 0 && (!u0 || !F || !dF || !X || !sig)) || n_scan < 1 || !B || tx < 0 || tx >= a->n_tx ||
        e < 0 || e >= a->n_elements || ray < 0 || ray >= a->rays_per_element)
        return -1;
    octx C;
    gctx G;
    int rc = ed_setup(a, s, attach, &C, &G);
    if (rc) return rc;
    G.g = g;
    const int np = (int)(s->n_mat + 3 * s->n_sph);
    for (int64_t i = 0; i < n; ++i) {
        ed_out o;
        F[i] = 0.0;
        for (int p = 0; p < np; ++p) dF[i * np + p] = 0.0;
        X[2 * i] = X[2 * i + 1] = NAN;
        sig[i] = 0;
        if (!ed_path(&G, tx, e, (uint32_t)ray, u0[i], &o)) continue;
        X[2 * i] = o.x[0].v;
        X[2 * i + 1] = o.x[1].v;
        sig[i] = o.sig;
        if (!o.inside || !(o.t.v < C.t_max) || o.t.v < 0.0) continue;
        const double *ch = g + (tx * a->n_elements + o.er) * a->n_samples;
        double gv, gs;
        double x = o.t.v * a->f_s;
        if (a->binning == 0) {
            int64_t k = (int64_t)floor(x);
            gv = (k >= 0 && k < a->n_samples) ? ch[k] : 0.0;
            gs = 0.0;
        } else {
            double tau = x - 0.5, f0 = floor(tau), f = tau - f0;
            int64_t k = (int64_t)f0;
            double g0 = (k >= 0 && k < a->n_samples) ? ch[k] : 0.0;
            double g1 = (k + 1 >= 0 && k + 1 < a->n_samples) ? ch[k + 1] : 0.0;
            gv = (1.0 - f) * g0 + f * g1;
            gs = (g1 - g0) * a->f_s;
        }
        F[i] = o.c.v * gv;
        for (int p = 0; p < np; ++p) dF[i * np + p] = o.c.t[1 + p] * gv + o.c.v * gs * o.t.t[1 + p];
    }
    for (int p = 0; p < np; ++p) B[p] = 0.0;
    ed_family(&G, g, tx, e, (uint32_t)ray, n_scan, B, np);
    ed_free(&C, &G);
    return 0;
}

/* ---------------------------------------------------------------- pulse Eq. 14 */
/* Analytic pulse h[m] = g(m/fs) (sin(2 pi fc m/fs) - i cos(2 pi fc m/fs)),
 * whose real part is Eq. 14 with the Gaussian written exp(-t^2/(2 sigma^2));
 * sigma is set so the envelope's full width at half maximum equals n_cycles
 * periods.  Taps |m| <= K = ceil(3 sigma fs). */
int or_pulse_taps(const or_acq *a, double *taps, int64_t cap)
{
    double sig = a->n_cycles / (2.0 * sqrt(2.0 * log(2.0)) * a->f_c);
    int K = (int)ceil(3.0 * sig * a->f_s);
    if (taps == NULL) return K;
    if (2 * K + 1 > cap) return -1;
    for (int m = -K; m <= K; ++m) {
        double tm = (double)m / a->f_s;
        double g = exp(-tm * tm / (2.0 * sig * sig));
        double ph = 2.0 * PI * a->f_c * tm;
        taps[2 * (m + K)] = g * sin(ph);
        taps[2 * (m + K) + 1] = -g * cos(ph);
    }
    return K;
}

/* ch_rf[n] = sum_m h[m] ch_raw[n - m], zero outside the record. */
int or_pulse(const or_acq *a, int64_t n_channels, const double *ch_raw, double *ch_rf)
{
    int K = or_pulse_taps(a, NULL, 0);
    double *h = (double *)malloc(sizeof(double) * (size_t)(2 * (2 * K + 1)));
    if (!h) return -2;
    or_pulse_taps(a, h, 2 * K + 1);
    int64_t S = a->n_samples, nch = n_channels;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t ch = 0; ch < nch; ++ch) {
        const double *x = ch_raw + ch * S;
        double *y = ch_rf + 2 * ch * S;
        for (int64_t n = 0; n < S; ++n) {
            double re = 0.0, im = 0.0;
            for (int m = -K; m <= K; ++m) {
                int64_t j = n - m;
                if (j < 0 || j >= S) continue;
                re += h[2 * (m + K)] * x[j];
                im += h[2 * (m + K) + 1] * x[j];
            }
            y[2 * n] = re;
            y[2 * n + 1] = im;
        }
    }
    free(h);
    return 0;
}

/* ------------------------------------------------------------------- DAS */
/* Plane-wave delay-and-sum with coherent compounding: the transmit delay is
 * the steered plane wavefront's arrival at the pixel, referenced like the
 * emission delays; the receive delay is the straight path back to each
 * element; both use c0.  Sample n stands for time (n + 1/2)/fs; the analytic
 * channel signal is linearly interpolated (zero outside [0, S-1)), weighted
 * by a Hann window over the receive aperture and summed over elements and
 * transmits. */
static void das_point(const or_acq *a, const double *xe, const double *ze, const double *apod, double x,
                      double z, const double *ch_rf, double out[2])
{
    int64_t E = a->n_elements, S = a->n_samples;
    double re = 0.0, im = 0.0;
    for (int64_t tx = 0; tx < a->n_tx; ++tx) {
        double st = sin(a->angles[tx]), ct = cos(a->angles[tx]);
        double ttx;
        if (a->radius > 0.0) {
            /* convex array: the plane front k.p, referenced like its delays */
            double ref = INFINITY;
            for (int64_t e = 0; e < E; ++e)
                if (xe[e] * st + ze[e] * ct < ref) ref = xe[e] * st + ze[e] * ct;
            ttx = (x * st + z * ct - ref) / a->c0;
        } else {
            double xref = st >= 0 ? xe[0] : xe[E - 1];
            ttx = ((x - xref) * st + z * ct) / a->c0;
        }
        for (int64_t e = 0; e < E; ++e) {
            double dx = x - xe[e], dz = z - ze[e];
            double trx = sqrt(dx * dx + dz * dz) / a->c0;
            double idx = (ttx + trx) * a->f_s - 0.5;
            double f0 = floor(idx);
            int64_t i0 = (int64_t)f0;
            double fr = idx - f0;
            if (i0 < 0 || i0 >= S - 1) continue;
            const double *p = ch_rf + 2 * ((tx * E + e) * S + i0);
            re += apod[e] * ((1.0 - fr) * p[0] + fr * p[2]);
            im += apod[e] * ((1.0 - fr) * p[1] + fr * p[3]);
        }
    }
    out[0] = re;
    out[1] = im;
}

static int das_tables(const or_acq *a, double **xe, double **ze, double **apod)
{
    int64_t E = a->n_elements;
    *xe = (double *)malloc(sizeof(double) * (size_t)E);
    *ze = (double *)malloc(sizeof(double) * (size_t)E);
    *apod = (double *)malloc(sizeof(double) * (size_t)E);
    if (!*xe || !*ze || !*apod) return -2;
    for (int64_t e = 0; e < E; ++e) {
        double g[4];
        or_element_geometry(a, e, g);
        (*xe)[e] = g[0];
        (*ze)[e] = g[1];
        (*apod)[e] = 0.5 - 0.5 * cos(2.0 * PI * ((double)e + 0.5) / (double)E);
    }
    return 0;
}

/* ---------------------------------------------- synthetic-aperture synthesis */
/* A steered plane wave is the sum over elements of each element's own
 * transmit delayed by its steering delay (Sec. 2.3 "Ray Emission", Fig. 3):
 * with synthetic-aperture data, element e's channels are shifted by
 * tau_k(e) fs samples, linearly interpolated between samples. */
int or_synthesize(const or_acq *a, const double *ch_sa, const double *angles, int64_t n_ang, double *out)
{
    const int64_t E = a->n_elements, S = a->n_samples;
    or_acq b = *a;
    b.angles = angles;
    b.n_tx = n_ang;
    b.scheme = 0;
    memset(out, 0, sizeof(double) * (size_t)(n_ang * E * S));
    for (int64_t k = 0; k < n_ang; ++k)
        for (int64_t e = 0; e < E; ++e) {
            double sh = or_delay(&b, k, e) * a->f_s;
            for (int64_t er = 0; er < E; ++er) {
                const double *x = ch_sa + (e * E + er) * S;
                double *y = out + (k * E + er) * S;
                for (int64_t s = 0; s < S; ++s) {
                    double u = (double)s - sh;
                    double f0 = floor(u);
                    int64_t i0 = (int64_t)f0;
                    double f = u - f0;
                    double v0 = (i0 >= 0 && i0 < S) ? x[i0] : 0.0;
                    double v1 = (i0 + 1 >= 0 && i0 + 1 < S) ? x[i0 + 1] : 0.0;
                    y[s] += (1.0 - f) * v0 + f * v1;
                }
            }
        }
    return 0;
}

int or_das(const or_acq *a, int64_t nx, int64_t nz, double x0, double x1, double z0, double z1,
           const double *ch_rf, int n_threads, double *iq)
{
    double *xe, *ze, *apod;
    if (das_tables(a, &xe, &ze, &apod)) return -2;
    double dx = nx > 1 ? (x1 - x0) / (double)(nx - 1) : 0.0;
    double dz = nz > 1 ? (z1 - z0) / (double)(nz - 1) : 0.0;
    int nt = n_threads;
#ifdef _OPENMP
    if (nt <= 0) nt = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
    for (int64_t ix = 0; ix < nx; ++ix) {
        for (int64_t iz = 0; iz < nz; ++iz)
            das_point(a, xe, ze, apod, x0 + (double)ix * dx, z0 + (double)iz * dz, ch_rf, iq + 2 * (ix * nz + iz));
    }
    (void)nt;
    free(xe);
    free(ze);
    free(apod);
    return 0;
}

int or_das_points(const or_acq *a, const double *xz, int64_t n, const double *ch_rf, double *iq)
{
    double *xe, *ze, *apod;
    if (das_tables(a, &xe, &ze, &apod)) return -2;
    for (int64_t i = 0; i < n; ++i) das_point(a, xe, ze, apod, xz[2 * i], xz[2 * i + 1], ch_rf, iq + 2 * i);
    free(xe);
    free(ze);
    free(apod);
    return 0;
}

/* Envelope |IQ| and log compression to a dynamic range of dr_db decibels. */
int or_envelope(int64_t n, const double *iq, double dr_db, double *env, double *bmode)
{
    double mx = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        env[i] = sqrt(iq[2 * i] * iq[2 * i] + iq[2 * i + 1] * iq[2 * i + 1]);
        if (env[i] > mx) mx = env[i];
    }
    if (!bmode) return 0;
    for (int64_t i = 0; i < n; ++i) {
        double db = (mx > 0.0 && env[i] > 0.0) ? 20.0 * log10(env[i] / mx) : -dr_db;
        bmode[i] = db < -dr_db ? -dr_db : db;
    }
    return 0;
}

/* ------------------------------------------------ sector grids (convex array) */
/* Pixel (i, j) of a sector grid sits at angle phi_i = p0 + i (p1 - p0)/(np - 1)
 * from +z and depth r_j = r0 + j (r1 - r0)/(nr - 1) below the array face,
 * along the ray from the centre of curvature (0, 0, -R):
 * (x, z) = (R + r) (sin phi, cos phi) - (0, R).  R = 0 gives a sector about
 * the origin. */
int or_sector_points(double radius, int64_t np, int64_t nr, double p0, double p1, double r0, double r1, double *xz)
{
    if (np < 1 || nr < 1 || radius < 0.0) return -1;
    double dp = np > 1 ? (p1 - p0) / (double)(np - 1) : 0.0, dr = nr > 1 ? (r1 - r0) / (double)(nr - 1) : 0.0;
    for (int64_t i = 0; i < np; ++i)
        for (int64_t j = 0; j < nr; ++j) {
            double ph = p0 + (double)i * dp, r = radius + r0 + (double)j * dr;
            xz[2 * (i * nr + j)] = r * sin(ph);
            xz[2 * (i * nr + j) + 1] = r * cos(ph) - radius;
        }
    return 0;
}

/* Scan conversion of a sector image img[np][nr] (grid as above) onto the
 * Cartesian grid x_k = x0 + k (x1 - x0)/(nx - 1), z_l likewise: each pixel
 * takes its polar coordinates about (0, 0, -R), phi = atan2(x, z + R) and
 * r = |(x, z + R)| - R, and interpolates the image bilinearly in (phi, r)
 * between the four surrounding samples; pixels outside the sector's closed
 * (phi, r) rectangle take `fill`. */
int or_scan_convert(double radius, int64_t np, int64_t nr, double p0, double p1, double r0, double r1,
                    const double *img, int64_t nx, int64_t nz, double x0, double x1, double z0, double z1,
                    double fill, double *out)
{
    if (np < 2 || nr < 2 || nx < 1 || nz < 1 || radius < 0.0 || !(p1 > p0) || !(r1 > r0)) return -1;
    double dp = (p1 - p0) / (double)(np - 1), dr = (r1 - r0) / (double)(nr - 1);
    double dx = nx > 1 ? (x1 - x0) / (double)(nx - 1) : 0.0, dz = nz > 1 ? (z1 - z0) / (double)(nz - 1) : 0.0;
    for (int64_t k = 0; k < nx; ++k)
        for (int64_t l = 0; l < nz; ++l) {
            double x = x0 + (double)k * dx, zc = z0 + (double)l * dz + radius;
            double fi = (atan2(x, zc) - p0) / dp, fj = (sqrt(x * x + zc * zc) - radius - r0) / dr;
            double v = fill;
            if (fi >= 0.0 && fi <= (double)(np - 1) && fj >= 0.0 && fj <= (double)(nr - 1)) {
                int64_t i0 = (int64_t)floor(fi), j0 = (int64_t)floor(fj);
                if (i0 > np - 2) i0 = np - 2;
                if (j0 > nr - 2) j0 = nr - 2;
                double a = fi - (double)i0, b = fj - (double)j0;
                v = (1.0 - a) * ((1.0 - b) * img[i0 * nr + j0] + b * img[i0 * nr + j0 + 1]) +
                    a * ((1.0 - b) * img[(i0 + 1) * nr + j0] + b * img[(i0 + 1) * nr + j0 + 1]);
            }
            out[k * nz + l] = v;
        }
    return 0;
}
