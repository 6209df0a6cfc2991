/*
 * ultraray.h -- C ABI of the MI355X (gfx950) full-path ultrasound ray tracer.
 *
 * The library computes the pressure signal P(e, t) received by every element
 * e of a linear or convex transducer array over time t for a plane-wave (or
 * element-by-element) acquisition pattern, and turns these per-element
 * signals into a B-mode image (UltraRay, arXiv 2501.05828, Sec. 2.1 problem
 * statement and Sec. 2.3 signal processing).
 *
 * Conventions shared by every entry point
 *   Units     metres, seconds, m/s; impedance Z in MRayl; attenuation in
 *             dB/(cm MHz); angles in radians.
 *   Frame     x lateral, y elevation, z depth.  A linear array's face is
 *             the plane z = 0 of the scene box and faces +z; element e has
 *             its centre at x_e = (e - (E-1)/2) * pitch, y = 0, z = 0.  A
 *             convex array (ur_probe_desc.radius > 0) lies on the cylinder
 *             of that radius about the y axis through (0, 0, -radius).
 *   Layouts   channel data [n_tx][n_elements][n_samples], samples
 *             contiguous; complex data interleaved (re, im) float pairs;
 *             images [nx][nz], depth contiguous.  Sample n of the channel
 *             data stands for arrival times in [n/fs, (n+1)/fs).
 *   Memory    "_dev" pointers are device (HIP) memory owned by the caller;
 *             other pointers are host memory, read (or written) before the
 *             call returns.  The library owns the uploaded scene, its
 *             acceleration structures and all workspace.
 *   Streams   "stream" is a hipStream_t (NULL = the default stream).  Device
 *             outputs are valid once the stream has reached the end of the
 *             call's work; entry points that fill host outputs synchronise
 *             the stream before returning.
 *   Errors    Every entry point returns a ur_status (0 = success).  On a
 *             validation failure nothing is launched and no output is
 *             written; ur_last_error() returns a message describing the last
 *             failure on that context (ur_last_error(NULL): the calling
 *             thread's last failed ur_context_create).  No C++ exception
 *             crosses the ABI.
 *   Threads   A context is used by one host thread at a time.
 */
#ifndef ULTRARAY_H
#define ULTRARAY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define UR_API __attribute__((visibility("default")))

typedef enum {
    UR_OK = 0,
    UR_ERR_INVALID_ARG = -1,   /* bad pointer, size, count or value            */
    UR_ERR_CALL_ORDER = -2,    /* e.g. trace before scene upload / setup       */
    UR_ERR_OOM = -3,           /* device or host allocation failed             */
    UR_ERR_HIP = -4,           /* a HIP runtime call failed                    */
    UR_ERR_SCENE = -5,         /* inconsistent scene (materials, geometry)     */
    UR_ERR_CAPACITY = -6,      /* a fixed-capacity table or buffer is too small */
    UR_ERR_UNSUPPORTED = -7    /* feature or size outside the supported range  */
} ur_status;

typedef struct ur_context ur_context;

/* Scene (host arrays, copied by ur_scene_upload).  Every surface separates a
 * "front" material (the side its geometric normal points to) from a "back"
 * material; a sphere's front is its outside.  Triangles use the normal
 * (v1 - v0) x (v2 - v0).  The axis-aligned box absorbs every ray that leaves
 * it; its face z = box[2] must be the transducer plane z = 0 for a linear
 * array and lie at or above the ends of a convex one (checked by
 * ur_transmit_setup).  Scatterers are points with a signed re-radiation
 * amplitude. */
typedef struct {
    int64_t n_mat, n_tri, n_sph, n_pln, n_scat, top_medium;
    const double *mat;        /* [n_mat][3] Z [MRayl], alpha [dB/(cm MHz)], c [m/s]; n_mat <= 16 */
    const double *box;        /* [6] xmin, ymin, zmin (<= 0), xmax, ymax, zmax               */
    const double *tri;        /* [n_tri][9] v0, v1, v2                                         */
    const int32_t *tri_mat;   /* [n_tri][2] front, back                                        */
    const double *sph;        /* [n_sph][4] centre, radius; n_sph <= 64                        */
    const int32_t *sph_mat;   /* [n_sph][2] outside, inside                                    */
    const double *pln;        /* [n_pln][4] unit normal n and d, plane n.x = d; n_pln <= 64    */
    const int32_t *pln_mat;   /* [n_pln][2] front (n side), back                               */
    const double *scat;       /* [n_scat][4] position, amplitude                               */
    const double *rough;      /* [n_mat] GGX roughness alpha of Eq. 12 per material, 0 = smooth,
                               * at most 10; NULL: all smooth.  A boundary is as rough as the
                               * rougher of its two materials (microfacet normal drawn from D(h),
                               * Walter et al. 2007 weight factor); not supported by the adjoint */
} ur_scene_desc;

/* Transducer array (Sec. 2.3 "Ray Emission": number of lateral elements,
 * elevational extent and radius; a linear array has infinite radius, given
 * here as radius = 0).  Linear: element centres on the x axis at
 * (e - (E-1)/2) pitch, all facing +z.  Convex: centre of curvature at
 * (0, 0, -radius), element e at angle phi_e = (e - (E-1)/2) pitch / radius
 * (pitch = arc length), centre (radius sin phi_e, 0, radius cos phi_e -
 * radius), facing (sin phi_e, 0, cos phi_e); rays start on the element's arc
 * and leave about the local outward normal, the array's cylinder absorbs the
 * rays that reach it, and the receive angle of Eq. 13 is taken to the normal
 * of the element hit or sampled.  The array must span less than 180 degrees. */
typedef struct {
    int64_t n_elements;       /* 1 .. 65535                        */
    double pitch;             /* element pitch [m] (arc length on a convex array) */
    double elevation;         /* element height along y [m]        */
    double f_c;               /* centre frequency [Hz]             */
    double radius;            /* 0: linear array; > 0: convex array radius [m] */
} ur_probe_desc;

#define UR_BIN_NEAREST 0      /* a record adds to the sample whose interval holds its time   */
#define UR_BIN_LINEAR 1       /* tent split between the two samples whose centres bracket it */

/* Plane-wave acquisition and tracer limits. */
typedef struct {
    int64_t n_tx;             /* number of steered plane waves, 1 .. 65535              */
    int64_t n_samples;        /* samples per channel                                     */
    int64_t rays_per_element; /* rays emitted per element and transmit, < 2^32           */
    int64_t max_bounces;      /* interface interactions before termination (Sec. 2.3)    */
    int64_t binning;          /* UR_BIN_NEAREST or UR_BIN_LINEAR                          */
    double f_s;               /* sampling frequency [Hz]                                  */
    double c0;                /* speed of sound for steering delays and beamforming [m/s] */
    double n_cycles;          /* pulse length in cycles (Eq. 14)                          */
    double r_s;               /* scatterer capture radius [m]                             */
    double max_path;          /* maximum path length [m]                                   */
    double alpha_m, alpha_c;  /* receive main-beam and cut-off angles (Eq. 13) [rad]       */
    const double *angles;     /* [n_tx] steering angles [rad] (host)                       */
    int64_t element_choice;   /* transducer sampling (Sec. 2.3): UR_ELEMENT_UNIFORM draws the
                               * target uniformly over all E element centres (weight E);
                               * UR_ELEMENT_CONE uniformly over the K elements whose centre the
                               * capture point's acceptance cone can reach (weight K, the same
                               * expectation, lower variance)                                 */
    int64_t scheme;           /* UR_SCHEME_PLANE_WAVE: n_tx steered plane waves (angles);
                               * UR_SCHEME_SYNTHETIC: synthetic aperture, n_tx = n_elements and
                               * transmit t fires element t alone without delay (angles unused),
                               * its rays drawn as in transmit 0 with the weights of a full-array
                               * transmit; see ur_synthesize                                   */
    int64_t rough_direct_only; /* 0: at every rough boundary a secondary ray goes to an element centre
                               * drawn as for scatterers, weighted by the boundary's scattering toward
                               * it (Sec. 2.3 transducer sampling at interaction points), balanced with
                               * the direct hit that may follow (balance heuristic); 1: direct hits only */
} ur_acq_desc;

#define UR_ELEMENT_UNIFORM 0
#define UR_ELEMENT_CONE 1
#define UR_SCHEME_PLANE_WAVE 0
#define UR_SCHEME_SYNTHETIC 1

#define UR_APOD_NONE 0
#define UR_APOD_HANN 1

/* Image grid: pixel (i, j) sits at x = x0 + i (x1-x0)/(nx-1), z = z0 + j (z1-z0)/(nz-1).
 * A sector grid (sector = 1, for convex arrays) places pixel (i, j) at angle
 * phi = x0 + i (x1-x0)/(nx-1) [rad] from +z and depth r = z0 + j (z1-z0)/(nz-1)
 * below the array face along the ray from the centre of curvature:
 * (x, z) = (R + r)(sin phi, cos phi) - (0, R), R the array radius (0: about the
 * origin).  Images are stored [nx][nz]. */
typedef struct {
    int64_t nx, nz, apod;
    double x0, x1, z0, z1;
    double dynamic_range_db;  /* log compression range for the B-mode output (90 dB in Sec. 4) */
    int64_t sector;           /* 0 Cartesian, 1 sector                                        */
} ur_grid_desc;

/* Counters of one trace call (filled only when requested). */
typedef struct {
    uint64_t rays, segments, reflect, transmit, tir, scatter_events, nee_zero, nee_cast, nee_blocked,
             direct_hits, records, dropped, edge_band, term_box, term_bounce, term_time, term_path,
             media_mismatch;
    uint64_t tri_nodes, tri_tests, scat_cells, scat_tests, shadow_nodes, shadow_tri_tests;
    uint64_t term_rough;      /* rays absorbed at a rough boundary (microfacet facing away, or new
                               * direction on the wrong side of the surface) */
    uint64_t surface_events;  /* transducer-sampling draws at rough boundaries                     */
    uint64_t surface_zero;    /* ... of them with zero weight (no element in the cone, or the drawn
                               * element outside it, or a direction the boundary cannot scatter to) */
    double kernel_ms;         /* time of the whole trace stage between HIP events on the call's stream */
} ur_trace_stats;

/* One entry of an explicit-ray path log (ur_trace_rays). */
typedef struct {
    int64_t kind;             /* 0 direct-hit record, 1 scatterer record, 2 reflect, 3 transmit, 4 end,
                               * 5 rough-boundary record (transducer sampling at a rough boundary) */
    int64_t tx, elem, seg, id;
    double t, value, x, y, z;
} ur_event;

/* Explicit ray for ur_trace_rays. */
typedef struct {
    double o[3], d[3], w, t;  /* origin, unit direction, weight, start time */
    int64_t tx, elem, ray, medium;
} ur_ray;

/* Creates a context bound to HIP device `hip_device`.  *out receives the
 * handle (NULL on failure); on failure ur_last_error(NULL) names the HIP call
 * or argument that failed. */
UR_API ur_status ur_context_create(int hip_device, ur_context **out);

/* Frees the context and everything the library allocated for it.  NULL is a no-op. */
UR_API void ur_context_destroy(ur_context *ctx);

/* Message of the last failed call on ctx ("" if none); valid until the next
 * call.  With ctx = NULL: the calling thread's last failed ur_context_create
 * ("" if the last one succeeded). */
UR_API const char *ur_last_error(const ur_context *ctx);

/* Library version string. */
UR_API const char *ur_version(void);

/* Validates and uploads the scene (Sec. 4 scene: meshes with per-material
 * impedance; point scatterers and frequency-dependent attenuation extend the
 * paper's surface-only model),
 * builds the triangle and scatterer bounding-volume hierarchies on the host
 * and copies them to the device.  Replaces any previous scene.  Synchronous. */
UR_API ur_status ur_scene_upload(ur_context *ctx, const ur_scene_desc *scene);

/* Replaces parameter values of the uploaded scene without rebuilding its
 * acceleration structures (for optimisation loops): mat [n_mat][3] (Z,
 * alpha, c as in ur_scene_desc), scat_amp [n_scat] (scatterer amplitudes),
 * sph [n_sph][4] (centre, radius); each is a host array or NULL (kept).
 * Scatterer positions, meshes, planes and material indices stay fixed.  On
 * an invalid value nothing is changed.  Synchronous. */
UR_API ur_status ur_scene_update(ur_context *ctx, const double *mat, const double *scat_amp, const double *sph);

/* Transmit setup: element centres, plane-wave steering delays (Sec. 2.3 "Ray
 * Emission", Fig. 3), pulse taps (Eq. 14) and tracer limits.  Requires a
 * scene (material count is checked against it).  Synchronous. */
UR_API ur_status ur_transmit_setup(ur_context *ctx, const ur_probe_desc *probe, const ur_acq_desc *acq);

/* Sets the emission-direction proposal: pdf_dev and cdf_dev are device arrays
 * [n_tx][n_elements][1024] over the 32x32 equal-area direction cells (pdf: the
 * probability of each cell, summing to 1; cdf: its inclusive prefix sum).
 * NULL, NULL restores uniform emission.  The arrays are read during later
 * traces and must stay alive until the proposal is replaced.  (Eq. 4's p_t.) */
UR_API ur_status ur_set_proposal(ur_context *ctx, const float *pdf_dev, const float *cdf_dev);

/* Traces every ray of every transmit (Sec. 2.2 Eq. 4 estimator with the
 * Sec. 2.3 emission, traversal and transducer sampling) and writes the
 * channel data ch_raw_dev [n_tx][n_elements][n_samples] (zero-filled first).
 * If ch_rf_dev is not NULL, also writes the pulse-shaped analytic channel
 * data [n_tx][n_elements][n_samples][2] (as ur_pulse).  Only rays with
 * index r = ray_offset + k * ray_stride are traced (stride 1, offset 0 traces
 * all; the estimator's normalisation is unchanged).  If stats is not NULL it
 * is filled (the counting kernel variant is used, which also counts
 * traversal work).  The call waits for its work on the stream to finish and
 * fails with UR_ERR_CAPACITY if a primary-ray segment found no slot in the
 * segment queue (sized for the worst case, so this signals a library
 * fault rather than a size limit). */
UR_API ur_status ur_trace(ur_context *ctx, uint64_t seed, int64_t ray_stride, int64_t ray_offset,
                          float *ch_raw_dev, float *ch_rf_dev, ur_trace_stats *stats, void *stream);

/* Work-size limits of later ur_trace calls.  A trace is cut into equal
 * launch ranges of at most min(rays_per_launch, 2^29) rays.  With scatterers
 * present, each launch queues its primary-ray segments for the scatterer walk
 * in library-owned device memory (96 bytes a segment, plus a chunk of 256 per
 * resident wavefront).  If the worst case of a range (max_bounces + 1
 * segments a ray) fits the segment budget (ur_set_segment_queue), the queue
 * holds that worst case; otherwise it holds the budget, and the launch admits
 * rays only while the worst case of the rays it has not finished still fits:
 * it ends early and the next launch goes on from there.  Up to
 * nee_queue_capacity transducer-sampling candidates (80 bytes each,
 * library-owned) are queued per launch before their secondary rays are cast;
 * a launch that produces more is traced again with the secondary rays cast
 * inline.  Results never depend on these limits.
 * Defaults: 2^30 rays; candidates: until this call sets it, the rays of one
 * range, but at least 2^25 and at most 2^27. */
UR_API ur_status ur_set_limits(ur_context *ctx, int64_t rays_per_launch, int64_t nee_queue_capacity);

/* Segment budget of later ur_trace calls: the segment queue holds at most
 * `segments` segments (96 bytes each) beyond its per-wavefront chunks; 0
 * (default) allows 1/8 of the device memory.  A budget below 1024 x
 * (max_bounces + 1) segments makes launches as short as the worst case needs
 * (but not below 2^16 rays).  segments < 0: UR_ERR_INVALID_ARG. */
UR_API ur_status ur_set_segment_queue(ur_context *ctx, int64_t segments);

/* Binning mode of later ur_trace calls (Sec. 2.3, each echo binned by its
 * arrival time into the channel data).  deterministic = 0 (default): every
 * record is added with device-wide float atomics, so the low bits of the
 * channel data depend on the order of arrival.  deterministic = 1: records
 * are staged (up to `capacity`, 24 bytes each, library-owned device memory)
 * and binned after the trace with exact 64-bit integer arithmetic at one
 * scale per call (below 1e-13 of the largest record for 1e5 records), so
 * the channel data are the same bits on every call with the same inputs.
 * A trace that offers more than `capacity` records returns
 * UR_ERR_CAPACITY.  ur_trace_rays always uses atomics. */
UR_API ur_status ur_set_binning(ur_context *ctx, int32_t deterministic, int64_t capacity);

/* Steered plane waves synthesised from synthetic-aperture channel data
 * (any acquisition scheme from one set of traces, Sec. 1; delays of
 * Sec. 2.3 / Fig. 3):
 * out[k][er][s] = sum over emitting elements e of ch_sa[e][er] at sample
 * s - tau_k(e) fs, linearly interpolated (zero outside [0, n_samples)), with
 * tau_k(e) = (x_e - x_ref) sin(theta_k) / c0 the plane-wave delays of the
 * current setup's probe.  ch_sa_dev [E][E][n_samples] FP32 (device, as traced
 * with UR_SCHEME_SYNTHETIC), angles [n_ang] (host), out_dev [n_ang][E][n_samples]
 * FP32 (device, overwritten), n_ang <= 128.  Accumulates in FP64.  Async on `stream`. */
UR_API ur_status ur_synthesize(ur_context *ctx, const float *ch_sa_dev, const double *angles, int64_t n_ang,
                               float *out_dev, void *stream);

/* Scan conversion for display of a sector image (Sec. 4's convex-probe
 * images): img_dev [sector->nx][sector->nz] (device, FP32, e.g. a B-mode
 * image from ur_beamform on that sector grid) resampled onto the Cartesian
 * grid `cart` into out_dev [cart->nx][cart->nz] (device).  Each output pixel
 * takes its angle and depth about the array's centre of curvature and
 * interpolates bilinearly between the four surrounding sector samples; pixels
 * outside the sector get `fill`.  Needs sector->sector = 1 with at least 2 x 2
 * samples and increasing x and z ranges, and cart->sector = 0.  Asynchronous
 * on `stream`. */
UR_API ur_status ur_scan_convert(ur_context *ctx, const ur_grid_desc *sector, const float *img_dev,
                                 const ur_grid_desc *cart, float fill, float *out_dev, void *stream);

/* Pulse shaping (Eq. 14): ch_rf = ch_raw convolved with the analytic pulse
 * g(t) (sin(2 pi f_c t) - i cos(2 pi f_c t)), Gaussian g with full width at
 * half maximum n_cycles / f_c, taps |m| <= ceil(3 sigma f_s), zero outside the
 * record.  ch_raw_dev [n_tx][E][n_samples] FP32, ch_rf_dev
 * [n_tx][E][n_samples][2] FP32 (overwritten); layouts as in ur_trace.
 * Asynchronous on `stream`. */
UR_API ur_status ur_pulse(ur_context *ctx, const float *ch_raw_dev, float *ch_rf_dev, void *stream);

/* Plane-wave delay-and-sum with coherent compounding over transmits,
 * followed by demodulation (envelope) and log compression (Sec. 2.3 "Phase
 * Calculation and Signal Processing").  ch_rf_dev as written by ur_pulse.
 * Outputs (any may be NULL, not all): iq_dev [nx][nz][2], env_dev [nx][nz],
 * bmode_dev [nx][nz] in dB within [-dynamic_range_db, 0]. */
UR_API ur_status ur_beamform(ur_context *ctx, const ur_grid_desc *grid, const float *ch_rf_dev, float *iq_dev,
                             float *env_dev, float *bmode_dev, void *stream);

/* ur_beamform for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, kernels and results, but no device allocation, no
 * hipFree and no allocating library routine in the call.  Its scratch (the
 * envelope when bmode_dev is given without env_dev, and the envelope's
 * maximum) lives in a static device array of 16 MiB + 256 bytes that every
 * device loading the library holds until the process ends.  A B-mode image
 * without env_dev is limited to nx * nz <= 4,194,304 pixels (UR_ERR_CAPACITY
 * beyond, nothing launched).  Every call on one device shares that array,
 * which keeps the last call's contents: calls that overlap on one device
 * (other streams, other contexts, other threads) race and must be ordered by
 * the caller. */
UR_API ur_status ur_beamform_static(ur_context *ctx, const ur_grid_desc *grid, const float *ch_rf_dev,
                                    float *iq_dev, float *env_dev, float *bmode_dev, void *stream);

/* Device time in milliseconds, between HIP events recorded on the call's
 * stream immediately around each kernel launch: the trace kernels of the
 * last ur_trace call (extend + scatter, summed over launches; secondary
 * rays and pulse shaping excluded) and the delay-and-sum kernel of the last
 * ur_beamform call; -1 where no such call was made.  Waits for those
 * events. */
UR_API ur_status ur_last_kernel_ms(ur_context *ctx, double *trace_ms, double *das_ms);

/* The trace kernels of the last ur_trace call separately (milliseconds,
 * summed over launches): extend (emission, closest hits, interface
 * events, direct hits), scatter (scatterer captures) and sampling (secondary
 * rays of the captures); -1 if no call was made.  launches receives the
 * number of launches (each kernel ran once per launch).  Any pointer may
 * be NULL. */
UR_API ur_status ur_last_trace_kernels_ms(ur_context *ctx, double *extend_ms, double *scatter_ms, double *sampling_ms,
                                          int64_t *launches);

/* Test and debugging aid: traces the given host rays one by one with the
 * same device code path as ur_trace and returns their path logs (host
 * events, at most cap; *n_events receives the total count).  If ch_raw_dev is
 * not NULL the records are also binned into it (zero-filled first).
 * Synchronous. */
UR_API ur_status ur_trace_rays(ur_context *ctx, uint64_t seed, const ur_ray *rays, int64_t n_rays,
                               ur_event *events, int64_t cap, int64_t *n_events, float *ch_raw_dev,
                               void *stream);

/* ---------------------------------------------------------------------------
 * Learned emission proposal (Eq. 4's direction pdf p_t, learned per
 * (transmit, element) row).  The network maps the row's normalised element
 * position and steering angle plus a 32-dimensional random Fourier encoding
 * [sin(2 pi B v), cos(2 pi B v)], B given as 16x2 floats, through three ReLU
 * layers of width 64 to a softmax over the 32x32 equal-area direction cells
 * (77,120 FP32 parameters in the order W1[34][64], b1[64], W2[64][64], b2,
 * W3[64][64], b3, W4[64][1024], b4[1024]).  Matrix products use BF16 operands
 * with FP32 accumulation.  Rows are r = tx * n_elements + e for the current
 * transmit setup; a new setup requires ur_mlp_init again.
 * ------------------------------------------------------------------------- */

/* Loads parameters (host, 77,120 floats) and the Fourier matrix (host,
 * 16x2 floats) and resets the Adam state.  Synchronous. */
UR_API ur_status ur_mlp_init(ur_context *ctx, const float *params, const float *rff);

/* Copies the current parameters to host memory (77,120 floats).  Synchronous. */
UR_API ur_status ur_mlp_get_params(ur_context *ctx, float *params);

/* Training state, for checkpoints: state (host, 3 x 77,120 floats) receives
 * the parameters, Adam's first moments and its second moments, in that
 * order, and *step the number of Adam steps taken (the bias corrections of
 * the next step depend on it).  Synchronous. */
UR_API ur_status ur_mlp_get_state(ur_context *ctx, float *state, int64_t *step);

/* Restores a state in the layout of ur_mlp_get_state (finite values, second
 * moments >= 0, step >= 0) after ur_mlp_init for the same transmit setup; the
 * Fourier matrix given to ur_mlp_init is kept.  UR_ERR_INVALID_ARG for a bad
 * state.  Synchronous. */
UR_API ur_status ur_mlp_set_state(ur_context *ctx, const float *state, int64_t step);

/* q_dev [rows][1024]: the network's direction distribution for every row. */
UR_API ur_status ur_mlp_forward(ur_context *ctx, float *q_dev, void *stream);

/* Weighted cross-entropy L = -sum H log q / sum H for the target histogram
 * hist_dev [rows][1024] (summed contribution magnitudes per emission cell),
 * its gradient grad_dev [77,120] and the loss loss_dev [1] (nullable). */
UR_API ur_status ur_mlp_loss_grad(ur_context *ctx, const float *hist_dev, float *grad_dev, float *loss_dev,
                                  void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the loss above. */
UR_API ur_status ur_mlp_train_step(ur_context *ctx, const float *hist_dev, float lr, float *loss_dev, void *stream);

/* Proposal tables for ur_set_proposal: pdf = (1 - eps) q + eps / 1024 (the
 * uniform component keeps every direction reachable, so the 1/pdf-weighted
 * estimator stays unbiased) and its inclusive prefix sum, [rows][1024]. */
UR_API ur_status ur_mlp_proposal_tables(ur_context *ctx, float eps, float *pdf_dev, float *cdf_dev, void *stream);

/* Recording of contributions during later ur_trace calls: every binned
 * contribution c appends {bin = (tx * n_elements + emitting element) * 1024 +
 * emission cell (uint32), |c| (float)} to rec_dev (8-byte entries, capacity
 * cap) and increments *count_dev (device, unsigned 64-bit; counts also the
 * records that did not fit).  rec_dev = NULL stops recording. */
UR_API ur_status ur_set_record(ur_context *ctx, void *rec_dev, int64_t cap, unsigned long long *count_dev);

/* Path-cost histogram for a cost-aware proposal: while cost_dev (device,
 * float [rows][1024], zeroed by the caller) is set, every primary ray of
 * later ur_trace calls adds its cost to the cell it was emitted in, with
 * cost = four-wide node visits + 2 per segment + 1.5 per scatterer-grid
 * cell edge of path length (a model of the time the ray takes in the
 * extend and scatter kernels).  NULL stops it. */
UR_API ur_status ur_set_cost_histogram(ur_context *ctx, float *cost_dev);

/* Cost-aware training target: replaces the |c| of every record in
 * rec_dev[0, n_rec) by c^2 / sqrt(S2 x mean cost) of its bin, where S2 is
 * the sum of c^2 over the bin's records and mean cost = cost_dev[bin] x 1024
 * / rays_per_row (uniform emission gives each cell rays_per_row / 1024 rays
 * in expectation).  The minibatch histograms of ur_record_histogram then
 * have expectation proportional to sqrt(S2 / mean cost) per cell, the
 * emission density that minimises variance x time for the recorded paths
 * (importance sampling with per-sample cost).  Async. */
UR_API ur_status ur_record_reweight(ur_context *ctx, void *rec_dev, int64_t n_rec, const float *cost_dev,
                                    double rays_per_row, void *stream);

/* Minibatch target: hist_dev [rows][1024] is zeroed, then `batch` records
 * drawn uniformly with replacement from rec_dev[0, n_rec) (Philox with key
 * `seed`, counter (draw, step)) add their value (|c|, or the weight set by
 * ur_record_reweight) to their bins. */
UR_API ur_status ur_record_histogram(ur_context *ctx, const void *rec_dev, int64_t n_rec, int64_t batch,
                                     uint64_t seed, uint32_t step, float *hist_dev, void *stream);

/* ---------------------------------------------------------------- adjoint
 * Gradients of a scalar loss L of the simulated data, for gradient-based
 * inversion (the differentiability the method is built for, Sec. 1 and
 * Sec. 3).  The signal chain is linear up to the envelope, and its adjoints
 * are the transposed operators; the trace adjoint regenerates every path from
 * its counters (path replay) and differentiates the contributions along it.
 *
 * Gradients are interior (frozen-decision) derivatives: the discontinuities
 * of the estimator in geometry (a path starting or ceasing to capture a
 * scatterer, to hit the aperture or a triangle) contribute no boundary term.
 */

/* Adjoint of ur_pulse: g_raw[k] = sum_m Re h[m] Re g_rf[k + m] + Im h[m] Im
 * g_rf[k + m] for every channel (the transpose of the Eq. 14 convolution).
 * g_rf_dev: complex float [n_tx][n_elements][n_samples] (interleaved re, im),
 * g_raw_dev: float [n_tx][n_elements][n_samples], overwritten.  Async. */
UR_API ur_status ur_pulse_adjoint(ur_context *ctx, const float *g_rf_dev, float *g_raw_dev, void *stream);

/* Adjoint of ur_beamform (delay-and-sum and envelope).  Give exactly one of
 * g_env_dev (float [nx][nz], dL/d envelope; needs iq_dev, the complex IQ
 * image [nx][nz] of the forward call) and g_iq_dev (complex float [nx][nz],
 * dL/d IQ).  g_rf_dev (complex float [n_tx][n_elements][n_samples]) is
 * overwritten with dL/d ch_rf; the grid and apodisation must be those of the
 * forward call.  Pixels with |IQ| = 0 pass no envelope gradient.  The
 * transpose scatters with float atomics, so its summation order (and the
 * last bits of g_rf) vary from call to call.  Async. */
UR_API ur_status ur_beamform_adjoint(ur_context *ctx, const ur_grid_desc *grid, const float *iq_dev,
                                     const float *g_env_dev, const float *g_iq_dev, float *g_rf_dev, void *stream);

/* Gradient outputs of ur_trace_adjoint (device pointers; NULL = not wanted).
 *   amp        float  [n_scat]      dL/d scatterer amplitude (scene order)
 *   alpha      double [n_mat]       dL/d attenuation alpha [per dB/(cm MHz)]
 *                                   (at most 8 materials)
 *   Z          double [n_mat]       dL/d acoustic impedance [per MRayl]
 *   sph_center double [n_sph][3]    dL/d sphere centre coordinates [per m]
 *   value      double [1]           J = sum of g(t) c over the contributions,
 *                                   accumulated in FP64 (the functional whose
 *                                   derivatives the other outputs are)
 * frozen_choice = 0: the reflect-or-transmit choice of Eqs. 7-11 keeps its
 * probability attached to the weight (R / value(R), (1 - R) / value(1 - R)),
 * which adds the derivative of the choice probability (the gradient of the
 * expectation over the choice); 1: the choice counts as fixed, giving the
 * derivative of the fixed-seed estimator between decision changes.
 * record_paths: with Z or sph_center requested, the paths go in ranges of
 * this many (0: as many as fit in 1/32 of the device memory); the value pass over
 * a range keeps each segment's closest primitive (16 bytes a segment) and up
 * to 8 contributing captures a path (8 bytes each), which the tangent passes
 * over the range replay.  The context keeps these buffers (grown, never
 * shrunk) until it is destroyed. */
typedef struct ur_grad_desc {
    float *amp;
    double *alpha;
    double *Z;
    double *sph_center;
    double *value;          /* [1] or NULL: J = sum g(t) c over the replayed contributions (FP64) */
    int32_t frozen_choice;
    int64_t record_paths;   /* >= 0; 0 = automatic */
} ur_grad_desc;

/* Path-replay adjoint of ur_trace for the same (seed, ray_stride,
 * ray_offset): with g_raw_dev = dL/d ch_raw (float [n_tx][n_elements]
 * [n_samples]), accumulates into each requested output of `grads` (each is
 * cleared first) the derivative of L through every binned contribution c at
 * arrival time t: g(t) dc + c g'(t) dt, where g' (the slope of g between
 * sample centres) is non-zero only with linear binning.  Amplitude and
 * attenuation gradients come from one replay; the impedances and sphere
 * coordinates come from forward-mode (dual number) replays, two parameter
 * directions per replay.  The same
 * proposal tables as the forward call must be set.  Rough boundaries
 * (Eq. 12) are supported when their echoes are received by direct hits only
 * (ur_acq_desc.rough_direct_only = 1): the GGX microfacet normal follows the
 * dual macro normal for the same random numbers and its weight factor is
 * differentiated; with transducer sampling at rough boundaries the call
 * returns UR_ERR_UNSUPPORTED.  Every decision (closest primitive, capture,
 * element drawn) is taken on values, so it is the same in every pass; the
 * tangent passes replay the value pass's record of them (record_paths).
 * Errors: UR_ERR_INVALID_ARG (no output, record_paths < 0, stride/offset),
 * UR_ERR_OOM (record buffers).  Async on `stream`. */
UR_API ur_status ur_trace_adjoint(ur_context *ctx, uint64_t seed, int64_t ray_stride, int64_t ray_offset,
                                  const float *g_raw_dev, const ur_grad_desc *grads, void *stream);

/* Visibility-boundary terms of the direct hits (the paper's differentiable
 * framework, Sec. 1 and Sec. 5), which ur_trace_adjoint's interior
 * derivative leaves out: a direct hit is binned into the element whose face
 * holds its landing point (Sec. 2.3), so its contribution jumps where that
 * point crosses an element edge, an end of the aperture or an elevation
 * edge, and impedances and sphere centres move the crossings.  The jumps are
 * integrated exactly along the emission origin's lateral coordinate u0 on
 * the element face (Eq. 4) of every path family of the same (seed,
 * ray_stride, ray_offset) paths: n_scan + 1 evenly spaced origins per family,
 * intervals whose ends follow different sequences of primitives and choices
 * halved, every crossing located by Newton steps and weighted by the Leibniz
 * rule, [F] dx/dtheta / |dx/du0|.  Accumulates (each output cleared first)
 * corr_z_dev (double [n_mat]) and corr_sph_dev (double [n_sph][3]), each
 * nullable; adding them to ur_trace_adjoint's Z and sph_center with the
 * choice attached (frozen_choice = 0) estimates the derivative of the
 * expected data when the direct hits carry the only discontinuities.
 * g_raw_dev as for ur_trace_adjoint.  Linear and convex arrays (on a convex
 * one the origin moves along the element's arc, the landing coordinate is
 * the arc angle and every element receives against its own normal);
 * plane-wave transmits, uniform emission, smooth boundaries, at most 32
 * impedances and sphere coordinates (else UR_ERR_UNSUPPORTED).  A family costs n_scan + 1
 * replays, about 48 more for every change of sequence along the origin
 * (meshes: a new triangle at every facet edge) and a few per crossing and
 * parameter.  Async on `stream`. */
UR_API ur_status ur_trace_grad_edges(ur_context *ctx, uint64_t seed, int64_t ray_stride, int64_t ray_offset,
                                     const float *g_raw_dev, int32_t n_scan, double *corr_z_dev, double *corr_sph_dev,
                                     void *stream);

/* Philox4x32-10 evaluated on the device for n counters (host arrays
 * ctr [n][4], out [n][4]) under key (key0, key1); for checking that the
 * device stream equals the published generator.  Synchronous. */
UR_API ur_status ur_philox(ur_context *ctx, const uint32_t *ctr, int64_t n, uint32_t key0, uint32_t key1,
                           uint32_t *out);

#ifdef __cplusplus
}
#endif
#endif
