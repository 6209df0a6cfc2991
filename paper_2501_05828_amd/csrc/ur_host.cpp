// Host runtime behind the C ABI (include/ultraray.h): context, validation,
// scene upload with BVH construction, transmit setup, kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ultraray.h"
#include "bvh.h"
#include "scatter_grid.h"
#include "ur_internal.h"

using namespace ur;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

// Scratch of ur_beamform_static, the allocation-free B-mode entry point: a
// 256-byte header whose first word is the running maximum of the envelope
// (FP32 bits), then an envelope buffer of at most kStaticPixels pixels.  HIP
// gives every device that loads the library its own copy, held until the
// process ends.  Host code never uses the symbol itself as an address: it
// takes each device's address once (static_scratch) and passes that.
// Share of the device memory the adjoint's record buffers may take (paths of
// one range times their decisions): longer ranges have fewer kernel tails (on
// the large scene 128 ranges of 512 MiB took 4.88 s, 8 ranges 4.29 s).
constexpr size_t kAdjRecShare = 32;

constexpr int64_t kStaticHeader = 64;                  // floats (256 bytes)
constexpr int64_t kStaticPixels = int64_t(1) << 22;    // 2048 x 2048 pixels, 16 MiB
static __device__ __align__(256) float scratch[kStaticHeader + kStaticPixels];

// Message of the calling thread's last failed ur_context_create (there is
// no context to hold it).
thread_local std::string t_create_err;

}  // namespace

struct ur_context {
    int device = 0;
    std::string err;
    // scene (host copies of what later calls need)
    bool has_scene = false;
    std::vector<double> mat;               // [n_mat][3]
    std::vector<double> rough;             // [n_mat] GGX roughness (0 = smooth)
    double box[6] = {0};
    int top_medium = 0;
    int64_t n_tri = 0, n_sph = 0, n_pln = 0, n_scat = 0;
    int n_tnodes = 0, n_tnodes4 = 0;
    float tree_lo[3] = {0, 0, 0}, tree_hi[3] = {0, 0, 0};   // root box of the binary tree
    std::vector<double> scat;              // [n_scat][4], kept for the r_s-dependent scatterer grid
    std::vector<double> sph;               // [n_sph][4]
    std::vector<int32_t> item_order;       // scatterer index of each grid item
    GridInfo grid{};
    DevBuf d_mat, d_sph, d_sph_mat, d_pln, d_pln_mat, d_tri, d_tri_n, d_tri_mat, d_tri_id, d_tnodes, d_tnodes4, d_cell_start, d_items,
        d_items_f, d_item_id, d_work;
    // setup
    bool has_setup = false;
    ur_probe_desc probe{};
    ur_acq_desc acq{};
    std::vector<double> angles;
    std::vector<double> xe_h, ze_h;        // element centres x, z (host copies)
    int K = 0;
    DevBuf d_xe, d_tau, d_taps, d_apod, d_txc, d_stats, d_stats2, d_maxbits, d_env, d_rays, d_events, d_evcount, d_ctr,
        d_nee, d_counters, d_segq, d_segc;
    int64_t rays_per_launch = int64_t(1) << 30;
    // proposal network (rows = transmits x elements of the current setup)
    bool mlp_ready = false;
    int mlp_rows = 0, mlp_step = 0;
    DevBuf d_giq;                          // adjoint of IQ inside ur_beamform_adjoint
    DevBuf d_adj_seg, d_adj_cap, d_adj_ncap;   // decisions of the adjoint's value pass over a range of paths
    DevBuf d_adj_next;                     // work counter of the adjoint's persistent replay
    DevBuf d_det, d_det_ctr, d_det_bins;   // deterministic binning: staged records, counters, integer bins
    bool det_mode = false;                 // bin by staged records instead of float atomics
    int64_t det_cap = 0;
    DevBuf d_elem, d_ze;                   // convex arrays: element centre / normal table, centre depths
    DevBuf d_theta, d_m, d_v, d_grad, d_rff, d_X, d_H1, d_H2, d_H3, d_Z, d_dZ, d_dH3, d_dH2, d_dH1, d_angles, d_scal;
    // contribution recording
    RecordEntry *rec = nullptr;
    float *cost = nullptr;                 // per-cell path-cost histogram (optional)
    DevBuf d_s2;
    unsigned long long *rec_count = nullptr;
    int64_t rec_cap = 0;
    std::vector<hipEvent_t> tev;           // [4 * launches]: before extend, after extend, after scatter, after sampling
    int n_tev = 0;
    int64_t nee_cap = int64_t(1) << 25;      // 80 B each: 2.7 GB (the cone choice casts nearly every capture)
    bool nee_auto = true;                    // capacity not set by the caller: at least one per ray of a range
    int64_t seg_budget = 0;                  // segments the segment queue may hold (0: 1/8 of device memory)
    const float *pdf = nullptr, *cdf = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool trace_timed = false, das_timed = false;
    float *scratch = nullptr;              // this device's copy of the static B-mode scratch

    ur_status fail(ur_status code, const char *fmt, ...) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }
    ur_status hip_fail(hipError_t e, const char *what) {
        return fail(UR_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    }
};

namespace {

#define HIP_TRY(ctx, call)                                 \
    do {                                                   \
        hipError_t _e = (call);                            \
        if (_e != hipSuccess) return (ctx)->hip_fail(_e, #call); \
    } while (0)

ur_status alloc(ur_context *c, DevBuf &b, size_t bytes) {
    if (b.bytes >= bytes && b.p) return UR_OK;
    b.release();
    if (bytes == 0) return UR_OK;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        return c->fail(UR_ERR_OOM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    b.bytes = bytes;
    return UR_OK;
}

template <class T>
ur_status upload(ur_context *c, DevBuf &b, const std::vector<T> &v) {
    ur_status s = alloc(c, b, v.size() * sizeof(T));
    if (s) return s;
    if (!v.empty()) HIP_TRY(c, hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return UR_OK;
}

bool finite_all(const double *p, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

ur_status set_device(ur_context *c) {
    HIP_TRY(c, hipSetDevice(c->device));
    return UR_OK;
}

// Material constants at the probe's centre frequency.
ur_status upload_materials(ur_context *c) {
    const int64_t nm = (int64_t)c->mat.size() / 3;
    std::vector<Material> m(nm);
    const double fmhz = c->has_setup ? c->probe.f_c * 1e-6 : 0.0;
    for (int64_t i = 0; i < nm; ++i) {
        m[i].Z = c->mat[3 * i];
        m[i].ka = c->mat[3 * i + 1] * fmhz * 100.0 * std::log(10.0) / 20.0;   // dB/(cm MHz) -> Np/m
        m[i].inv_c = 1.0 / c->mat[3 * i + 2];
        m[i].rough = i < (int64_t)c->rough.size() ? c->rough[i] : 0.0;
    }
    return upload(c, c->d_mat, m);
}

template <class F>
ur_status guarded(ur_context *c, F &&f) {
    if (!c) return UR_ERR_INVALID_ARG;
    try {
        ur_status s = set_device(c);
        if (s) return s;
        return f();
    } catch (const std::bad_alloc &) {
        return c->fail(UR_ERR_OOM, "host allocation failed");
    } catch (...) {
        return c->fail(UR_ERR_INVALID_ARG, "unexpected host exception");
    }
}

ur_status fill_params(ur_context *c, TraceParams &P, uint64_t seed) {
    const ur_acq_desc &a = c->acq;
    const ur_probe_desc &pr = c->probe;
    std::memset(&P, 0, sizeof(P));
    P.E = (int)pr.n_elements;
    P.T = (int)a.n_tx;
    P.S = (int)a.n_samples;
    P.binning = (int)a.binning;
    P.n_el = (uint32_t)a.rays_per_element;
    P.B = (int)a.max_bounces;
    P.proposal = c->cdf != nullptr;
    P.key0 = (uint32_t)seed;
    P.key1 = (uint32_t)(seed >> 32);
    P.pitch = pr.pitch;
    P.elev = pr.elevation;
    P.fs = a.f_s;
    P.t_max = (double)a.n_samples / a.f_s;
    P.max_path = a.max_path;
    P.alpha_m = a.alpha_m;
    P.alpha_c = a.alpha_c;
    P.cos_alpha_c = std::cos(a.alpha_c);
    // the cone-restricted choice needs alpha_c < 90 degrees; above that every
    // element can receive and the uniform choice is the same thing
    P.elem_choice = a.element_choice == UR_ELEMENT_CONE && a.alpha_c < 0.5 * M_PI ? UR_ELEMENT_CONE
                                                                                   : UR_ELEMENT_UNIFORM;
    P.tan_alpha_c = std::tan(a.alpha_c);
    P.sin_alpha_c = std::sin(a.alpha_c);
    P.sa = a.scheme == UR_SCHEME_SYNTHETIC;
    P.convex = pr.radius > 0.0;
    P.rough_nee = a.rough_direct_only == 0;
    P.radius = pr.radius;
    P.dphi = P.convex ? pr.pitch / pr.radius : 0.0;
    P.half_arc = 0.5 * (double)pr.n_elements * P.dphi;
    P.elem = (const double4 *)c->d_elem.p;
    P.r_s2 = a.r_s * a.r_s;
    P.n_per_tx = (double)pr.n_elements * (double)a.rays_per_element;
    P.half_ap = 0.5 * (double)pr.n_elements * pr.pitch;
    P.area_e = pr.pitch * pr.elevation;
    P.xe = (const double *)c->d_xe.p;
    P.tau = (const double *)c->d_tau.p;
    P.pdf = c->pdf;
    P.cdf = c->cdf;
    P.n_mat = (int)(c->mat.size() / 3);
    P.n_sph = (int)c->n_sph;
    P.n_pln = (int)c->n_pln;
    P.top_medium = c->top_medium;
    P.id_sph0 = c->n_tri;
    P.id_pln0 = c->n_tri + c->n_sph;
    P.id_box = c->n_tri + c->n_sph + c->n_pln;
    for (int i = 0; i < 6; ++i) P.box[i] = c->box[i];
    P.mat = (const Material *)c->d_mat.p;
    P.sph = (const double *)c->d_sph.p;
    P.sph_mat = (const int *)c->d_sph_mat.p;
    P.pln = (const double *)c->d_pln.p;
    P.pln_mat = (const int *)c->d_pln_mat.p;
    P.tri = (const double *)c->d_tri.p;
    P.tri_n = (const double4 *)c->d_tri_n.p;
    P.tri_mat = (const int *)c->d_tri_mat.p;
    P.tri_id = (const int *)c->d_tri_id.p;
    P.tnodes = (const BvhNode *)c->d_tnodes.p;
    P.tnodes4 = (const Bvh4NodeQ *)c->d_tnodes4.p;
    P.n_tnodes4 = c->n_tnodes4;
    P.n_tri = (int)c->n_tri;
    P.n_tnodes = c->n_tnodes;
    for (int k = 0; k < 3; ++k) {
        P.tree_lo_f[k] = c->tree_lo[k];
        P.tree_hi_f[k] = c->tree_hi[k];
    }
    P.grid = c->grid;
    for (int k = 0; k < 3; ++k) {
        const double lo = c->grid.lo[k] - 1e-5, hi = c->grid.lo[k] + (double)c->grid.n[k] * c->grid.h + 1e-5;
        float fl = (float)lo, fh = (float)hi;
        if ((double)fl > lo) fl = std::nextafter(fl, -INFINITY);
        if ((double)fh < hi) fh = std::nextafter(fh, INFINITY);
        P.grid_lo_f[k] = fl;
        P.grid_hi_f[k] = fh;
    }
    P.grid_wa_f = std::nextafter((float)(c->grid.wy_a + 5e-5), INFINITY);
    P.grid_wb_f = c->grid.wy_b < 0.0 ? -1.0f : std::nextafter((float)(c->grid.wy_b * (1.0 + 1e-6)), INFINITY);
    P.cell_start = (const int *)c->d_cell_start.p;
    P.items = (const double4 *)c->d_items.p;
    P.items_f = (const float4 *)c->d_items_f.p;
    {
        double ext = 0.0;
        for (int i = 0; i < 6; ++i) ext = std::max(ext, std::fabs(c->box[i]));
        const double m = 1e-6 + 4e-6 * ext, r = std::sqrt(P.r_s2) + m;
        P.pre_m = (float)m;
        P.pre_r2 = (float)(r * r * (1.0 + 1e-5));
    }
    P.item_id = (const int *)c->d_item_id.p;
    P.n_scat = c->item_order.empty() ? 0 : (int)c->n_scat;   // no registered scatterer: no captures
    P.any_rough = 0;
    for (double r : c->rough) P.any_rough |= r > 0.0;
    P.work_next = (unsigned long long *)c->d_work.p;
    P.cost = c->cost;
    return UR_OK;
}

__global__ void k_zero_f32(float *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

__global__ void k_zero_u64(unsigned long long *p, int n) {
    const int i = threadIdx.x;
    if (i < n) p[i] = 0ull;
}

hipError_t zero_f32(float *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace

extern "C" {

UR_API const char *ur_version(void) { return "ultraray-mi355x 0.1 (gfx950)"; }

static ur_status create_fail(ur_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    t_create_err = buf;
    return code;
}

// Each device's address of the static scratch, taken once with that device
// current (kMaxDevices devices at most).
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static float *g_scratch[kMaxDevices] = {};

static hipError_t static_scratch(int device, float **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[device] = (float *)p;
    }
    *out = g_scratch[device];
    return hipSuccess;
}

UR_API ur_status ur_context_create(int hip_device, ur_context **out) {
    if (!out) return create_fail(UR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return create_fail(UR_ERR_HIP, "hipGetDeviceCount: %s", hipGetErrorString(e));
    if (n <= 0) return create_fail(UR_ERR_HIP, "hipGetDeviceCount: no HIP device");
    if (hip_device < 0 || hip_device >= n || hip_device >= kMaxDevices)
        return create_fail(UR_ERR_INVALID_ARG, "hip_device %d out of range (%d devices)", hip_device, n);
    ur_context *c = new (std::nothrow) ur_context();
    if (!c) return create_fail(UR_ERR_OOM, "host allocation failed");
    c->device = hip_device;
    if ((e = hipSetDevice(hip_device)) != hipSuccess) {
        delete c;
        return create_fail(UR_ERR_HIP, "hipSetDevice(%d): %s", hip_device, hipGetErrorString(e));
    }
    for (auto &ev : c->ev) {
        if ((e = hipEventCreate(&ev)) != hipSuccess) {
            ur_context_destroy(c);
            return create_fail(UR_ERR_HIP, "hipEventCreate: %s", hipGetErrorString(e));
        }
    }
    if ((e = static_scratch(hip_device, &c->scratch)) != hipSuccess) {
        ur_context_destroy(c);
        return create_fail(UR_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    }
    t_create_err.clear();
    *out = c;
    return UR_OK;
}

UR_API void ur_context_destroy(ur_context *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (DevBuf *b : {&c->d_mat, &c->d_sph, &c->d_sph_mat, &c->d_pln, &c->d_pln_mat, &c->d_tri, &c->d_tri_n, &c->d_tri_mat,
                      &c->d_tri_id, &c->d_tnodes, &c->d_tnodes4, &c->d_cell_start, &c->d_items, &c->d_items_f, &c->d_s2, &c->d_item_id, &c->d_work, &c->d_xe, &c->d_tau,
                      &c->d_taps, &c->d_apod, &c->d_txc, &c->d_stats, &c->d_stats2, &c->d_maxbits, &c->d_env,
                      &c->d_rays, &c->d_events, &c->d_evcount, &c->d_ctr, &c->d_nee, &c->d_counters, &c->d_theta,
                      &c->d_m, &c->d_v, &c->d_grad, &c->d_rff, &c->d_X, &c->d_H1, &c->d_H2, &c->d_H3, &c->d_Z,
                      &c->d_dZ, &c->d_dH3, &c->d_dH2, &c->d_dH1, &c->d_angles, &c->d_scal, &c->d_segq, &c->d_segc,
                      &c->d_giq, &c->d_elem, &c->d_ze, &c->d_adj_seg, &c->d_adj_cap, &c->d_adj_ncap, &c->d_adj_next, &c->d_det, &c->d_det_ctr, &c->d_det_bins})
        b->release();
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : c->tev)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

UR_API const char *ur_last_error(const ur_context *c) { return c ? c->err.c_str() : t_create_err.c_str(); }

UR_API ur_status ur_scene_upload(ur_context *c, const ur_scene_desc *s) {
    return guarded(c, [&]() -> ur_status {
        if (!s) return c->fail(UR_ERR_INVALID_ARG, "scene is NULL");
        if (s->n_mat < 1 || s->n_mat > kMaxMat) return c->fail(UR_ERR_UNSUPPORTED, "n_mat must be in [1, %d]", kMaxMat);
        if (s->n_tri < 0 || s->n_sph < 0 || s->n_pln < 0 || s->n_scat < 0)
            return c->fail(UR_ERR_INVALID_ARG, "negative primitive count");
        if (s->n_sph > kMaxSph || s->n_pln > kMaxPln)
            return c->fail(UR_ERR_UNSUPPORTED, "at most %d spheres and %d planes", kMaxSph, kMaxPln);
        if (s->n_tri >= (1 << 27) || s->n_scat >= (1 << 27))
            return c->fail(UR_ERR_UNSUPPORTED, "at most 2^27 triangles / scatterers");
        if (!s->mat || !s->box || (s->n_tri && (!s->tri || !s->tri_mat)) || (s->n_sph && (!s->sph || !s->sph_mat)) ||
            (s->n_pln && (!s->pln || !s->pln_mat)) || (s->n_scat && !s->scat))
            return c->fail(UR_ERR_INVALID_ARG, "NULL array for a non-empty primitive set");
        if (!finite_all(s->mat, 3 * s->n_mat) || !finite_all(s->box, 6) || !finite_all(s->tri, 9 * s->n_tri) ||
            !finite_all(s->sph, 4 * s->n_sph) || !finite_all(s->pln, 4 * s->n_pln) ||
            !finite_all(s->scat, 4 * s->n_scat))
            return c->fail(UR_ERR_INVALID_ARG, "non-finite scene value");
        for (int64_t m = 0; m < s->n_mat; ++m)
            if (!(s->mat[3 * m] > 0) || !(s->mat[3 * m + 1] >= 0) || !(s->mat[3 * m + 2] > 0))
                return c->fail(UR_ERR_SCENE, "material %lld needs Z > 0, alpha >= 0, c > 0", (long long)m);
        if (s->rough)
            for (int64_t m = 0; m < s->n_mat; ++m)
                if (!(s->rough[m] >= 0.0 && s->rough[m] <= 10.0))
                    return c->fail(UR_ERR_SCENE, "material %lld roughness must be in [0, 10]", (long long)m);
        for (int i = 0; i < 3; ++i)
            if (!(s->box[i] < s->box[3 + i])) return c->fail(UR_ERR_SCENE, "box min must be below max");
        if (!(s->box[2] <= 0.0))
            return c->fail(UR_ERR_SCENE, "the box top z = box[2] must be at or above the array (z <= 0)");
        if (s->top_medium < 0 || s->top_medium >= s->n_mat) return c->fail(UR_ERR_SCENE, "top_medium out of range");
        auto bad_mat = [&](const int32_t *m, int64_t n) {
            for (int64_t i = 0; i < 2 * n; ++i)
                if (m[i] < 0 || m[i] >= s->n_mat) return true;
            return false;
        };
        if (bad_mat(s->tri_mat, s->n_tri) || bad_mat(s->sph_mat, s->n_sph) || bad_mat(s->pln_mat, s->n_pln))
            return c->fail(UR_ERR_SCENE, "material index out of range");
        for (int64_t j = 0; j < s->n_sph; ++j)
            if (!(s->sph[4 * j + 3] > 0)) return c->fail(UR_ERR_SCENE, "sphere %lld radius must be > 0", (long long)j);
        for (int64_t j = 0; j < s->n_pln; ++j) {
            const double *p = s->pln + 4 * j;
            if (std::fabs(std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]) - 1.0) > 1e-9)
                return c->fail(UR_ERR_SCENE, "plane %lld normal is not unit length", (long long)j);
        }
        c->has_scene = false;
        c->mat.assign(s->mat, s->mat + 3 * s->n_mat);
        if (s->rough) c->rough.assign(s->rough, s->rough + s->n_mat);
        else c->rough.assign((size_t)s->n_mat, 0.0);
        std::memcpy(c->box, s->box, sizeof(c->box));
        c->top_medium = (int)s->top_medium;
        c->n_tri = s->n_tri;
        c->n_sph = s->n_sph;
        c->n_pln = s->n_pln;
        c->n_scat = s->n_scat;
        c->scat.assign(s->scat, s->scat + 4 * s->n_scat);
        c->sph.assign(s->sph, s->sph + 4 * s->n_sph);
        ur_status st;
        if ((st = upload_materials(c))) return st;
        if ((st = upload(c, c->d_sph, std::vector<double>(s->sph, s->sph + 4 * s->n_sph)))) return st;
        if ((st = upload(c, c->d_sph_mat, std::vector<int32_t>(s->sph_mat, s->sph_mat + 2 * s->n_sph)))) return st;
        if ((st = upload(c, c->d_pln, std::vector<double>(s->pln, s->pln + 4 * s->n_pln)))) return st;
        if ((st = upload(c, c->d_pln_mat, std::vector<int32_t>(s->pln_mat, s->pln_mat + 2 * s->n_pln)))) return st;
        // triangles: BVH with leaves of <= 4, 1 um dilation
        {
            std::vector<PrimBounds> pb(s->n_tri);
            for (int64_t i = 0; i < s->n_tri; ++i) {
                const double *v = s->tri + 9 * i;
                for (int k = 0; k < 3; ++k) {
                    pb[i].lo[k] = std::min(v[k], std::min(v[3 + k], v[6 + k]));
                    pb[i].hi[k] = std::max(v[k], std::max(v[3 + k], v[6 + k]));
                }
            }
            // one triangle per leaf: a four-wide FP32 node visit costs less
            // than the FP64 triangle tests a larger leaf would add
            BvhResult r = build_bvh(pb, 1, 1e-6);
            std::vector<double> tri(9 * s->n_tri);
            std::vector<int32_t> tm(2 * s->n_tri), tid(s->n_tri);
            std::vector<double4> tn(s->n_tri);
            for (int64_t k = 0; k < s->n_tri; ++k) {
                const int o = r.order[k];
                const double *v = s->tri + 9 * (int64_t)o;
                for (int j = 0; j < 3; ++j) {
                    tri[9 * k + j] = v[j];
                    tri[9 * k + 3 + j] = v[3 + j] - v[j];
                    tri[9 * k + 6 + j] = v[6 + j] - v[j];
                }
                // unit normal: (e1 x e2) / |e1 x e2| in FP64
                const double *e1 = &tri[9 * k + 3], *e2 = &tri[9 * k + 6];
                const double n0 = e1[1] * e2[2] - e1[2] * e2[1];
                const double n1 = e1[2] * e2[0] - e1[0] * e2[2];
                const double n2 = e1[0] * e2[1] - e1[1] * e2[0];
                const double l = std::sqrt(n0 * n0 + n1 * n1 + n2 * n2);
                tn[k] = make_double4(n0 / l, n1 / l, n2 / l, 0.0);
                tm[2 * k] = s->tri_mat[2 * o];
                tm[2 * k + 1] = s->tri_mat[2 * o + 1];
                tid[k] = o;
            }
            c->n_tnodes = (int)r.nodes.size();
            for (int k = 0; k < 3 && !r.nodes.empty(); ++k) {
                c->tree_lo[k] = r.nodes[0].lo[k];
                c->tree_hi[k] = r.nodes[0].hi[k];
            }
            const std::vector<Bvh4NodeQ> wide = quantize_bvh4(collapse_bvh4(r.nodes));
            c->n_tnodes4 = (int)wide.size();
            if ((st = upload(c, c->d_tnodes4, wide))) return st;
            if ((st = upload(c, c->d_tri, tri))) return st;
            if ((st = upload(c, c->d_tri_n, tn))) return st;
            if ((st = upload(c, c->d_tri_mat, tm))) return st;
            if ((st = upload(c, c->d_tri_id, tid))) return st;
            if ((st = upload(c, c->d_tnodes, r.nodes))) return st;
        }
        c->has_scene = true;   // the scatterer grid depends on r_s: built at transmit setup
        if (c->has_setup) {
            c->has_setup = false;
            ur_acq_desc a = c->acq;
            a.angles = c->angles.data();
            ur_probe_desc p = c->probe;
            return ur_transmit_setup(c, &p, &a);
        }
        return UR_OK;
    });
}

UR_API ur_status ur_scene_update(ur_context *c, const double *mat, const double *scat_amp, const double *sph) {
    return guarded(c, [&]() -> ur_status {
        if (!c->has_scene) return c->fail(UR_ERR_CALL_ORDER, "upload a scene first");
        const int64_t nm = (int64_t)c->mat.size() / 3;
        if (mat) {
            if (!finite_all(mat, 3 * nm)) return c->fail(UR_ERR_INVALID_ARG, "non-finite material value");
            for (int64_t m = 0; m < nm; ++m)
                if (!(mat[3 * m] > 0) || !(mat[3 * m + 1] >= 0) || !(mat[3 * m + 2] > 0))
                    return c->fail(UR_ERR_SCENE, "material %lld needs Z > 0, alpha >= 0, c > 0", (long long)m);
        }
        if (scat_amp && !finite_all(scat_amp, c->n_scat)) return c->fail(UR_ERR_INVALID_ARG, "non-finite amplitude");
        if (sph) {
            if (!finite_all(sph, 4 * c->n_sph)) return c->fail(UR_ERR_INVALID_ARG, "non-finite sphere value");
            for (int64_t j = 0; j < c->n_sph; ++j)
                if (!(sph[4 * j + 3] > 0)) return c->fail(UR_ERR_SCENE, "sphere %lld radius must be > 0", (long long)j);
        }
        ur_status st;
        if (mat) {
            c->mat.assign(mat, mat + 3 * nm);
            if ((st = upload_materials(c))) return st;
        }
        if (sph) {
            c->sph.assign(sph, sph + 4 * c->n_sph);
            if ((st = upload(c, c->d_sph, c->sph))) return st;
        }
        if (scat_amp) {
            for (int64_t k = 0; k < c->n_scat; ++k) c->scat[4 * k + 3] = scat_amp[k];
            if (c->has_setup) {
                std::vector<double4> items(c->item_order.size());
                for (size_t k = 0; k < items.size(); ++k) {
                    const double *q = c->scat.data() + 4 * (int64_t)c->item_order[k];
                    items[k] = make_double4(q[0], q[1], q[2], q[3]);
                }
                if ((st = upload(c, c->d_items, items))) return st;
            }
        }
        return UR_OK;
    });
}

UR_API ur_status ur_transmit_setup(ur_context *c, const ur_probe_desc *p, const ur_acq_desc *a) {
    return guarded(c, [&]() -> ur_status {
        if (!c->has_scene) return c->fail(UR_ERR_CALL_ORDER, "upload a scene before transmit setup");
        if (!p || !a || !a->angles) return c->fail(UR_ERR_INVALID_ARG, "probe, acquisition and angles are required");
        if (p->n_elements < 1 || p->n_elements > 65535) return c->fail(UR_ERR_INVALID_ARG, "n_elements must be in [1, 65535]");
        if (!(p->pitch > 0) || !(p->elevation > 0) || !(p->f_c > 0) || !std::isfinite(p->pitch) ||
            !std::isfinite(p->elevation) || !std::isfinite(p->f_c))
            return c->fail(UR_ERR_INVALID_ARG, "pitch, elevation and f_c must be positive");
        if (!(p->radius >= 0.0) || !std::isfinite(p->radius))
            return c->fail(UR_ERR_INVALID_ARG, "radius must be 0 (linear) or positive (convex)");
        if (p->radius > 0.0) {
            const double hp = 0.5 * (double)p->n_elements * p->pitch / p->radius, h = std::sin(0.5 * hp);
            if (!(hp < 0.5 * M_PI)) return c->fail(UR_ERR_INVALID_ARG, "a convex array must span less than 180 degrees");
            if (!(c->box[2] <= -2.0 * p->radius * h * h))
                return c->fail(UR_ERR_SCENE, "the box top z = %g must lie at or above the convex array's ends (z = %g)",
                               c->box[2], -2.0 * p->radius * h * h);
        } else if (c->box[2] != 0.0) {
            return c->fail(UR_ERR_SCENE, "with a linear array the box top z = box[2] must be the array plane z = 0");
        }
        if (a->n_tx < 1 || a->n_tx > 65535) return c->fail(UR_ERR_INVALID_ARG, "n_tx must be in [1, 65535]");
        if (a->n_samples < 2 || a->n_samples > (1 << 24)) return c->fail(UR_ERR_INVALID_ARG, "n_samples must be in [2, 2^24]");
        if (a->rays_per_element < 0 || a->rays_per_element > 0xFFFFFFFFll)
            return c->fail(UR_ERR_INVALID_ARG, "rays_per_element must be in [0, 2^32)");
        if (a->max_bounces < 0 || a->max_bounces > 65535) return c->fail(UR_ERR_INVALID_ARG, "max_bounces must be in [0, 65535]");
        if (a->binning != UR_BIN_NEAREST && a->binning != UR_BIN_LINEAR) return c->fail(UR_ERR_INVALID_ARG, "unknown binning mode");
        const double v[] = {a->f_s, a->c0, a->n_cycles, a->max_path};
        for (double x : v)
            if (!(x > 0) || !std::isfinite(x)) return c->fail(UR_ERR_INVALID_ARG, "f_s, c0, n_cycles and max_path must be positive");
        if (!(a->r_s >= 0) || !std::isfinite(a->r_s)) return c->fail(UR_ERR_INVALID_ARG, "r_s must be >= 0");
        if (a->scheme != UR_SCHEME_PLANE_WAVE && a->scheme != UR_SCHEME_SYNTHETIC)
            return c->fail(UR_ERR_INVALID_ARG, "scheme must be UR_SCHEME_PLANE_WAVE or UR_SCHEME_SYNTHETIC");
        if (a->scheme == UR_SCHEME_SYNTHETIC && a->n_tx != p->n_elements)
            return c->fail(UR_ERR_INVALID_ARG, "the synthetic-aperture scheme needs n_tx = n_elements");
        if (a->rough_direct_only != 0 && a->rough_direct_only != 1)
            return c->fail(UR_ERR_INVALID_ARG, "rough_direct_only must be 0 or 1");
        if (a->element_choice != UR_ELEMENT_UNIFORM && a->element_choice != UR_ELEMENT_CONE)
            return c->fail(UR_ERR_INVALID_ARG, "element_choice must be UR_ELEMENT_UNIFORM or UR_ELEMENT_CONE");
        if (!(a->alpha_m >= 0) || !(a->alpha_c >= a->alpha_m) || !(a->alpha_c <= M_PI))
            return c->fail(UR_ERR_INVALID_ARG, "need 0 <= alpha_m <= alpha_c <= pi");
        for (int64_t t = 0; t < a->n_tx; ++t)
            if (!std::isfinite(a->angles[t]) || std::fabs(a->angles[t]) >= M_PI / 2)
                return c->fail(UR_ERR_INVALID_ARG, "steering angle %lld must be finite and within (-pi/2, pi/2)", (long long)t);
        const double sig = a->n_cycles / (2.0 * std::sqrt(2.0 * std::log(2.0)) * p->f_c);
        const int K = (int)std::ceil(3.0 * sig * a->f_s);
        if (K > 512) return c->fail(UR_ERR_UNSUPPORTED, "pulse needs %d half-taps, at most 512 are supported", K);
        const double work = (double)a->n_tx * (double)p->n_elements * (double)a->rays_per_element;
        if (work > 9.0e15) return c->fail(UR_ERR_UNSUPPORTED, "too many rays");

        c->has_setup = false;
        c->probe = *p;
        c->acq = *a;
        c->angles.assign(a->angles, a->angles + a->n_tx);
        c->acq.angles = nullptr;
        c->K = K;
        const int64_t E = p->n_elements, T = a->n_tx;
        // element centres and plane-wave delays referenced to the first-firing
        // element.  A convex array of radius R has its centre of curvature at
        // (0, 0, -R) and the pitch is the arc length: element e sits at angle
        // phi_e = (e - (E-1)/2) pitch / R, at (R sin phi_e, -2 R sin^2(phi_e/2)),
        // facing (sin phi_e, 0, cos phi_e); it fires when the plane front
        // k = (sin theta, 0, cos theta) passes its centre.
        const bool convex = p->radius > 0.0;
        std::vector<double> xe(E), ze(E), tau(T * E), kref(T);
        std::vector<double4> elem(E);
        for (int64_t e = 0; e < E; ++e) {
            const double off = (double)e - 0.5 * (double)(E - 1);
            if (convex) {
                const double ph = off * p->pitch / p->radius, h = std::sin(0.5 * ph);
                xe[e] = p->radius * std::sin(ph);
                ze[e] = -2.0 * p->radius * h * h;
                elem[e] = make_double4(xe[e], ze[e], std::sin(ph), std::cos(ph));
            } else {
                xe[e] = off * p->pitch;
                ze[e] = 0.0;
                elem[e] = make_double4(xe[e], 0.0, 0.0, 1.0);
            }
        }
        for (int64_t t = 0; t < T; ++t) {
            const double st = std::sin(c->angles[t]), ct = std::cos(c->angles[t]);
            if (convex) {
                double ref = INFINITY;
                for (int64_t e = 0; e < E; ++e) ref = std::min(ref, xe[e] * st + ze[e] * ct);
                kref[t] = ref;
                for (int64_t e = 0; e < E; ++e)
                    tau[t * E + e] = a->scheme == UR_SCHEME_SYNTHETIC ? 0.0 : (xe[e] * st + ze[e] * ct - ref) / a->c0;
            } else {
                const double xref = st >= 0 ? xe[0] : xe[E - 1];
                kref[t] = xref * st;
                for (int64_t e = 0; e < E; ++e)
                    tau[t * E + e] = a->scheme == UR_SCHEME_SYNTHETIC ? 0.0 : (xe[e] - xref) * st / a->c0;
            }
        }
        // analytic pulse taps (Eq. 14), Gaussian with FWHM of n_cycles periods
        std::vector<float2> taps(2 * K + 1);
        for (int m = -K; m <= K; ++m) {
            const double tm = (double)m / a->f_s;
            const double g = std::exp(-tm * tm / (2.0 * sig * sig));
            const double ph = 2.0 * M_PI * p->f_c * tm;
            taps[m + K] = make_float2((float)(g * std::sin(ph)), (float)(-g * std::cos(ph)));
        }
        // beamforming constants per transmit: idx = x*A + z*B + C + r*fs/c0
        std::vector<double4> txc(T);
        const double k = a->f_s / a->c0;
        for (int64_t t = 0; t < T; ++t) {
            const double st = std::sin(c->angles[t]), ct = std::cos(c->angles[t]);
            if (convex) {
                txc[t] = make_double4(st * k, ct * k, -kref[t] * k - 0.5, 0.0);
            } else {
                const double xref = st >= 0 ? xe[0] : xe[E - 1];
                txc[t] = make_double4(st * k, ct * k, -xref * st * k - 0.5, 0.0);
            }
        }
        // receive apodisation tables: [0, E) uniform, [E, 2E) Hann over the full aperture
        std::vector<float> apod(2 * E);
        for (int64_t e = 0; e < E; ++e) {
            apod[e] = 1.0f;
            apod[E + e] = (float)(0.5 - 0.5 * std::cos(2.0 * M_PI * ((double)e + 0.5) / (double)E));
        }
        ur_status st;
        if ((st = upload(c, c->d_apod, apod))) return st;
        c->xe_h = xe;
        c->ze_h = ze;
        if ((st = upload(c, c->d_xe, xe))) return st;
        if ((st = upload(c, c->d_ze, ze))) return st;
        if ((st = upload(c, c->d_elem, elem))) return st;
        if ((st = upload(c, c->d_tau, tau))) return st;
        if ((st = upload(c, c->d_taps, taps))) return st;
        if ((st = upload(c, c->d_txc, txc))) return st;
        if ((st = alloc(c, c->d_stats, kNumStats * sizeof(unsigned long long)))) return st;
        if ((st = alloc(c, c->d_stats2, kNumStats * sizeof(unsigned long long)))) return st;
        if ((st = alloc(c, c->d_counters, 8 * sizeof(unsigned long long)))) return st;
        if ((st = alloc(c, c->d_maxbits, 256))) return st;
        if ((st = upload(c, c->d_angles, c->angles))) return st;
        if (c->mlp_ready && T * E != c->mlp_rows) {
            c->mlp_ready = false;   // the network's rows follow the acquisition
            c->pdf = c->cdf = nullptr;
        }
        c->has_setup = true;
        if ((st = upload_materials(c))) return st;
        // scatterers: uniform grid; each registered in the cells its capture
        // ball (radius r_s plus a 1 um margin) overlaps.  Scatterers that no
        // element can hear (Eq. 13 zero over the whole grown ball for every
        // element) are left out: their captures only ever yield zero-valued
        // secondary rays.
        {
            RxCone rx{xe[0], xe[E - 1], a->alpha_c};
            if (convex) {
                rx.radius = p->radius;
                rx.phi_lo = (0.0 - 0.5 * (double)(E - 1)) * p->pitch / p->radius;
                rx.phi_hi = ((double)(E - 1) - 0.5 * (double)(E - 1)) * p->pitch / p->radius;
            }
            ScatterGrid g = build_scatter_grid(c->box, c->scat.data(), (long)c->n_scat, a->r_s, a->r_s * 1e-5 + 1e-6,
                                               &rx);
            std::vector<double4> items(g.items.size());
            std::vector<float4> items_f(g.items.size());
            for (size_t k = 0; k < g.items.size(); ++k) {
                const double *q = c->scat.data() + 4 * (int64_t)g.items[k];
                items[k] = make_double4(q[0], q[1], q[2], q[3]);
                items_f[k] = make_float4((float)q[0], (float)q[1], (float)q[2], 0.0f);
            }
            c->grid = g.info;
            c->item_order = g.items;
            if ((st = upload(c, c->d_cell_start, g.cell_start))) return st;
            if ((st = upload(c, c->d_items, items))) return st;
            if ((st = upload(c, c->d_items_f, items_f))) return st;
            if ((st = upload(c, c->d_item_id, g.items))) return st;
            if ((st = alloc(c, c->d_work, 256))) return st;
        }
        return UR_OK;
    });
}

UR_API ur_status ur_set_proposal(ur_context *c, const float *pdf_dev, const float *cdf_dev) {
    return guarded(c, [&]() -> ur_status {
        if ((pdf_dev == nullptr) != (cdf_dev == nullptr))
            return c->fail(UR_ERR_INVALID_ARG, "pdf and cdf must both be set or both be NULL");
        c->pdf = pdf_dev;
        c->cdf = cdf_dev;
        return UR_OK;
    });
}

UR_API ur_status ur_trace(ur_context *c, uint64_t seed, int64_t ray_stride, int64_t ray_offset, float *ch_raw_dev,
                          float *ch_rf_dev, ur_trace_stats *stats, void *stream) {
    return guarded(c, [&]() -> ur_status {
        if (!c->has_setup) return c->fail(UR_ERR_CALL_ORDER, "call ur_scene_upload and ur_transmit_setup first");
        if (!ch_raw_dev) return c->fail(UR_ERR_INVALID_ARG, "ch_raw_dev is NULL");
        if (ray_stride < 1 || ray_offset < 0 || ray_offset >= ray_stride)
            return c->fail(UR_ERR_INVALID_ARG, "need ray_stride >= 1 and 0 <= ray_offset < ray_stride");
        hipStream_t s = (hipStream_t)stream;
        TraceParams P;
        fill_params(c, P, seed);
        const int64_t nel = c->acq.rays_per_element;
        P.stride = ray_stride;
        P.offset = ray_offset;
        P.per_el = nel > ray_offset ? (nel - ray_offset + ray_stride - 1) / ray_stride : 0;
        P.n_work = (int64_t)(P.sa ? 1 : P.T) * P.E * P.per_el;   // synthetic aperture: one element per transmit
        P.ch_raw = ch_raw_dev;
        const int64_t n_ch = (int64_t)P.T * P.E * P.S;
        ur_status st;
        HIP_TRY(c, zero_f32(ch_raw_dev, n_ch, s));
        unsigned long long *ctr = (unsigned long long *)c->d_counters.p;
        P.nee_count = ctr + 2;
        P.rec = c->rec;
        P.rec_count = c->rec_count;
        P.rec_cap = c->rec_cap;
        unsigned long long *st1 = stats ? (unsigned long long *)c->d_stats.p : nullptr;
        unsigned long long *st2 = stats ? (unsigned long long *)c->d_stats2.p : nullptr;
        if (stats) {
            hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, st1, kNumStats);
            hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, st2, kNumStats);
            HIP_TRY(c, hipGetLastError());
        }
        // Launch ranges: fewer, longer ranges have fewer kernel tails (each
        // range boundary costs about 1.3 ms on the bone frame).  The segment
        // queue between the extend and scatter kernels stays within its
        // budget (1/8 of the device memory unless ur_set_segment_queue set
        // one).  If that holds the worst case of a range (every ray queueing
        // all B + 1 segments, plus one partly used chunk per wavefront), every
        // launch takes its whole range; otherwise the queue takes the whole
        // budget and the extend kernel admits rays only while the worst case
        // of the rays not yet finished still fits, so a launch ends where the
        // queue would fill and the next one starts there.
        int64_t range = std::max<int64_t>(1, std::min<int64_t>(c->rays_per_launch, kSplitRays));
        bool admit = false;
        if (P.n_scat > 0) {
            const int64_t waves = ur_extend_max_waves();
            if (waves < 0) return c->fail(UR_ERR_HIP, "occupancy query failed");
            const int64_t slack = waves * kSegChunk;
            int64_t budget = c->seg_budget;
            if (budget == 0) {
                size_t free_b = 0, total_b = 0;
                HIP_TRY(c, hipMemGetInfo(&free_b, &total_b));
                budget = (int64_t)(total_b / 8 / (sizeof(SegHot) + sizeof(SegCold))) - slack;
            }
            const int64_t n_first = std::min<int64_t>(range, std::max<int64_t>(P.n_work, 1));
            int64_t cap = n_first * (int64_t)(P.B + 1) + slack;
            if (cap > budget + slack) {
                // admission needs room for the first chunk of rays at least
                if (budget >= (int64_t)kRayChunk * (P.B + 1)) {
                    admit = true;
                    cap = budget + slack;
                } else {
                    const int64_t fit = budget / (int64_t)(P.B + 1);
                    range = std::min(range, std::max<int64_t>(int64_t(1) << 16, fit));
                    cap = std::min<int64_t>(range, std::max<int64_t>(P.n_work, 1)) * (int64_t)(P.B + 1) + slack;
                }
            }
            if ((st = alloc(c, c->d_segq, (size_t)cap * sizeof(SegHot)))) return st;
            if ((st = alloc(c, c->d_segc, (size_t)cap * sizeof(SegCold)))) return st;
            P.segq = (SegHot *)c->d_segq.p;
            P.segc = (SegCold *)c->d_segc.p;
            P.seg_cap = cap;
            if (admit) {
                P.seg_commit = ctr + 7;
                P.seg_limit = (unsigned long long)(cap - slack);
            }
        }
        {
            const int64_t launches = (P.n_work + range - 1) / range;
            if (launches > 1) range = (P.n_work + launches - 1) / launches;   // equal ranges
        }
        // the transducer-sampling queue: a range that overflows it is traced
        // again, so by default it holds one candidate per ray of a range, at
        // least 2^25 and at most 2^27 (10.7 GB)
        const int64_t nee_cap =
            c->nee_auto ? std::max<int64_t>(c->nee_cap, std::min<int64_t>({range, P.n_work, int64_t(1) << 27}))
                        : c->nee_cap;
        if ((st = alloc(c, c->d_nee, (size_t)nee_cap * sizeof(NeeEntry)))) return st;
        P.nee = (NeeEntry *)c->d_nee.p;
        P.nee_cap = nee_cap;
        c->n_tev = 0;
        c->trace_timed = false;
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, ctr + 6, 1);
        P.seg_lost = ctr + 6;
        if (c->det_mode) {
            if ((st = alloc(c, c->d_det, (size_t)c->det_cap * sizeof(DetRecord)))) return st;
            if ((st = alloc(c, c->d_det_ctr, 2 * sizeof(unsigned long long)))) return st;
            if ((st = alloc(c, c->d_det_bins, (size_t)n_ch * sizeof(long long)))) return st;
            hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, (unsigned long long *)c->d_det_ctr.p, 2);
            HIP_TRY(c, zero_f32((float *)c->d_det_bins.p, 2 * n_ch, s));   // int64 zeros are float zeros twice
            HIP_TRY(c, hipGetLastError());
            P.det = (DetRecord *)c->d_det.p;
            P.det_count = (unsigned long long *)c->d_det_ctr.p;
            P.det_cap = c->det_cap;
        }
        HIP_TRY(c, hipEventRecord(c->ev[0], s));
        // Work is launched in ranges: extend (closest hits, shading, segment
        // queue), scatter (captures into the transducer-sampling queue), cast
        // the sampling queue, then (only if that queue overflowed) re-trace
        // the range casting the sampling rays inline without direct hits.
        for (int64_t begin = 0; begin < P.n_work;) {
            P.work_begin = begin;
            P.work_end = std::min(P.n_work, begin + range);
            while ((int64_t)c->tev.size() < 4 * (c->n_tev + 1)) {
                hipEvent_t e;
                HIP_TRY(c, hipEventCreate(&e));
                c->tev.push_back(e);
            }
            hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, ctr, 6);
            if (admit) hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, ctr + 7, 1);
            HIP_TRY(c, hipGetLastError());
            P.work_next = ctr;
            P.seg_count = ctr + 3;
            P.seg_next = ctr + 4;
            P.stats = st1;
            hipEvent_t *ev = &c->tev[4 * c->n_tev];
            HIP_TRY(c, hipEventRecord(ev[0], s));
            HIP_TRY(c, ur_launch_extend(P, stats != nullptr, s));
            HIP_TRY(c, hipEventRecord(ev[1], s));
            if (admit) {
                // the rays this launch took: [0, work_next) of the range, all
                // of them traced (a wavefront takes a chunk only once admitted)
                unsigned long long next = 0;
                HIP_TRY(c, hipMemcpyAsync(&next, ctr, sizeof(next), hipMemcpyDeviceToHost, s));
                HIP_TRY(c, hipStreamSynchronize(s));
                const int64_t taken = std::min<int64_t>((int64_t)next, P.work_end - P.work_begin);
                if (taken <= 0) return c->fail(UR_ERR_CAPACITY, "segment queue admits no rays");
                P.work_end = P.work_begin + taken;
            }
            begin = P.work_end;
            if (P.n_scat > 0) HIP_TRY(c, ur_launch_scatter(P, stats != nullptr, s));
            HIP_TRY(c, hipEventRecord(ev[2], s));
            HIP_TRY(c, ur_launch_nee(P, stats != nullptr, s));
            HIP_TRY(c, hipEventRecord(ev[3], s));
            ++c->n_tev;
            TraceParams P2 = P;
            P2.work_next = ctr + 1;
            P2.stats = st2;
            HIP_TRY(c, ur_launch_trace(P2, stats != nullptr, kInlineNeeOnly, s));
        }
        if (c->det_mode)
            HIP_TRY(c, ur_launch_det_bin(P.det, P.det_cap, P.det_count, (long long *)c->d_det_bins.p, ch_raw_dev,
                                         (int64_t)P.T * P.E, P.S, P.binning, s));
        HIP_TRY(c, hipEventRecord(c->ev[1], s));
        c->trace_timed = c->n_tev > 0;
        if (ch_rf_dev) HIP_TRY(c, ur_launch_pulse(ch_raw_dev, (float2 *)ch_rf_dev, (const float2 *)c->d_taps.p, c->K,
                                                  (int64_t)P.T * P.E, P.S, s));
        // every call checks the segment queue's lost count (one 8-byte read),
        // and in the deterministic mode the staged records offered
        unsigned long long lost = 0, offered = 0;
        HIP_TRY(c, hipMemcpyAsync(&lost, ctr + 6, sizeof(lost), hipMemcpyDeviceToHost, s));
        if (c->det_mode) HIP_TRY(c, hipMemcpyAsync(&offered, P.det_count, sizeof(offered), hipMemcpyDeviceToHost, s));
        if (stats) {
            unsigned long long h[kNumStats], h2[kNumStats];
            HIP_TRY(c, hipMemcpyAsync(h, st1, sizeof(h), hipMemcpyDeviceToHost, s));
            HIP_TRY(c, hipMemcpyAsync(h2, st2, sizeof(h2), hipMemcpyDeviceToHost, s));
            HIP_TRY(c, hipStreamSynchronize(s));
            if (lost) return c->fail(UR_ERR_CAPACITY, "segment queue overflow (%llu segments lost)", lost);
            if ((int64_t)offered > c->det_cap && c->det_mode)
                return c->fail(UR_ERR_CAPACITY, "deterministic binning: %llu records for a capacity of %lld", offered,
                               (long long)c->det_cap);
            // the overflow re-trace contributes only its transducer-sampling work
            uint64_t *dst = &stats->rays;
            for (int k = 0; k < kNumStats; ++k) dst[k] = h[k];
            stats->nee_cast += h2[7];
            stats->nee_blocked += h2[8];
            stats->records += h2[10];
            stats->dropped += h2[11];
            stats->edge_band += h2[12];
            stats->shadow_nodes += h2[22];
            stats->shadow_tri_tests += h2[23];
            float ms = 0.f;
            HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
            stats->kernel_ms = ms;
        } else {
            HIP_TRY(c, hipStreamSynchronize(s));
            if (lost) return c->fail(UR_ERR_CAPACITY, "segment queue overflow (%llu segments lost)", lost);
            if ((int64_t)offered > c->det_cap && c->det_mode)
                return c->fail(UR_ERR_CAPACITY, "deterministic binning: %llu records for a capacity of %lld", offered,
                               (long long)c->det_cap);
        }
        return UR_OK;
    });
}

UR_API ur_status ur_set_binning(ur_context *c, int32_t deterministic, int64_t capacity) {
    return guarded(c, [&]() -> ur_status {
        if (deterministic != 0 && deterministic != 1) return c->fail(UR_ERR_INVALID_ARG, "deterministic must be 0 or 1");
        if (deterministic && capacity < 1) return c->fail(UR_ERR_INVALID_ARG, "need a capacity >= 1");
        c->det_mode = deterministic == 1;
        c->det_cap = deterministic ? capacity : 0;
        return UR_OK;
    });
}

UR_API ur_status ur_set_segment_queue(ur_context *c, int64_t segments) {
    return guarded(c, [&]() -> ur_status {
        if (segments < 0) return c->fail(UR_ERR_INVALID_ARG, "need segments >= 0");
        c->seg_budget = segments;
        c->d_segq.release();
        c->d_segc.release();
        return UR_OK;
    });
}

UR_API ur_status ur_set_limits(ur_context *c, int64_t rays_per_launch, int64_t nee_queue_capacity) {
    return guarded(c, [&]() -> ur_status {
        if (rays_per_launch < 1 || nee_queue_capacity < 1 || nee_queue_capacity > (int64_t(1) << 31))
            return c->fail(UR_ERR_INVALID_ARG, "need rays_per_launch >= 1 and 1 <= nee_queue_capacity <= 2^31");
        c->rays_per_launch = rays_per_launch;
        c->nee_cap = nee_queue_capacity;
        c->nee_auto = false;
        c->d_nee.release();
        return UR_OK;
    });
}

UR_API ur_status ur_synthesize(ur_context *c, const float *ch_sa_dev, const double *angles, int64_t n_ang,
                               float *out_dev, void *stream) {
    return guarded(c, [&]() -> ur_status {
        if (!c->has_setup) return c->fail(UR_ERR_CALL_ORDER, "call ur_transmit_setup first");
        if (!ch_sa_dev || !out_dev || !angles) return c->fail(UR_ERR_INVALID_ARG, "NULL buffer");
        if (n_ang < 1 || n_ang > 128) return c->fail(UR_ERR_INVALID_ARG, "need 1 <= n_ang <= 128");
        for (int64_t k = 0; k < n_ang; ++k)
            if (!std::isfinite(angles[k]) || std::fabs(angles[k]) >= M_PI / 2)
                return c->fail(UR_ERR_INVALID_ARG, "angle %lld must be finite and within (-pi/2, pi/2)", (long long)k);
        const bool convex = c->probe.radius > 0.0;
        HIP_TRY(c, ur_launch_synth_angles(ch_sa_dev, angles, (int)n_ang, (int)c->probe.n_elements,
                                          (int)c->acq.n_samples, c->xe_h.data(), convex ? c->ze_h.data() : nullptr,
                                          (const double *)c->d_xe.p, (const double *)c->d_ze.p, c->acq.c0,
                                          c->acq.f_s, out_dev, (hipStream_t)stream));
        return UR_OK;
    });
}

UR_API ur_status ur_scan_convert(ur_context *c, const ur_grid_desc *sector, const float *img_dev,
                                 const ur_grid_desc *cart, float fill, float *out_dev, void *stream) {
    return guarded(c, [&]() -> ur_status {
        if (!c->has_setup) return c->fail(UR_ERR_CALL_ORDER, "call ur_transmit_setup first");
        if (!sector || !cart || !img_dev || !out_dev) return c->fail(UR_ERR_INVALID_ARG, "NULL argument");
        if (sector->sector != 1 || cart->sector != 0)
            return c->fail(UR_ERR_INVALID_ARG, "need a sector source grid and a Cartesian target grid");
        if (sector->nx < 2 || sector->nz < 2 || sector->nx > 65535 || sector->nz > (1 << 24) || cart->nx < 1 ||
            cart->nz < 1 || cart->nx > 65535 || cart->nz > (1 << 24))
            return c->fail(UR_ERR_INVALID_ARG, "grid size out of range");
        const double gv[] = {sector->x0, sector->x1, sector->z0, sector->z1, cart->x0, cart->x1, cart->z0, cart->z1};
        if (!finite_all(gv, 8) || !std::isfinite(fill)) return c->fail(UR_ERR_INVALID_ARG, "non-finite grid value");
        if (!(sector->x1 > sector->x0) || !(sector->z1 > sector->z0))
            return c->fail(UR_ERR_INVALID_ARG, "the sector grid needs x1 > x0 and z1 > z0");
        HIP_TRY(c, ur_launch_scan_convert(c->probe.radius, (int)sector->nx, (int)sector->nz, sector->x0, sector->x1,
                                          sector->z0, sector->z1, img_dev, (int)cart->nx, (int)cart->nz, cart->x0,
                                          cart->x1, cart->z0, cart->z1, fill, out_dev, (hipStream_t)stream));
        return UR_OK;
    });
}

UR_API ur_status ur_pulse(ur_context *c, const float *ch_raw_dev, float *ch_rf_dev, void *stream) {
    return guarded(c, [&]() -> ur_status {
        if (!c->has_setup) return c->fail(UR_ERR_CALL_ORDER, "call ur_transmit_setup first");
        if (!ch_raw_dev || !ch_rf_dev) return c->fail(UR_ERR_INVALID_ARG, "NULL channel buffer");
        HIP_TRY(c, ur_launch_pulse(ch_raw_dev, (float2 *)ch_rf_dev, (const float2 *)c->d_taps.p, c->K,
                                   c->acq.n_tx * c->probe.n_elements, (int)c->acq.n_samples, (hipStream_t)stream));
        return UR_OK;
    });
}

// Delay-and-sum constants of an image grid.  A sector grid places pixel
// (i, j) at angle x0 + i dx and depth z0 + j dz along the ray from the
// array's centre of curvature (the origin for a linear array).
static DasParams das_params(const ur_context *c, const ur_grid_desc *g) {
    const int64_t E = c->probe.n_elements;
    DasParams P;
    P.E = (int)E;
    P.T = (int)c->acq.n_tx;
    P.S = (int)c->acq.n_samples;
    P.nx = (int)g->nx;
    P.nz = (int)g->nz;
    P.sector = g->sector != 0;
    P.radius = c->probe.radius;
    P.x0 = g->x0;
    P.dx = g->nx > 1 ? (g->x1 - g->x0) / (double)(g->nx - 1) : 0.0;
    P.z0 = g->z0;
    P.dz = g->nz > 1 ? (g->z1 - g->z0) / (double)(g->nz - 1) : 0.0;
    P.fs_over_c0 = c->acq.f_s / c->acq.c0;
    P.fs = c->acq.f_s;
    P.xe = (const double *)c->d_xe.p;
    P.ze = c->probe.radius > 0.0 ? (const double *)c->d_ze.p : nullptr;
    P.apod = (const float *)c->d_apod.p + (g->apod == UR_APOD_HANN ? E : 0);
    P.txc = (const double4 *)c->d_txc.p;
    P.rf = nullptr;
    P.iq = nullptr;
    P.env = nullptr;
    return P;
}

static ur_status check_beamform(ur_context *c, const ur_grid_desc *g, const float *ch_rf_dev, const float *iq_dev,
                                const float *env_dev, const float *bmode_dev) {
    if (!c->has_setup) return c->fail(UR_ERR_CALL_ORDER, "call ur_transmit_setup first");
    if (!g || !ch_rf_dev) return c->fail(UR_ERR_INVALID_ARG, "grid and ch_rf_dev are required");
    if (!iq_dev && !env_dev && !bmode_dev) return c->fail(UR_ERR_INVALID_ARG, "no output requested");
    if (g->nx < 1 || g->nz < 1 || g->nx > 65535 || g->nz > (1 << 24))
        return c->fail(UR_ERR_INVALID_ARG, "grid size out of range");
    const double gv[] = {g->x0, g->x1, g->z0, g->z1, g->dynamic_range_db};
    if (!finite_all(gv, 5)) return c->fail(UR_ERR_INVALID_ARG, "non-finite grid value");
    if (bmode_dev && !(g->dynamic_range_db > 0)) return c->fail(UR_ERR_INVALID_ARG, "dynamic range must be > 0");
    if (g->apod != UR_APOD_NONE && g->apod != UR_APOD_HANN) return c->fail(UR_ERR_INVALID_ARG, "unknown apodisation");
    if (g->sector != 0 && g->sector != 1) return c->fail(UR_ERR_INVALID_ARG, "sector must be 0 or 1");
    return UR_OK;
}

// DAS + envelope into iq / env, then (if bmode) log compression of env with
// its maximum reduced into *max_bits.
static ur_status run_beamform(ur_context *c, const ur_grid_desc *g, const float *ch_rf_dev, float *iq_dev, float *env,
                              float *bmode_dev, unsigned int *max_bits, hipStream_t s) {
    DasParams P = das_params(c, g);
    P.rf = (const float2 *)ch_rf_dev;
    P.iq = (float2 *)iq_dev;
    P.env = env;
    HIP_TRY(c, hipEventRecord(c->ev[2], s));
    HIP_TRY(c, ur_launch_das(P, s));
    HIP_TRY(c, hipEventRecord(c->ev[3], s));
    c->das_timed = true;
    if (bmode_dev)
        HIP_TRY(c, ur_launch_bmode(env, bmode_dev, g->nx * g->nz, (float)g->dynamic_range_db, max_bits, s));
    return UR_OK;
}

UR_API ur_status ur_beamform(ur_context *c, const ur_grid_desc *g, const float *ch_rf_dev, float *iq_dev, float *env_dev,
                             float *bmode_dev, void *stream) {
    return guarded(c, [&]() -> ur_status {
        ur_status st = check_beamform(c, g, ch_rf_dev, iq_dev, env_dev, bmode_dev);
        if (st) return st;
        float *env = env_dev;
        if (!env && bmode_dev) {
            if ((st = alloc(c, c->d_env, g->nx * g->nz * sizeof(float)))) return st;
            env = (float *)c->d_env.p;
        }
        return run_beamform(c, g, ch_rf_dev, iq_dev, env, bmode_dev, (unsigned int *)c->d_maxbits.p,
                            (hipStream_t)stream);
    });
}

UR_API ur_status ur_beamform_static(ur_context *c, const ur_grid_desc *g, const float *ch_rf_dev, float *iq_dev,
                                    float *env_dev, float *bmode_dev, void *stream) {
    return guarded(c, [&]() -> ur_status {
        ur_status st = check_beamform(c, g, ch_rf_dev, iq_dev, env_dev, bmode_dev);
        if (st) return st;
        if (!c->scratch) return c->fail(UR_ERR_HIP, "no static scratch on device %d", c->device);
        float *env = env_dev;
        if (!env && bmode_dev) {
            if (g->nx * g->nz > kStaticPixels)
                return c->fail(UR_ERR_CAPACITY,
                               "ur_beamform_static: %lld pixels exceed the static envelope buffer of %lld pixels "
                               "(pass env_dev, or use ur_beamform)",
                               (long long)(g->nx * g->nz), (long long)kStaticPixels);
            env = c->scratch + kStaticHeader;
        }
        // the maximum's word is cleared by ur_launch_bmode's own fill kernel
        return run_beamform(c, g, ch_rf_dev, iq_dev, env, bmode_dev, (unsigned int *)c->scratch, (hipStream_t)stream);
    });
}

UR_API ur_status ur_last_kernel_ms(ur_context *c, double *trace_ms, double *das_ms) {
    return guarded(c, [&]() -> ur_status {
        float ms = 0.f;
        if (trace_ms) {
            *trace_ms = -1.0;
            if (c->trace_timed) {
                double sum = 0.0;
                for (int i = 0; i < c->n_tev; ++i) {
                    HIP_TRY(c, hipEventSynchronize(c->tev[4 * i + 2]));
                    HIP_TRY(c, hipEventElapsedTime(&ms, c->tev[4 * i], c->tev[4 * i + 2]));
                    sum += ms;
                }
                *trace_ms = sum;
            }
        }
        if (das_ms) {
            *das_ms = -1.0;
            if (c->das_timed) {
                HIP_TRY(c, hipEventSynchronize(c->ev[3]));
                HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[2], c->ev[3]));
                *das_ms = ms;
            }
        }
        return UR_OK;
    });
}

UR_API ur_status ur_last_trace_kernels_ms(ur_context *c, double *extend_ms, double *scatter_ms, double *sampling_ms,
                                          int64_t *launches) {
    return guarded(c, [&]() -> ur_status {
        double acc[3] = {0.0, 0.0, 0.0};
        if (!c->trace_timed) {
            acc[0] = acc[1] = acc[2] = -1.0;
        } else {
            for (int i = 0; i < c->n_tev; ++i) {
                HIP_TRY(c, hipEventSynchronize(c->tev[4 * i + 3]));
                for (int k = 0; k < 3; ++k) {
                    float ms = 0.f;
                    HIP_TRY(c, hipEventElapsedTime(&ms, c->tev[4 * i + k], c->tev[4 * i + k + 1]));
                    acc[k] += ms;
                }
            }
        }
        if (extend_ms) *extend_ms = acc[0];
        if (scatter_ms) *scatter_ms = acc[1];
        if (sampling_ms) *sampling_ms = acc[2];
        if (launches) *launches = c->trace_timed ? c->n_tev : 0;
        return UR_OK;
    });
}

UR_API ur_status ur_trace_rays(ur_context *c, uint64_t seed, const ur_ray *rays, int64_t n, ur_event *events, int64_t cap,
                               int64_t *n_events, float *ch_raw_dev, void *stream) {
    return guarded(c, [&]() -> ur_status {
        if (!c->has_setup) return c->fail(UR_ERR_CALL_ORDER, "call ur_transmit_setup first");
        if (n < 0 || cap < 0 || (n > 0 && !rays) || (cap > 0 && !events))
            return c->fail(UR_ERR_INVALID_ARG, "bad ray or event buffer");
        const int64_t nm = (int64_t)c->mat.size() / 3;
        for (int64_t i = 0; i < n; ++i) {
            const ur_ray &r = rays[i];
            if (r.tx < 0 || r.tx >= c->acq.n_tx || r.elem < 0 || r.elem >= c->probe.n_elements || r.medium < 0 ||
                r.medium >= nm || r.ray < 0 || r.ray > 0xFFFFFFFFll || !finite_all(r.o, 3) || !finite_all(r.d, 3) ||
                !std::isfinite(r.w) || !std::isfinite(r.t))
                return c->fail(UR_ERR_INVALID_ARG, "ray %lld has an out-of-range field", (long long)i);
            const double l = std::sqrt(r.d[0] * r.d[0] + r.d[1] * r.d[1] + r.d[2] * r.d[2]);
            if (std::fabs(l - 1.0) > 1e-9) return c->fail(UR_ERR_INVALID_ARG, "ray %lld direction is not unit", (long long)i);
            for (int k = 0; k < 3; ++k)
                if (r.o[k] < c->box[k] || r.o[k] > c->box[3 + k])
                    return c->fail(UR_ERR_INVALID_ARG, "ray %lld starts outside the box", (long long)i);
        }
        hipStream_t s = (hipStream_t)stream;
        ur_status st;
        if ((st = alloc(c, c->d_rays, std::max<int64_t>(n, 1) * sizeof(ur_ray)))) return st;
        if ((st = alloc(c, c->d_events, std::max<int64_t>(cap, 1) * sizeof(ur_event)))) return st;
        if ((st = alloc(c, c->d_evcount, 64))) return st;
        TraceParams P;
        fill_params(c, P, seed);
        const int64_t n_ch = (int64_t)P.T * P.E * P.S;
        float *raw = ch_raw_dev;
        DevBuf tmp;
        if (!raw) {
            if ((st = alloc(c, tmp, n_ch * sizeof(float)))) return st;
            raw = (float *)tmp.p;
        }
        P.ch_raw = raw;
        P.stats = (unsigned long long *)c->d_stats.p;
        if (n) HIP_TRY(c, hipMemcpy(c->d_rays.p, rays, n * sizeof(ur_ray), hipMemcpyHostToDevice));
        HIP_TRY(c, zero_f32(raw, n_ch, s));
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, (unsigned long long *)c->d_evcount.p, 1);
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, P.stats, kNumStats);
        EventLog L{c->d_events.p, (unsigned long long *)c->d_evcount.p, cap};
        HIP_TRY(c, ur_launch_trace_rays(P, c->d_rays.p, n, L, s));
        unsigned long long cnt = 0;
        HIP_TRY(c, hipMemcpyAsync(&cnt, c->d_evcount.p, sizeof(cnt), hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        const int64_t keep = std::min<int64_t>((int64_t)cnt, cap);
        if (keep) HIP_TRY(c, hipMemcpy(events, c->d_events.p, keep * sizeof(ur_event), hipMemcpyDeviceToHost));
        if (n_events) *n_events = (int64_t)cnt;
        tmp.release();
        return UR_OK;
    });
}

UR_API ur_status ur_philox(ur_context *c, const uint32_t *ctr, int64_t n, uint32_t key0, uint32_t key1, uint32_t *out) {
    return guarded(c, [&]() -> ur_status {
        if (n < 0 || (n > 0 && (!ctr || !out))) return c->fail(UR_ERR_INVALID_ARG, "bad counter buffer");
        if (n == 0) return UR_OK;
        ur_status st;
        if ((st = alloc(c, c->d_ctr, 2 * n * 4 * sizeof(uint32_t)))) return st;
        uint32_t *dc = (uint32_t *)c->d_ctr.p, *dout = dc + 4 * n;
        HIP_TRY(c, hipMemcpy(dc, ctr, 4 * n * sizeof(uint32_t), hipMemcpyHostToDevice));
        HIP_TRY(c, ur_launch_philox(dc, dout, n, key0, key1, nullptr));
        HIP_TRY(c, hipDeviceSynchronize());
        HIP_TRY(c, hipMemcpy(out, dout, 4 * n * sizeof(uint32_t), hipMemcpyDeviceToHost));
        return UR_OK;
    });
}


// ------------------------------------------------------------ adjoint
UR_API ur_status ur_pulse_adjoint(ur_context *c, const float *g_rf_dev, float *g_raw_dev, void *stream) {
    return guarded(c, [&]() -> ur_status {
        if (!c->has_setup) return c->fail(UR_ERR_CALL_ORDER, "call ur_transmit_setup first");
        if (!g_rf_dev || !g_raw_dev) return c->fail(UR_ERR_INVALID_ARG, "NULL channel buffer");
        HIP_TRY(c, ur_launch_pulse_adj((const float2 *)g_rf_dev, g_raw_dev, (const float2 *)c->d_taps.p, c->K,
                                       c->acq.n_tx * c->probe.n_elements, (int)c->acq.n_samples, (hipStream_t)stream));
        return UR_OK;
    });
}

UR_API ur_status ur_beamform_adjoint(ur_context *c, const ur_grid_desc *g, const float *iq_dev, const float *g_env_dev,
                                     const float *g_iq_dev, float *g_rf_dev, void *stream) {
    return guarded(c, [&]() -> ur_status {
        if (!c->has_setup) return c->fail(UR_ERR_CALL_ORDER, "call ur_transmit_setup first");
        if (!g || !g_rf_dev) return c->fail(UR_ERR_INVALID_ARG, "grid and g_rf_dev are required");
        if ((g_env_dev == nullptr) == (g_iq_dev == nullptr))
            return c->fail(UR_ERR_INVALID_ARG, "give exactly one of g_env_dev and g_iq_dev");
        if (g_env_dev && !iq_dev) return c->fail(UR_ERR_INVALID_ARG, "the envelope adjoint needs iq_dev");
        if (g->nx < 1 || g->nz < 1 || g->nx > 65535 || g->nz > (1 << 24))
            return c->fail(UR_ERR_INVALID_ARG, "grid size out of range");
        const double gv[] = {g->x0, g->x1, g->z0, g->z1};
        if (!finite_all(gv, 4)) return c->fail(UR_ERR_INVALID_ARG, "non-finite grid value");
        if (g->apod != UR_APOD_NONE && g->apod != UR_APOD_HANN) return c->fail(UR_ERR_INVALID_ARG, "unknown apodisation");
        if (g->sector != 0 && g->sector != 1) return c->fail(UR_ERR_INVALID_ARG, "sector must be 0 or 1");
        hipStream_t s = (hipStream_t)stream;
        const int64_t E = c->probe.n_elements, npx = g->nx * g->nz;
        const float2 *giq = (const float2 *)g_iq_dev;
        if (g_env_dev) {
            ur_status st;
            if ((st = alloc(c, c->d_giq, npx * sizeof(float2)))) return st;
            HIP_TRY(c, ur_launch_env_adj((const float2 *)iq_dev, g_env_dev, (float2 *)c->d_giq.p, npx, s));
            giq = (const float2 *)c->d_giq.p;
        }
        DasParams P = das_params(c, g);
        P.rf = nullptr;
        P.iq = nullptr;
        P.env = nullptr;
        HIP_TRY(c, zero_f32(g_rf_dev, 2 * (int64_t)P.T * E * P.S, s));
        HIP_TRY(c, ur_launch_das_adj(P, giq, g_rf_dev, s));
        return UR_OK;
    });
}

UR_API ur_status ur_trace_adjoint(ur_context *c, uint64_t seed, int64_t ray_stride, int64_t ray_offset,
                                  const float *g_raw_dev, const ur_grad_desc *grads, void *stream) {
    return guarded(c, [&]() -> ur_status {
        if (!c->has_setup) return c->fail(UR_ERR_CALL_ORDER, "call ur_scene_upload and ur_transmit_setup first");
        if (!g_raw_dev || !grads) return c->fail(UR_ERR_INVALID_ARG, "g_raw_dev and grads are required");
        if (!c->acq.rough_direct_only)
            for (double r : c->rough)
                if (r > 0.0)
                    return c->fail(UR_ERR_UNSUPPORTED, "the adjoint supports rough boundaries only with their echoes "
                                                       "received by direct hits (rough_direct_only = 1)");
        if (!grads->amp && !grads->alpha && !grads->Z && !grads->sph_center && !grads->value)
            return c->fail(UR_ERR_INVALID_ARG, "no output requested");
        if (ray_stride < 1 || ray_offset < 0 || ray_offset >= ray_stride)
            return c->fail(UR_ERR_INVALID_ARG, "need ray_stride >= 1 and 0 <= ray_offset < ray_stride");
        if (grads->record_paths < 0) return c->fail(UR_ERR_INVALID_ARG, "record_paths must be >= 0");
        const int n_mat = (int)(c->mat.size() / 3);
        if (grads->alpha && n_mat > kAdjMaxMat)
            return c->fail(UR_ERR_UNSUPPORTED, "attenuation gradients support at most %d materials", kAdjMaxMat);
        hipStream_t s = (hipStream_t)stream;
        TraceParams P;
        fill_params(c, P, seed);
        const int64_t nel = c->acq.rays_per_element;
        P.stride = ray_stride;
        P.offset = ray_offset;
        P.per_el = nel > ray_offset ? (nel - ray_offset + ray_stride - 1) / ray_stride : 0;
        P.n_work = (int64_t)(P.sa ? 1 : P.T) * P.E * P.per_el;   // synthetic aperture: one element per transmit
        const double kappa = c->probe.f_c * 1e-6 * 100.0 * std::log(10.0) / 20.0;
        if (grads->amp) HIP_TRY(c, zero_f32(grads->amp, c->n_scat, s));
        if (grads->alpha) HIP_TRY(c, ur_launch_zero_f64(grads->alpha, n_mat, s));
        if (grads->value) HIP_TRY(c, ur_launch_zero_f64(grads->value, 1, s));
        if (grads->Z) HIP_TRY(c, ur_launch_zero_f64(grads->Z, n_mat, s));
        if (grads->sph_center) HIP_TRY(c, ur_launch_zero_f64(grads->sph_center, 3 * (int)c->n_sph, s));
        std::vector<AdjTangent> tans;
        if (grads->Z)
            for (int m = 0; m < n_mat; ++m) tans.push_back(AdjTangent{1, m, 0, grads->Z + m});
        if (grads->sph_center)
            for (int j = 0; j < (int)c->n_sph; ++j)
                for (int k = 0; k < 3; ++k) tans.push_back(AdjTangent{2, j, k, grads->sph_center + 3 * j + k});
        const int n_tan = (int)tans.size();
        const bool value_pass = grads->amp || grads->alpha || grads->value;
        // With tangent passes the paths go in ranges: the value pass over a
        // range records its decisions and the tangent passes replay them.
        // Element and segment indices are kept in 16 bits.
        ur_status st;
        const bool use_rec = n_tan > 0 && P.E <= 65535 && P.B < 65535;
        const size_t per_ray = (size_t)(P.B + 1) * sizeof(AdjSeg) + kAdjCapRec * sizeof(AdjCap) + 1;
        size_t free_b = 0, total_b = 0;
        HIP_TRY(c, hipMemGetInfo(&free_b, &total_b));
        const int64_t fit = std::max<int64_t>(1, (int64_t)(total_b / kAdjRecShare / per_ray));
        const int64_t range = !use_rec ? std::max<int64_t>(1, P.n_work)
                                       : std::max<int64_t>(1, std::min(P.n_work, grads->record_paths > 0
                                                                                      ? grads->record_paths
                                                                                      : fit));
        if ((st = alloc(c, c->d_adj_next, sizeof(unsigned long long)))) return st;
        if (use_rec) {
            if ((st = alloc(c, c->d_adj_seg, (size_t)range * (P.B + 1) * sizeof(AdjSeg)))) return st;
            if ((st = alloc(c, c->d_adj_cap, (size_t)range * kAdjCapRec * sizeof(AdjCap)))) return st;
            if ((st = alloc(c, c->d_adj_ncap, (size_t)range))) return st;
        }
        for (int64_t b0 = 0; b0 < P.n_work; b0 += range) {
            AdjRecord rec{0, b0, std::min(P.n_work, b0 + range), nullptr, nullptr, nullptr,
                          (unsigned long long *)c->d_adj_next.p};
            if (use_rec) {
                rec.seg = (AdjSeg *)c->d_adj_seg.p;
                rec.cap = (AdjCap *)c->d_adj_cap.p;
                rec.ncap = (unsigned char *)c->d_adj_ncap.p;
                rec.mode = 1;
            }
            if (value_pass || use_rec)
                HIP_TRY(c, ur_launch_replay(P, 0, nullptr, g_raw_dev, grads->amp, grads->alpha, grads->value, kappa, 1,
                                            rec, s));
            if (use_rec) rec.mode = 2;
            if (!tans.empty())
                HIP_TRY(c, ur_launch_replay(P, (int)tans.size(), tans.data(), g_raw_dev, nullptr, nullptr, nullptr,
                                            kappa, !grads->frozen_choice, rec, s));
        }
        return UR_OK;
    });
}

UR_API ur_status ur_trace_grad_edges(ur_context *c, uint64_t seed, int64_t ray_stride, int64_t ray_offset,
                                     const float *g_raw_dev, int32_t n_scan, double *corr_z_dev, double *corr_sph_dev,
                                     void *stream) {
    return guarded(c, [&]() -> ur_status {
        if (!c->has_setup) return c->fail(UR_ERR_CALL_ORDER, "call ur_scene_upload and ur_transmit_setup first");
        if (!g_raw_dev || (!corr_z_dev && !corr_sph_dev))
            return c->fail(UR_ERR_INVALID_ARG, "g_raw_dev and at least one output are required");
        if (n_scan < 1) return c->fail(UR_ERR_INVALID_ARG, "n_scan must be >= 1");
        if (ray_stride < 1 || ray_offset < 0 || ray_offset >= ray_stride)
            return c->fail(UR_ERR_INVALID_ARG, "need ray_stride >= 1 and 0 <= ray_offset < ray_stride");
        TraceParams P;
        fill_params(c, P, seed);
        if (P.sa || P.proposal || P.any_rough)
            return c->fail(UR_ERR_UNSUPPORTED, "the edge terms need plane-wave transmits, uniform emission and "
                                               "smooth boundaries");
        const int n_mat = (int)(c->mat.size() / 3);
        const int64_t nel = c->acq.rays_per_element;
        P.stride = ray_stride;
        P.offset = ray_offset;
        P.per_el = nel > ray_offset ? (nel - ray_offset + ray_stride - 1) / ray_stride : 0;
        P.n_work = (int64_t)P.T * P.E * P.per_el;
        hipStream_t s = (hipStream_t)stream;
        if (n_mat + 3 * (int)c->n_sph > 32)
            return c->fail(UR_ERR_UNSUPPORTED, "the edge terms support at most 32 impedances and sphere coordinates");
        if (corr_z_dev) HIP_TRY(c, ur_launch_zero_f64(corr_z_dev, n_mat, s));
        if (corr_sph_dev) HIP_TRY(c, ur_launch_zero_f64(corr_sph_dev, 3 * (int)c->n_sph, s));
        HIP_TRY(c, ur_launch_edges(P, corr_z_dev, corr_sph_dev, g_raw_dev, n_scan, s));
        return UR_OK;
    });
}

// ------------------------------------------------------------ proposal network
namespace {
constexpr int kIn = 34, kHid = 64, kOut = 1024, kParams = 77120;
constexpr int oW1 = 0, ob1 = oW1 + kIn * kHid, oW2 = ob1 + kHid, ob2 = oW2 + kHid * kHid, oW3 = ob2 + kHid,
              ob3 = oW3 + kHid * kHid, oW4 = ob3 + kHid, ob4 = oW4 + kHid * kOut;
static_assert(ob4 + kOut == kParams, "parameter layout");

ur_status mlp_forward(ur_context *c, hipStream_t s) {
    const int R = c->mlp_rows;
    const float *th = (const float *)c->d_theta.p;
    double amax = 0.0;
    for (double a : c->angles) amax = std::max(amax, std::fabs(a));
    if (amax == 0.0) amax = 1.0;
    HIP_TRY(c, ur_mlp_features((const double *)c->d_xe.p, (const double *)c->d_angles.p, (int)c->probe.n_elements,
                               (int)c->acq.n_tx, 0.5 * (double)c->probe.n_elements * c->probe.pitch, amax,
                               (const float *)c->d_rff.p, (float *)c->d_X.p, s));
    float *X = (float *)c->d_X.p, *H1 = (float *)c->d_H1.p, *H2 = (float *)c->d_H2.p, *H3 = (float *)c->d_H3.p;
    HIP_TRY(c, ur_mlp_gemm(X, kIn, 1, th + oW1, kHid, 1, H1, R, kHid, kIn, th + ob1, nullptr, 1, s));
    HIP_TRY(c, ur_mlp_gemm(H1, kHid, 1, th + oW2, kHid, 1, H2, R, kHid, kHid, th + ob2, nullptr, 1, s));
    HIP_TRY(c, ur_mlp_gemm(H2, kHid, 1, th + oW3, kHid, 1, H3, R, kHid, kHid, th + ob3, nullptr, 1, s));
    HIP_TRY(c, ur_mlp_gemm(H3, kHid, 1, th + oW4, kOut, 1, (float *)c->d_Z.p, R, kOut, kHid, th + ob4, nullptr, 0, s));
    return UR_OK;
}

// Loss and gradient of the weighted cross-entropy into grad (device).
ur_status mlp_backward(ur_context *c, const float *hist, float *grad, float *loss, hipStream_t s) {
    const int R = c->mlp_rows;
    const float *th = (const float *)c->d_theta.p;
    float *X = (float *)c->d_X.p, *H1 = (float *)c->d_H1.p, *H2 = (float *)c->d_H2.p, *H3 = (float *)c->d_H3.p;
    float *dZ = (float *)c->d_dZ.p, *d3 = (float *)c->d_dH3.p, *d2 = (float *)c->d_dH2.p, *d1 = (float *)c->d_dH1.p;
    float *tot = (float *)c->d_scal.p;
    ur_status st;
    if ((st = mlp_forward(c, s))) return st;
    HIP_TRY(c, ur_mlp_sum(hist, (int64_t)R * kOut, tot, s));
    if (loss) HIP_TRY(c, ur_mlp_fill(loss, 1, 0.f, s));
    HIP_TRY(c, ur_mlp_softmax_ce((const float *)c->d_Z.p, hist, tot, nullptr, dZ, loss, R, s));
    HIP_TRY(c, ur_mlp_gemm(H3, 1, kHid, dZ, kOut, 1, grad + oW4, kHid, kOut, R, nullptr, nullptr, 0, s));
    HIP_TRY(c, ur_mlp_colsum(dZ, R, kOut, grad + ob4, s));
    HIP_TRY(c, ur_mlp_gemm(dZ, kOut, 1, th + oW4, 1, kOut, d3, R, kHid, kOut, nullptr, H3, 0, s));
    HIP_TRY(c, ur_mlp_gemm(H2, 1, kHid, d3, kHid, 1, grad + oW3, kHid, kHid, R, nullptr, nullptr, 0, s));
    HIP_TRY(c, ur_mlp_colsum(d3, R, kHid, grad + ob3, s));
    HIP_TRY(c, ur_mlp_gemm(d3, kHid, 1, th + oW3, 1, kHid, d2, R, kHid, kHid, nullptr, H2, 0, s));
    HIP_TRY(c, ur_mlp_gemm(H1, 1, kHid, d2, kHid, 1, grad + oW2, kHid, kHid, R, nullptr, nullptr, 0, s));
    HIP_TRY(c, ur_mlp_colsum(d2, R, kHid, grad + ob2, s));
    HIP_TRY(c, ur_mlp_gemm(d2, kHid, 1, th + oW2, 1, kHid, d1, R, kHid, kHid, nullptr, H1, 0, s));
    HIP_TRY(c, ur_mlp_gemm(X, 1, kIn, d1, kHid, 1, grad + oW1, kIn, kHid, R, nullptr, nullptr, 0, s));
    HIP_TRY(c, ur_mlp_colsum(d1, R, kHid, grad + ob1, s));
    return UR_OK;
}

ur_status mlp_check(ur_context *c) {
    if (!c->has_setup) return c->fail(UR_ERR_CALL_ORDER, "call ur_transmit_setup first");
    if (!c->mlp_ready) return c->fail(UR_ERR_CALL_ORDER, "call ur_mlp_init after the transmit setup");
    return UR_OK;
}
}  // namespace

UR_API ur_status ur_mlp_init(ur_context *c, const float *params, const float *rff) {
    return guarded(c, [&]() -> ur_status {
        if (!c->has_setup) return c->fail(UR_ERR_CALL_ORDER, "call ur_transmit_setup first");
        if (!params || !rff) return c->fail(UR_ERR_INVALID_ARG, "params and rff are required");
        for (int i = 0; i < kParams; ++i)
            if (!std::isfinite(params[i])) return c->fail(UR_ERR_INVALID_ARG, "non-finite parameter %d", i);
        const int64_t R = c->acq.n_tx * c->probe.n_elements;
        if (R > (1 << 20)) return c->fail(UR_ERR_UNSUPPORTED, "at most 2^20 (transmit, element) rows");
        c->mlp_rows = (int)R;
        ur_status st;
        const size_t P = kParams * sizeof(float);
        if ((st = alloc(c, c->d_theta, P)) || (st = alloc(c, c->d_m, P)) || (st = alloc(c, c->d_v, P)) ||
            (st = alloc(c, c->d_grad, P)) || (st = alloc(c, c->d_rff, 32 * sizeof(float))) ||
            (st = alloc(c, c->d_X, R * kIn * sizeof(float))) || (st = alloc(c, c->d_H1, R * kHid * sizeof(float))) ||
            (st = alloc(c, c->d_H2, R * kHid * sizeof(float))) || (st = alloc(c, c->d_H3, R * kHid * sizeof(float))) ||
            (st = alloc(c, c->d_Z, R * kOut * sizeof(float))) || (st = alloc(c, c->d_dZ, R * kOut * sizeof(float))) ||
            (st = alloc(c, c->d_dH3, R * kHid * sizeof(float))) || (st = alloc(c, c->d_dH2, R * kHid * sizeof(float))) ||
            (st = alloc(c, c->d_dH1, R * kHid * sizeof(float))) || (st = alloc(c, c->d_scal, 64)))
            return st;
        HIP_TRY(c, hipMemcpy(c->d_theta.p, params, P, hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(c->d_rff.p, rff, 32 * sizeof(float), hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemset(c->d_m.p, 0, P));
        HIP_TRY(c, hipMemset(c->d_v.p, 0, P));
        HIP_TRY(c, hipDeviceSynchronize());
        c->mlp_step = 0;
        c->mlp_ready = true;
        return UR_OK;
    });
}

UR_API ur_status ur_mlp_get_params(ur_context *c, float *params) {
    return guarded(c, [&]() -> ur_status {
        ur_status st;
        if ((st = mlp_check(c))) return st;
        if (!params) return c->fail(UR_ERR_INVALID_ARG, "params is NULL");
        HIP_TRY(c, hipDeviceSynchronize());
        HIP_TRY(c, hipMemcpy(params, c->d_theta.p, kParams * sizeof(float), hipMemcpyDeviceToHost));
        return UR_OK;
    });
}

UR_API ur_status ur_mlp_get_state(ur_context *c, float *state, int64_t *step) {
    return guarded(c, [&]() -> ur_status {
        ur_status st;
        if ((st = mlp_check(c))) return st;
        if (!state || !step) return c->fail(UR_ERR_INVALID_ARG, "state and step are required");
        HIP_TRY(c, hipDeviceSynchronize());
        const size_t P = kParams * sizeof(float);
        HIP_TRY(c, hipMemcpy(state, c->d_theta.p, P, hipMemcpyDeviceToHost));
        HIP_TRY(c, hipMemcpy(state + kParams, c->d_m.p, P, hipMemcpyDeviceToHost));
        HIP_TRY(c, hipMemcpy(state + 2 * kParams, c->d_v.p, P, hipMemcpyDeviceToHost));
        *step = c->mlp_step;
        return UR_OK;
    });
}

UR_API ur_status ur_mlp_set_state(ur_context *c, const float *state, int64_t step) {
    return guarded(c, [&]() -> ur_status {
        ur_status st;
        if ((st = mlp_check(c))) return st;
        if (!state) return c->fail(UR_ERR_INVALID_ARG, "state is NULL");
        if (step < 0 || step > INT32_MAX) return c->fail(UR_ERR_INVALID_ARG, "step %lld out of range", (long long)step);
        for (int i = 0; i < 3 * kParams; ++i)
            if (!std::isfinite(state[i])) return c->fail(UR_ERR_INVALID_ARG, "non-finite state entry %d", i);
        for (int i = 2 * kParams; i < 3 * kParams; ++i)
            if (state[i] < 0.0f) return c->fail(UR_ERR_INVALID_ARG, "negative second moment at %d", i - 2 * kParams);
        HIP_TRY(c, hipDeviceSynchronize());
        const size_t P = kParams * sizeof(float);
        HIP_TRY(c, hipMemcpy(c->d_theta.p, state, P, hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(c->d_m.p, state + kParams, P, hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(c->d_v.p, state + 2 * kParams, P, hipMemcpyHostToDevice));
        c->mlp_step = (int)step;
        return UR_OK;
    });
}

UR_API ur_status ur_mlp_forward(ur_context *c, float *q_dev, void *stream) {
    return guarded(c, [&]() -> ur_status {
        ur_status st;
        if ((st = mlp_check(c))) return st;
        if (!q_dev) return c->fail(UR_ERR_INVALID_ARG, "q_dev is NULL");
        hipStream_t s = (hipStream_t)stream;
        if ((st = mlp_forward(c, s))) return st;
        HIP_TRY(c, ur_mlp_softmax_ce((const float *)c->d_Z.p, nullptr, nullptr, q_dev, nullptr, nullptr, c->mlp_rows, s));
        return UR_OK;
    });
}

UR_API ur_status ur_mlp_loss_grad(ur_context *c, const float *hist_dev, float *grad_dev, float *loss_dev, void *stream) {
    return guarded(c, [&]() -> ur_status {
        ur_status st;
        if ((st = mlp_check(c))) return st;
        if (!hist_dev || !grad_dev) return c->fail(UR_ERR_INVALID_ARG, "hist_dev and grad_dev are required");
        return mlp_backward(c, hist_dev, grad_dev, loss_dev, (hipStream_t)stream);
    });
}

UR_API ur_status ur_mlp_train_step(ur_context *c, const float *hist_dev, float lr, float *loss_dev, void *stream) {
    return guarded(c, [&]() -> ur_status {
        ur_status st;
        if ((st = mlp_check(c))) return st;
        if (!hist_dev) return c->fail(UR_ERR_INVALID_ARG, "hist_dev is NULL");
        if (!(lr > 0.f) || !std::isfinite(lr)) return c->fail(UR_ERR_INVALID_ARG, "learning rate must be positive");
        hipStream_t s = (hipStream_t)stream;
        if ((st = mlp_backward(c, hist_dev, (float *)c->d_grad.p, loss_dev, s))) return st;
        ++c->mlp_step;
        const double b1 = 0.9, b2 = 0.999;
        HIP_TRY(c, ur_mlp_adam((float *)c->d_theta.p, (float *)c->d_m.p, (float *)c->d_v.p, (const float *)c->d_grad.p,
                               kParams, lr, (float)b1, (float)b2, 1e-8f, (float)(1.0 - std::pow(b1, c->mlp_step)),
                               (float)(1.0 - std::pow(b2, c->mlp_step)), s));
        return UR_OK;
    });
}

UR_API ur_status ur_mlp_proposal_tables(ur_context *c, float eps, float *pdf_dev, float *cdf_dev, void *stream) {
    return guarded(c, [&]() -> ur_status {
        ur_status st;
        if ((st = mlp_check(c))) return st;
        if (!pdf_dev || !cdf_dev) return c->fail(UR_ERR_INVALID_ARG, "pdf_dev and cdf_dev are required");
        if (!(eps > 0.f && eps <= 1.f)) return c->fail(UR_ERR_INVALID_ARG, "uniform mixture weight must be in (0, 1]");
        hipStream_t s = (hipStream_t)stream;
        if ((st = mlp_forward(c, s))) return st;
        HIP_TRY(c, ur_mlp_softmax_ce((const float *)c->d_Z.p, nullptr, nullptr, (float *)c->d_dZ.p, nullptr, nullptr,
                                     c->mlp_rows, s));
        HIP_TRY(c, ur_mlp_tables((const float *)c->d_dZ.p, c->mlp_rows, eps, pdf_dev, cdf_dev, s));
        return UR_OK;
    });
}

UR_API ur_status ur_set_record(ur_context *c, void *rec_dev, int64_t cap, unsigned long long *count_dev) {
    return guarded(c, [&]() -> ur_status {
        if (rec_dev && (cap < 1 || !count_dev)) return c->fail(UR_ERR_INVALID_ARG, "need cap >= 1 and a count pointer");
        c->rec = (RecordEntry *)rec_dev;
        c->rec_cap = rec_dev ? cap : 0;
        c->rec_count = rec_dev ? count_dev : nullptr;
        return UR_OK;
    });
}

UR_API ur_status ur_set_cost_histogram(ur_context *c, float *cost_dev) {
    return guarded(c, [&]() -> ur_status {
        c->cost = cost_dev;
        return UR_OK;
    });
}

UR_API ur_status ur_record_reweight(ur_context *c, void *rec_dev, int64_t n_rec, const float *cost_dev,
                                    double rays_per_row, void *stream) {
    return guarded(c, [&]() -> ur_status {
        if (!c->has_setup) return c->fail(UR_ERR_CALL_ORDER, "call ur_transmit_setup first");
        if ((n_rec > 0 && !rec_dev) || n_rec < 0 || !cost_dev || !(rays_per_row > 0))
            return c->fail(UR_ERR_INVALID_ARG, "need records, a cost histogram and rays_per_row > 0");
        const int64_t bins = c->acq.n_tx * c->probe.n_elements * kOut;
        ur_status st;
        if ((st = alloc(c, c->d_s2, (size_t)bins * sizeof(float)))) return st;
        HIP_TRY(c, ur_mlp_record_reweight((RecordEntry *)rec_dev, n_rec, cost_dev, rays_per_row, (float *)c->d_s2.p,
                                          bins, (hipStream_t)stream));
        return UR_OK;
    });
}

UR_API ur_status ur_record_histogram(ur_context *c, const void *rec_dev, int64_t n_rec, int64_t batch, uint64_t seed,
                                     uint32_t step, float *hist_dev, void *stream) {
    return guarded(c, [&]() -> ur_status {
        if (!c->has_setup) return c->fail(UR_ERR_CALL_ORDER, "call ur_transmit_setup first");
        if (!hist_dev || (n_rec > 0 && !rec_dev) || n_rec < 0 || batch < 0)
            return c->fail(UR_ERR_INVALID_ARG, "bad record or histogram buffer");
        const int64_t bins = c->acq.n_tx * c->probe.n_elements * kOut;
        HIP_TRY(c, ur_mlp_record_hist((const RecordEntry *)rec_dev, n_rec, batch, seed, step, bins, hist_dev,
                                      (hipStream_t)stream));
        return UR_OK;
    });
}

}  // extern "C"
