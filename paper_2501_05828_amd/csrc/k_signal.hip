// Signal processing on gfx950: pulse shaping (Eq. 14), plane-wave
// delay-and-sum with coherent compounding, envelope and log compression
// (UltraRay, arXiv 2501.05828, Sec. 2.3 "Phase Calculation and Signal
// Processing").
#include <algorithm>

#include "ur_internal.h"

namespace {
using namespace ur;

constexpr int kFirTile = 256;
constexpr int kMaxHalfTaps = 512;

// ch_rf[ch][n] = sum_{|m|<=K} h[m] ch_raw[ch][n-m].  One block filters a
// 256-sample tile of one channel; the tile plus its 2K halo is staged in LDS
// with coalesced loads, taps sit in LDS, every lane produces one complex
// output.
__global__ __launch_bounds__(kFirTile) void k_pulse(const float *__restrict__ raw, float2 *__restrict__ rf,
                                                     const float2 *__restrict__ taps, int K, int S) {
    __shared__ float xs[kFirTile + 2 * kMaxHalfTaps];
    __shared__ float2 hs[2 * kMaxHalfTaps + 1];
    const int64_t ch = blockIdx.y;
    const int n0 = blockIdx.x * kFirTile;
    const float *x = raw + ch * S;
    for (int i = threadIdx.x; i < kFirTile + 2 * K; i += kFirTile) {
        const int n = n0 - K + i;
        xs[i] = (n >= 0 && n < S) ? x[n] : 0.0f;
    }
    for (int i = threadIdx.x; i < 2 * K + 1; i += kFirTile) hs[i] = taps[i];
    __syncthreads();
    const int n = n0 + threadIdx.x;
    if (n >= S) return;
    float re = 0.0f, im = 0.0f;
    // output n reads input n - m = xs[threadIdx.x + K - m]
    for (int m = -K; m <= K; ++m) {
        const float v = xs[threadIdx.x + K - m];
        const float2 h = hs[m + K];
        re = fmaf(h.x, v, re);
        im = fmaf(h.y, v, im);
    }
    rf[ch * S + n] = make_float2(re, im);
}

// Pixel position: a Cartesian grid point, or on a sector grid the point at
// angle x0 + ix dx and depth z0 + iz dz along the ray from the centre of
// curvature (0, 0, -R): (R + r) (sin phi, cos phi) - (0, R).
__device__ __forceinline__ void das_pixel(const DasParams &p, int ix, int iz, double &x, double &z) {
    if (p.sector) {
        double sp, cp;
        sincos(p.x0 + (double)ix * p.dx, &sp, &cp);
        const double r = p.radius + (p.z0 + (double)iz * p.dz);
        x = r * sp;
        z = r * cp - p.radius;
    } else {
        x = p.x0 + (double)ix * p.dx;
        z = p.z0 + (double)iz * p.dz;
    }
}

// A fractional sample index split into its floor (exact, FP64) and its
// fraction in [0, 1) (FP32).  Indices far outside any record are clamped,
// so the conversion stays within int range; they fail the range test.
struct SplitIdx {
    int n;
    float f;
};
__device__ __forceinline__ SplitIdx split_idx(double v) {
    v = fmin(fmax(v, -1073741824.0), 1073741824.0);
    const double fl = floor(v);
    return SplitIdx{(int)fl, (float)(v - fl)};
}

// The DAS sample index of one (pixel, transmit, element) term is the sum of
// a transmit part t_tx fs (per pixel and transmit) and a receive part
// t_rx fs (per pixel and element), each split as above: floor parts add
// exactly and the two fractions add in FP32 (error below 2.4e-7 samples), so
// i0 = floor of the FP64 sum except within that distance of an integer,
// where linear interpolation is continuous.  Returns the interpolation
// weight of sample i0 + 1 and whether 0 <= i0 < S - 1.
__device__ __forceinline__ bool das_term_index(SplitIdx rx, SplitIdx tx, int S, int &i0, float &fr) {
    const float f = rx.f + tx.f;          // in [0, 2)
    // (the hardware fraction f - floor(f): exact here, f or f - 1)
    fr = __builtin_amdgcn_fractf(f);
    i0 = rx.n + tx.n + (f >= 1.0f ? 1 : 0);
    return (unsigned)i0 < (unsigned)(S - 1);
}

__device__ __forceinline__ SplitIdx das_rx(const DasParams &p, double x, double z, int e) {
    const double dxe = x - p.xe[e];
    // (elements off z = 0 only on a convex array)
    const double dze = p.ze ? z - p.ze[e] : z;
    return split_idx(sqrt(dxe * dxe + dze * dze) * p.fs_over_c0);
}

__device__ __forceinline__ SplitIdx das_tx(const DasParams &p, double x, double z, int tx) {
    const double4 c = p.txc[tx];
    return split_idx(x * c.x + z * c.y + c.z);
}

// Buffer resource word 3 of a raw (unformatted, unswizzled) buffer on gfx9.
constexpr int kRawBufferWord3 = 0x00020000;

// Delay-and-sum over K transmits t0 .. t0 + K - 1 of one pixel: for every
// element, the K gathers of the two neighbouring complex samples are issued
// together, then interpolated and summed, and the sum is weighted by the
// element's apodisation.  Each gather is one 16-byte buffer load through a
// resource spanning exactly the channel's S samples (its base is the same for
// the whole wavefront, so the lane adds only a 32-bit offset).  A term whose
// index is outside the record loads from offset 2^31, beyond the resource,
// where the hardware returns zeros: it adds nothing, whatever its weights.
template <int K>
__device__ __forceinline__ void das_transmits(const DasParams &p, double x, double z, int t0, float &re, float &im) {
    SplitIdx tt[K];
#pragma unroll
    for (int k = 0; k < K; ++k) tt[k] = das_tx(p, x, z, t0 + k);
    const int64_t tstride = (int64_t)p.E * p.S;
    for (int e = 0; e < p.E; ++e) {
        const SplitIdx rx = das_rx(p, x, z, e);
        const float2 *ch = p.rf + ((int64_t)t0 * p.E + e) * p.S;
        float2 v0[K], v1[K], wt[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            int i0;
            float fr;
            const bool in = das_term_index(rx, tt[k], p.S, i0, fr);
            const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<float2 *>(ch + k * tstride), (short)0, p.S * 8, kRawBufferWord3);
            const auto q = __builtin_amdgcn_raw_buffer_load_b128(r, (int)(in ? (uint32_t)i0 * 8u : 0x80000000u), 0, 0);
            v0[k] = make_float2(__uint_as_float(q[0]), __uint_as_float(q[1]));
            v1[k] = make_float2(__uint_as_float(q[2]), __uint_as_float(q[3]));
            wt[k] = make_float2(1.0f - fr, fr);
        }
        float er = 0.0f, ei = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            er = fmaf(wt[k].x, v0[k].x, fmaf(wt[k].y, v1[k].x, er));
            ei = fmaf(wt[k].x, v0[k].y, fmaf(wt[k].y, v1[k].y, ei));
        }
        const float a = p.apod[e];
        re = fmaf(a, er, re);
        im = fmaf(a, ei, im);
    }
}

// Delay-and-sum with coherent compounding (one lane per pixel).  A block of
// 256 lanes covers a 16 x 16 tile of the image and each wavefront an 8 x 8
// sub-tile (8 consecutive depths per lateral position), so the samples that
// one gather of a wavefront touches lie within a few cache lines.  The
// transmits are taken in register batches of 11 and one batch of the rest;
// the receive delay (one FP64 square root per pixel and element) is formed
// once per batch.  The interpolation and accumulation are FP32.
constexpr int kDasTile = 16;
__global__ __launch_bounds__(256) void k_das(DasParams p) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int ix = blockIdx.y * kDasTile + (w & 1) * 8 + (l >> 3);
    const int iz = blockIdx.x * kDasTile + (w >> 1) * 8 + (l & 7);
    if (ix >= p.nx || iz >= p.nz) return;   // (no block-wide synchronisation below)
    double x, z;
    das_pixel(p, ix, iz, x, z);
    float re = 0.0f, im = 0.0f;
    int t0 = 0;
    for (; t0 + 11 <= p.T; t0 += 11) das_transmits<11>(p, x, z, t0, re, im);
    // the remaining transmits in one batch (one receive delay per element)
    switch (p.T - t0) {
    case 10: das_transmits<10>(p, x, z, t0, re, im); break;
    case 9: das_transmits<9>(p, x, z, t0, re, im); break;
    case 8: das_transmits<8>(p, x, z, t0, re, im); break;
    case 7: das_transmits<7>(p, x, z, t0, re, im); break;
    case 6: das_transmits<6>(p, x, z, t0, re, im); break;
    case 5: das_transmits<5>(p, x, z, t0, re, im); break;
    case 4: das_transmits<4>(p, x, z, t0, re, im); break;
    case 3: das_transmits<3>(p, x, z, t0, re, im); break;
    case 2: das_transmits<2>(p, x, z, t0, re, im); break;
    case 1: das_transmits<1>(p, x, z, t0, re, im); break;
    default: break;
    }
    const int64_t o = (int64_t)ix * p.nz + iz;
    if (p.iq) p.iq[o] = make_float2(re, im);
    if (p.env) p.env[o] = sqrtf(re * re + im * im);
}

// Non-negative floats order like their bit patterns.
__global__ void k_absmax(const float *env, int64_t n, unsigned int *max_bits) {
    __shared__ unsigned int red[256];
    unsigned int m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, __float_as_uint(fmaxf(env[i], 0.0f)));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(max_bits, red[0]);
}

__global__ void k_logcompress(const float *env, float *bmode, int64_t n, float dr, const unsigned int *max_bits) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float mx = __uint_as_float(*max_bits);
    const float v = env[i];
    float db = (mx > 0.0f && v > 0.0f) ? 20.0f * log10f(v / mx) : -dr;
    bmode[i] = db < -dr ? -dr : db;
}

__global__ void k_zero_u32(unsigned int *p) { *p = 0u; }

// ------------------------------------------------------------- adjoints
// Envelope |IQ|: dL/dIQ = dL/denv * IQ / |IQ| (zero where |IQ| = 0).
__global__ void k_env_adj(const float2 *iq, const float *g_env, float2 *g_iq, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 z = iq[i];
    const float a = sqrtf(z.x * z.x + z.y * z.y);
    const float s = a > 0.f ? g_env[i] / a : 0.f;
    g_iq[i] = make_float2(s * z.x, s * z.y);
}

// Transpose of the delay-and-sum: every (pixel, transmit, element) term
// w_e ((1 - f) rf[i0] + f rf[i0 + 1]) scatters w_e (1 - f) g and w_e f g
// into the channel-data adjoint (float atomics; same indices as k_das).
__global__ __launch_bounds__(256) void k_das_adj(DasParams p, const float2 *g_iq, float *g_rf) {
    const int iz = blockIdx.x * blockDim.x + threadIdx.x;
    const int ix = blockIdx.y;
    if (iz >= p.nz) return;
    const float2 g = g_iq[(int64_t)ix * p.nz + iz];
    if (g.x == 0.f && g.y == 0.f) return;
    double x, z;
    das_pixel(p, ix, iz, x, z);
    for (int e = 0; e < p.E; ++e) {
        const SplitIdx rx = das_rx(p, x, z, e);
        const float a = p.apod[e];
        for (int tx = 0; tx < p.T; ++tx) {
            int i0;
            float fr;
            if (!das_term_index(rx, das_tx(p, x, z, tx), p.S, i0, fr)) continue;
            float *s = g_rf + 2 * (((int64_t)tx * p.E + e) * p.S + i0);
            const float w0 = a * (1.f - fr), w1 = a * fr;
            unsafeAtomicAdd(s, w0 * g.x);
            unsafeAtomicAdd(s + 1, w0 * g.y);
            unsafeAtomicAdd(s + 2, w1 * g.x);
            unsafeAtomicAdd(s + 3, w1 * g.y);
        }
    }
}

// Transpose of the pulse convolution: g_raw[k] = sum_m Re(h[m]) g_re[k + m]
// + Im(h[m]) g_im[k + m] (a correlation), staged like k_pulse.
__global__ __launch_bounds__(kFirTile) void k_pulse_adj(const float2 *__restrict__ g_rf, float *__restrict__ g_raw,
                                                        const float2 *__restrict__ taps, int K, int S) {
    __shared__ float2 gs[kFirTile + 2 * kMaxHalfTaps];
    __shared__ float2 hs[2 * kMaxHalfTaps + 1];
    const int64_t ch = blockIdx.y;
    const int n0 = blockIdx.x * kFirTile;
    const float2 *g = g_rf + ch * S;
    for (int i = threadIdx.x; i < kFirTile + 2 * K; i += kFirTile) {
        const int n = n0 - K + i;
        gs[i] = (n >= 0 && n < S) ? g[n] : make_float2(0.f, 0.f);
    }
    for (int i = threadIdx.x; i < 2 * K + 1; i += kFirTile) hs[i] = taps[i];
    __syncthreads();
    const int k = n0 + threadIdx.x;
    if (k >= S) return;
    float acc = 0.f;
    for (int m = -K; m <= K; ++m) {
        const float2 v = gs[threadIdx.x + K + m];
        const float2 h = hs[m + K];
        acc = fmaf(h.x, v.x, fmaf(h.y, v.y, acc));
    }
    g_raw[ch * S + k] = acc;
}

}  // namespace

hipError_t ur_launch_pulse(const float *raw, float2 *rf, const float2 *taps, int K, int64_t n_ch, int S,
                           hipStream_t s) {
    if (K > kMaxHalfTaps) return hipErrorInvalidValue;
    if (n_ch <= 0 || S <= 0) return hipSuccess;
    for (int64_t c0 = 0; c0 < n_ch; c0 += 65535) {   // grid.y is limited to 65535 channels per launch
        const int64_t nc = std::min<int64_t>(65535, n_ch - c0);
        dim3 grid((unsigned)((S + kFirTile - 1) / kFirTile), (unsigned)nc);
        hipLaunchKernelGGL(k_pulse, grid, dim3(kFirTile), 0, s, raw + c0 * S, rf + c0 * S, taps, K, S);
    }
    return hipGetLastError();
}

hipError_t ur_launch_env_adj(const float2 *iq, const float *g_env, float2 *g_iq, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_env_adj, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, iq, g_env, g_iq, n);
    return hipGetLastError();
}

hipError_t ur_launch_das_adj(const ur::DasParams &p, const float2 *g_iq, float *g_rf, hipStream_t s) {
    dim3 grid((unsigned)((p.nz + 255) / 256), (unsigned)p.nx);
    hipLaunchKernelGGL(k_das_adj, grid, dim3(256), 0, s, p, g_iq, g_rf);
    return hipGetLastError();
}

hipError_t ur_launch_pulse_adj(const float2 *g_rf, float *g_raw, const float2 *taps, int K, int64_t n_ch, int S,
                               hipStream_t s) {
    if (K > kMaxHalfTaps) return hipErrorInvalidValue;
    if (n_ch <= 0 || S <= 0) return hipSuccess;
    for (int64_t c0 = 0; c0 < n_ch; c0 += 65535) {
        const int64_t nc = std::min<int64_t>(65535, n_ch - c0);
        dim3 grid((unsigned)((S + kFirTile - 1) / kFirTile), (unsigned)nc);
        hipLaunchKernelGGL(k_pulse_adj, grid, dim3(kFirTile), 0, s, g_rf + c0 * S, g_raw + c0 * S, taps, K, S);
    }
    return hipGetLastError();
}

hipError_t ur_launch_das(const ur::DasParams &p, hipStream_t s) {
    if (p.nx <= 0 || p.nz <= 0) return hipSuccess;
    dim3 grid((unsigned)((p.nz + kDasTile - 1) / kDasTile), (unsigned)((p.nx + kDasTile - 1) / kDasTile));
    hipLaunchKernelGGL(k_das, grid, dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t ur_launch_bmode(const float *env, float *bmode, int64_t n, float dr_db, unsigned int *max_bits,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, max_bits);
    const int64_t blocks = std::min<int64_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(k_absmax, dim3((unsigned)blocks), dim3(256), 0, s, env, n, max_bits);
    hipLaunchKernelGGL(k_logcompress, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, env, bmode, n, dr_db,
                       max_bits);
    return hipGetLastError();
}

// ------------------------------------------- synthetic-aperture synthesis
// Steered plane waves from element-by-element data: each output sample sums
// over the emitting elements the element's channel shifted by its steering
// delay (Sec. 2.3, Fig. 3) times fs, linearly interpolated, in FP64.  The
// delay is (x_e - x_ref) sin(theta) / c0 on a linear array and
// (x_e sin(theta) + z_e cos(theta) - min over elements) / c0 on a convex one.  One thread per output sample; for each
// emitting element the threads of a block read neighbouring samples of one
// channel.
namespace {
constexpr int kSynthMaxAngles = 128;   // 2 KB of kernel arguments
struct SynthAngles {
    double st[kSynthMaxAngles];     // sin(theta_k)
    double ct[kSynthMaxAngles];     // cos(theta_k)
    double ref[kSynthMaxAngles];    // linear: x of the first-firing element; convex: min_e k.c_e
};

__global__ __launch_bounds__(256) void k_synth(const float *sa, int E, int S, const double *xe_tab,
                                               const double *ze_tab, double c0, double fs, SynthAngles A,
                                               float *out) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    const int er = blockIdx.y, k = blockIdx.z;
    if (s >= S) return;
    double acc = 0.0;
    for (int e = 0; e < E; ++e) {
        const double xe = xe_tab[e];
        const double sh = ze_tab ? (xe * A.st[k] + ze_tab[e] * A.ct[k] - A.ref[k]) / c0 * fs
                                 : (xe - A.ref[k]) * A.st[k] / c0 * fs;
        const double u = (double)s - sh, f0 = floor(u), f = u - f0;
        const int i0 = (int)f0;
        const float *x = sa + ((int64_t)e * E + er) * S;
        const double v0 = (i0 >= 0 && i0 < S) ? (double)x[i0] : 0.0;
        const double v1 = (i0 + 1 >= 0 && i0 + 1 < S) ? (double)x[i0 + 1] : 0.0;
        acc += (1.0 - f) * v0 + f * v1;
    }
    out[((int64_t)k * E + er) * S + s] = (float)acc;
}
}  // namespace

hipError_t ur_launch_synth_angles(const float *sa, const double *angles, int n_ang, int E, int S,
                                  const double *xe_host, const double *ze_host, const double *xe_dev,
                                  const double *ze_dev, double c0, double fs, float *out, hipStream_t s) {
    if (n_ang <= 0 || E <= 0 || S <= 0) return hipSuccess;
    if (n_ang > kSynthMaxAngles || E > 65535) return hipErrorInvalidValue;
    SynthAngles A;
    for (int k = 0; k < n_ang; ++k) {
        A.st[k] = std::sin(angles[k]);
        A.ct[k] = std::cos(angles[k]);
        if (ze_host) {
            double ref = INFINITY;
            for (int e = 0; e < E; ++e) ref = std::min(ref, xe_host[e] * A.st[k] + ze_host[e] * A.ct[k]);
            A.ref[k] = ref;
        } else {
            A.ref[k] = A.st[k] >= 0 ? xe_host[0] : xe_host[E - 1];
        }
    }
    dim3 grid((unsigned)((S + 255) / 256), (unsigned)E, (unsigned)n_ang);
    hipLaunchKernelGGL(k_synth, grid, dim3(256), 0, s, sa, E, S, xe_dev, ze_host ? ze_dev : nullptr, c0, fs, A, out);
    return hipGetLastError();
}

// ------------------------------------------------------- scan conversion
// Sector image [np][nr] (angle-major, as the sector grid of k_das) resampled
// onto a Cartesian grid [nx][nz]: each pixel's polar coordinates about the
// centre of curvature (0, 0, -R), phi = atan2(x, z + R) and
// r = |(x, z + R)| - R, index the sector grid; the value is the bilinear
// blend of the four surrounding samples (weights and blend in FP64), and
// pixels outside the sector's closed (phi, r) rectangle take `fill`.  One
// lane per pixel, lanes of a wavefront down one column.
namespace {
struct ScanParams {
    int np, nr, nx, nz;
    double radius, p0, dp, r0, dr, x0, dx, z0, dz;
    float fill;
};

__global__ __launch_bounds__(256) void k_scan_convert(ScanParams q, const float *__restrict__ img,
                                                      float *__restrict__ out) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (l >= q.nz) return;
    const double x = q.x0 + (double)k * q.dx, zc = q.z0 + (double)l * q.dz + q.radius;
    const double fi = (atan2(x, zc) - q.p0) / q.dp, fj = (sqrt(x * x + zc * zc) - q.radius - q.r0) / q.dr;
    float v = q.fill;
    if (fi >= 0.0 && fi <= (double)(q.np - 1) && fj >= 0.0 && fj <= (double)(q.nr - 1)) {
        const int i0 = min((int)floor(fi), q.np - 2), j0 = min((int)floor(fj), q.nr - 2);
        const double a = fi - (double)i0, b = fj - (double)j0;
        const float *s0 = img + (int64_t)i0 * q.nr + j0, *s1 = s0 + q.nr;
        v = (float)((1.0 - a) * ((1.0 - b) * (double)s0[0] + b * (double)s0[1]) +
                    a * ((1.0 - b) * (double)s1[0] + b * (double)s1[1]));
    }
    out[(int64_t)k * q.nz + l] = v;
}
}  // namespace

hipError_t ur_launch_scan_convert(double radius, int np, int nr, double p0, double p1, double r0, double r1,
                                  const float *img, int nx, int nz, double x0, double x1, double z0, double z1,
                                  float fill, float *out, hipStream_t s) {
    if (np < 2 || nr < 2 || nx < 1 || nz < 1) return hipErrorInvalidValue;
    ScanParams q;
    q.np = np;
    q.nr = nr;
    q.nx = nx;
    q.nz = nz;
    q.radius = radius;
    q.p0 = p0;
    q.dp = (p1 - p0) / (double)(np - 1);
    q.r0 = r0;
    q.dr = (r1 - r0) / (double)(nr - 1);
    q.x0 = x0;
    q.dx = nx > 1 ? (x1 - x0) / (double)(nx - 1) : 0.0;
    q.z0 = z0;
    q.dz = nz > 1 ? (z1 - z0) / (double)(nz - 1) : 0.0;
    q.fill = fill;
    dim3 grid((unsigned)((nz + 255) / 256), (unsigned)nx);
    hipLaunchKernelGGL(k_scan_convert, grid, dim3(256), 0, s, q, img, out);
    return hipGetLastError();
}
