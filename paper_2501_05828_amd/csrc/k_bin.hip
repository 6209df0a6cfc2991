// Deterministic binning of the channel data (UltraRay, arXiv 2501.05828,
// Sec. 2.3, Phase Calculation): the trace stages its records, and they are
// binned here with exact integer arithmetic, so that the channel data do not
// depend on the order in which the records arrived (float atomics round in
// arrival order).  Every bin contribution (nearest: v into floor(x); linear:
// (1 - f) v and f v into the two neighbouring samples) is rounded to a
// 64-bit integer at one scale 2^k per trace, chosen from the largest |v| M
// and the record count n so that no bin can overflow (n M 2^k < 2^61):
// integer addition is associative, and the rounding error of a contribution
// is at most 2^-k-1 < n M 2^-61, about 1e-14 of M for 1e5 records.  The
// bins are then scaled back to FP32.
#include <algorithm>

#include "ur_internal.h"
#include "ultraray.h"

namespace {
using namespace ur;

__device__ __forceinline__ int64_t det_n(const unsigned long long *ctr, int64_t cap) {
    const int64_t n = (int64_t)ctr[0];
    return n < cap ? n : cap;
}

// 2^k with n M 2^k < 2^61 (1 if there is nothing to bin).
__device__ __forceinline__ double det_scale(const unsigned long long *ctr, int64_t cap) {
    const double M = __longlong_as_double((long long)ctr[1]);
    const int64_t n = det_n(ctr, cap);
    if (!(M > 0.0) || n <= 0) return 1.0;
    return ldexp(1.0, 60 - ilogb(M * (double)n));
}

__global__ void k_det_max(const DetRecord *r, int64_t cap, unsigned long long *ctr) {
    const int64_t n = det_n(ctr, cap);
    unsigned long long m = 0ull;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long b = (unsigned long long)__double_as_longlong(fabs(r[i].v));
        m = b > m ? b : m;   // |v| >= 0: the bit patterns order as the values
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off, 64);
        m = o > m ? o : m;
    }
    if ((threadIdx.x & 63) == 0 && m) atomicMax(ctr + 1, m);
}

__global__ void k_det_bin(const DetRecord *r, int64_t cap, const unsigned long long *ctr, long long *bins, int S,
                          int binning) {
    const int64_t n = det_n(ctr, cap);
    const double scale = det_scale(ctr, cap);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const DetRecord q = r[i];
        long long *ch = bins + q.ch * S;
        if (binning == UR_BIN_NEAREST) {
            const int k = (int)floor(q.x);
            if (k >= 0 && k < S) atomicAdd((unsigned long long *)(ch + k), (unsigned long long)llrint(q.v * scale));
        } else {
            const double tau = q.x - 0.5, f0 = floor(tau), f = tau - f0;
            const int k = (int)f0;
            if (k >= 0 && k < S)
                atomicAdd((unsigned long long *)(ch + k), (unsigned long long)llrint((1.0 - f) * q.v * scale));
            if (k + 1 >= 0 && k + 1 < S)
                atomicAdd((unsigned long long *)(ch + k + 1), (unsigned long long)llrint(f * q.v * scale));
        }
    }
}

__global__ void k_det_out(const long long *bins, int64_t cap, const unsigned long long *ctr, float *out, int64_t n) {
    const double inv = 1.0 / det_scale(ctr, cap);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)((double)bins[i] * inv);
}
}  // namespace

hipError_t ur_launch_det_bin(const ur::DetRecord *rec, int64_t cap, unsigned long long *ctr, long long *bins,
                             float *ch_raw, int64_t n_ch, int S, int binning, hipStream_t s) {
    const int64_t n_out = n_ch * S;
    const unsigned g_rec = (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (cap + 255) / 256));
    const unsigned g_out = (unsigned)std::min<int64_t>(8192, std::max<int64_t>(1, (n_out + 255) / 256));
    hipLaunchKernelGGL(k_det_max, dim3(g_rec), dim3(256), 0, s, rec, cap, ctr);
    hipLaunchKernelGGL(k_det_bin, dim3(g_rec), dim3(256), 0, s, rec, cap, ctr, bins, S, binning);
    hipLaunchKernelGGL(k_det_out, dim3(g_out), dim3(256), 0, s, bins, cap, ctr, ch_raw, n_out);
    return hipGetLastError();
}
