// k_prep.hip -- column standardisation used before the simulations of
// Section V-C: every feature is centred to zero median and scaled to unit
// variance.  One workgroup per column: the median is found exactly by a
// four-pass radix selection on order-preserving integer keys of the FP32
// values (an LDS histogram of one byte per pass), the variance by a
// compensated two-pass sum in a fixed order.
#include "common.hpp"
#include "kernels.hpp"

namespace gmds {

namespace {

constexpr int kPW = 256;

// Order-preserving map of FP32 bits to uint32 (negative values reversed).
__device__ __forceinline__ uint32_t fkey(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float funkey(uint32_t k) {
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(u);
}

// k-th smallest value (0-based) of column `col`.
__device__ float select_kth(const float* __restrict__ X, int64_t n, int64_t ldx, int64_t col, int64_t k,
                            uint32_t* hist, uint32_t* sh) {
    uint32_t prefix = 0u, mask = 0u;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        for (int b = threadIdx.x; b < 256; b += kPW) hist[b] = 0u;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < n; i += kPW) {
            const uint32_t key = fkey(X[i * ldx + col]);
            if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t cum = 0;
            int b = 0;
            for (; b < 255; ++b) {
                if (cum + (int64_t)hist[b] > k) break;
                cum += hist[b];
            }
            sh[0] = (uint32_t)b;
            sh[1] = (uint32_t)(k - cum);
        }
        __syncthreads();
        prefix |= sh[0] << shift;
        mask |= 255u << shift;
        k = (int64_t)sh[1];
        __syncthreads();
    }
    return funkey(prefix);
}

__device__ Comp block_sum(Comp acc, float* lds) {
    const int t = threadIdx.x;
    lds[2 * t] = acc.hi;
    lds[2 * t + 1] = acc.lo;
    __syncthreads();
    for (int st = kPW / 2; st > 0; st >>= 1) {
        if (t < st) {
            Comp a, b;
            a.hi = lds[2 * t];
            a.lo = lds[2 * t + 1];
            b.hi = lds[2 * (t + st)];
            b.lo = lds[2 * (t + st) + 1];
            a.add(b);
            lds[2 * t] = a.hi;
            lds[2 * t + 1] = a.lo;
        }
        __syncthreads();
    }
    Comp r;
    r.hi = lds[0];
    r.lo = lds[1];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kPW) void k_standardise(const float* __restrict__ X, int64_t n, int64_t ldx,
                                                     float* __restrict__ Y, int64_t ldy, float* __restrict__ stats) {
    __shared__ uint32_t hist[256];
    __shared__ uint32_t sh[2];
    __shared__ float lds[2 * kPW];
    const int64_t col = blockIdx.x;
    // median: the middle order statistic, or the mean of the two middle ones
    const float lo = select_kth(X, n, ldx, col, (n - 1) / 2, hist, sh);
    const float hi = (n % 2) ? lo : select_kth(X, n, ldx, col, n / 2, hist, sh);
    const float med = (n % 2) ? lo : 0.5f * lo + 0.5f * hi;
    // population variance about the mean
    Comp s;
    for (int64_t i = threadIdx.x; i < n; i += kPW) s.add(X[i * ldx + col]);
    const float mean = block_sum(s, lds).value() / (float)n;
    Comp v;
    for (int64_t i = threadIdx.x; i < n; i += kPW) {
        const float d = X[i * ldx + col] - mean;
        v.add(d * d);
    }
    const float var = block_sum(v, lds).value() / (float)n;
    const float sd = sqrtf(var);
    const float inv = (sd > 0.f) ? 1.f / sd : 1.f;
    for (int64_t i = threadIdx.x; i < n; i += kPW) Y[i * ldy + col] = (X[i * ldx + col] - med) * inv;
    if (stats && threadIdx.x == 0) {
        stats[2 * col] = med;
        stats[2 * col + 1] = sd;
    }
}

}  // namespace

hipError_t launch_standardise(const float* X, int64_t n, int m, int64_t ldx, float* Y, int64_t ldy, float* stats,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_standardise, dim3((unsigned)m), dim3(kPW), 0, s, X, n, ldx, Y, ldy, stats);
    return hipGetLastError();
}

}  // namespace gmds
