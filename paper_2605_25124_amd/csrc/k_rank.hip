// k_rank.hip -- doubled midranks of the coordinates of each row (Definition 1
// with the tie rule of Section III-A):
//     t_c = 2 * #{c' : v_c' < v_c} + #{c' : v_c' == v_c} + 1.
// Each thread counts for its own coordinates against the whole row, staged in
// LDS so that the threads of a row read the same word at the same time
// (broadcast).  The result is an integer function of FP32 comparisons, so it is
// bit-exact by construction.
#include "common.hpp"
#include "kernels.hpp"

namespace gmds {

constexpr int kRWG = 256;

// d <= 256: 256 / DP rows per workgroup (DP = d rounded up to a power of two).
__global__ __launch_bounds__(kRWG) void k_rank_small(const float* __restrict__ V, int64_t rows, int d, int dp,
                                                     int64_t ldv, int32_t* __restrict__ t, int64_t ldr) {
    __shared__ float row[kRWG];
    const int rpb = kRWG / dp;
    const int lr = threadIdx.x / dp;
    const int c = threadIdx.x % dp;
    const int64_t r = (int64_t)blockIdx.x * rpb + lr;
    const bool live = (r < rows) && (c < d);
    row[threadIdx.x] = live ? V[r * ldv + c] : 0.f;
    __syncthreads();
    if (!live) return;
    const float x = row[threadIdx.x];
    const float* rw = row + lr * dp;
    int less = 0, eq = 0;
    for (int k = 0; k < d; ++k) {
        const float y = rw[k];
        less += (y < x) ? 1 : 0;
        eq += (y == x) ? 1 : 0;
    }
    t[r * ldr + c] = 2 * less + eq + 1;
}

// d > 256: one row per workgroup; each thread owns up to 8 coordinates per
// batch and the row streams through LDS in chunks.
constexpr int kRankChunk = 4096;
constexpr int kRankEPT = 8;

__global__ __launch_bounds__(kRWG) void k_rank_large(const float* __restrict__ V, int d, int64_t ldv,
                                                     int32_t* __restrict__ t, int64_t ldr) {
    __shared__ float chunk[kRankChunk];
    const int64_t r = blockIdx.x;
    const float* src = V + r * ldv;
    for (int base = 0; base < d; base += kRWG * kRankEPT) {
        float x[kRankEPT];
        int less[kRankEPT], eq[kRankEPT];
#pragma unroll
        for (int e = 0; e < kRankEPT; ++e) {
            const int c = base + e * kRWG + threadIdx.x;
            x[e] = (c < d) ? src[c] : 0.f;
            less[e] = 0;
            eq[e] = 0;
        }
        for (int c0 = 0; c0 < d; c0 += kRankChunk) {
            const int len = (d - c0) < kRankChunk ? (d - c0) : kRankChunk;
            __syncthreads();
            for (int k = threadIdx.x; k < len; k += kRWG) chunk[k] = src[c0 + k];
            __syncthreads();
            for (int k = 0; k < len; ++k) {
                const float y = chunk[k];
#pragma unroll
                for (int e = 0; e < kRankEPT; ++e) {
                    less[e] += (y < x[e]) ? 1 : 0;
                    eq[e] += (y == x[e]) ? 1 : 0;
                }
            }
        }
#pragma unroll
        for (int e = 0; e < kRankEPT; ++e) {
            const int c = base + e * kRWG + threadIdx.x;
            if (c < d) t[r * ldr + c] = 2 * less[e] + eq[e] + 1;
        }
    }
}

hipError_t launch_rank(const float* V, int64_t rows, int d, int64_t ldv, int32_t* t, int64_t ldr,
                       hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    if (d <= kRWG) {
        int dp = 1;
        while (dp < d) dp <<= 1;
        const int rpb = kRWG / dp;
        const int64_t blocks = (rows + rpb - 1) / rpb;
        hipLaunchKernelGGL(k_rank_small, dim3((unsigned)blocks), dim3(kRWG), 0, s, V, rows, d, dp, ldv, t, ldr);
    } else {
        hipLaunchKernelGGL(k_rank_large, dim3((unsigned)rows), dim3(kRWG), 0, s, V, d, ldv, t, ldr);
    }
    return hipGetLastError();
}

}  // namespace gmds
