// k_rank.hip -- doubled midranks of the coordinates of each row (Definition 1
// with the tie rule of Section III-A):
//     t_c = 2 * #{c' : v_c' < v_c} + #{c' : v_c' == v_c} + 1.
// Short rows (d <= 256): each thread counts for its own coordinate against the
// whole row, staged in LDS so that the threads of a row read the same word at
// the same time (broadcast).  Longer rows: sorted chunks and binary search
// (below).  Either way the result is an integer function of FP32
// comparisons, so it is bit-exact by construction.
#include <algorithm>

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

// d > 256: sort, then count by binary search.  The row is cut into chunks of
// kRankChunk coordinates; k_rank_sort sorts every chunk (one workgroup, a
// bitonic network in LDS) into scratch, and k_rank_count gives each
// coordinate the number of keys below it and equal to it in every sorted
// chunk (lower and upper bound by binary search in LDS).  Keys are the FP32
// bit patterns mapped to unsigned integers in the order of the values, with
// -0 taken as +0, so that integer < and == are the IEEE comparisons of
// finite values.  O(d log d) per chunk pair instead of O(d^2).
constexpr int kRankChunk = 4096;

__device__ __forceinline__ uint32_t order_key(float x) {
    const uint32_t u = __float_as_uint(x == 0.f ? 0.f : x);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ __launch_bounds__(kRWG) void k_rank_sort(const float* __restrict__ V, int d, int64_t ldv,
                                                    uint32_t* __restrict__ sorted, int64_t lds_row) {
    __shared__ uint32_t key[kRankChunk];
    const int64_t r = blockIdx.x;
    const int c0 = blockIdx.y * kRankChunk;
    const int len = min(kRankChunk, d - c0);
    int P = 1;
    while (P < len) P <<= 1;
    for (int k = threadIdx.x; k < P; k += kRWG) key[k] = (k < len) ? order_key(V[r * ldv + c0 + k]) : 0xFFFFFFFFu;
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1)
        for (int st = size >> 1; st > 0; st >>= 1) {
            for (int x = threadIdx.x; x < P / 2; x += kRWG) {
                const int lo = 2 * x - (x & (st - 1));          // lower index of the x-th pair
                const int hi = lo + st;
                const bool up = (lo & size) == 0;
                const uint32_t a = key[lo], b = key[hi];
                if ((a > b) == up) {
                    key[lo] = b;
                    key[hi] = a;
                }
            }
            __syncthreads();
        }
    for (int k = threadIdx.x; k < len; k += kRWG) sorted[r * lds_row + c0 + k] = key[k];
}

__global__ __launch_bounds__(kRWG) void k_rank_count(const float* __restrict__ V, int d, int64_t ldv,
                                                     const uint32_t* __restrict__ sorted, int64_t lds_row,
                                                     int32_t* __restrict__ t, int64_t ldr) {
    __shared__ uint32_t key[kRankChunk];
    const int64_t r = blockIdx.x;
    const int c = blockIdx.y * kRWG + threadIdx.x;
    const uint32_t x = (c < d) ? order_key(V[r * ldv + c]) : 0u;
    int less = 0, eq = 0;
    for (int c0 = 0; c0 < d; c0 += kRankChunk) {
        const int len = min(kRankChunk, d - c0);
        __syncthreads();
        for (int k = threadIdx.x; k < len; k += kRWG) key[k] = sorted[r * lds_row + c0 + k];
        __syncthreads();
        int lo = 0, hi = len;                       // first key >= x
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (key[mid] < x) lo = mid + 1;
            else hi = mid;
        }
        int lo2 = lo, hi2 = len;                    // first key > x
        while (lo2 < hi2) {
            const int mid = (lo2 + hi2) >> 1;
            if (key[mid] <= x) lo2 = mid + 1;
            else hi2 = mid;
        }
        less += lo;
        eq += lo2 - lo;
    }
    if (c < d) t[r * ldr + c] = 2 * less + eq + 1;
}

constexpr int64_t kRankScratchWords = (int64_t)1 << 24;      // 64 MiB of sorted chunks at most

int64_t rank_scratch_words(int64_t rows, int d) {
    if (d <= kRWG) return 0;
    return std::min<int64_t>(rows, std::max<int64_t>(1, kRankScratchWords / d)) * (int64_t)d;
}

hipError_t launch_rank(const float* V, int64_t rows, int d, int64_t ldv, int32_t* t, int64_t ldr, uint32_t* scratch,
                       hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    if (d <= kRWG) {
        int dp = 1;
        while (dp < d) dp <<= 1;
        const int rpb = kRWG / dp;
        const int64_t blocks = (rows + rpb - 1) / rpb;
        hipLaunchKernelGGL(k_rank_small, dim3((unsigned)blocks), dim3(kRWG), 0, s, V, rows, d, dp, ldv, t, ldr);
        return hipGetLastError();
    }
    // rows in batches, so that the sorted chunks take at most kRankScratchWords
    const unsigned chunks = (unsigned)((d + kRankChunk - 1) / kRankChunk);
    const int64_t batch = std::max<int64_t>(1, kRankScratchWords / d);
    for (int64_t r0 = 0; r0 < rows; r0 += batch) {
        const unsigned nr = (unsigned)std::min<int64_t>(batch, rows - r0);
        hipLaunchKernelGGL(k_rank_sort, dim3(nr, chunks), dim3(kRWG), 0, s, V + r0 * ldv, d, ldv, scratch, (int64_t)d);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_rank_count, dim3(nr, (unsigned)((d + kRWG - 1) / kRWG)), dim3(kRWG), 0, s, V + r0 * ldv,
                           d, ldv, scratch, (int64_t)d, t + r0 * ldr, ldr);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace gmds
