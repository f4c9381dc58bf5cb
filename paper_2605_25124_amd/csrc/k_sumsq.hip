// k_sumsq.hip -- sum_{i<j} Delta_ij^2, the normaliser of the Kruskal stress
// (Section IV-B), and sum_{i<j} Delta_ij, the normaliser of the Sammon stress,
// for one or more stacked matrices.
//
// Pass 1: the strict upper triangle's rows 0 .. n-2 are taken in pairs
// (r, n-2-r), which together hold n entries, so equal numbers of pairs give
// equal work.  Each workgroup owns a contiguous run of row pairs; a thread
// reads the columns j = i+1+tid, +kSqWG, ... of a row (coalesced) and adds
// each entry (power 1) or its square (power 2, split exactly into v*v and the
// FMA residual) to a compensated accumulator.  The workgroup's accumulators are combined by a fixed tree and
// written as one (hi, lo) partial.  Pass 2: one workgroup per matrix sums the
// partials, again in a fixed order, so the result does not depend on timing.
#include "common.hpp"
#include "kernels.hpp"

namespace gmds {

namespace {

constexpr int kSqWG = 256;

__device__ Comp block_combine(Comp acc, float* lds) {
    const int tid = threadIdx.x;
    lds[tid] = acc.hi;
    lds[kSqWG + tid] = acc.lo;
    __syncthreads();
    for (int st = kSqWG / 2; st > 0; st >>= 1) {
        if (tid < st) {
            Comp u;
            u.hi = lds[tid];
            u.lo = lds[kSqWG + tid];
            Comp w;
            w.hi = lds[tid + st];
            w.lo = lds[kSqWG + tid + st];
            u.add(w);
            lds[tid] = u.hi;
            lds[kSqWG + tid] = u.lo;
        }
        __syncthreads();
    }
    Comp r;
    r.hi = lds[0];
    r.lo = lds[kSqWG];
    return r;
}

template <int POW>
__global__ __launch_bounds__(kSqWG) void k_sumsq_part(const float* __restrict__ Delta, int64_t n, int64_t ldd,
                                                      int64_t stride, int64_t pairs_per_block, float* part) {
    __shared__ float lds[2 * kSqWG];
    const float* D = Delta + (int64_t)blockIdx.y * stride;
    const int64_t npairs = n / 2;                      // rows 0..n-2 as (r, n-2-r)
    const int64_t r0 = (int64_t)blockIdx.x * pairs_per_block;
    const int64_t r1 = min(npairs, r0 + pairs_per_block);
    Comp acc;
    for (int64_t r = r0; r < r1; ++r) {
        for (int h = 0; h < 2; ++h) {
            const int64_t i = h ? n - 2 - r : r;
            if (h && i == r) break;                    // the middle row of an odd count
            const float* row = D + i * ldd;
            for (int64_t j = i + 1 + threadIdx.x; j < n; j += kSqWG) {
                const float v = row[j];
                if constexpr (POW == 1) {
                    acc.add(v);
                } else {
                    const float sq = v * v;
                    acc.add(sq);
                    acc.lo += fmaf(v, v, -sq);
                }
            }
        }
    }
    const Comp tot = block_combine(acc, lds);
    if (threadIdx.x == 0) {
        float* o = part + 2 * ((int64_t)blockIdx.y * gridDim.x + blockIdx.x);
        o[0] = tot.hi;
        o[1] = tot.lo;
    }
}

__global__ __launch_bounds__(kSqWG) void k_sumsq_final(const float* __restrict__ part, int64_t blocks, float* out) {
    __shared__ float lds[2 * kSqWG];
    const float* P = part + 2 * (int64_t)blockIdx.x * blocks;
    Comp acc;
    for (int64_t b = threadIdx.x; b < blocks; b += kSqWG) {
        Comp w;
        w.hi = P[2 * b];
        w.lo = P[2 * b + 1];
        acc.add(w);
    }
    const Comp tot = block_combine(acc, lds);
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = tot.hi;
        out[2 * blockIdx.x + 1] = tot.lo;
    }
}

// Largest row sum of 1 / Delta_ij over j != i with Delta_ij > 0 (full rows):
// each workgroup sums its rows in a fixed order and keeps their maximum.
__global__ __launch_bounds__(kSqWG) void k_rowinv_max(const float* __restrict__ Delta, int64_t n, int64_t ldd,
                                                      int64_t rows_per_block, float* part) {
    __shared__ float lds[2 * kSqWG];
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(n, r0 + rows_per_block);
    float mx = 0.f;
    for (int64_t i = r0; i < r1; ++i) {
        const float* row = Delta + i * ldd;
        Comp acc;
        for (int64_t j = threadIdx.x; j < n; j += kSqWG) {
            const float v = row[j];
            if (j != i && v > 0.f) acc.add(1.f / v);
        }
        const Comp tot = block_combine(acc, lds);
        mx = fmaxf(mx, tot.value());
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = mx;
}

__global__ __launch_bounds__(kSqWG) void k_max_final(const float* __restrict__ part, int64_t blocks, float* out) {
    __shared__ float lds[kSqWG];
    float mx = 0.f;
    for (int64_t b = threadIdx.x; b < blocks; b += kSqWG) mx = fmaxf(mx, part[b]);
    lds[threadIdx.x] = mx;
    __syncthreads();
    for (int st = kSqWG / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) lds[threadIdx.x] = fmaxf(lds[threadIdx.x], lds[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = lds[0];
}

constexpr int64_t kSqMaxBlocks = 2048;

int64_t pairs_per_block(int64_t n) {
    const int64_t npairs = n / 2;
    return std::max<int64_t>(1, (npairs + kSqMaxBlocks - 1) / kSqMaxBlocks);
}

}  // namespace

int64_t sumsq_blocks(int64_t n) {
    const int64_t npairs = n / 2;
    if (npairs == 0) return 0;
    const int64_t ppb = pairs_per_block(n);
    return (npairs + ppb - 1) / ppb;
}

hipError_t launch_sumsq(const float* Delta, int64_t n, int64_t ldd, int n_mat, int64_t stride, float* part,
                        float* out, int power, hipStream_t s) {
    const int64_t blocks = sumsq_blocks(n);
    if (blocks == 0) return launch_fill_u32(reinterpret_cast<uint32_t*>(out), 2 * (int64_t)n_mat, 0u, s);
    if (power == 1)
        hipLaunchKernelGGL(k_sumsq_part<1>, dim3((unsigned)blocks, (unsigned)n_mat), dim3(kSqWG), 0, s, Delta, n, ldd,
                           stride, pairs_per_block(n), part);
    else
        hipLaunchKernelGGL(k_sumsq_part<2>, dim3((unsigned)blocks, (unsigned)n_mat), dim3(kSqWG), 0, s, Delta, n, ldd,
                           stride, pairs_per_block(n), part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sumsq_final, dim3((unsigned)n_mat), dim3(kSqWG), 0, s, part, blocks, out);
    return hipGetLastError();
}

int64_t rowinv_blocks(int64_t n) { return std::min<int64_t>(n, kSqMaxBlocks); }

hipError_t launch_rowinv_max(const float* Delta, int64_t n, int64_t ldd, float* part, float* out, hipStream_t s) {
    const int64_t blocks = rowinv_blocks(n);
    const int64_t rpb = (n + blocks - 1) / blocks;
    hipLaunchKernelGGL(k_rowinv_max, dim3((unsigned)blocks), dim3(kSqWG), 0, s, Delta, n, ldd, rpb, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(kSqWG), 0, s, part, blocks, out);
    return hipGetLastError();
}

}  // namespace gmds
