// k_cmds.hip -- the kernels of classical MDS (Section IV-A): the Gram matrix
// B = -1/2 H D^2 H of the squared dissimilarities is never formed; subspace
// iteration applies it to an n x q block V (q <= 8) as
//     Y = -1/2 H (D^2 V),   D^2 = Delta .* Delta,
// one streaming pass over the rows of Delta per application.  With q this
// small the product is a bandwidth-bound matrix-vector sweep, not a dense
// contraction, so it runs on the vector ALUs.  Every sum has a fixed shape
// (compensated per thread, then a fixed tree), so results are reproducible.
#include "common.hpp"
#include "kernels.hpp"

namespace gmds {

namespace {

constexpr int kCW = 256;           // threads of a row workgroup
constexpr int kQ = kMaxCmdsQ;      // widest block handled

// out[i, c] = sum_j Delta_ij^2 V[j, c], j != i (full rows of Delta).  A
// workgroup takes kRows consecutive rows, so that every element of V it loads
// serves kRows rows (V is read from L2 n / kRows times per pass instead of n).
// Each row's sum has the same shape as with one row per workgroup: thread t
// adds j = t, t + kCW, ... in order (compensated), then a fixed tree over the
// threads.
constexpr int kRows = 4;

__global__ __launch_bounds__(kCW) void k_d2v(const float* __restrict__ Delta, int64_t n, int64_t ldd,
                                             const float* __restrict__ V, int q, float* __restrict__ out) {
    __shared__ float lds[2 * kCW * kQ];
    const int64_t i0 = (int64_t)blockIdx.x * kRows;
    const int nr = (int)min<int64_t>(kRows, n - i0);
    Comp acc[kRows][kQ];
    for (int64_t j = threadIdx.x; j < n; j += kCW) {
        float vj[kQ];
#pragma unroll
        for (int c = 0; c < kQ; ++c) vj[c] = (c < q) ? V[j * q + c] : 0.f;
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            if (r >= nr || j == i0 + r) continue;
            const float d = Delta[(i0 + r) * ldd + j];
            const float d2 = d * d;
#pragma unroll
            for (int c = 0; c < kQ; ++c)
                if (c < q) acc[r][c].add(d2 * vj[c]);
        }
    }
    const int t = threadIdx.x;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        if (r >= nr) break;                    // nr is the same for the whole workgroup
#pragma unroll
        for (int c = 0; c < kQ; ++c) {
            lds[(c * kCW + t) * 2] = acc[r][c].hi;
            lds[(c * kCW + t) * 2 + 1] = acc[r][c].lo;
        }
        __syncthreads();
        for (int st = kCW / 2; st > 0; st >>= 1) {
            if (t < st) {
#pragma unroll
                for (int c = 0; c < kQ; ++c) {
                    Comp a, b;
                    a.hi = lds[(c * kCW + t) * 2];
                    a.lo = lds[(c * kCW + t) * 2 + 1];
                    b.hi = lds[(c * kCW + t + st) * 2];
                    b.lo = lds[(c * kCW + t + st) * 2 + 1];
                    a.add(b);
                    lds[(c * kCW + t) * 2] = a.hi;
                    lds[(c * kCW + t) * 2 + 1] = a.lo;
                }
            }
            __syncthreads();
        }
        if (t < q) out[(i0 + r) * q + t] = lds[(t * kCW) * 2] + lds[(t * kCW) * 2 + 1];
        __syncthreads();
    }
}

// Partial sums over a block of rows of A^T B (qa x qb entries, compensated,
// fixed order): part[block][a * qb + b] as (hi, lo).  B == nullptr sums the
// columns of A (qb = 1 with B_i = 1).
__global__ __launch_bounds__(kCW) void k_gram_part(const float* __restrict__ A, int qa, const float* __restrict__ B,
                                                   int qb, int64_t n, int64_t rows_per_block, float* part) {
    __shared__ float lds[2 * kCW];
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(n, r0 + rows_per_block);
    for (int e = 0; e < qa * qb; ++e) {
        const int a = e / qb, b = e % qb;
        Comp acc;
        for (int64_t i = r0 + threadIdx.x; i < r1; i += kCW)
            acc.add(A[i * qa + a] * (B ? B[i * qb + b] : 1.f));
        const int t = threadIdx.x;
        lds[2 * t] = acc.hi;
        lds[2 * t + 1] = acc.lo;
        __syncthreads();
        for (int st = kCW / 2; st > 0; st >>= 1) {
            if (t < st) {
                Comp x, y;
                x.hi = lds[2 * t];
                x.lo = lds[2 * t + 1];
                y.hi = lds[2 * (t + st)];
                y.lo = lds[2 * (t + st) + 1];
                x.add(y);
                lds[2 * t] = x.hi;
                lds[2 * t + 1] = x.lo;
            }
            __syncthreads();
        }
        if (t == 0) {
            part[((int64_t)blockIdx.x * qa * qb + e) * 2] = lds[0];
            part[((int64_t)blockIdx.x * qa * qb + e) * 2 + 1] = lds[1];
        }
        __syncthreads();
    }
}

// out[e] = sum over blocks of part[block][e] (fixed order), as (hi, lo).
__global__ __launch_bounds__(kCW) void k_gram_final(const float* __restrict__ part, int64_t blocks, int ne,
                                                    float* out) {
    const int e = blockIdx.x * kCW + threadIdx.x;
    if (e >= ne) return;
    Comp acc;
    for (int64_t b = 0; b < blocks; ++b) {
        Comp x;
        x.hi = part[(b * ne + e) * 2];
        x.lo = part[(b * ne + e) * 2 + 1];
        acc.add(x);
    }
    out[2 * e] = acc.hi;
    out[2 * e + 1] = acc.lo;
}

// out[i, :] = (alpha * (A[i, :] - shift)) M, with M qa x qb (row-major) and
// shift (qa) in device memory.
__global__ __launch_bounds__(kCW) void k_rowmat(const float* __restrict__ A, int qa, const float* __restrict__ shift,
                                                float alpha, const float* __restrict__ M, int qb, int64_t n,
                                                float* __restrict__ out, int64_t ldo) {
    const int64_t i = (int64_t)blockIdx.x * kCW + threadIdx.x;
    if (i >= n) return;
    float a[kQ];
#pragma unroll
    for (int c = 0; c < kQ; ++c) a[c] = (c < qa) ? alpha * (A[i * qa + c] - (shift ? shift[c] : 0.f)) : 0.f;
    for (int b = 0; b < qb; ++b) {
        float s = 0.f;
#pragma unroll
        for (int c = 0; c < kQ; ++c)
            if (c < qa) s = fmaf(a[c], M[c * qb + b], s);
        out[i * ldo + b] = s;
    }
}

// shift[c] = (hi + lo) / n of the compensated column sums (hi, lo) in sums.
__global__ void k_colmean(const float* __restrict__ sums, int q, int64_t n, float* __restrict__ shift) {
    const int c = threadIdx.x;
    if (c < q) shift[c] = (float)(((double)sums[2 * c] + (double)sums[2 * c + 1]) / (double)n);
}

}  // namespace

hipError_t launch_colmean(const float* sums, int q, int64_t n, float* shift, hipStream_t s) {
    hipLaunchKernelGGL(k_colmean, dim3(1), dim3(64), 0, s, sums, q, n, shift);
    return hipGetLastError();
}

hipError_t launch_d2v(const float* Delta, int64_t n, int64_t ldd, const float* V, int q, float* out,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_d2v, dim3((unsigned)((n + kRows - 1) / kRows)), dim3(kCW), 0, s, Delta, n, ldd, V, q, out);
    return hipGetLastError();
}

int64_t gram_blocks(int64_t n) { return std::min<int64_t>(256, (n + kCW - 1) / kCW); }

hipError_t launch_gram(const float* A, int qa, const float* B, int qb, int64_t n, float* part, float* out,
                       hipStream_t s) {
    const int64_t blocks = gram_blocks(n);
    const int64_t rpb = (n + blocks - 1) / blocks;
    hipLaunchKernelGGL(k_gram_part, dim3((unsigned)blocks), dim3(kCW), 0, s, A, qa, B, qb, n, rpb, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int ne = qa * qb;
    hipLaunchKernelGGL(k_gram_final, dim3((unsigned)((ne + kCW - 1) / kCW)), dim3(kCW), 0, s, part, blocks, ne,
                       out);
    return hipGetLastError();
}

hipError_t launch_rowmat(const float* A, int qa, const float* shift, float alpha, const float* M, int qb, int64_t n,
                         float* out, int64_t ldo, hipStream_t s) {
    hipLaunchKernelGGL(k_rowmat, dim3((unsigned)((n + kCW - 1) / kCW)), dim3(kCW), 0, s, A, qa, shift, alpha, M, qb,
                       n, out, ldo);
    return hipGetLastError();
}

}  // namespace gmds
