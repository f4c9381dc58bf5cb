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
// serves kRows rows.  Thread t reads the column quads j0 = 4 (t + kCW k) of
// each row (one 16-byte load per row and quad when the rows are aligned) and
// the four rows of V they meet (q 16-byte loads), and accumulates the
// products in FP64 (full rate on this GPU, so no compensation is needed);
// the threads' sums are combined by a fixed tree, so every row's sum has one
// fixed shape.
constexpr int kRows = 4;

template <bool VEC, int Q>
__global__ __launch_bounds__(kCW) void k_d2v(const float* __restrict__ Delta, int64_t n, int64_t ldd,
                                             const float* __restrict__ V, float* __restrict__ out) {
    constexpr int kQB = Q;             // the block width, a compile-time constant
    constexpr int q = Q;
    __shared__ double lds[kCW * kQB];
    const int64_t i0 = (int64_t)blockIdx.x * kRows;
    const int nr = (int)min<int64_t>(kRows, n - i0);
    double acc[kRows][kQB];
#pragma unroll
    for (int r = 0; r < kRows; ++r)
#pragma unroll
        for (int c = 0; c < kQB; ++c) acc[r][c] = 0.0;
    for (int64_t j0 = 4 * (int64_t)threadIdx.x; j0 < n; j0 += 4 * kCW) {
        float d[kRows][4];
        const bool full = j0 + 3 < n;
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const float* row = Delta + (i0 + (r < nr ? r : 0)) * ldd;
            if (VEC && full) {
                const float4 v = *reinterpret_cast<const float4*>(row + j0);
                d[r][0] = v.x;
                d[r][1] = v.y;
                d[r][2] = v.z;
                d[r][3] = v.w;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) d[r][e] = (j0 + e < n) ? row[j0 + e] : 0.f;
            }
            if (r >= nr) {
#pragma unroll
                for (int e = 0; e < 4; ++e) d[r][e] = 0.f;
            }
        }
        if (j0 < i0 + kRows && i0 < j0 + 4) {        // the quad meets the diagonal: leave out j == i
#pragma unroll
            for (int r = 0; r < kRows; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (j0 + e == i0 + r) d[r][e] = 0.f;
        }
        // rows j0 .. j0+3 of V: 4q consecutive floats, 16-byte aligned
        float v[4 * kQB];
        if (full) {
#pragma unroll
            for (int k = 0; k < kQB; ++k) {
                const float4 w = *reinterpret_cast<const float4*>(V + j0 * q + 4 * k);
                v[4 * k] = w.x;
                v[4 * k + 1] = w.y;
                v[4 * k + 2] = w.z;
                v[4 * k + 3] = w.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4 * kQB; ++k) v[k] = (j0 * q + k < n * q) ? V[j0 * q + k] : 0.f;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int r = 0; r < kRows; ++r) {
                const double d2 = (double)(d[r][e] * d[r][e]);
#pragma unroll
                for (int c = 0; c < kQB; ++c) acc[r][c] = fma(d2, (double)v[e * q + c], acc[r][c]);
            }
    }
    const int t = threadIdx.x;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        if (r >= nr) break;                    // nr is the same for the whole workgroup
#pragma unroll
        for (int c = 0; c < kQB; ++c) lds[c * kCW + t] = acc[r][c];
        __syncthreads();
        for (int st = kCW / 2; st > 0; st >>= 1) {
            if (t < st) {
#pragma unroll
                for (int c = 0; c < kQB; ++c) lds[c * kCW + t] += lds[c * kCW + t + st];
            }
            __syncthreads();
        }
        if (t < q) out[(i0 + r) * q + t] = (float)lds[t * kCW];
        __syncthreads();
    }
}

// out (qa*qb (hi, lo) pairs, entry a*qb + b) = A^T B over n rows, B == nullptr
// meaning the column sums of A (qb = 1); a launch may carry a second product
// of the same shape (blockIdx.y = 1).  Block k of a product sums the rows
// [k R, (k+1) R): thread t takes entry t % ne and the rows t / ne,
// t / ne + S, ... of the block (S = kCW / ne row slices, eight loads in
// flight), compensated; the S slice sums are added in slice order into the
// block's partial.  k_gram_final adds the kGB partials of every entry in
// block order, so every entry has one fixed shape.
constexpr int kGB = 128;           // blocks per product

__global__ __launch_bounds__(kCW) void k_gram_part(const float* __restrict__ A0, const float* __restrict__ B0,
                                                   const float* __restrict__ A1, const float* __restrict__ B1,
                                                   int qa, int qb, int64_t n, int64_t rows_per_block,
                                                   float* __restrict__ part) {
    __shared__ float lds[2 * kCW];
    const float* A = blockIdx.y ? A1 : A0;
    const float* B = blockIdx.y ? B1 : B0;
    const int ne = qa * qb;
    const int S = kCW / ne;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(n, r0 + rows_per_block);
    const int t = threadIdx.x;
    const int e = t % ne, sl = t / ne;
    Comp acc;
    if (sl < S) {
        const int a = e / qb, b = e % qb;
        constexpr int kB = 8;
        for (int64_t i0 = r0 + sl; i0 < r1; i0 += (int64_t)kB * S) {
            float x[kB];
#pragma unroll
            for (int k = 0; k < kB; ++k) {
                const int64_t i = i0 + (int64_t)k * S;
                x[k] = (i < r1) ? A[i * qa + a] * (B ? B[i * qb + b] : 1.f) : 0.f;
            }
#pragma unroll
            for (int k = 0; k < kB; ++k) acc.add(x[k]);
        }
    }
    lds[2 * t] = acc.hi;
    lds[2 * t + 1] = acc.lo;
    __syncthreads();
    if (t < ne) {
        Comp tot;
        for (int k = 0; k < S; ++k) {
            Comp x;
            x.hi = lds[2 * (k * ne + t)];
            x.lo = lds[2 * (k * ne + t) + 1];
            tot.add(x);
        }
        float* pp = part + 2 * (((int64_t)blockIdx.y * kGB + blockIdx.x) * ne + t);
        pp[0] = tot.hi;
        pp[1] = tot.lo;
    }
}

// out_y[e] = sum over blocks of part[y][block][e] in block order, (hi, lo).
__global__ __launch_bounds__(kCW) void k_gram_final(const float* __restrict__ part, int ne, int nprod,
                                                    float* __restrict__ out0, float* __restrict__ out1) {
    const int x = threadIdx.x;
    if (x >= ne * nprod) return;
    const int y = x / ne, e = x % ne;
    float* out = y ? out1 : out0;
    float h[kGB], l[kGB];
#pragma unroll
    for (int k = 0; k < kGB; ++k) {
        h[k] = part[2 * (((int64_t)y * kGB + k) * ne + e)];
        l[k] = part[2 * (((int64_t)y * kGB + k) * ne + e) + 1];
    }
    Comp acc;
#pragma unroll
    for (int k = 0; k < kGB; ++k) {
        Comp v;
        v.hi = h[k];
        v.lo = l[k];
        acc.add(v);
    }
    out[2 * e] = acc.hi;
    out[2 * e + 1] = acc.lo;
}

// out[i, :] = (alpha * (A[i, :] - mean)) M, with M qa x qb (row-major) in
// device memory and mean[c] = (sums[2c] + sums[2c+1]) / n from column sums
// (hi, lo) of A (sums == nullptr: no centring).
__global__ __launch_bounds__(kCW) void k_rowmat(const float* __restrict__ A, int qa, const float* __restrict__ sums,
                                                float alpha, const float* __restrict__ M, int qb, int64_t n,
                                                float* __restrict__ out, int64_t ldo) {
    const int64_t i = (int64_t)blockIdx.x * kCW + threadIdx.x;
    if (i >= n) return;
    float a[kQ];
#pragma unroll
    for (int c = 0; c < kQ; ++c) {
        float mean = 0.f;
        if (sums && c < qa) mean = (float)(((double)sums[2 * c] + (double)sums[2 * c + 1]) / (double)n);
        a[c] = (c < qa) ? alpha * (A[i * qa + c] - mean) : 0.f;
    }
    for (int b = 0; b < qb; ++b) {
        float s = 0.f;
#pragma unroll
        for (int c = 0; c < kQ; ++c)
            if (c < qa) s = fmaf(a[c], M[c * qb + b], s);
        out[i * ldo + b] = s;
    }
}

// Orthonormalising map of a block Y from its Gram matrix G = Y^T Y (q x q,
// compensated (hi, lo) sums, symmetrised): the Cholesky factor G = R^T R,
// column by column in FP64, and M = R^-1, so that Y M has orthonormal
// columns spanning those of Y.  G is only as accurate as the FP32 entries of
// Y (relative 1e-7), so a column whose part orthogonal to the earlier ones
// has less than kDepTol of its squared norm is taken to lie in their span
// (its orthogonal part is rounding noise) and becomes a zero column of Y M.
// One thread; everything in registers.
constexpr double kDepTol = 1e-5;

__global__ __launch_bounds__(64) void k_chol_orth(const float* __restrict__ g, int q, float* __restrict__ M) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double A[kQ][kQ], R[kQ][kQ], Mi[kQ][kQ];
    bool keep[kQ];
    double mx = 0.0;
#pragma unroll
    for (int i = 0; i < kQ; ++i)
#pragma unroll
        for (int j = 0; j < kQ; ++j) {
            double v = 0.0;
            if (i < q && j < q) {
                const double a = (double)g[2 * (i * q + j)] + (double)g[2 * (i * q + j) + 1];
                const double b = (double)g[2 * (j * q + i)] + (double)g[2 * (j * q + i) + 1];
                v = 0.5 * (a + b);
            }
            A[i][j] = v;
            R[i][j] = 0.0;
            Mi[i][j] = 0.0;
        }
#pragma unroll
    for (int i = 0; i < kQ; ++i) mx = fmax(mx, A[i][i]);
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        double d = A[k][k];
#pragma unroll
        for (int l = 0; l < k; ++l) d -= R[l][k] * R[l][k];
        keep[k] = k < q && mx > 0.0 && d > kDepTol * A[k][k];
        const double rkk = keep[k] ? sqrt(d) : 1.0;
        R[k][k] = keep[k] ? rkk : 0.0;
#pragma unroll
        for (int j = k + 1; j < kQ; ++j) {
            double v = A[k][j];
#pragma unroll
            for (int l = 0; l < k; ++l) v -= R[l][k] * R[l][j];
            R[k][j] = keep[k] ? v / rkk : 0.0;
        }
    }
    // M = R^-1 by back substitution, column by column; dropped rows and
    // columns stay zero
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        if (!keep[k]) continue;
        Mi[k][k] = 1.0 / R[k][k];
#pragma unroll
        for (int i = k - 1; i >= 0; --i) {
            if (!keep[i]) continue;
            double v = 0.0;
#pragma unroll
            for (int l = i + 1; l <= k; ++l) v += R[i][l] * Mi[l][k];
            Mi[i][k] = -v / R[i][i];
        }
    }
#pragma unroll
    for (int i = 0; i < kQ; ++i)
#pragma unroll
        for (int k = 0; k < kQ; ++k)
            if (i < q && k < q) M[i * q + k] = (float)Mi[i][k];
}

}  // namespace

template <int Q>
static void d2v_q(bool vec, dim3 grid, hipStream_t s, const float* Delta, int64_t n, int64_t ldd, const float* V,
                  float* out) {
    if (vec) hipLaunchKernelGGL((k_d2v<true, Q>), grid, dim3(kCW), 0, s, Delta, n, ldd, V, out);
    else hipLaunchKernelGGL((k_d2v<false, Q>), grid, dim3(kCW), 0, s, Delta, n, ldd, V, out);
}

hipError_t launch_d2v(const float* Delta, int64_t n, int64_t ldd, const float* V, int q, float* out,
                      hipStream_t s) {
    const dim3 grid((unsigned)((n + kRows - 1) / kRows));
    const bool vec = (reinterpret_cast<uintptr_t>(Delta) & 15u) == 0 && (ldd % 4) == 0;
    switch (q) {
        case 1: d2v_q<1>(vec, grid, s, Delta, n, ldd, V, out); break;
        case 2: d2v_q<2>(vec, grid, s, Delta, n, ldd, V, out); break;
        case 3: d2v_q<3>(vec, grid, s, Delta, n, ldd, V, out); break;
        case 4: d2v_q<4>(vec, grid, s, Delta, n, ldd, V, out); break;
        case 5: d2v_q<5>(vec, grid, s, Delta, n, ldd, V, out); break;
        case 6: d2v_q<6>(vec, grid, s, Delta, n, ldd, V, out); break;
        case 7: d2v_q<7>(vec, grid, s, Delta, n, ldd, V, out); break;
        default: d2v_q<8>(vec, grid, s, Delta, n, ldd, V, out); break;
    }
    return hipGetLastError();
}

hipError_t launch_gram(const float* A, int qa, const float* B, int qb, int64_t n, float* part, float* out,
                       hipStream_t s, const float* A2, const float* B2, float* out2) {
    const int nprod = A2 ? 2 : 1;
    const int64_t rpb = (n + kGB - 1) / kGB;
    hipLaunchKernelGGL(k_gram_part, dim3(kGB, nprod), dim3(kCW), 0, s, A, B, A2, B2, qa, qb, n, rpb, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gram_final, dim3(1), dim3(kCW), 0, s, part, qa * qb, nprod, out, out2);
    return hipGetLastError();
}

int64_t gram_part_floats() { return 2 * (int64_t)kGB * 2 * kQ * kQ; }

hipError_t launch_chol_orth(const float* g, int q, float* M, hipStream_t s) {
    hipLaunchKernelGGL(k_chol_orth, dim3(1), dim3(64), 0, s, g, q, M);
    return hipGetLastError();
}

hipError_t launch_rowmat(const float* A, int qa, const float* sums, float alpha, const float* M, int qb, int64_t n,
                         float* out, int64_t ldo, hipStream_t s) {
    hipLaunchKernelGGL(k_rowmat, dim3((unsigned)((n + kCW - 1) / kCW)), dim3(kCW), 0, s, A, qa, sums, alpha, M, qb,
                       n, out, ldo);
    return hipGetLastError();
}

}  // namespace gmds
