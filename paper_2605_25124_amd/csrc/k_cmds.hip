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

// out[i, c] = sum_j Delta_ij^2 V[j, c], j != i (full rows of Delta), in
// FP64.  A workgroup takes kRows consecutive rows, so that every element of V
// it loads serves kRows rows.  Thread t reads the column quads
// j0 = 4 (t + kCW k) of each row (one 16-byte load per row and quad when the
// rows are aligned) and the four rows of V they meet (q 16-byte loads), and
// accumulates the products in FP64 (full rate on this GPU, so no compensation
// is needed).  The 64 lane sums of a wave are combined by a butterfly (every
// lane ends with the same value), then the four waves' sums are added in wave
// order, so every row's sum has one fixed shape.
// (eight rows for q <= 6, four for wider blocks, whose accumulators would
// leave room for one wave per SIMD).
__host__ __device__ constexpr int d2v_rows(int q) { return q <= 6 ? 8 : 4; }

template <bool VEC, int Q>
__global__ __launch_bounds__(kCW) __attribute__((amdgpu_waves_per_eu(2))) void k_d2v(const float* __restrict__ Delta, int64_t n, int64_t ldd,
                                             const float* __restrict__ V, double* __restrict__ out, int rev) {
    constexpr int q = Q;
    constexpr int kRows = d2v_rows(Q);
    constexpr int kW = kCW / 64;
    __shared__ double lds[kW][kRows * Q];
    // rev: the row blocks are taken last to first, so that a pass starts on
    // the rows the previous pass read last (still in the memory-side cache)
    const int64_t i0 = (int64_t)(rev ? gridDim.x - 1 - blockIdx.x : blockIdx.x) * kRows;
    const int nr = (int)min<int64_t>(kRows, n - i0);
    double acc[kRows][Q];
#pragma unroll
    for (int r = 0; r < kRows; ++r)
#pragma unroll
        for (int c = 0; c < Q; ++c) acc[r][c] = 0.0;
    const float* rows[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) rows[r] = Delta + (i0 + (r < nr ? r : nr - 1)) * ldd;   // clamped
    // products of one quad: rows past the block's last hold the clamped
    // row's values and are masked here, as is the diagonal j == i
    auto accumulate = [&](int64_t j0, const float (&d)[kRows][4], const float (&v)[4 * Q]) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int r = 0; r < kRows; ++r) {
                const bool live = r < nr && j0 + e != i0 + r;
                const double d2 = live ? (double)(d[r][e] * d[r][e]) : 0.0;
#pragma unroll
                for (int c = 0; c < Q; ++c) acc[r][c] = fma(d2, (double)v[e * q + c], acc[r][c]);
            }
    };
    // Whole quads (16-byte loads of Delta and V): the next quad's loads are
    // issued before the current quad is computed, so that they are in flight
    // during the arithmetic.
    const int64_t nfull = VEC ? (n & ~(int64_t)3) : 0;
    auto load_quad = [&](int64_t j, float (&dd)[kRows][4], float (&vv)[4 * Q]) {
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const float4 x = *reinterpret_cast<const float4*>(rows[r] + j);
            dd[r][0] = x.x;
            dd[r][1] = x.y;
            dd[r][2] = x.z;
            dd[r][3] = x.w;
        }
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const float4 w = *reinterpret_cast<const float4*>(V + j * q + 4 * k);
            vv[4 * k] = w.x;
            vv[4 * k + 1] = w.y;
            vv[4 * k + 2] = w.z;
            vv[4 * k + 3] = w.w;
        }
    };
    {
        float dn[kRows][4], vn[4 * Q];
        int64_t j0 = 4 * (int64_t)threadIdx.x;
        if (j0 < nfull) load_quad(j0, dn, vn);
        for (; j0 < nfull; j0 += 4 * kCW) {
            float d[kRows][4], v[4 * Q];
#pragma unroll
            for (int r = 0; r < kRows; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e) d[r][e] = dn[r][e];
#pragma unroll
            for (int k = 0; k < 4 * Q; ++k) v[k] = vn[k];
            if (j0 + 4 * kCW < nfull) load_quad(j0 + 4 * kCW, dn, vn);
            accumulate(j0, d, v);
        }
    }
    // the rest (a last partial quad; every quad without 16-byte alignment):
    // element loads at clamped addresses, masked past n
    for (int64_t j0 = nfull + 4 * (int64_t)threadIdx.x; j0 < n; j0 += 4 * kCW) {
        float d[kRows][4], v[4 * Q];
#pragma unroll
        for (int r = 0; r < kRows; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) d[r][e] = rows[r][min<int64_t>(j0 + e, n - 1)];
#pragma unroll
        for (int k = 0; k < 4 * Q; ++k) v[k] = V[min<int64_t>(j0 * q + k, n * q - 1)];
#pragma unroll
        for (int r = 0; r < kRows; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (j0 + e >= n) d[r][e] = 0.f;
#pragma unroll
        for (int k = 0; k < 4 * Q; ++k)
            if (j0 * q + k >= n * q) v[k] = 0.f;
        accumulate(j0, d, v);
    }
    const int t = threadIdx.x;
#pragma unroll
    for (int r = 0; r < kRows; ++r)
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            double x = acc[r][c];
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
            acc[r][c] = x;
        }
    if ((t & 63) == 0) {
#pragma unroll
        for (int r = 0; r < kRows; ++r)
#pragma unroll
            for (int c = 0; c < Q; ++c) lds[t >> 6][r * Q + c] = acc[r][c];
    }
    __syncthreads();
    if (t < nr * Q) {
        double x = lds[0][t];
#pragma unroll
        for (int w = 1; w < kW; ++w) x += lds[w][t];
        out[i0 * q + t] = x;
    }
}

// The sums one subspace step needs, over the n rows of Y = D^2 V (FP64) and
// V, for the centring identities of the caller: product y = 0: c = Y^T 1
// (q entries), y = 1: s = V^T 1 (q), y = 2: V^T Y (q x q, entry a*q + b),
// y = 3: Y^T Y.  Block k of a product sums the rows [k R, (k+1) R): thread t
// takes entry t % ne and the rows t / ne, t / ne + S, ... of the block
// (S = kCW / ne row slices, eight loads in flight) in FP64; the S slice sums
// are added in slice order into the block's partial, and k_step_orth adds the
// kGB partials of every entry in block order: one fixed shape per entry.
constexpr int kGB = 128;           // blocks per product

__global__ __launch_bounds__(kCW) void k_step_part(const double* __restrict__ Y, const float* __restrict__ V, int q,
                                                   int64_t n, int64_t rows_per_block, double* __restrict__ part) {
    __shared__ double lds[kCW];
    const int y = blockIdx.y;
    const int ne = y < 2 ? q : q * q;
    const int S = kCW / ne;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(n, r0 + rows_per_block);
    const int t = threadIdx.x;
    const int e = t % ne, sl = t / ne;
    const int a = e / q, b = e % q;
    double acc = 0.0;
    if (sl < S) {
        constexpr int kB = 8;
        for (int64_t i0 = r0 + sl; i0 < r1; i0 += (int64_t)kB * S) {
            double x[kB];
#pragma unroll
            for (int k = 0; k < kB; ++k) {
                const int64_t i = i0 + (int64_t)k * S;
                double v = 0.0;
                if (i < r1) {
                    if (y == 0) v = Y[i * q + e];
                    else if (y == 1) v = (double)V[i * q + e];
                    else if (y == 2) v = (double)V[i * q + a] * Y[i * q + b];
                    else v = Y[i * q + a] * Y[i * q + b];
                }
                x[k] = v;
            }
#pragma unroll
            for (int k = 0; k < kB; ++k) acc += x[k];
        }
    }
    lds[t] = acc;
    __syncthreads();
    if (t < ne) {
        double tot = 0.0;
        for (int k = 0; k < S; ++k) tot += lds[k * ne + t];
        part[((int64_t)y * kGB + blockIdx.x) * (kQ * kQ) + t] = tot;
    }
}

// out (qa*qb (hi, lo) pairs, entry a*qb + b) = A^T B over n rows, B == nullptr
// meaning the column sums of A (qb = 1); used for the start block.  The same
// blocking as k_step_part, with compensated FP32 sums; k_gram_final adds the
// kGB partials of every entry in block order, so every entry has one fixed
// shape.

__global__ __launch_bounds__(kCW) void k_gram_part(const float* __restrict__ A, const float* __restrict__ B, int qa,
                                                   int qb, int64_t n, int64_t rows_per_block,
                                                   float* __restrict__ part) {
    __shared__ float lds[2 * kCW];
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
        float* pp = part + 2 * ((int64_t)blockIdx.x * ne + t);
        pp[0] = tot.hi;
        pp[1] = tot.lo;
    }
}

// out[e] = sum over blocks of part[block][e] in block order, (hi, lo).
__global__ __launch_bounds__(kCW) void k_gram_final(const float* __restrict__ part, int ne, float* __restrict__ out) {
    const int e = threadIdx.x;
    if (e >= ne) return;
    float h[kGB], l[kGB];
#pragma unroll
    for (int k = 0; k < kGB; ++k) {
        h[k] = part[2 * ((int64_t)k * ne + e)];
        l[k] = part[2 * ((int64_t)k * ne + e) + 1];
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
// symmetric, FP64): the Cholesky factor G = R^T R, column by column, and
// Mi = R^-1, so that Y Mi has orthonormal columns spanning those of Y.  G is
// only as accurate as the entries of Y, so a column whose part orthogonal to
// the earlier ones has less than kDepTol of its squared norm is taken to lie
// in their span (its orthogonal part is rounding noise) and becomes a zero
// column of Y Mi.  One thread; everything in registers.
constexpr double kDepTol = 1e-5;

__device__ void chol_inverse(const double (&A)[kQ][kQ], int q, double (&Mi)[kQ][kQ]) {
    double R[kQ][kQ];
    bool keep[kQ];
    double mx = 0.0;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        mx = fmax(mx, A[i][i]);
#pragma unroll
        for (int j = 0; j < kQ; ++j) {
            R[i][j] = 0.0;
            Mi[i][j] = 0.0;
        }
    }
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
    // Mi = R^-1 by back substitution, column by column; dropped rows and
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
}

// The same map from launch_gram's compensated (hi, lo) Gram matrix, in FP32.
__global__ __launch_bounds__(64) void k_chol_orth(const float* __restrict__ g, int q, float* __restrict__ M) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double A[kQ][kQ], Mi[kQ][kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i)
#pragma unroll
        for (int j = 0; j < kQ; ++j) {
            double v = 0.0;
            if (i < q && j < q) {
                const double x = (double)g[2 * (i * q + j)] + (double)g[2 * (i * q + j) + 1];
                const double y = (double)g[2 * (j * q + i)] + (double)g[2 * (j * q + i) + 1];
                v = 0.5 * (x + y);
            }
            A[i][j] = v;
        }
    chol_inverse(A, q, Mi);
#pragma unroll
    for (int i = 0; i < kQ; ++i)
#pragma unroll
        for (int k = 0; k < kQ; ++k)
            if (i < q && k < q) M[i * q + k] = (float)Mi[i][k];
}

// One subspace step from k_step_part's partials.  With Y = D^2 V,
// c = Y^T 1, s = V^T 1 and the centred block Yh = B V = -1/2 (Y - 1 c^T / n):
//     T = V^T Yh    = -1/2 (V^T Y - s c^T / n)     (the Rayleigh-Ritz matrix),
//     G = Yh^T Yh   =  1/4 (Y^T Y - c c^T / n),
// all in FP64 from FP64 sums of the unrounded Y.  Writes T (q x q doubles),
// M = -1/2 R^-1 from the Cholesky factor of G and mean = c / n, so that
// V_next = (Y - 1 mean^T) M = Yh R^-1 (k_rowmat64).
// 256 threads: one wave per SIMD, so that the one thread doing the Cholesky
// keeps its FP64 arrays in registers
constexpr int kOrthWG = 256;

__global__ __launch_bounds__(kOrthWG) void k_step_orth(const double* __restrict__ part, int q, int64_t n,
                                                       double* __restrict__ T, double* __restrict__ M,
                                                       double* __restrict__ mean) {
    __shared__ double tot[4][kQ * kQ];
    __shared__ double sl_sum[kOrthWG];
    const int t = threadIdx.x;
    // entries: c (q), s (q), V^T Y (q*q), Y^T Y (q*q); thread t takes entry
    // t % ne and the partials sl, sl + S, ... (sl = t / ne, S = kOrthWG / ne
    // slices); the slices are then added in slice order
    const int ne = 2 * q + 2 * q * q;
    const int S = kOrthWG / ne;
    const int x = t % ne, sl = t / ne;
    int y, e;
    if (x < q) { y = 0; e = x; }
    else if (x < 2 * q) { y = 1; e = x - q; }
    else if (x < 2 * q + q * q) { y = 2; e = x - 2 * q; }
    else { y = 3; e = x - 2 * q - q * q; }
    double acc = 0.0;
    if (sl < S) {
        const double* pp = part + (int64_t)y * kGB * (kQ * kQ) + e;
        constexpr int kB = 16;
        for (int k0 = sl; k0 < kGB; k0 += kB * S) {
            double v[kB];
#pragma unroll
            for (int k = 0; k < kB; ++k) {
                const int kk = k0 + k * S;
                v[k] = kk < kGB ? pp[(int64_t)kk * (kQ * kQ)] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < kB; ++k) acc += v[k];
        }
    }
    sl_sum[t] = acc;
    __syncthreads();
    if (t < ne) {
        double a = 0.0;
        for (int k = 0; k < S; ++k) a += sl_sum[k * ne + t];
        tot[y][e] = a;
    }
    __syncthreads();
    if (t != 0) return;
    const double inv_n = 1.0 / (double)n;
    double A[kQ][kQ], Mi[kQ][kQ];
#pragma unroll
    for (int a = 0; a < kQ; ++a)
#pragma unroll
        for (int b = 0; b < kQ; ++b) {
            double g = 0.0;
            if (a < q && b < q) {
                T[a * q + b] = -0.5 * (tot[2][a * q + b] - tot[1][a] * tot[0][b] * inv_n);
                g = 0.25 * (tot[3][a * q + b] - tot[0][a] * tot[0][b] * inv_n);
            }
            A[a][b] = g;
        }
    chol_inverse(A, q, Mi);
#pragma unroll
    for (int a = 0; a < kQ; ++a) {
        if (a < q) mean[a] = tot[0][a] * inv_n;
#pragma unroll
        for (int b = 0; b < kQ; ++b)
            if (a < q && b < q) M[a * q + b] = -0.5 * Mi[a][b];
    }
}

// out[i, :] = (Y[i, :] - mean) M in FP64, rounded to FP32 (V of the next step).
__global__ __launch_bounds__(kCW) void k_rowmat64(const double* __restrict__ Y, int q,
                                                  const double* __restrict__ mean, const double* __restrict__ M,
                                                  int64_t n, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kCW + threadIdx.x;
    if (i >= n) return;
    double a[kQ];
#pragma unroll
    for (int c = 0; c < kQ; ++c) a[c] = (c < q) ? Y[i * q + c] - mean[c] : 0.0;
    for (int b = 0; b < q; ++b) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < kQ; ++c)
            if (c < q) s = fma(a[c], M[c * q + b], s);
        out[i * q + b] = (float)s;
    }
}

// The start block: entry k of the n x q array is a value in [-1/2, 1/2) from
// the SplitMix64 finaliser of k (a fixed, reproducible pseudo-random block).
__global__ __launch_bounds__(kCW) void k_start_block(float* __restrict__ V, int64_t count) {
    const int64_t k = (int64_t)blockIdx.x * kCW + threadIdx.x;
    if (k >= count) return;
    uint64_t z = (uint64_t)k * 0x9E3779B97F4A7C15ull + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    V[k] = (float)((double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5);
}

}  // namespace

hipError_t launch_start_block(float* V, int64_t count, hipStream_t s) {
    hipLaunchKernelGGL(k_start_block, dim3((unsigned)((count + kCW - 1) / kCW)), dim3(kCW), 0, s, V, count);
    return hipGetLastError();
}

template <int Q>
static void d2v_q(bool vec, hipStream_t s, const float* Delta, int64_t n, int64_t ldd, const float* V,
                  double* out, int rev) {
    const dim3 grid((unsigned)((n + d2v_rows(Q) - 1) / d2v_rows(Q)));
    if (vec) hipLaunchKernelGGL((k_d2v<true, Q>), grid, dim3(kCW), 0, s, Delta, n, ldd, V, out, rev);
    else hipLaunchKernelGGL((k_d2v<false, Q>), grid, dim3(kCW), 0, s, Delta, n, ldd, V, out, rev);
}

hipError_t launch_d2v(const float* Delta, int64_t n, int64_t ldd, const float* V, int q, double* out,
                      hipStream_t s, bool reverse) {
    const bool vec = (reinterpret_cast<uintptr_t>(Delta) & 15u) == 0 && (ldd % 4) == 0;
    const int rev = reverse ? 1 : 0;
    switch (q) {
        case 1: d2v_q<1>(vec, s, Delta, n, ldd, V, out, rev); break;
        case 2: d2v_q<2>(vec, s, Delta, n, ldd, V, out, rev); break;
        case 3: d2v_q<3>(vec, s, Delta, n, ldd, V, out, rev); break;
        case 4: d2v_q<4>(vec, s, Delta, n, ldd, V, out, rev); break;
        case 5: d2v_q<5>(vec, s, Delta, n, ldd, V, out, rev); break;
        case 6: d2v_q<6>(vec, s, Delta, n, ldd, V, out, rev); break;
        case 7: d2v_q<7>(vec, s, Delta, n, ldd, V, out, rev); break;
        default: d2v_q<8>(vec, s, Delta, n, ldd, V, out, rev); break;
    }
    return hipGetLastError();
}

int64_t step_part_doubles() { return 4 * (int64_t)kGB * kQ * kQ; }

hipError_t launch_subspace_step(const double* Y, const float* V, int q, int64_t n, double* part, double* T,
                                double* M, double* mean, float* Vnext, hipStream_t s) {
    const int64_t rpb = (n + kGB - 1) / kGB;
    hipLaunchKernelGGL(k_step_part, dim3(kGB, 4), dim3(kCW), 0, s, Y, V, q, n, rpb, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_step_orth, dim3(1), dim3(kOrthWG), 0, s, part, q, n, T, M, mean);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rowmat64, dim3((unsigned)((n + kCW - 1) / kCW)), dim3(kCW), 0, s, Y, q, mean, M, n, Vnext);
    return hipGetLastError();
}

hipError_t launch_gram(const float* A, int qa, const float* B, int qb, int64_t n, float* part, float* out,
                       hipStream_t s) {
    const int64_t rpb = (n + kGB - 1) / kGB;
    hipLaunchKernelGGL(k_gram_part, dim3(kGB), dim3(kCW), 0, s, A, B, qa, qb, n, rpb, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gram_final, dim3(1), dim3(kCW), 0, s, part, qa * qb, out);
    return hipGetLastError();
}

int64_t gram_part_floats() { return 2 * (int64_t)kGB * kQ * kQ; }

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
