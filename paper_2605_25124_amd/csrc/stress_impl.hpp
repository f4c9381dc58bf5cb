// stress_impl.hpp -- the stress kernels: fused stress forward + backward over
// the upper triangle of Delta, the deterministic reduction of its partial sums
// and the persistent multi-instance solver, templated on the loss (raw stress
// or Sammon stress).  k_stress.hip instantiates the raw stress and holds the
// host-side launchers; k_stress_sammon.hip instantiates the Sammon stress.
//
// Work decomposition.  The strict upper triangle {i < j} of an n x n problem is
// cut into T x T tiles (I, J), I <= J, enumerated row by row (tri_index), and
// every tile into T/UR work units of UR consecutive rows.  One 256-thread
// workgroup streams one unit of Delta exactly once.  Sixteen lanes (one DPP
// row) cover a tile row: lane c4 owns the columns 4*(c4 + 16q) .. +3, q < T/64,
// read as 16-byte global loads, so each load instruction fetches 256 contiguous
// bytes of the row; the workgroup walks 16 rows per step and the loads of the
// next step are in flight while the current one is computed.  For each pair it
// re-ranks the p latent coordinates of u = Z_i - Z_j, forms the latent distance
// delta, the residual r = delta - Delta_ij, r^2 and the gradient term
// r * d delta / d Z_i (added to row i, subtracted from column j; the common
// factor 2 -- 2 * 2^(1-nu) for p = 2 Gini -- is applied once per point).  The
// Sammon stress weighs both by 1 / Delta_ij and divides by sum_{i<j} Delta_ij.
//
// Reduction.  A unit writes one partial per row (complete for that tile), one
// partial per column and its stress.  A second launch sums, for every point, the
// row partials of its tile row and the column partials of its tile column in a
// fixed order (sixteen interleaved Neumaier sums, one wave each over 64
// consecutive points, combined in index order), and either writes the
// gradient or takes the descent step.  No floating-point
// atomics anywhere: results are bitwise reproducible and independent of
// scheduling and of how many instances share a launch.
#pragma once

#include <hip/hip_ext.h>

#include "common.hpp"
#include "kernels.hpp"

namespace gmds {

constexpr int kWG = 256;
constexpr int kLPR = 16;                 // lanes per tile row = one DPP row
constexpr int kRPS = kWG / kLPR;         // rows per step
constexpr int kSplit = 16;               // interleaved partial sums per point in the reduction
constexpr int kBatch = 8;                // loads in flight per stress-slice sum
constexpr int kWaves = kStressWaves;     // waves per workgroup (one stress partial each)
static_assert(kWaves * 64 == kWG, "one stress partial per wave");

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const f4v gf4;
typedef __attribute__((address_space(1))) const float gfl;
typedef __attribute__((address_space(1))) float gflw;

__device__ __forceinline__ gfl* gp(const float* p) { return (gfl*)p; }
__device__ __forceinline__ gflw* gpw(float* p) { return (gflw*)p; }

template <int T, int P> struct TileShape {
    static constexpr int CPT = T / kLPR;      // columns per thread
    static constexpr int NQ = CPT / 4;        // 16-byte loads per thread and row
    static constexpr int UR = unit_rows(T, P);  // rows per work unit
    static constexpr int STEPS = UR / kRPS;   // pipelined steps per unit
    static constexpr int UNITS = T / UR;      // work units per tile
    // Delta steps in flight per thread: the whole unit while that costs at
    // most 8 loads (32 registers), else two
    static constexpr int DEPTH = (NQ * STEPS <= 8) ? STEPS : 2;
    // LDS of the row reduction: lane c4's sum of component c for unit row r
    // at ((c * kLPR + c4) * RS + r) + c * PAD; the strides keep the writes of
    // a half-wave and the reads of the final sums on distinct banks
    static constexpr int RS = UR + 2;
    static constexpr int PLANE = kLPR * RS + 11;
};

template <int P, int LAT>
struct PG_ { static constexpr int value = (P == 2 && LAT == 0) ? 1 : P; };

// Sum over the 16 lanes of a DPP row by rotations; every lane ends with a
// total and lane 0 of the row is the one used (fixed order).
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float row16_sum(float x) {
    x += dpp_f<0x128>(x);   // row_ror:8
    x += dpp_f<0x124>(x);   // row_ror:4
    x += dpp_f<0x122>(x);   // row_ror:2
    x += dpp_f<0x121>(x);   // row_ror:1
    return x;
}

// Stress term of one pair, added to sst with one FMA, and its gradient term g
// (without the common factor), both weighted by the loss's pair weight w:
// w r^2 and w r d delta / d Z_i.
// MASK: `valid` zeroes pairs outside the strict upper triangle or past n.
// u_c = fl32(Z_i,c - Z_j,c).  Gini: doubled midranks t_c of u over its p
// coordinates, a_c = (p/2) W_p[t_c], delta = sum_c u_c a_c, g = r a.
// Euclid: delta = |u|, g = r u / |u| (0 when u = 0).
// Weighted residual: Sammon's weight 1/Delta_ij (a pair with Delta_ij = 0
// carries none); the raw stress weighs every pair by 1.
template <int LOSS>
__device__ __forceinline__ float weigh(float r, float d) {
    if constexpr (LOSS == kLossSammon) return (d > 0.f) ? r * __builtin_amdgcn_rcpf(d) : 0.f;
    else return r;
}

// h with its sign flipped where s is negative (s a coordinate difference):
// one bit operation.
__device__ __forceinline__ float signed_as(float h, float s) {
    return __int_as_float(__float_as_int(h) ^ (__float_as_int(s) & (int)0x80000000u));
}

template <int P, int LAT, int LOSS, bool GRAD, bool MASK>
__device__ __forceinline__ void pair_term(const float (&zi)[P], const float (&zj)[P], float d, bool valid,
                                          int p, const InstDesc& D, float (&g)[PG_<P, LAT>::value], float& sst) {
    constexpr int PG = PG_<P, LAT>::value;
    float u[P];
#pragma unroll
    for (int c = 0; c < P; ++c) u[c] = zi[c] - zj[c];
    if constexpr (P == 2 && LAT == 0) {
        // t = (2,4) if u1 < u2, (4,2) if u1 > u2, (3,3) on a tie, hence
        // delta = 2^(1-nu) |u2 - u1| and a = 2^(1-nu) sgn(u2 - u1) (-1, +1);
        // g keeps r sgn(u2 - u1), the second component.
        const float w = u[1] - u[0];
        float r = fmaf(D.c2, fabsf(w), -d);
        if constexpr (MASK) r = valid ? r : 0.f;
        const float rw = weigh<LOSS>(r, d);
        if constexpr (GRAD) g[0] = (w > 0.f) ? rw : ((w < 0.f) ? -rw : 0.f);
        sst = fmaf(r, rw, sst);
    } else if constexpr (P == 3 && LAT == 0) {
        // Untied u takes the doubled midranks (2, 4, 6) in sorted order, and the
        // middle weight is exactly 0, so delta = a_max (u_max - u_min) with
        // a_max = (3/2) W_3[6] = -a_min.  A tie (rare) takes the general rule.
        const float mx = fmaxf(fmaxf(u[0], u[1]), u[2]);
        const float mn = fminf(fminf(u[0], u[1]), u[2]);
        const bool tie = (u[0] == u[1]) || (u[1] == u[2]) || (u[0] == u[2]);
        float r, a[3];
        if (!tie) {
            const float wmax = D.wtab[4], wmin = D.wtab[0];
            r = fmaf(wmax, mx - mn, -d);
#pragma unroll
            for (int c = 0; c < 3; ++c) a[c] = (u[c] == mx) ? wmax : ((u[c] == mn) ? wmin : 0.f);
        } else {
            float delta = 0.f;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                int t = 1;
#pragma unroll
                for (int k = 0; k < 3; ++k) t += (u[k] < u[c]) ? 2 : ((u[k] == u[c]) ? 1 : 0);
                float w = D.wtab[0];
#pragma unroll
                for (int q = 1; q < 5; ++q) w = (t - 2 == q) ? D.wtab[q] : w;
                a[c] = w;
                delta = fmaf(u[c], w, delta);
            }
            r = delta - d;
        }
        if constexpr (MASK) r = valid ? r : 0.f;
        const float rw = weigh<LOSS>(r, d);
        if constexpr (GRAD) {
#pragma unroll
            for (int c = 0; c < 3; ++c) g[c] = rw * a[c];
        }
        sst = fmaf(r, rw, sst);
    } else if constexpr (LAT == 0) {
        float a[P];
        float delta = 0.f;
#pragma unroll
        for (int c = 0; c < P; ++c) {
            int t = 1;
#pragma unroll
            for (int k = 0; k < P; ++k)
                if (P != kMaxP || k < p) t += (u[k] < u[c]) ? 2 : ((u[k] == u[c]) ? 1 : 0);
            float w = D.wtab[0];
#pragma unroll
            for (int q = 1; q < 2 * P - 1; ++q) w = (t - 2 == q) ? D.wtab[q] : w;
            if (P == kMaxP && c >= p) w = 0.f;
            a[c] = w;
            delta = fmaf(u[c], w, delta);
        }
        float r = delta - d;
        if constexpr (MASK) r = valid ? r : 0.f;
        const float rw = weigh<LOSS>(r, d);
        if constexpr (GRAD) {
#pragma unroll
            for (int c = 0; c < PG; ++c) g[c] = rw * a[c];
        }
        sst = fmaf(r, rw, sst);
    } else {
        float ss = 0.f;
#pragma unroll
        for (int c = 0; c < P; ++c) ss = fmaf(u[c], u[c], ss);
        const float rs = (ss > 0.f) ? rsqrtf(ss) : 0.f;
        float r = fmaf(ss, rs, -d);
        if constexpr (MASK) r = valid ? r : 0.f;
        const float rw = weigh<LOSS>(r, d);
        if constexpr (GRAD) {
            const float f = rw * rs;
#pragma unroll
            for (int c = 0; c < PG; ++c) g[c] = f * u[c];
        }
        sst = fmaf(r, rw, sst);
    }
}

// Fixed-shape workgroup sum of compensated pairs; every thread gets the total.
__device__ Comp wg_sum(Comp v, float* lds) {
    const int tid = threadIdx.x;
    __syncthreads();
    lds[tid] = v.hi;
    lds[kWG + tid] = v.lo;
    __syncthreads();
#pragma unroll
    for (int st = kWG / 2; st > 0; st >>= 1) {
        if (tid < st) {
            Comp a;
            a.hi = lds[tid];
            a.lo = lds[kWG + tid];
            Comp b;
            b.hi = lds[tid + st];
            b.lo = lds[kWG + tid + st];
            a.add(b);
            lds[tid] = a.hi;
            lds[kWG + tid] = a.lo;
        }
        __syncthreads();
    }
    Comp r;
    r.hi = lds[0];
    r.lo = lds[kWG];
    __syncthreads();
    return r;
}

// LDS floats used by one unit: the latent rows and columns of the unit, the
// column reduction (16 row groups x T) and the stress tree.
template <int P, int T>
constexpr int unit_lds_floats() {
    constexpr int ROWS = P * TileShape<T, P>::PLANE;
    constexpr int COLS = kRPS * T;
    return TileShape<T, P>::UR * P + T * P + (ROWS > COLS ? ROWS : COLS);
}

// Stream unit `sub` (rows I*T + sub*UR ..) of tile lt = (I, J) of instance D:
// row partials rowpart[lt][row], column partials colpart[lt][sub][col] (GRAD)
// and its stress, one (hi, lo) per wave: sigpart[(lt*UNITS + sub)*kWaves + w].
template <int P, int LAT, int LOSS, int T, bool GRAD, bool MASK>
__device__ void unit_body(const InstDesc& D, int64_t lt, int sub, int64_t I, int64_t J, float* lds) {
    constexpr int CPT = TileShape<T, P>::CPT;
    constexpr int NQ = TileShape<T, P>::NQ;
    constexpr int UNITS = TileShape<T, P>::UNITS;
    constexpr int UR = TileShape<T, P>::UR;
    constexpr int STEPS = TileShape<T, P>::STEPS;
    constexpr int PG = PG_<P, LAT>::value;
    const int tid = threadIdx.x;
    const int c4 = tid % kLPR;
    const int rr = tid / kLPR;
    const int64_t n = D.n;
    const int64_t i0 = I * T + sub * UR;
    const int64_t j0 = J * T;
    const int p = (P == kMaxP) ? D.p : P;
    gfl* Zg = gp(D.Z);
    float* zrow = lds;                                  // [UR][P]
    float* zcol = lds + UR * P;                         // [T][P]
    float* red = zcol + T * P;                          // row sums during the steps, then the column sums

    // Delta loads for one step of the unit (unmasked: 16-byte global loads)
    // Masked tiles (the diagonal, and the last tile row or column) decide
    // validity in 32-bit tile-local coordinates: pair (il, jl) exists if
    // il < rows_left, jl < cols_left and, on a diagonal tile, jl > il.  Off
    // the diagonal every column lies above every row.
    const int rows_left = (int)min<int64_t>(n - I * T, (int64_t)T);
    const int cols_left = (int)min<int64_t>(n - j0, (int64_t)T);
    const bool diag = (I == J);
    auto load_step = [&](int s, f4v (&buf)[NQ]) {
        const int64_t i = i0 + s * kRPS + rr;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            if constexpr (!MASK) {
                const int64_t jb = j0 + 4 * (c4 + q * kLPR);
                buf[q] = *(gf4*)(D.Delta + i * D.ldd + jb);
            } else {
                const int il = sub * UR + s * kRPS + rr;
                const int jbl = 4 * (c4 + q * kLPR);
                f4v v = {0.f, 0.f, 0.f, 0.f};
                if (il < rows_left && jbl < cols_left && (!diag || jbl + 3 > il)) {
                    const float* Dr = D.Delta + i * D.ldd + j0;
                    if (D.vec && jbl + 3 < cols_left) {
                        v = *(gf4*)(Dr + jbl);
                    } else {
                        if (jbl + 0 < cols_left && (!diag || jbl + 0 > il)) v.x = gp(Dr)[jbl + 0];
                        if (jbl + 1 < cols_left && (!diag || jbl + 1 > il)) v.y = gp(Dr)[jbl + 1];
                        if (jbl + 2 < cols_left && (!diag || jbl + 2 > il)) v.z = gp(Dr)[jbl + 2];
                        if (jbl + 3 < cols_left && (!diag || jbl + 3 > il)) v.w = gp(Dr)[jbl + 3];
                    }
                }
                buf[q] = v;
            }
        }
    };
    // The latent rows and columns of the unit are requested first (coalesced),
    // then the first DEPTH steps of Delta, so that both are in flight together
    // while the coordinates wait for their LDS slots; afterwards step
    // s + DEPTH is loaded into the slot that step s has just been computed from.
    constexpr int NZR = (UR * P + kWG - 1) / kWG;
    constexpr int NZC = (T * P + kWG - 1) / kWG;
    float zr_[NZR], zc_[NZC];
#pragma unroll
    for (int k = 0; k < NZR; ++k) {
        const int x = tid + k * kWG;
        const int r = x / P, c = x % P;
        const int64_t i = i0 + r;
        zr_[k] = (x < UR * P && c < p && (!MASK || i < n)) ? Zg[i * D.ldz + c] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < NZC; ++k) {
        const int x = tid + k * kWG;
        const int r = x / P, c = x % P;
        const int64_t j = j0 + r;
        zc_[k] = (x < T * P && c < p && (!MASK || j < n)) ? Zg[j * D.ldz + c] : 0.f;
    }
    constexpr int DEPTH = TileShape<T, P>::DEPTH;
    f4v buf[DEPTH][NQ];
#pragma unroll
    for (int s = 0; s < DEPTH; ++s) load_step(s, buf[s]);
#pragma unroll
    for (int k = 0; k < NZR; ++k)
        if (tid + k * kWG < UR * P) zrow[tid + k * kWG] = zr_[k];
#pragma unroll
    for (int k = 0; k < NZC; ++k)
        if (tid + k * kWG < T * P) zcol[tid + k * kWG] = zc_[k];
    __syncthreads();
    float zj[CPT][P];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int c = 0; c < P; ++c) zj[q * 4 + e][c] = zcol[(4 * (c4 + q * kLPR) + e) * P + c];
    float colacc[CPT][PG];
#pragma unroll
    for (int x = 0; x < CPT; ++x)
#pragma unroll
        for (int c = 0; c < PG; ++c) colacc[x][c] = -0.f;   // -0 + x == x: the first add folds away
    Comp sig;

    auto compute_step = [&](int s, const f4v (&buf)[NQ]) {
        const int il = sub * UR + s * kRPS + rr;           // row within the tile
        float zi[P];
#pragma unroll
        for (int c = 0; c < P; ++c) zi[c] = zrow[(s * kRPS + rr) * P + c];
        float rowacc[PG];
#pragma unroll
        for (int c = 0; c < PG; ++c) rowacc[c] = -0.f;
        float sst = 0.f;
        // p = 2 Gini on an interior tile: unless some pair of the step is tied
        // (w = u2 - u1 = 0) somewhere in the wave, the gradient term is the
        // weighted residual with the sign of w flipped in (sign-bit xor),
        // which equals the general rule's select bit for bit.
        bool fast = false;
        float w2[CPT];
        if constexpr (P == 2 && LAT == 0 && !MASK) {
            bool tie = false;
#pragma unroll
            for (int x = 0; x < CPT; ++x) {
                w2[x] = (zi[1] - zj[x][1]) - (zi[0] - zj[x][0]);
                tie |= (w2[x] == 0.f);
            }
            fast = __builtin_amdgcn_ballot_w64(tie) == 0;
        }
        if (fast) {
            if constexpr (P == 2 && LAT == 0 && !MASK) {
#pragma unroll
                for (int q = 0; q < NQ; ++q)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int x = q * 4 + e;
                        const float d = buf[q][e];
                        const float r = fmaf(D.c2, fabsf(w2[x]), -d);
                        const float rw = weigh<LOSS>(r, d);
                        sst = fmaf(r, rw, sst);
                        if constexpr (GRAD) {
                            const float g = __int_as_float(__float_as_int(rw) ^
                                                           (__float_as_int(w2[x]) & (int)0x80000000u));
                            rowacc[0] += g;
                            colacc[x][0] += g;
                        }
                    }
            }
        } else if constexpr (P == 3 && LAT == 0) {
            // p = 3 Gini.  Untied u takes the doubled midranks (2, 4, 6) in
            // sorted order and the middle weight is exactly 0, so
            // delta = a (u_max - u_min) with a = (3/2) W_3[6]; over the
            // coordinate differences d_ab = u_a - u_b, u_max - u_min is
            // max |d_ab| (the same rounded difference).  The gradient term is
            // +h on the largest coordinate, -h on the smallest and 0 on the
            // middle one (h = a times the weighted residual rw).  The terms
            // are accumulated in units of a/2, the reduction applying that
            // factor once per point: with s_ab = rw carrying the sign of
            // d_ab, the term of coordinate a is s_ab + s_ac, and rw + rw and
            // rw - rw are exact, so every accumulated term is exact and no
            // component is recovered from the others.  A tied pair (some
            // d_ab == 0) or a pair outside the triangle gets r = 0 here and
            // adds nothing; if some lane of the wave holds a tied pair of the
            // triangle, the step's tied pairs then take the general midrank
            // rule, converted to the same units.
            const float wmax = D.wtab[4];
            bool tied = false;
#pragma unroll
            for (int q = 0; q < NQ; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int x = q * 4 + e;
                    const float d = buf[q][e];
                    const float u0 = zi[0] - zj[x][0], u1 = zi[1] - zj[x][1], u2 = zi[2] - zj[x][2];
                    const float d01 = u0 - u1, d02 = u0 - u2, d12 = u1 - u2;
                    const float span = fmaxf(fmaxf(fabsf(d01), fabsf(d02)), fabsf(d12));
                    const float gap = fminf(fminf(fabsf(d01), fabsf(d02)), fabsf(d12));
                    bool valid = true;
                    if constexpr (MASK) {
                        const int jl = 4 * (c4 + q * kLPR) + e;
                        valid = (il < rows_left) && (jl < cols_left) && (!diag || jl > il);
                    }
                    const bool tie = gap == 0.f;
                    tied |= valid && tie;
                    float r = fmaf(wmax, span, -d);
                    r = (valid && !tie) ? r : 0.f;
                    const float rw = weigh<LOSS>(r, d);
                    sst = fmaf(r, rw, sst);
                    if constexpr (GRAD) {
                        const float s01 = signed_as(rw, d01), s02 = signed_as(rw, d02), s12 = signed_as(rw, d12);
                        const float g0 = s01 + s02, g1 = s12 - s01, g2 = -(s02 + s12);
                        rowacc[0] += g0;
                        rowacc[1] += g1;
                        rowacc[2] += g2;
                        colacc[x][0] += g0;
                        colacc[x][1] += g1;
                        colacc[x][2] += g2;
                    }
                }
            if (__builtin_amdgcn_ballot_w64(tied) != 0) {
                const float to_units = wmax > 0.f ? 2.f / wmax : 0.f;
#pragma unroll
                for (int q = 0; q < NQ; ++q)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int x = q * 4 + e;
                        const int jl = 4 * (c4 + q * kLPR) + e;
                        const bool valid = !MASK || ((il < rows_left) && (jl < cols_left) && (!diag || jl > il));
                        const float u0 = zi[0] - zj[x][0], u1 = zi[1] - zj[x][1], u2 = zi[2] - zj[x][2];
                        const bool tie = (u0 == u1) || (u0 == u2) || (u1 == u2);
                        float g[PG];
                        pair_term<P, LAT, LOSS, GRAD, true>(zi, zj[x], buf[q][e], valid && tie, p, D, g, sst);
                        if constexpr (GRAD) {
#pragma unroll
                            for (int c = 0; c < PG; ++c) {
                                rowacc[c] += g[c] * to_units;
                                colacc[x][c] += g[c] * to_units;
                            }
                        }
                    }
            }
        } else {
#pragma unroll
            for (int q = 0; q < NQ; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int x = q * 4 + e;
                    const int jl = 4 * (c4 + q * kLPR) + e;
                    const bool valid = !MASK || ((il < rows_left) && (jl < cols_left) && (!diag || jl > il));
                    float g[PG];
                    pair_term<P, LAT, LOSS, GRAD, MASK>(zi, zj[x], buf[q][e], valid, p, D, g, sst);
                    if constexpr (GRAD) {
#pragma unroll
                        for (int c = 0; c < PG; ++c) {
                            rowacc[c] += g[c];
                            colacc[x][c] += g[c];
                        }
                    }
                }
        }
        if constexpr (GRAD) {
            // the 16 lanes' sums of this row are added after the last step
            constexpr int RS = TileShape<T, P>::RS, PLANE = TileShape<T, P>::PLANE;
#pragma unroll
            for (int c = 0; c < PG; ++c) red[c * PLANE + c4 * RS + s * kRPS + rr] = rowacc[c];
        }
        sig.add(sst);
    };

#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
        compute_step(s, buf[s % DEPTH]);
        if (s + DEPTH < STEPS) load_step(s + DEPTH, buf[s % DEPTH]);
    }

    if constexpr (GRAD) {
        // row partials: the sums of the 16 lanes of each row, in lane order
        {
            constexpr int RS = TileShape<T, P>::RS, PLANE = TileShape<T, P>::PLANE;
            __syncthreads();
            for (int x = tid; x < UR * PG; x += kWG) {
                const int rl = x / PG, c = x % PG;
                const float* src = red + c * PLANE + rl;
                float acc = src[0];
#pragma unroll
                for (int l = 1; l < kLPR; ++l) acc += src[l * RS];
                const int il = sub * UR + rl;
                if (!MASK || il < rows_left) gpw(D.rowpart)[(lt * T + il) * PG + c] = acc;
            }
        }
        // column partials: the 16 row groups hold partial sums of each column
#pragma unroll
        for (int c = 0; c < PG; ++c) {
            __syncthreads();
#pragma unroll
            for (int q = 0; q < NQ; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) red[rr * T + 4 * (c4 + q * kLPR) + e] = colacc[q * 4 + e][c];
            __syncthreads();
            for (int x = tid; x < T; x += kWG) {
                float acc = 0.f;
#pragma unroll
                for (int r = 0; r < kRPS; ++r) acc += red[r * T + x];
                gpw(D.colpart)[((lt * UNITS + sub) * T + x) * PG + c] = acc;
            }
        }
    }
    // stress: one partial per wave.  Each lane's compensated pair (hi, lo) is
    // summed over the wave part by part, in a fixed tree: rotation sums within
    // each row of 16 lanes, then the four rows.
    {
        float h = row16_sum(sig.hi), l = row16_sum(sig.lo);
        h += __shfl_xor(h, 16, 64);
        l += __shfl_xor(l, 16, 64);
        h += __shfl_xor(h, 32, 64);
        l += __shfl_xor(l, 32, 64);
        sig.hi = h;
        sig.lo = l;
    }
    if ((tid & 63) == 0) {
        const int64_t slot = (lt * UNITS + sub) * kWaves + (tid >> 6);
        gpw(D.sigpart)[2 * slot + 0] = sig.hi;
        gpw(D.sigpart)[2 * slot + 1] = sig.lo;
    }
}

template <int P, int LAT, int LOSS, int T, bool GRAD>
__device__ __forceinline__ void stress_unit(const InstDesc& D, int64_t lu, float* lds) {
    constexpr int UNITS = TileShape<T, P>::UNITS;
    const int64_t lt = lu / UNITS;
    const int sub = (int)(lu % UNITS);
    int64_t I, J;
    tri_decode(lt, D.nb, I, J);
    if (I * T + (int64_t)sub * TileShape<T, P>::UR >= D.n) return;   // rows past n: nothing to do
    const bool interior = D.vec && (I < J) && ((J + 1) * T <= D.n);
    if (interior) unit_body<P, LAT, LOSS, T, GRAD, false>(D, lt, sub, I, J, lds);
    else unit_body<P, LAT, LOSS, T, GRAD, true>(D, lt, sub, I, J, lds);
}

// ---------------------------------------------------------------- reduction
// Every sum below has a fixed shape that does not depend on how many threads
// execute it, so the reduction launch (kRedWG threads) and the persistent
// solver (kWG threads) produce bitwise identical results.
constexpr int kRedWG = 1024;             // threads of a reduction block for large instances
constexpr int kRedWGSmall = 256;         // ... and when every instance of the launch is small
constexpr int kNPT = 64;                 // points per reduction group (one per lane)
constexpr int kVT = 1024;                // virtual threads of a stress slice

// Common factor of every gradient term: 2 for the raw stress, 2 / sum Delta
// for the Sammon stress.
__device__ __forceinline__ float loss_factor(const InstDesc& D) {
    if (D.loss == kLossSammon) return (float)(2.0 / ((double)D.dsum[0] + (double)D.dsum[1]));
    return 2.f;
}

// Loads in flight per partial gradient sum: 8 for one or two stored
// components (more only add masked loads for small instances), fewer for
// wider gradients to bound the registers.
__host__ __device__ constexpr int red_batch(int pg) { return pg <= 2 ? 8 : (pg <= 4 ? 4 : 2); }

// Partial gradient of point k: terms t = s, s + kSplit, ... of the sequence
// "row partials of its tile row (tiles (b, b..nb-1)), then column partials of
// its tile column (every unit of tiles (0..b, b))", summed (Neumaier) in
// increasing t.  The loads of a batch are in flight together; an absent term
// adds an exact 0.
template <int P, int LAT, int T>
__device__ __forceinline__ void point_partial(const InstDesc& D, int64_t k, int s, Comp (&acc)[PG_<P, LAT>::value]) {
    constexpr int PG = PG_<P, LAT>::value;
    constexpr int UNITS = TileShape<T, P>::UNITS;
    constexpr int RB = red_batch(PG);
    // Tile and unit indices fit 32 bits: the host caps an instance's work
    // units at 2^31 - 1, so nb^2 < 2^32; element offsets are taken in 64 bits.
    const uint32_t b = (uint32_t)(k / T);
    const int64_t kl = k % T;
    const uint32_t nb = (uint32_t)D.nb;
    const int nrow = (int)(nb - b);
    const int nterm = nrow + (int)(b + 1) * UNITS;
    gfl* rbase = gp(D.rowpart) + (tri_index(b, b, nb) * T + kl) * PG;   // row tiles (b, b..) are consecutive
    gfl* cbase = gp(D.colpart) + kl * PG;
    for (int t0 = s; t0 < nterm; t0 += kSplit * RB) {
        float v[RB][PG];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int t = t0 + q * kSplit;
            if (t < nrow) {
#pragma unroll
                for (int c = 0; c < PG; ++c) v[q][c] = rbase[t * (T * PG) + c];
            } else {
                const uint32_t tc = (uint32_t)(t - nrow);
                const uint32_t I = tc / UNITS;
                const uint32_t u = tc % UNITS;
                const uint32_t lt = I * nb - (I * (I - 1)) / 2 + (b - I);
                // units past n (only in the last tile) were never written
                const bool ok = (t < nterm) && !(I == nb - 1 && (int64_t)I * T + (int64_t)u * TileShape<T, P>::UR >= D.n);
                const uint64_t off = (uint64_t)(lt * UNITS + u) * (T * PG);
#pragma unroll
                for (int c = 0; c < PG; ++c) v[q][c] = ok ? -cbase[off + c] : 0.f;
            }
        }
#pragma unroll
        for (int q = 0; q < RB; ++q)
#pragma unroll
            for (int c = 0; c < PG; ++c) acc[c].add(v[q][c]);
    }
}

// Gradient of the kNPT points k0 .. k0+kNPT-1: the kSplit partial sums of each
// point (one wave per partial sum: 64 consecutive points, coalesced loads)
// are added in index order, scaled by the common factor and applied.  NT is
// the number of threads executing the call.  LDS: 2 * kSplit * kNPT * PG floats.
template <int P, int LAT, int T, int NT>
__device__ void reduce_group(const InstDesc& D, int64_t k0, int mode, float* lds) {
    constexpr int PG = PG_<P, LAT>::value;
    const int tid = threadIdx.x;
    const int p = (P == kMaxP) ? D.p : P;
    // the combining threads fetch what they update before the partial sums
    // arrive, so that its latency overlaps theirs
    const bool comb = tid < kNPT && k0 + tid < D.n;
    float zold[P];
    float sc = 1.f;
    if (comb) {
        if (mode == kModeGrad) {
            if (D.grad_out) sc = *D.grad_out;
        } else {
#pragma unroll
            for (int c = 0; c < P; ++c) zold[c] = (c < p) ? D.Z[(k0 + tid) * D.ldz + c] : 0.f;
        }
    }
    for (int item = tid; item < kSplit * kNPT; item += NT) {
        const int sp = item / kNPT;
        const int pl = item % kNPT;
        const int64_t k = k0 + pl;
        Comp acc[PG];
        if (k < D.n) point_partial<P, LAT, T>(D, k, sp, acc);
#pragma unroll
        for (int c = 0; c < PG; ++c) {
            lds[((c * kSplit + sp) * kNPT + pl) * 2] = acc[c].hi;
            lds[((c * kSplit + sp) * kNPT + pl) * 2 + 1] = acc[c].lo;
        }
    }
    __syncthreads();
    if (comb) {
        const int pl = tid;
        const int64_t k = k0 + pl;
        Comp tot[PG];
#pragma unroll
        for (int c = 0; c < PG; ++c)
#pragma unroll 4
            for (int q = 0; q < kSplit; ++q) {
                Comp x;
                x.hi = lds[((c * kSplit + q) * kNPT + pl) * 2];
                x.lo = lds[((c * kSplit + q) * kNPT + pl) * 2 + 1];
                tot[c].add(x);
            }
        float G[P];
        if constexpr (P == 2 && LAT == 0) {
            const float v = loss_factor(D) * D.c2 * tot[0].value();
            G[0] = -v;
            G[1] = v;
        } else if constexpr (P == 3 && LAT == 0) {
            // the p = 3 Gini terms were accumulated in units of a/2 (a = (3/2) W_3[6])
            const float f = loss_factor(D) * (0.5f * D.wtab[4]);
#pragma unroll
            for (int c = 0; c < P; ++c) G[c] = f * tot[c].value();
        } else {
#pragma unroll
            for (int c = 0; c < P; ++c) G[c] = loss_factor(D) * tot[c].value();
        }
        if (mode == kModeGrad) {
#pragma unroll
            for (int c = 0; c < P; ++c)
                if (c < p) D.gradZ[k * D.ldg + c] = sc * G[c];
        } else {
#pragma unroll
            for (int c = 0; c < P; ++c)
                if (c < p) D.Z[k * D.ldz + c] = zold[c] - D.eta * G[c];
        }
    }
    __syncthreads();
}

// Stress of instance D from the per-wave unit partials (units past n, only in
// the last tile, hold nothing), in contiguous slices.  A slice is a fixed
// shape sum: virtual thread v < kVT adds partials a+v, a+v+kVT, ... in order,
// then a fixed binary tree over the kVT values; slices are added in order
// (at most kSigSlices of them, the room the host reserves per instance).

template <int T, int P>
__device__ __forceinline__ int64_t sigma_count(const InstDesc& D) {
    return tri_count(D.nb) * TileShape<T, P>::UNITS * kWaves;
}
// At most kVT * kBatch partials per slice (one batch of loads per virtual
// thread), at most kSigSlices slices (one slice -- written directly, no
// combining step -- for small instances).
template <int T, int P>
__device__ __forceinline__ int sigma_slices(const InstDesc& D) {
    const int64_t s = (sigma_count<T, P>(D) + kVT * kBatch - 1) / (kVT * kBatch);
    return (int)(s < 1 ? 1 : (s > kSigSlices ? kSigSlices : s));
}

// LDS: 2 * kVT floats.  All NT threads return the slice sum.
template <int T, int P, int NT>
__device__ Comp sigma_slice(const InstDesc& D, int slice, float* lds) {
    constexpr int UNITS = TileShape<T, P>::UNITS;
    const int64_t nt = tri_count(D.nb);
    const int64_t cnt = sigma_count<T, P>(D);
    const int ns = sigma_slices<T, P>(D);
    const int64_t a = cnt * slice / ns;
    const int64_t e = cnt * (slice + 1) / ns;
    gfl* sp = gp(D.sigpart);
    for (int vt = threadIdx.x; vt < kVT; vt += NT) {
        Comp acc;
        for (int64_t t0 = a + vt; t0 < e; t0 += (int64_t)kVT * kBatch) {
            float hv[kBatch], lv[kBatch];
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
                const int64_t t = t0 + (int64_t)q * kVT;
                const int64_t lu = t / kWaves;
                const int u = (int)(lu % UNITS);
                const bool ok = (t < e) && !(lu / UNITS == nt - 1 && (D.nb - 1) * T + (int64_t)u * TileShape<T, P>::UR >= D.n);
                hv[q] = ok ? sp[2 * t] : 0.f;
                lv[q] = ok ? sp[2 * t + 1] : 0.f;
            }
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
                Comp x;
                x.hi = hv[q];
                x.lo = lv[q];
                acc.add(x);
            }
        }
        lds[vt] = acc.hi;
        lds[kVT + vt] = acc.lo;
    }
    __syncthreads();
    // The tree's last six levels (64 values) take one wave and its shuffles
    // when every value has a thread of its own (the same additions in the
    // same order as through LDS, without a barrier per level).
    constexpr int STW = (NT >= kVT) ? 64 : 1;
    for (int st = kVT / 2; st >= STW; st >>= 1) {
        for (int x = threadIdx.x; x < st; x += NT) {
            Comp u;
            u.hi = lds[x];
            u.lo = lds[kVT + x];
            Comp w;
            w.hi = lds[x + st];
            w.lo = lds[kVT + x + st];
            u.add(w);
            lds[x] = u.hi;
            lds[kVT + x] = u.lo;
        }
        __syncthreads();
    }
    if constexpr (NT >= kVT) {
        if (threadIdx.x < 64) {
            Comp u;
            u.hi = lds[threadIdx.x];
            u.lo = lds[kVT + threadIdx.x];
            for (int st = 32; st > 0; st >>= 1) {
                Comp w;
                w.hi = __shfl_down(u.hi, st, 64);
                w.lo = __shfl_down(u.lo, st, 64);
                u.add(w);
            }
            if (threadIdx.x == 0) {
                lds[0] = u.hi;
                lds[kVT] = u.lo;
            }
        }
        __syncthreads();
    }
    Comp r;
    r.hi = lds[0];
    r.lo = lds[kVT];
    __syncthreads();
    return r;
}

template <int T, int P, int NT>
__device__ Comp instance_sigma(const InstDesc& D, float* lds) {
    const int ns = sigma_slices<T, P>(D);
    if (ns == 1) return sigma_slice<T, P, NT>(D, 0, lds);
    Comp tot;
    for (int sl = 0; sl < ns; ++sl) tot.add(sigma_slice<T, P, NT>(D, sl, lds));
    return tot;
}

__device__ __forceinline__ void write_sigma(const InstDesc& D, int mode, int it, const Comp& s_in) {
    if (threadIdx.x != 0) return;
    // Sammon stress: the weighted sum over the sum of the dissimilarities
    Comp s = s_in;
    if (D.loss == kLossSammon) {
        const double v = ((double)s_in.hi + (double)s_in.lo) / ((double)D.dsum[0] + (double)D.dsum[1]);
        s.hi = (float)v;
        s.lo = (float)(v - (double)s.hi);
    }
    if (mode == kModeDescent) {
        if (D.sigma_hist) D.sigma_hist[it] = s.hi + s.lo;
        if (D.ks_hist) {
            const double den = (double)D.dsumsq[0] + (double)D.dsumsq[1];
            const double num = (double)s.hi + (double)s.lo;
            D.ks_hist[it] = den > 0.0 ? (float)sqrt(num / den) : 0.f;
        }
    } else if (D.out_sigma) {
        D.out_sigma[0] = s.hi;
        D.out_sigma[1] = s.lo;
    }
}

// Map a global unit index to its instance (descriptors sorted by tile_off,
// which counts units).
__device__ __forceinline__ int find_instance(const InstDesc* dd, int n_inst, int64_t q) {
    int lo = 0, hi = n_inst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (dd[mid].tile_off <= q) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Waves per SIMD asked of the register allocator: the raw stress with the
// Gini latent at p = 2 and p = 3 on 128-wide tiles.  The masked path of the
// edge and diagonal tiles sets the register count (88 and 153 against 75 and
// 114 for the interior path); under the cap the allocator spills a few
// registers instead (16 and 104 bytes per lane), and the extra wave per SIMD
// pays for it (about 3 % and 7 %).  The Sammon kernels would spill more, so
// they keep the default.
template <int P, int LAT, int LOSS, int T>
constexpr int units_waves() {
    if (LOSS != kLossRaw || T != 128 || LAT != 0) return 1;
    return P == 2 ? 6 : (P == 3 ? 4 : 1);
}

template <int P, int LAT, int LOSS, int T, bool GRAD>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(units_waves<P, LAT, LOSS, T>())))
void k_stress_units(const InstDesc* __restrict__ dd, int n_inst, int64_t q_base, int rev) {
    __shared__ float lds[unit_lds_floats<P, T>()];
    // rev: the launch takes its units last to first, so that it starts on the
    // tiles the previous launch read last (still in the memory-side cache)
    const int64_t q = (int64_t)(rev ? gridDim.x - 1 - blockIdx.x : blockIdx.x) + q_base;
    const int k = find_instance(dd, n_inst, q);
    const InstDesc D = dd[k];
    stress_unit<P, LAT, LOSS, T, GRAD>(D, q - D.tile_off, lds);
}

template <int PG>
constexpr int reduce_lds_floats() {
    return 2 * kSplit * kNPT * PG > 2 * kVT ? 2 * kSplit * kNPT * PG : 2 * kVT;
}

// Reduction launch over the concatenated blocks of all instances (block
// offsets in red_off).  The first blocks of an instance sum one slice of its
// stress each (with several slices, the last to finish adds them in order);
// the following blocks take kNPT points each.
template <int P, int LAT, int T, int NT>
__global__ __launch_bounds__(NT) void k_stress_reduce(const InstDesc* __restrict__ dd, int n_inst,
                                                      const int32_t* __restrict__ bmap, int64_t q_base, int mode,
                                                      int it) {
    constexpr int PG = PG_<P, LAT>::value;
    __shared__ float lds[reduce_lds_floats<PG>()];
    __shared__ int last;
    const int64_t q = (int64_t)blockIdx.x + q_base;
    // the instance of this block: from the host's block map when there is one
    // (one load instead of a chain of dependent ones), else by binary search
    int lo = 0;
    if (bmap) {
        lo = bmap[q];
    } else {
        int hi = n_inst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (dd[mid].red_off <= q) lo = mid;
            else hi = mid - 1;
        }
    }
    const InstDesc& D = dd[lo];
    const int64_t b = q - D.red_off;
    const int ns = sigma_slices<T, P>(D);
    if (b < ns) {
        const Comp part = sigma_slice<T, P, NT>(D, (int)b, lds);
        if (threadIdx.x == 0) {
            if (ns == 1) {
                write_sigma(D, mode, it, part);
            } else {
                gpw(D.sigslice)[2 * b] = part.hi;
                gpw(D.sigslice)[2 * b + 1] = part.lo;
                __threadfence();
                last = (atomicAdd(D.instcnt, 1u) + 1 == (uint32_t)ns) ? 1 : 0;
            }
        }
        if (ns == 1) return;
        __syncthreads();
        if (last && threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            Comp tot;
            for (int sl = 0; sl < ns; ++sl) {
                Comp x;
                x.hi = gp(D.sigslice)[2 * sl];
                x.lo = gp(D.sigslice)[2 * sl + 1];
                tot.add(x);
            }
            write_sigma(D, mode, it, tot);
            __hip_atomic_store(D.instcnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }
    if (mode == kModeSigma) return;
    reduce_group<P, LAT, T, NT>(D, (b - ns) * kNPT, mode, lds);
}

// Persistent solver.  Queue item q = (iteration it, instance k, local unit),
// iteration-major, instances in the host's order.  A workgroup pops q, waits
// until instance k has finished iteration it-1 (epoch[k] >= it), streams the
// unit and counts it done (release fence, integer counter); the workgroup that
// completes the last unit of (k, it) reduces the whole instance with the same
// fixed-order sums as the reduction launch, takes the step, resets the counter
// and publishes epoch[k] = it + 1.  Items are popped in queue order and every
// item waits only on items popped before it, whose workgroups are already
// running, so the queue drains whatever the number of resident workgroups.  A
// wait longer than spin_limit ticks of the constant-rate device clock sets the
// abort status; every workgroup then stops popping work and the kernel ends.
template <int P, int LAT, int LOSS, int T>
__global__ __launch_bounds__(kWG) void k_solve_persistent(const InstDesc* __restrict__ dd, int n_inst,
                                                          const int64_t* __restrict__ prefix,
                                                          int64_t per_iter, int iters, SolveCtl* ctl,
                                                          uint32_t* epoch, int64_t spin_limit) {
    constexpr int PG = PG_<P, LAT>::value;
    constexpr int UNITS = TileShape<T, P>::UNITS;
    constexpr int NL1 = unit_lds_floats<P, T>();
    constexpr int NL2 = reduce_lds_floats<PG>();
    __shared__ float lds[NL1 > NL2 ? NL1 : NL2];
    __shared__ int64_t sh_q;
    __shared__ int sh_flag;
    const int tid = threadIdx.x;
    const int64_t total = per_iter * (int64_t)iters;
    for (;;) {
        if (tid == 0) {
            const uint32_t st = __hip_atomic_load(&ctl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int64_t q = total;
            if (st == kStatusOk) q = (int64_t)atomicAdd(&ctl->head, 1ull);
            sh_q = q;
        }
        __syncthreads();
        const int64_t q = sh_q;
        __syncthreads();
        if (q >= total) break;
        const int it = (int)(q / per_iter);
        const int64_t r = q % per_iter;
        int lo = 0, hi = n_inst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= r) lo = mid;
            else hi = mid - 1;
        }
        const int k = lo;
        const int64_t lu = r - prefix[k];
        if (tid == 0) {
            int ok = 1;
            if (__hip_atomic_load(&epoch[k], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < (uint32_t)it) {
                // Every poll is an acquire, which invalidates this XCD's L2
                // (the lines the running units stream from included), so the
                // pause between polls grows, up to about 8000 cycles.
                const uint64_t t0 = wall_clock64();
                int naps = 1;
                while (__hip_atomic_load(&epoch[k], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < (uint32_t)it) {
                    for (int j = 0; j < naps; ++j) __builtin_amdgcn_s_sleep(8);
                    naps = naps < 16 ? 2 * naps : 16;
                    if (__hip_atomic_load(&ctl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != kStatusOk) {
                        ok = 0;
                        break;
                    }
                    if ((int64_t)(wall_clock64() - t0) > spin_limit) {
                        __hip_atomic_store(&ctl->status, (uint32_t)kStatusTimeout, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                        ok = 0;
                        break;
                    }
                }
            }
            sh_flag = ok;
        }
        __syncthreads();
        if (!sh_flag) {
            __syncthreads();
            continue;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const InstDesc D = dd[k];
        stress_unit<P, LAT, LOSS, T, true>(D, lu, lds);
        // every wave's stores have reached this XCD's L2 at the barrier; one
        // device-scope release (an L2 writeback) by one thread then publishes
        // them all with the count (a fence in every wave cost four)
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const uint32_t old = atomicAdd(D.instcnt, 1u);
            sh_flag = (old + 1 == (uint32_t)(tri_count(D.nb) * UNITS)) ? 1 : 0;
        }
        __syncthreads();
        if (sh_flag) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const Comp s = instance_sigma<T, P, kWG>(D, lds);
            write_sigma(D, kModeDescent, it, s);
            for (int64_t k0 = 0; k0 < D.n; k0 += kNPT) reduce_group<P, LAT, T, kWG>(D, k0, kModeDescent, lds);
            __syncthreads();
            if (tid == 0) {      // the release store publishes the workgroup's updates of Z
                __hip_atomic_store(D.instcnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&epoch[k], (uint32_t)(it + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
    }
}


// ------------------------------------------------- launch helpers (per unit)
static inline int p_bucket(int p) { return p <= 4 ? p : kMaxP; }

// A launch on stream s; with both events set (profiling), the runtime stamps
// them at the start and the end of the kernel itself.
struct Launch {
    hipStream_t s;
    LaunchTimer tm;
    bool small = false;     // reduction launch: every instance has at most kSmallReduceN points
    bool rev = false;       // stress-units launch: units in reverse order
};

// Up to this many points per instance the reduction runs in blocks of
// kRedWGSmall threads: the same fixed-shape sums, each thread taking several
// of them, and a quarter of the waves.
constexpr int64_t kSmallReduceN = 4096;

template <typename K, typename... A>
static hipError_t launch_k(K kernel, dim3 grid, dim3 block, const Launch& L, A... args) {
    if (L.tm.start && L.tm.stop)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, L.s, L.tm.start, L.tm.stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, L.s, args...);
    return hipGetLastError();
}

template <int P, int LAT, int LOSS, int T>
static hipError_t units_impl(const InstDesc* dd, int n_inst, int64_t count, int64_t qb, bool grad, const Launch& L) {
    if (count <= 0) return hipSuccess;
    if (grad)
        return launch_k(k_stress_units<P, LAT, LOSS, T, true>, dim3((unsigned)count), dim3(kWG), L, dd, n_inst, qb,
                        (int)L.rev);
    return launch_k(k_stress_units<P, LAT, LOSS, T, false>, dim3((unsigned)count), dim3(kWG), L, dd, n_inst, qb,
                    (int)L.rev);
}

template <int LOSS, int LAT, int T>
static hipError_t units_dispatch_p(const InstDesc* dd, int n_inst, int64_t count, int64_t qb, int p, bool grad,
                                   const Launch& L) {
    switch (p_bucket(p)) {
        case 1: return units_impl<1, LAT, LOSS, T>(dd, n_inst, count, qb, grad, L);
        case 2: return units_impl<2, LAT, LOSS, T>(dd, n_inst, count, qb, grad, L);
        case 3: return units_impl<3, LAT, LOSS, T>(dd, n_inst, count, qb, grad, L);
        case 4: return units_impl<4, LAT, LOSS, T>(dd, n_inst, count, qb, grad, L);
        default: return units_impl<kMaxP, LAT, LOSS, T>(dd, n_inst, count, qb, grad, L);
    }
}

template <int LOSS, int T>
static hipError_t units_dispatch_lat(const InstDesc* dd, int n_inst, int64_t count, int64_t qb, int p, int latent,
                                     bool grad, const Launch& L) {
    if (latent == 0) return units_dispatch_p<LOSS, 0, T>(dd, n_inst, count, qb, p, grad, L);
    return units_dispatch_p<LOSS, 1, T>(dd, n_inst, count, qb, p, grad, L);
}

template <int LOSS>
static hipError_t units_dispatch(const InstDesc* dd, int n_inst, int64_t count, int64_t qb, int p, int latent, int T,
                                 bool grad, const Launch& L) {
    if (T == 64) return units_dispatch_lat<LOSS, 64>(dd, n_inst, count, qb, p, latent, grad, L);
    if (T == 128) return units_dispatch_lat<LOSS, 128>(dd, n_inst, count, qb, p, latent, grad, L);
    return units_dispatch_lat<LOSS, 256>(dd, n_inst, count, qb, p, latent, grad, L);
}

template <int P, int LAT, int LOSS, int T>
static const void* persistent_fn() {
    return reinterpret_cast<const void*>(&k_solve_persistent<P, LAT, LOSS, T>);
}

template <int LOSS, int LAT, int T>
static const void* persistent_table_p(int p) {
    switch (p_bucket(p)) {
        case 1: return persistent_fn<1, LAT, LOSS, T>();
        case 2: return persistent_fn<2, LAT, LOSS, T>();
        case 3: return persistent_fn<3, LAT, LOSS, T>();
        case 4: return persistent_fn<4, LAT, LOSS, T>();
        default: return persistent_fn<kMaxP, LAT, LOSS, T>();
    }
}

template <int LOSS>
static const void* persistent_table(int p, int latent, int T) {
    if (latent == 0) {
        if (T == 64) return persistent_table_p<LOSS, 0, 64>(p);
        if (T == 128) return persistent_table_p<LOSS, 0, 128>(p);
        return persistent_table_p<LOSS, 0, 256>(p);
    }
    if (T == 64) return persistent_table_p<LOSS, 1, 64>(p);
    if (T == 128) return persistent_table_p<LOSS, 1, 128>(p);
    return persistent_table_p<LOSS, 1, 256>(p);
}

// Defined in k_stress_sammon.hip (the Sammon-stress instantiations).
hipError_t launch_units_sammon(const InstDesc* dd, int n_inst, int64_t count, int64_t q_base, int p, int latent,
                               int T, bool grad, hipStream_t s, LaunchTimer tm, bool reverse);
const void* persistent_ptr_sammon(int p, int latent, int T);

}  // namespace gmds
