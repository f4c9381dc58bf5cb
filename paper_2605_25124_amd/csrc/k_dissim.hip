// k_dissim.hip -- generalised Gini pseudo-distances between all pairs of rows.
//
// For a pair (i, j) with z = fl32(X_i - X_j) the symmetrised distance is
//     Delta = (m/2) * sum_c z_c W[t_c],  t = doubled midranks of z,
// and W is increasing in t, so it only depends on z in sorted order: a run of
// equal values at sorted positions a..b (0-based) shares t = a + b + 2.  Each
// pair is therefore sorted once (for every nu of the call) and never
// un-permuted.  The kernels never touch a pow(): the host passes the table
// W_{m,nu}[t], t = 2..2m, per nu.
//
//   m <= 64   k_dissim_lane : one lane per pair, z in registers, Batcher's
//             odd-even merge network pruned to a size bucket B >= m
//             (comparators all put the minimum first, so +inf padding never
//             moves and comparators past B can be dropped).  Weights of untied positions are wave-uniform; a run
//             of ties is corrected in a branch the wave only takes when one of
//             its lanes holds a tie.
//   m <= 4096 k_dissim_group: G lanes per pair (G = 16, 32 or 64), E = P/G values
//             per lane (P the padded power of two), bitonic sort in registers
//             with cross-lane exchanges, run bounds by segmented max/min scans
//             across the G lanes, weights read from LDS.
//
// Both kernels work on 32 x 32 (lane) or 16 x 16 (group) tiles of the pair
// triangle, stage the results in LDS and write Delta[i, j] and its mirror
// Delta[j, i] with coalesced row segments; the diagonal is written as 0.
#include <utility>

#include "common.hpp"
#include "kernels.hpp"

namespace gmds {

constexpr int kDWG = 256;
constexpr int kNuChunk = 8;

__device__ __forceinline__ void cex(float& a, float& b) {
    const float lo = fminf(a, b);
    const float hi = fmaxf(a, b);
    a = lo;
    b = hi;
}

// Compile-time loop: f(std::integral_constant<int, I>) for I = 0 .. N-1, so that
// every register-array index inside f is a constant.
template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

constexpr int ilog2(int x) {
    int r = 0;
    while ((1 << r) < x) ++r;
    return r;
}

// ------------------------------------------------ odd-even merge network
constexpr int next_pow2(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

template <int M>
struct OEMNet {
    static constexpr int N = next_pow2(M);
    // Batcher's odd-even merge sort on N inputs, keeping comparators whose
    // both ends are < M.
    template <bool FILL, typename F>
    static constexpr int walk(F&& f) {
        int c = 0;
        for (int p = 1; p < N; p <<= 1)
            for (int k = p; k >= 1; k >>= 1)
                for (int j = k % p; j + k < N; j += 2 * k)
                    for (int i = 0; i < k && i + j + k < N; ++i)
                        if ((i + j) / (2 * p) == (i + j + k) / (2 * p) && i + j + k < M) {
                            if (FILL) f(c, i + j, i + j + k);
                            ++c;
                        }
        return c;
    }
    static constexpr int count() {
        return walk<false>([](int, int, int) {});
    }
    static constexpr int C = count();
    struct Net {
        short a[C > 0 ? C : 1];
        short b[C > 0 ? C : 1];
    };
    static constexpr Net make() {
        Net r{};
        int c = 0;
        for (int p = 1; p < N; p <<= 1)
            for (int k = p; k >= 1; k >>= 1)
                for (int j = k % p; j + k < N; j += 2 * k)
                    for (int i = 0; i < k && i + j + k < N; ++i)
                        if ((i + j) / (2 * p) == (i + j + k) / (2 * p) && i + j + k < M) {
                            r.a[c] = (short)(i + j);
                            r.b[c] = (short)(i + j + k);
                            ++c;
                        }
        return r;
    }
    static constexpr Net net = make();
};

template <int M, int I>
__device__ __forceinline__ void cex_at(float (&v)[M]) {
    constexpr int a = OEMNet<M>::net.a[I];
    constexpr int b = OEMNet<M>::net.b[I];
    cex(v[a], v[b]);
}

template <int M, int... Is>
__device__ __forceinline__ void apply_net(float (&v)[M], std::integer_sequence<int, Is...>) {
    (cex_at<M, Is>(v), ...);
}

template <int M>
__device__ __forceinline__ void sort_lane(float (&v)[M]) {
    if constexpr (OEMNet<M>::C > 0) apply_net<M>(v, std::make_integer_sequence<int, OEMNet<M>::C>{});
}

// ----------------------------------------------------------- write phase
// out[q][r][c] (row stride TS+1) holds Delta for pair (I*TS + r, J*TS + c).
template <int TS>
__device__ void write_tile(const DissimArgs& A, int nu0, int nq, const float* out, int64_t I, int64_t J) {
    const int64_t n = A.n;
    for (int q = 0; q < nq; ++q) {
        float* D = A.Delta + (int64_t)(nu0 + q) * A.stride_nu;
        const float* o = out + q * TS * (TS + 1);
        for (int idx = threadIdx.x; idx < TS * TS; idx += kDWG) {
            const int a = idx / TS, b = idx % TS;
            // direct: Delta[I*TS + a][J*TS + b] = pair (a, b)
            int64_t i = I * TS + a, j = J * TS + b;
            if (i < n && j < n) {
                if (I < J || a < b) D[i * A.ldd + j] = o[a * (TS + 1) + b];
                else if (a == b) D[i * A.ldd + j] = 0.f;
            }
            // mirror: Delta[J*TS + a][I*TS + b] = pair (b, a)
            i = J * TS + a;
            j = I * TS + b;
            if (i < n && j < n && (I < J || b < a)) D[i * A.ldd + j] = o[b * (TS + 1) + a];
        }
    }
}

// ------------------------------------------------------- lane per pair
// B is a size bucket (compile time), m <= B the runtime length; positions
// m..B-1 hold +inf, which the all-ascending network never moves.
template <int B, bool LIN>
__global__ __launch_bounds__(kDWG) void k_dissim_lane(DissimArgs A, int nu0, int nq) {
    constexpr int TS = 32;
    __shared__ float xs[2 * TS * 65];
    __shared__ float out[kNuChunk * TS * (TS + 1)];
    const int m0 = A.m;
    const int S = m0 | 1;                               // odd LDS row stride: no bank conflicts
    const int64_t n = A.n;
    const int64_t nb = (n + TS - 1) / TS;
    int64_t I, J;
    tri_decode(blockIdx.x, nb, I, J);
    const int tid = threadIdx.x;
    for (int idx = tid; idx < 2 * TS * m0; idx += kDWG) {
        const int row = idx / m0, c = idx % m0;
        const int64_t g = (row < TS) ? (I * TS + row) : (J * TS + row - TS);
        xs[row * S + c] = (g < n) ? A.X[g * A.ldx + c] : 0.f;
    }
    __syncthreads();
    const int c = tid % TS;
    const float inf = __builtin_inff();
    const int wlen = 2 * m0 - 1;
#pragma unroll 1
    for (int sidx = 0; sidx < TS * TS / kDWG; ++sidx) {
        // m is made opaque at every pair row (and every nu below), so that the
        // wave-uniform tests k < m of the unrolled loops are formed where they
        // are used instead of being kept live across the loops (hundreds of
        // SGPRs, spilled)
        int m = m0;
        asm volatile("" : "+s"(m));
        const int r = tid / TS + sidx * (kDWG / TS);
        const int64_t i = I * TS + r, j = J * TS + c;
        const bool valid = (i < n) && (j < n) && (I < J || r < c);
        float* o = out + r * (TS + 1) + c;
        if (!valid) {
            for (int q = 0; q < nq; ++q) o[q * TS * (TS + 1)] = 0.f;
            continue;
        }
        float v[B];
        static_for<B>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            v[k] = (k < m) ? (xs[r * S + k] - xs[(TS + c) * S + k]) : inf;
        });
        sort_lane<B>(v);
        bool tie = false;
        if constexpr (!LIN) {
            static_for<B - 1>([&](auto kc) {
                constexpr int k = decltype(kc)::value + 1;
                tie = tie || ((k < m) && (v[k] == v[k - 1]));
            });
        }
        // untied positions: t = 2k + 2, weight index 2k, the same for every lane
        // (scalar loads; one nu at a time keeps them within the SGPR budget)
#pragma unroll 1
        for (int q = 0; q < kNuChunk; ++q) {
            asm volatile("" : "+s"(m));
            if (q < nq) {
                const float* U = A.wtab + (int64_t)(nu0 + q) * wlen;
                float acc[4] = {0.f, 0.f, 0.f, 0.f};
                static_for<B>([&](auto kc) {
                    constexpr int k = decltype(kc)::value;
                    if (k < m) acc[k & 3] = fmaf(v[k], U[2 * k], acc[k & 3]);
                });
                o[q * TS * (TS + 1)] = A.half_m * ((acc[0] + acc[1]) + (acc[2] + acc[3]));
            }
        }
        if (!LIN && __any(tie)) {
            if (tie) {
                // With ties the lane recomputes the sum run by run: a run a..b
                // of equal values z contributes (b-a+1) z W[a+b+2].
                for (int q = 0; q < nq; ++q) {
                    asm volatile("" : "+s"(m));
                    const float* W = A.wtab + (int64_t)(nu0 + q) * wlen;
                    int rs = 0;
                    float acc = 0.f;
                    static_for<B>([&](auto kc) {
                        constexpr int k = decltype(kc)::value;
                        if (k < m) {
                            const bool end = (k + 1 >= m) || (v[k + 1 < B ? k + 1 : k] != v[k]);
                            if (end) {
                                acc = fmaf(v[k], (float)(k - rs + 1) * W[rs + k], acc);
                                rs = k + 1;
                            }
                        }
                    });
                    o[q * TS * (TS + 1)] = A.half_m * acc;
                }
            }
        }
    }
    __syncthreads();
    write_tile<TS>(A, nu0, nq, out, I, J);
}

// ---------------------------------------------------- G lanes per pair
// Element e = g*E + r of the virtual array lives in register r of group lane g.
// Every compare-exchange whose direction is only known at run time (per lane)
// is one median-of-three per output: med3(a, b, -inf) = min(a, b) and
// med3(a, b, +inf) = max(a, b), so a lane keeps the minimum or the maximum by
// the sign of one constant instead of computing both and selecting.
__device__ __forceinline__ float med3(float a, float b, float c) { return __builtin_amdgcn_fmed3f(a, b, c); }

template <int G, int E>
__device__ __forceinline__ void bitonic_blocked(float (&v)[E], int g) {
    constexpr int N = G * E;
    const float inf = __builtin_inff();
    static_for<ilog2(N)>([&](auto kc) {
        constexpr int k = 2 << decltype(kc)::value;
        // blocks of size k with (e & k) != 0 are sorted descending; for
        // k >= E that is the same for every register of a lane
        const bool lane_desc = (k >= E) && (k < N) && (((g * E) & k) != 0);
        const float ld = lane_desc ? inf : -inf;          // first of a pair keeps max if descending
        static_for<ilog2(k)>([&](auto sc) {
            constexpr int st = (k >> 1) >> decltype(sc)::value;
            if constexpr (st >= E) {
                const int ls = st / E;
                const bool lower = (g & ls) == 0;
                const float keep = (lower != lane_desc) ? -inf : inf;   // -inf keeps the minimum
                static_for<E>([&](auto rc) {
                    constexpr int r = decltype(rc)::value;
                    const float o = __shfl_xor(v[r], ls, G);
                    v[r] = med3(v[r], o, keep);
                });
            } else {
                static_for<E>([&](auto rc) {
                    constexpr int r = decltype(rc)::value;
                    if constexpr ((r & st) == 0) {
                        if constexpr (k < E) {
                            constexpr bool desc = (r & k) != 0;
                            if constexpr (desc) cex(v[r | st], v[r]);
                            else cex(v[r], v[r | st]);
                        } else {
                            const float a = v[r], b = v[r | st];
                            v[r] = med3(a, b, ld);
                            v[r | st] = med3(a, b, -ld);
                        }
                    }
                });
            }
        });
    });
}

template <int G>
__device__ __forceinline__ int scan_max_excl(int x, int g) {
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        const int y = __shfl_up(x, o, G);
        if (g >= o) x = max(x, y);
    }
    const int y = __shfl_up(x, 1, G);
    return g > 0 ? y : -1;
}

template <int G>
__device__ __forceinline__ int scan_min_excl_rev(int x, int g) {
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        const int y = __shfl_down(x, o, G);
        if (g + o < G) x = min(x, y);
    }
    const int y = __shfl_down(x, 1, G);
    return g + 1 < G ? y : 0x7fffffff;
}

// LDS index of weight W[t] (t - 2 = ti) in the skewed table of one nu; the skew
// spreads the untied positions of the G lanes (stride 2E) over distinct banks.
template <int E>
__device__ __forceinline__ int wskew(int ti) {
    return ti + ti / (2 * E);
}

// G = 32, E = 32 (m in (512, 1024]) is asked for 5 waves per SIMD: 96
// registers with a few spilled (72 bytes per lane) measure 3 % faster than
// 126 registers at 4 waves.
template <int G, int E>
constexpr int dissim_group_waves() { return (G == 32 && E == 32) ? 5 : 1; }

template <int G, int E, bool LIN>
__global__ __launch_bounds__(kDWG) __attribute__((amdgpu_waves_per_eu(dissim_group_waves<G, E>())))
void k_dissim_group(DissimArgs A, int nu0, int nq) {
    constexpr int TS = 16;
    constexpr int NG = kDWG / G;
    extern __shared__ float dyn[];
    const int m = A.m;
    const int wlen = 2 * m - 1;
    const int wstride = wlen + wlen / (2 * E) + 1;
    float* wt = dyn;                                   // [nq][wstride]
    float* out = dyn + nq * wstride;                   // [nq][TS][TS+1]
    const int64_t n = A.n;
    const int64_t nb = (n + TS - 1) / TS;
    int64_t I, J;
    tri_decode(blockIdx.x, nb, I, J);
    const int tid = threadIdx.x;
    for (int q = 0; q < nq; ++q)
        for (int ti = tid; ti < wlen; ti += kDWG)
            wt[q * wstride + wskew<E>(ti)] = A.wtab[(int64_t)(nu0 + q) * wlen + ti];
    __syncthreads();
    const int g0 = tid % G;
    const int grp = tid / G;
    const float inf = __builtin_inff();
#pragma unroll 1
    for (int pq = grp; pq < TS * TS; pq += NG) {
        // g is made opaque at every pair, so that the compiler recomputes the
        // per-stage lane masks of the sort where they are used instead of
        // keeping some sixty of them live across the loop (SGPR spills and
        // one wave less per SIMD)
        int g = g0;
        asm volatile("" : "+v"(g));
        const int r = pq / TS, c = pq % TS;
        const int64_t i = I * TS + r, j = J * TS + c;
        const bool valid = (i < n) && (j < n) && (I < J || r < c);
        if (!valid) {
            if (g == 0)
                for (int q = 0; q < nq; ++q) out[q * TS * (TS + 1) + r * (TS + 1) + c] = 0.f;
            continue;
        }
        float v[E];
        const float* xi = A.X + i * A.ldx;
        const float* xj = A.X + j * A.ldx;
        if (A.vecx) {
            // lane g takes the coordinates g*E .. g*E+E-1 in 16-byte loads
            // (which value starts at which position does not matter: they
            // are sorted next)
            const int c0 = g * E;
            static_for<E / 4>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                const int cc = c0 + 4 * q;
                if (cc + 3 < m) {
                    const float4 a = *reinterpret_cast<const float4*>(xi + cc);
                    const float4 b = *reinterpret_cast<const float4*>(xj + cc);
                    v[4 * q] = a.x - b.x;
                    v[4 * q + 1] = a.y - b.y;
                    v[4 * q + 2] = a.z - b.z;
                    v[4 * q + 3] = a.w - b.w;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[4 * q + e] = (cc + e < m) ? (xi[cc + e] - xj[cc + e]) : inf;
                }
            });
        } else {
            static_for<E>([&](auto rc) {
                constexpr int rr = decltype(rc)::value;
                const int cc = rr * G + g;
                v[rr] = (cc < m) ? (xi[cc] - xj[cc]) : inf;
            });
        }
        bitonic_blocked<G, E>(v, g);
        const int e0 = g * E;
        int a[E];
        if constexpr (LIN) {
            // weights linear in t: a run of ties gets the same total weight
            // with every element at its own sorted position (t = 2e + 2) as
            // with all of them at the run's midrank, so no run is needed
            static_for<E>([&](auto rc) {
                constexpr int rr = decltype(rc)::value;
                a[rr] = (e0 + rr < m) ? wskew<E>(2 * (e0 + rr)) : -1;
            });
        } else {
        // run starts (forward)
        const float prevv = __shfl_up(v[E - 1], 1, G);
        const float nextv = __shfl_down(v[0], 1, G);
        // a[rr]: start of the run holding element e0+rr (-1: begins in an earlier lane)
        int run = -1;
        int first_end = 0x7fffffff;
        static_for<E>([&](auto rc) {
            constexpr int rr = decltype(rc)::value;
            bool start, end;
            if constexpr (rr == 0) start = (g == 0) || (v[0] != prevv);
            else start = v[rr] != v[rr - 1];
            if constexpr (rr == E - 1) end = (g == G - 1) || (v[E - 1] != nextv);
            else end = v[rr] != v[rr + 1];
            if (start) run = e0 + rr;
            a[rr] = run;
            if (end && first_end == 0x7fffffff) first_end = e0 + rr;
        });
        const int carry_a = scan_max_excl<G>(run, g);
        const int carry_b = scan_min_excl_rev<G>(first_end, g);
        // a[rr] <- t - 2 = run start + run end; -1 for padding
        int bcur = (g < G - 1 && v[E - 1] == nextv) ? carry_b : (e0 + E - 1);
        static_for<E>([&](auto xc) {
            constexpr int rr = E - 1 - decltype(xc)::value;
            if constexpr (rr < E - 1) {
                if (v[rr] != v[rr + 1]) bcur = e0 + rr;
            }
            const int aa = a[rr] < 0 ? carry_a : a[rr];
            // clamp: finite inputs keep a + b in [0, 2m-2] already
            const int ti = min(max(aa + bcur, 0), 2 * m - 2);
            a[rr] = (e0 + rr < m) ? wskew<E>(ti) : -1;
        });
        }
        for (int q = 0; q < nq; ++q) {
            const float* wq = wt + q * wstride;
            float s0 = 0.f, s1 = 0.f;
            static_for<E>([&](auto rc) {
                constexpr int rr = decltype(rc)::value;
                if (a[rr] >= 0) {
                    if constexpr (rr & 1) s1 = fmaf(v[rr], wq[a[rr]], s1);
                    else s0 = fmaf(v[rr], wq[a[rr]], s0);
                }
            });
            const float tot = group_sum<G>(s0 + s1);
            if (g == 0) out[q * TS * (TS + 1) + r * (TS + 1) + c] = A.half_m * tot;
        }
    }
    __syncthreads();
    write_tile<TS>(A, nu0, nq, out, I, J);
}

// --------------------------------------------------------------- launch
template <int B>
static hipError_t lane_impl(const DissimArgs& a, int nu0, int nq, hipStream_t s) {
    const int64_t nb = (a.n + 31) / 32;
    if (a.lin) hipLaunchKernelGGL((k_dissim_lane<B, true>), dim3((unsigned)tri_count(nb)), dim3(kDWG), 0, s, a, nu0, nq);
    else hipLaunchKernelGGL((k_dissim_lane<B, false>), dim3((unsigned)tri_count(nb)), dim3(kDWG), 0, s, a, nu0, nq);
    return hipGetLastError();
}

static hipError_t lane_dispatch(const DissimArgs& a, int nu0, int nq, hipStream_t s) {
    const int m = a.m;
    if (m <= 4) return lane_impl<4>(a, nu0, nq, s);
    if (m <= 8) return lane_impl<8>(a, nu0, nq, s);
    if (m <= 12) return lane_impl<12>(a, nu0, nq, s);
    if (m <= 16) return lane_impl<16>(a, nu0, nq, s);
    if (m <= 24) return lane_impl<24>(a, nu0, nq, s);
    if (m <= 32) return lane_impl<32>(a, nu0, nq, s);
    if (m <= 48) return lane_impl<48>(a, nu0, nq, s);
    return lane_impl<64>(a, nu0, nq, s);
}

template <int G, int E>
static hipError_t group_impl(const DissimArgs& a, int nu0, int nq, hipStream_t s) {
    const int64_t nb = (a.n + 15) / 16;
    const int wlen = 2 * a.m - 1;
    const int wstride = wlen + wlen / (2 * E) + 1;
    const size_t shm = sizeof(float) * ((size_t)nq * wstride + (size_t)nq * 16 * 17);
    if (a.lin) hipLaunchKernelGGL((k_dissim_group<G, E, true>), dim3((unsigned)tri_count(nb)), dim3(kDWG), shm, s, a, nu0,
                                  nq);
    else hipLaunchKernelGGL((k_dissim_group<G, E, false>), dim3((unsigned)tri_count(nb)), dim3(kDWG), shm, s, a, nu0,
                            nq);
    return hipGetLastError();
}

static int group_max_nu(int m, int E) {
    const int wlen = 2 * m - 1;
    const int wstride = wlen + wlen / (2 * E) + 1;
    const int per = (wstride + 16 * 17) * (int)sizeof(float);
    int k = (48 * 1024) / per;
    if (k > kNuChunk) k = kNuChunk;
    return k < 1 ? 1 : k;
}

hipError_t launch_dissim(const DissimArgs& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    if (a.n == 1) {
        // a single row: only the zero diagonal
        for (int q = 0; q < a.n_nu; ++q) {
            hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(a.Delta + (int64_t)q * a.stride_nu), 1, 0u, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    const int m = a.m;
    if (m <= 64) {
        for (int nu0 = 0; nu0 < a.n_nu; nu0 += kNuChunk) {
            const int nq = (a.n_nu - nu0) < kNuChunk ? (a.n_nu - nu0) : kNuChunk;
            hipError_t e = lane_dispatch(a, nu0, nq, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    int G, E;
    if (m <= 128) { G = 16; E = 8; }
    else if (m <= 256) { G = 16; E = 16; }
    else if (m <= 512) { G = 16; E = 32; }
    else if (m <= 1024) { G = 32; E = 32; }
    else if (m <= 2048) { G = 64; E = 32; }
    else { G = 64; E = 64; }
    const int chunk = group_max_nu(m, E);
    for (int nu0 = 0; nu0 < a.n_nu; nu0 += chunk) {
        const int nq = (a.n_nu - nu0) < chunk ? (a.n_nu - nu0) : chunk;
        hipError_t e;
        if (G == 16 && E == 8) e = group_impl<16, 8>(a, nu0, nq, s);
        else if (G == 16 && E == 16) e = group_impl<16, 16>(a, nu0, nq, s);
        else if (G == 16 && E == 32) e = group_impl<16, 32>(a, nu0, nq, s);
        else if (G == 32 && E == 32) e = group_impl<32, 32>(a, nu0, nq, s);
        else if (G == 64 && E == 32) e = group_impl<64, 32>(a, nu0, nq, s);
        else e = group_impl<64, 64>(a, nu0, nq, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace gmds
