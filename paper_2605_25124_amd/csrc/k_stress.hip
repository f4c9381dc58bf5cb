// k_stress.hip -- fused raw-stress forward + backward over the upper triangle of
// Delta, its deterministic reduction, and the persistent multi-instance solver.
//
// Work decomposition.  The strict upper triangle {i < j} of an n x n problem is
// cut into T x T tiles (I, J), I <= J, enumerated row by row (tri_index).  One
// 256-thread workgroup streams one tile of Delta exactly once: every thread owns
// CPT consecutive-in-groups-of-4 columns of the tile (16-byte loads, LPR lanes
// cover one 4*LPR*... row segment contiguously) and walks down the rows.  For
// each pair it re-ranks the p latent coordinates of u = Z_i - Z_j, forms the
// latent distance delta, the residual r = delta - Delta_ij, r^2, and the
// gradient contribution g = 2 r * d delta / d Z_i (added to row i and
// subtracted from column j).  Per tile it writes row partials, column partials
// and the stress (hi, lo) to scratch; a second pass sums them in a fixed order
// (Neumaier), so every result is deterministic and independent of scheduling.
#include "common.hpp"
#include "kernels.hpp"

namespace gmds {

constexpr int kWG = 256;

template <int T> struct TileShape;
template <> struct TileShape<64> { static constexpr int CPT = 4; };
template <> struct TileShape<128> { static constexpr int CPT = 8; };
template <> struct TileShape<256> { static constexpr int CPT = 8; };

template <int P, int LAT>
struct PG_ { static constexpr int value = (P == 2 && LAT == 0) ? 1 : P; };

// LDS floats needed by stress_tile.
template <int P, int LAT, int T>
constexpr int tile_lds_floats() {
    return (kWG / (T / TileShape<T>::CPT)) * T * PG_<P, LAT>::value;
}

// Latent distance and residual for one pair.  `valid` masks pairs outside the
// strict upper triangle or past n: they contribute exactly zero.
//   u_c = fl32(Z_i,c - Z_j,c); Gini: doubled midranks t_c of u over its p
//   coordinates, a_c = (p/2) W_p[t_c], delta = sum_c u_c a_c; Euclid:
//   delta = |u|, a = u / |u| (0 when u = 0).  g_c = 2 r a_c.
template <int P, int LAT, bool GRAD>
__device__ __forceinline__ float pair_term(const float (&zi)[P], const float (&zj)[P], float d, bool valid,
                                           int p, const InstDesc& D, float (&g)[PG_<P, LAT>::value]) {
    constexpr int PG = PG_<P, LAT>::value;
    float u[P];
#pragma unroll
    for (int c = 0; c < P; ++c) u[c] = zi[c] - zj[c];
    if constexpr (P == 2 && LAT == 0) {
        // p = 2: t = (2,4) if u1 < u2, (4,2) if u1 > u2, (3,3) on a tie, so
        // delta = 2^(1-nu) |u2 - u1| and a = 2^(1-nu) sgn(u2 - u1) (-1, +1).
        const float w = u[1] - u[0];
        const float delta = D.c2 * fabsf(w);
        const float r = valid ? (delta - d) : 0.f;
        if constexpr (GRAD) {
            const float s = (w > 0.f) ? 1.f : ((w < 0.f) ? -1.f : 0.f);
            g[0] = 2.f * D.c2 * r * s;
        }
        return r * r;
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
        const float r = valid ? (delta - d) : 0.f;
        if constexpr (GRAD) {
#pragma unroll
            for (int c = 0; c < PG; ++c) g[c] = 2.f * r * a[c];
        }
        return r * r;
    } else {
        float ss = 0.f;
#pragma unroll
        for (int c = 0; c < P; ++c) ss = fmaf(u[c], u[c], ss);
        const float rs = (ss > 0.f) ? rsqrtf(ss) : 0.f;
        const float delta = ss * rs;
        const float r = valid ? (delta - d) : 0.f;
        if constexpr (GRAD) {
            const float f = 2.f * r * rs;
#pragma unroll
            for (int c = 0; c < PG; ++c) g[c] = f * u[c];
        }
        return r * r;
    }
}

// Stream one tile (local index lt of instance D) of Delta.
template <int P, int LAT, int T, bool GRAD>
__device__ void stress_tile(const InstDesc& D, int64_t lt, float* lds) {
    constexpr int CPT = TileShape<T>::CPT;
    constexpr int LPR = T / CPT;          // lanes per tile row
    constexpr int RPS = kWG / LPR;        // rows per step
    constexpr int STEPS = T / RPS;
    constexpr int NQ = CPT / 4;
    constexpr int PG = PG_<P, LAT>::value;
    static_assert(LPR <= 64 && (64 % LPR) == 0, "a tile row must sit inside one wave");

    const int tid = threadIdx.x;
    const int c4 = tid % LPR;
    const int rr = tid / LPR;
    int64_t I, J;
    tri_decode(lt, D.nb, I, J);
    const int64_t n = D.n;
    const int64_t i0 = I * T;
    const int64_t j0 = J * T;
    const int p = (P == kMaxP) ? D.p : P;

    float zj[CPT][P];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t j = j0 + 4 * (c4 + q * LPR) + e;
#pragma unroll
            for (int c = 0; c < P; ++c)
                zj[q * 4 + e][c] = (j < n && c < p) ? D.Z[j * D.ldz + c] : 0.f;
        }

    float colacc[CPT][PG];
#pragma unroll
    for (int x = 0; x < CPT; ++x)
#pragma unroll
        for (int c = 0; c < PG; ++c) colacc[x][c] = 0.f;
    Comp sig;

#pragma unroll 2
    for (int s = 0; s < STEPS; ++s) {
        const int il = s * RPS + rr;
        const int64_t i = i0 + il;
        float rowacc[PG];
#pragma unroll
        for (int c = 0; c < PG; ++c) rowacc[c] = 0.f;
        float sst = 0.f;
        if (i < n) {
            float zi[P];
#pragma unroll
            for (int c = 0; c < P; ++c) zi[c] = (c < p) ? D.Z[i * D.ldz + c] : 0.f;
            const float* Dr = D.Delta + i * D.ldd;
            float dv[CPT];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int64_t jb = j0 + 4 * (c4 + q * LPR);
                dv[q * 4 + 0] = dv[q * 4 + 1] = dv[q * 4 + 2] = dv[q * 4 + 3] = 0.f;
                if (jb + 3 > i && jb < n) {
                    if (D.vec && jb + 3 < n) {
                        const float4 v = *reinterpret_cast<const float4*>(Dr + jb);
                        dv[q * 4 + 0] = v.x;
                        dv[q * 4 + 1] = v.y;
                        dv[q * 4 + 2] = v.z;
                        dv[q * 4 + 3] = v.w;
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (jb + e < n && jb + e > i) dv[q * 4 + e] = Dr[jb + e];
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int x = q * 4 + e;
                    const int64_t j = j0 + 4 * (c4 + q * LPR) + e;
                    const bool valid = (j > i) && (j < n);
                    float g[PG];
                    sst += pair_term<P, LAT, GRAD>(zi, zj[x], dv[x], valid, p, D, g);
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
#pragma unroll
            for (int c = 0; c < PG; ++c) {
                const float tot = group_sum<LPR>(rowacc[c]);
                if (c4 == 0 && i < n) D.rowpart[(lt * T + il) * PG + c] = tot;
            }
        }
        sig.add(sst);
    }

    if constexpr (GRAD) {
        // Column partials: RPS row groups hold partial sums for each column.
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int col = 4 * (c4 + q * LPR) + e;
#pragma unroll
                for (int c = 0; c < PG; ++c) lds[(rr * T + col) * PG + c] = colacc[q * 4 + e][c];
            }
        __syncthreads();
        for (int x = tid; x < T * PG; x += kWG) {
            float acc = 0.f;
#pragma unroll 4
            for (int r = 0; r < RPS; ++r) acc += lds[r * T * PG + x];
            D.colpart[lt * T * PG + x] = acc;
        }
        __syncthreads();
    }
    // Stress of the tile: fixed-shape tree over the workgroup.
    lds[tid] = sig.hi;
    lds[kWG + tid] = sig.lo;
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
    if (tid == 0) {
        D.sigpart[2 * lt + 0] = lds[0];
        D.sigpart[2 * lt + 1] = lds[kWG];
    }
    __syncthreads();
}

// Gradient of point k from the tile partials, in a fixed order: the row
// partials of its tile row, then minus the column partials of its tile column.
template <int P, int LAT, int T>
__device__ __forceinline__ void reduce_point(const InstDesc& D, int64_t k, float (&G)[P]) {
    constexpr int PG = PG_<P, LAT>::value;
    const int64_t b = k / T;
    const int64_t kl = k % T;
    const int64_t nb = D.nb;
    Comp acc[PG];
    for (int64_t J = b; J < nb; ++J) {
        const int64_t lt = tri_index(b, J, nb);
#pragma unroll
        for (int c = 0; c < PG; ++c) acc[c].add(D.rowpart[(lt * T + kl) * PG + c]);
    }
    for (int64_t I = 0; I <= b; ++I) {
        const int64_t lt = tri_index(I, b, nb);
#pragma unroll
        for (int c = 0; c < PG; ++c) acc[c].add(-D.colpart[(lt * T + kl) * PG + c]);
    }
    if constexpr (P == 2 && LAT == 0) {
        const float v = acc[0].value();
        G[0] = -v;
        G[1] = v;
    } else {
#pragma unroll
        for (int c = 0; c < P; ++c) G[c] = acc[c].value();
    }
}

// Stress of instance D from its tile partials; executed by one whole workgroup.
__device__ void reduce_sigma(const InstDesc& D, float* lds, float& hi, float& lo) {
    const int tid = threadIdx.x;
    const int64_t nt = tri_count(D.nb);
    Comp acc;
    for (int64_t t = tid; t < nt; t += kWG) {
        Comp x;
        x.hi = D.sigpart[2 * t];
        x.lo = D.sigpart[2 * t + 1];
        acc.add(x);
    }
    lds[tid] = acc.hi;
    lds[kWG + tid] = acc.lo;
    __syncthreads();
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
    hi = lds[0];
    lo = lds[kWG];
    __syncthreads();
}

// Map a global tile index to its instance (descriptors sorted by tile_off).
__device__ __forceinline__ int find_instance(const InstDesc* dd, int n_inst, int64_t q) {
    int lo = 0, hi = n_inst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (dd[mid].tile_off <= q) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int P, int LAT, int T, bool GRAD>
__global__ __launch_bounds__(kWG) void k_stress_tiles(const InstDesc* __restrict__ dd, int n_inst, int64_t q_base) {
    __shared__ float lds[tile_lds_floats<P, LAT, T>() > 2 * kWG ? tile_lds_floats<P, LAT, T>() : 2 * kWG];
    const int64_t q = (int64_t)blockIdx.x + q_base;
    const int k = find_instance(dd, n_inst, q);
    const InstDesc D = dd[k];
    stress_tile<P, LAT, T, GRAD>(D, q - D.tile_off, lds);
}

// mode 0: write gradZ (scaled by *grad_out) and out_sigma; mode 1: descent
// step Z -= eta G and sigma_hist[it]; mode 2: out_sigma only.  blockIdx.y =
// instance; block nblk in x reduces the stress, blocks below it the points.
template <int P, int LAT, int T>
__global__ __launch_bounds__(kWG) void k_stress_reduce(const InstDesc* __restrict__ dd, int mode, int it) {
    __shared__ float lds[2 * kWG];
    const InstDesc& D = dd[blockIdx.y];
    const int64_t n = D.n;
    const int64_t nblk = (n + kWG - 1) / kWG;
    const int p = (P == kMaxP) ? D.p : P;
    if ((int64_t)blockIdx.x == nblk) {
        float hi, lo;
        reduce_sigma(D, lds, hi, lo);
        if (threadIdx.x == 0) {
            if (mode != 1) {
                if (D.out_sigma) {
                    D.out_sigma[0] = hi;
                    D.out_sigma[1] = lo;
                }
            } else if (D.sigma_hist) {
                D.sigma_hist[it] = hi + lo;
            }
        }
        return;
    }
    if ((int64_t)blockIdx.x > nblk || mode == 2) return;
    const int64_t k = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (k >= n) return;
    float G[P];
    reduce_point<P, LAT, T>(D, k, G);
    if (mode == 0) {
        const float sc = D.grad_out ? *D.grad_out : 1.f;
#pragma unroll
        for (int c = 0; c < P; ++c)
            if (c < p) D.gradZ[k * D.ldg + c] = sc * G[c];
    } else {
#pragma unroll
        for (int c = 0; c < P; ++c)
            if (c < p) D.Z[k * D.ldz + c] -= D.eta * G[c];
    }
}

// Persistent solver.  Queue item q = (iteration it, instance k, local tile lt),
// iteration-major, instances in the host's order.  A workgroup pops q, waits
// until instance k has finished iteration it-1 (epoch[k] >= it), streams the
// tile, and counts it done; the workgroup that completes the last tile of
// (k, it) reduces the partials, takes the descent step, resets the counter and
// publishes epoch[k] = it + 1.  Items are popped in queue order and every item
// waits only on items popped before it, whose workgroups are already running,
// so the queue drains whatever the number of resident workgroups.  A wait that
// exceeds spin_limit ticks of the constant-rate device clock sets the abort status;
// every workgroup then stops popping work and the kernel ends.
template <int P, int LAT, int T>
__global__ __launch_bounds__(kWG) void k_solve_persistent(const InstDesc* __restrict__ dd, int n_inst,
                                                          const int64_t* __restrict__ prefix,
                                                          int64_t per_iter, int iters, SolveCtl* ctl,
                                                          uint32_t* cnt, uint32_t* epoch, int64_t spin_limit) {
    constexpr int NL = tile_lds_floats<P, LAT, T>() > 2 * kWG ? tile_lds_floats<P, LAT, T>() : 2 * kWG;
    __shared__ float lds[NL];
    __shared__ int64_t sh_q;
    __shared__ int sh_flag;
    const int tid = threadIdx.x;
    const int64_t total = per_iter * (int64_t)iters;
    unsigned long long* head = &ctl->head;
    for (;;) {
        if (tid == 0) {
            const uint32_t st = __hip_atomic_load(&ctl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int64_t q = total;
            if (st == kStatusOk) q = (int64_t)atomicAdd(head, 1ull);
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
        const int64_t lt = r - prefix[k];
        if (tid == 0) {
            int ok = 1;
            if (__hip_atomic_load(&epoch[k], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < (uint32_t)it) {
                const uint64_t t0 = wall_clock64();
                while (__hip_atomic_load(&epoch[k], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < (uint32_t)it) {
                    __builtin_amdgcn_s_sleep(2);
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
        stress_tile<P, LAT, T, true>(D, lt, lds);
        __threadfence();
        __syncthreads();
        if (tid == 0) {
            const uint32_t old = atomicAdd(&cnt[k], 1u);
            sh_flag = (old + 1 == (uint32_t)tri_count(D.nb)) ? 1 : 0;
        }
        __syncthreads();
        if (sh_flag) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            float shi, slo;
            reduce_sigma(D, lds, shi, slo);
            if (tid == 0 && D.sigma_hist) D.sigma_hist[it] = shi + slo;
            const int p = (P == kMaxP) ? D.p : P;
            for (int64_t pt = tid; pt < D.n; pt += kWG) {
                float G[P];
                reduce_point<P, LAT, T>(D, pt, G);
#pragma unroll
                for (int c = 0; c < P; ++c)
                    if (c < p) D.Z[pt * D.ldz + c] -= D.eta * G[c];
            }
            __threadfence();
            __syncthreads();
            if (tid == 0) {
                __hip_atomic_store(&cnt[k], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&epoch[k], (uint32_t)(it + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------- dispatch
template <int P, int LAT, int T>
static hipError_t tiles_impl(const InstDesc* dd, int n_inst, int64_t total, int64_t qb, bool grad, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    if (grad)
        hipLaunchKernelGGL((k_stress_tiles<P, LAT, T, true>), dim3((unsigned)total), dim3(kWG), 0, s, dd, n_inst, qb);
    else
        hipLaunchKernelGGL((k_stress_tiles<P, LAT, T, false>), dim3((unsigned)total), dim3(kWG), 0, s, dd, n_inst, qb);
    return hipGetLastError();
}

static int p_bucket(int p) { return p <= 4 ? p : kMaxP; }

template <int LAT, int T>
static hipError_t tiles_p(const InstDesc* dd, int n_inst, int64_t total, int64_t qb, int p, bool grad,
                          hipStream_t s) {
    switch (p_bucket(p)) {
        case 1: return tiles_impl<1, LAT, T>(dd, n_inst, total, qb, grad, s);
        case 2: return tiles_impl<2, LAT, T>(dd, n_inst, total, qb, grad, s);
        case 3: return tiles_impl<3, LAT, T>(dd, n_inst, total, qb, grad, s);
        case 4: return tiles_impl<4, LAT, T>(dd, n_inst, total, qb, grad, s);
        default: return tiles_impl<kMaxP, LAT, T>(dd, n_inst, total, qb, grad, s);
    }
}

hipError_t launch_stress_tiles(const InstDesc* dd, int n_inst, int64_t count, int64_t q_base, int p, int latent,
                               int T, bool grad, hipStream_t s) {
    if (latent == 0) {
        if (T == 64) return tiles_p<0, 64>(dd, n_inst, count, q_base, p, grad, s);
        if (T == 128) return tiles_p<0, 128>(dd, n_inst, count, q_base, p, grad, s);
        return tiles_p<0, 256>(dd, n_inst, count, q_base, p, grad, s);
    }
    if (T == 64) return tiles_p<1, 64>(dd, n_inst, count, q_base, p, grad, s);
    if (T == 128) return tiles_p<1, 128>(dd, n_inst, count, q_base, p, grad, s);
    return tiles_p<1, 256>(dd, n_inst, count, q_base, p, grad, s);
}

template <int P, int LAT, int T>
static hipError_t reduce_impl(const InstDesc* dd, int n_inst, int64_t max_n, int mode, int it, hipStream_t s) {
    const unsigned gx = (unsigned)((max_n + kWG - 1) / kWG + 1);
    hipLaunchKernelGGL((k_stress_reduce<P, LAT, T>), dim3(gx, (unsigned)n_inst), dim3(kWG), 0, s, dd, mode, it);
    return hipGetLastError();
}

template <int LAT, int T>
static hipError_t reduce_p(const InstDesc* dd, int n_inst, int64_t max_n, int p, int mode, int it, hipStream_t s) {
    switch (p_bucket(p)) {
        case 1: return reduce_impl<1, LAT, T>(dd, n_inst, max_n, mode, it, s);
        case 2: return reduce_impl<2, LAT, T>(dd, n_inst, max_n, mode, it, s);
        case 3: return reduce_impl<3, LAT, T>(dd, n_inst, max_n, mode, it, s);
        case 4: return reduce_impl<4, LAT, T>(dd, n_inst, max_n, mode, it, s);
        default: return reduce_impl<kMaxP, LAT, T>(dd, n_inst, max_n, mode, it, s);
    }
}

hipError_t launch_stress_reduce(const InstDesc* dd, const InstDesc* hd, int n_inst, int p, int latent, int T,
                                int mode, int it, hipStream_t s) {
    int64_t max_n = 0;
    for (int k = 0; k < n_inst; ++k) max_n = hd[k].n > max_n ? hd[k].n : max_n;
    if (latent == 0) {
        if (T == 64) return reduce_p<0, 64>(dd, n_inst, max_n, p, mode, it, s);
        if (T == 128) return reduce_p<0, 128>(dd, n_inst, max_n, p, mode, it, s);
        return reduce_p<0, 256>(dd, n_inst, max_n, p, mode, it, s);
    }
    if (T == 64) return reduce_p<1, 64>(dd, n_inst, max_n, p, mode, it, s);
    if (T == 128) return reduce_p<1, 128>(dd, n_inst, max_n, p, mode, it, s);
    return reduce_p<1, 256>(dd, n_inst, max_n, p, mode, it, s);
}

template <int P, int LAT, int T>
static const void* persistent_fn() {
    return reinterpret_cast<const void*>(&k_solve_persistent<P, LAT, T>);
}

static const void* persistent_ptr(int p, int latent, int T) {
#define GMDS_PT(LAT, TT)                                             \
    switch (p_bucket(p)) {                                           \
        case 1: return persistent_fn<1, LAT, TT>();                  \
        case 2: return persistent_fn<2, LAT, TT>();                  \
        case 3: return persistent_fn<3, LAT, TT>();                  \
        case 4: return persistent_fn<4, LAT, TT>();                  \
        default: return persistent_fn<kMaxP, LAT, TT>();             \
    }
    if (latent == 0) {
        if (T == 64) { GMDS_PT(0, 64) }
        if (T == 128) { GMDS_PT(0, 128) }
        GMDS_PT(0, 256)
    }
    if (T == 64) { GMDS_PT(1, 64) }
    if (T == 128) { GMDS_PT(1, 128) }
    GMDS_PT(1, 256)
#undef GMDS_PT
}

int persistent_max_blocks_per_cu(int p, int latent, int T) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, persistent_ptr(p, latent, T), kWG, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

hipError_t launch_solve_persistent(const InstDesc* dd, int n_inst, const int64_t* d_tile_prefix,
                                   int64_t tiles_per_iter, int iters, int p, int latent, int T, int grid,
                                   SolveCtl* ctl, uint32_t* counters, uint32_t* epochs, int64_t spin_limit,
                                   hipStream_t s) {
    if (iters <= 0 || tiles_per_iter <= 0) return hipSuccess;
    const void* fn = persistent_ptr(p, latent, T);
    void* args[] = {(void*)&dd, (void*)&n_inst, (void*)&d_tile_prefix, (void*)&tiles_per_iter, (void*)&iters,
                    (void*)&ctl, (void*)&counters, (void*)&epochs, (void*)&spin_limit};
    return hipLaunchKernel(fn, dim3((unsigned)grid), dim3(kWG), args, 0, s);
}

}  // namespace gmds
