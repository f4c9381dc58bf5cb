// k_stress.hip -- raw-stress instantiations of the stress kernels (the
// templates live in stress_impl.hpp), the reduction launch, and the host-side
// launchers of both losses.
#include "stress_impl.hpp"

namespace gmds {

__global__ void k_fill_u32(uint32_t* p, int64_t count, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

template <int P, int LAT, int T>
static hipError_t reduce_impl(const InstDesc* dd, int n_inst, const int32_t* bmap, int64_t blocks, int64_t qb,
                              int mode, int it, const Launch& L) {
    if (blocks <= 0) return hipSuccess;
    if (L.small)
        return launch_k(k_stress_reduce<P, LAT, T, kRedWGSmall>, dim3((unsigned)blocks), dim3(kRedWGSmall), L, dd,
                        n_inst, bmap, qb, mode, it);
    return launch_k(k_stress_reduce<P, LAT, T, kRedWG>, dim3((unsigned)blocks), dim3(kRedWG), L, dd, n_inst, bmap,
                    qb, mode, it);
}

template <int LAT, int T>
static hipError_t reduce_dispatch_p(const InstDesc* dd, int n_inst, const int32_t* bmap, int64_t blocks, int64_t qb,
                                    int p, int mode, int it, const Launch& L) {
    switch (p_bucket(p)) {
        case 1: return reduce_impl<1, LAT, T>(dd, n_inst, bmap, blocks, qb, mode, it, L);
        case 2: return reduce_impl<2, LAT, T>(dd, n_inst, bmap, blocks, qb, mode, it, L);
        case 3: return reduce_impl<3, LAT, T>(dd, n_inst, bmap, blocks, qb, mode, it, L);
        case 4: return reduce_impl<4, LAT, T>(dd, n_inst, bmap, blocks, qb, mode, it, L);
        default: return reduce_impl<kMaxP, LAT, T>(dd, n_inst, bmap, blocks, qb, mode, it, L);
    }
}

template <int T>
static hipError_t reduce_dispatch_lat(const InstDesc* dd, int n_inst, const int32_t* bmap, int64_t blocks,
                                      int64_t qb, int p, int latent, int mode, int it, const Launch& L) {
    if (latent == 0) return reduce_dispatch_p<0, T>(dd, n_inst, bmap, blocks, qb, p, mode, it, L);
    return reduce_dispatch_p<1, T>(dd, n_inst, bmap, blocks, qb, p, mode, it, L);
}

hipError_t launch_stress_units(const InstDesc* dd, int n_inst, int64_t count, int64_t q_base, int p, int latent, int T,
                               bool grad, int loss, hipStream_t s, LaunchTimer tm, bool reverse) {
    if (loss == kLossSammon)
        return launch_units_sammon(dd, n_inst, count, q_base, p, latent, T, grad, s, tm, reverse);
    return units_dispatch<kLossRaw>(dd, n_inst, count, q_base, p, latent, T, grad, Launch{s, tm, false, reverse});
}

hipError_t launch_stress_reduce(const InstDesc* dd, int n_inst, int64_t blocks, int64_t q_base, int p, int latent,
                                int T, int mode, int it, int64_t max_n, hipStream_t s, LaunchTimer tm,
                                const int32_t* bmap, int red_wg) {
    const Launch L{s, tm, red_wg ? red_wg == kRedWGSmall : max_n <= kSmallReduceN};
    if (T == 64) return reduce_dispatch_lat<64>(dd, n_inst, bmap, blocks, q_base, p, latent, mode, it, L);
    if (T == 128) return reduce_dispatch_lat<128>(dd, n_inst, bmap, blocks, q_base, p, latent, mode, it, L);
    return reduce_dispatch_lat<256>(dd, n_inst, bmap, blocks, q_base, p, latent, mode, it, L);
}

// Host mirror of reduce_blocks (must agree with the device functions above).
int units_per_tile(int T, int p) { return T / unit_rows(T, p_bucket(p)); }

int64_t reduce_block_count(int64_t n, int64_t nb, int T, int p) {
    const int64_t cnt = tri_count(nb) * units_per_tile(T, p) * kWaves;
    int64_t ns = (cnt + kVT * kBatch - 1) / (kVT * kBatch);
    ns = ns < 1 ? 1 : (ns > kSigSlices ? kSigSlices : ns);
    return ns + (n + kNPT - 1) / kNPT;
}

hipError_t launch_fill_u32(uint32_t* ptr, int64_t count, uint32_t value, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, ptr, count, value);
    return hipGetLastError();
}

static const void* persistent_ptr(int p, int latent, int T, int loss) {
    if (loss == kLossSammon) return persistent_ptr_sammon(p, latent, T);
    return persistent_table<kLossRaw>(p, latent, T);
}

int persistent_max_blocks_per_cu(int p, int latent, int T, int loss) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, persistent_ptr(p, latent, T, loss), kWG, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

hipError_t launch_solve_persistent(const InstDesc* dd, int n_inst, const int64_t* d_unit_prefix,
                                   int64_t units_per_iter, int iters, int p, int latent, int T, int loss, int grid,
                                   SolveCtl* ctl, uint32_t* epochs, int64_t spin_limit, hipStream_t s,
                                   LaunchTimer tm) {
    if (iters <= 0 || units_per_iter <= 0) return hipSuccess;
    const void* fn = persistent_ptr(p, latent, T, loss);
    void* args[] = {(void*)&dd, (void*)&n_inst, (void*)&d_unit_prefix, (void*)&units_per_iter, (void*)&iters,
                    (void*)&ctl, (void*)&epochs, (void*)&spin_limit};
    if (tm.start && tm.stop)
        return hipExtLaunchKernel(fn, dim3((unsigned)grid), dim3(kWG), args, 0, s, tm.start, tm.stop, 0);
    return hipLaunchKernel(fn, dim3((unsigned)grid), dim3(kWG), args, 0, s);
}

}  // namespace gmds
