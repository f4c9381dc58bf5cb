// kernels.hpp -- launch interface between the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gmds {

constexpr int kMaxP = 8;           // latent dimensions supported by the stress kernels
constexpr int kMaxNu = 64;         // nu values per gini_dissim call

// Per-instance description of one stress evaluation / descent problem.
// Built on the host, read by the kernels.
struct InstDesc {
    const float* Delta;    // n x n, leading dimension ldd (upper triangle read)
    float* Z;              // n x p, leading dimension ldz
    float* sigma_hist;     // per-iteration sigma (descent only), or nullptr
    float* gradZ;          // n x p gradient output (single evaluation), or nullptr
    const float* grad_out; // device scalar multiplying gradZ, or nullptr
    float* out_sigma;      // device (hi, lo), or nullptr
    float* rowpart;        // scratch: [ntiles][T][pg] row partial gradients
    float* colpart;        // scratch: [ntiles][T][pg] column partial gradients
    float* sigpart;        // scratch: [ntiles][2] partial stress (hi, lo)
    int64_t n, ldd, ldz, ldg;
    int64_t nb;            // tiles per side = ceil(n / T)
    int64_t tile_off;      // first global tile index of this instance
    int32_t p;
    int32_t vec;           // Delta rows 16-byte aligned and ldd % 4 == 0
    float eta;             // descent step
    float c2;              // p = 2 Gini latent: 2^(1-nu)
    float wtab[2 * kMaxP - 1];  // Gini latent: (p/2) W_{p,nu}[t], t = 2 .. 2p
};

// Device-side status word of a persistent solve.
enum : uint32_t { kStatusOk = 0, kStatusTimeout = 1 };

// Persistent-solve control block (device memory, owned by the context).
struct SolveCtl {
    unsigned long long head;  // next queue item
    uint32_t status;          // kStatus*
    uint32_t pad[13];
};

struct DissimArgs {
    const float* X;
    float* Delta;
    const float* wtab;     // [n_nu][2m-1] W_{m,nu}[t] for t = 2 .. 2m (device)
    int64_t n, ldx, ldd, stride_nu;
    int32_t m, n_nu;
    float half_m;          // m / 2
};

// ---- launchers (return hipSuccess or the launch error) ----
hipError_t launch_rank(const float* V, int64_t rows, int d, int64_t ldv, int32_t* t, int64_t ldr,
                       hipStream_t s);

hipError_t launch_dissim(const DissimArgs& a, hipStream_t s);

// Evaluate global tiles q_base .. q_base+count-1 of the n_inst instances
// described by `dd` (device; sorted by tile_off).
hipError_t launch_stress_tiles(const InstDesc* dd, int n_inst, int64_t count, int64_t q_base, int p, int latent,
                               int T, bool grad, hipStream_t s);
// Reduce tile partials: mode 0 writes gradZ and out_sigma, mode 1 takes a
// descent step and records sigma_hist[it], mode 2 writes out_sigma only.
hipError_t launch_stress_reduce(const InstDesc* dd, const InstDesc* hd, int n_inst, int p, int latent,
                                int T, int mode, int it, hipStream_t s);
// One launch: all instances, all iterations.
hipError_t launch_solve_persistent(const InstDesc* dd, int n_inst, const int64_t* d_tile_prefix,
                                   int64_t tiles_per_iter, int iters, int p, int latent, int T, int grid,
                                   SolveCtl* ctl, uint32_t* counters, uint32_t* epochs, int64_t spin_limit,
                                   hipStream_t s);
int persistent_max_blocks_per_cu(int p, int latent, int T);

// Gradient components the stress kernels store per point in the tile
// partials: the p = 2 Gini gradient is (-g, g), so one; p <= 4 has its own
// kernel; larger p runs the kMaxP kernel, which stores kMaxP.
inline int stored_components(int p, int latent) {
    if (p == 2 && latent == 0) return 1;
    return p <= 4 ? p : kMaxP;
}

}  // namespace gmds
