// kernels.hpp -- launch interface between the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gmds {

constexpr int kMaxP = 8;           // latent dimensions supported by the stress kernels
constexpr int kMaxNu = 64;         // nu values per gini_dissim call
constexpr int kStressWaves = 4;    // waves per stress workgroup (one stress partial each)
constexpr int kSigSlices = 32;     // most stress slices one instance's reduction sums (scratch: 2 floats each)
constexpr int kMaxCmdsQ = 8;       // widest subspace of the classical-MDS iteration
constexpr int kLossRaw = 0;        // raw stress sum (delta - Delta)^2
constexpr int kLossSammon = 1;     // Sammon stress sum (delta - Delta)^2 / Delta over sum Delta

// Per-instance description of one stress evaluation / descent problem.
// Built on the host, read by the kernels.
struct InstDesc {
    const float* Delta;    // n x n, leading dimension ldd (upper triangle read)
    float* Z;              // n x p, leading dimension ldz
    float* sigma_hist;     // per-iteration sigma (descent only), or nullptr
    float* gradZ;          // n x p gradient output (single evaluation), or nullptr
    const float* grad_out; // device scalar multiplying gradZ, or nullptr
    float* out_sigma;      // device (hi, lo), or nullptr
    const float* dsumsq;   // device (hi, lo) of sum_{i<j} Delta_ij^2 (Kruskal normaliser), or nullptr
    float* ks_hist;        // per-iteration Kruskal stress (descent only), or nullptr
    const float* dsum;     // device (hi, lo) of sum_{i<j} Delta_ij (Sammon normaliser), or nullptr
    float* rowpart;        // scratch: [ntiles][T][pg] row partial gradients (one per row and tile)
    float* colpart;        // scratch: [ntiles][units][T][pg] column partial gradients (one per unit)
    float* sigpart;        // scratch: [ntiles][units][kStressWaves][2] partial stress (hi, lo) per wave
    float* sigslice;       // scratch: [kSigSlices][2] stress slices of the reduction launch
    uint32_t* instcnt;     // [1] finished stress slices / units; zero between launches
    int64_t n, ldd, ldz, ldg;
    int64_t nb;            // tiles per side = ceil(n / T)
    int64_t tile_off;      // first global work unit of this instance
    int64_t red_off;       // first block of this instance in a reduction launch
    int32_t p;
    int32_t loss;          // kLossRaw or kLossSammon
    int32_t vec;           // Delta rows 16-byte aligned and ldd % 4 == 0
    float eta;             // descent step
    float c2;              // p = 2 Gini latent: 2^(1-nu)
    float wtab[2 * kMaxP - 1];  // Gini latent: (p/2) W_{p,nu}[t], t = 2 .. 2p
};

// Optional events stamped by the runtime at the start and the end of one
// kernel (profiling); both null for a plain launch.
struct LaunchTimer {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};

// What a stress launch produces once every tile of an instance is done.
enum StressMode : int {
    kModeGrad = 0,      // gradZ (scaled by *grad_out) and out_sigma
    kModeDescent = 1,   // Z -= eta * grad and sigma_hist[it]
    kModeSigma = 2      // out_sigma only (no gradient work)
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
    int32_t lin;           // every nu of the call is 2: the weights are linear in t (ties need no runs)
    int32_t vecx;          // X rows start on 16 bytes (16-byte loads)
};

// ---- launchers (return hipSuccess or the launch error) ----
// scratch: rank_scratch_words(rows, d) words (device; the sorted chunks of
// rows longer than 256).
int64_t rank_scratch_words(int64_t rows, int d);
hipError_t launch_rank(const float* V, int64_t rows, int d, int64_t ldv, int32_t* t, int64_t ldr, uint32_t* scratch,
                       hipStream_t s);

hipError_t launch_dissim(const DissimArgs& a, hipStream_t s);

// Stream global work units q_base .. q_base+count-1 of the n_inst instances
// described by `dd` (device; sorted by tile_off): tile partials only.
// reverse: workgroups take the units last to first (the partials and sums do
// not depend on the order).
hipError_t launch_stress_units(const InstDesc* dd, int n_inst, int64_t count, int64_t q_base, int p, int latent, int T,
                               bool grad, int loss, hipStream_t s, LaunchTimer tm = {}, bool reverse = false);
// Reduce the partials of every instance; `blocks` is the sum over instances
// of reduce_block_count (instances sorted by red_off); blocks are numbered
// from q_base; max_n is the largest n among them (it sizes the blocks);
// bmap (device, optional) holds the instance of every block.
// StressMode says what is produced; `it` indexes sigma_hist in descent mode.
// red_wg: threads per block, 256 or 1024 (the sums have the same shape
// either way); 0 takes 256 when max_n <= 4096, else 1024.
hipError_t launch_stress_reduce(const InstDesc* dd, int n_inst, int64_t blocks, int64_t q_base, int p, int latent,
                                int T, int mode, int it, int64_t max_n, hipStream_t s, LaunchTimer tm = {},
                                const int32_t* bmap = nullptr, int red_wg = 0);
int64_t reduce_block_count(int64_t n, int64_t nb, int T, int p);
int units_per_tile(int T, int p);
// One launch: all instances, all iterations of the descent.
hipError_t launch_solve_persistent(const InstDesc* dd, int n_inst, const int64_t* d_unit_prefix,
                                   int64_t units_per_iter, int iters, int p, int latent, int T, int loss, int grid,
                                   SolveCtl* ctl, uint32_t* epochs, int64_t spin_limit, hipStream_t s,
                                   LaunchTimer tm = {});
int persistent_max_blocks_per_cu(int p, int latent, int T, int loss);
// Set `count` words to `value` (counters, epochs).
hipError_t launch_fill_u32(uint32_t* ptr, int64_t count, uint32_t value, hipStream_t s);
// sum_{i<j} Delta_ij^power (power 1 or 2) of n_mat stacked matrices into
// out[2k], out[2k+1] (hi, lo); `part` holds 2 * n_mat * sumsq_blocks(n) floats.
int64_t sumsq_blocks(int64_t n);
// max_i sum_{j != i, Delta_ij > 0} 1 / Delta_ij over full rows into out[0];
// `part` holds rowinv_blocks(n) floats.
int64_t rowinv_blocks(int64_t n);
hipError_t launch_rowinv_max(const float* Delta, int64_t n, int64_t ldd, float* part, float* out, hipStream_t s);
hipError_t launch_sumsq(const float* Delta, int64_t n, int64_t ldd, int n_mat, int64_t stride, float* part,
                        float* out, int power, hipStream_t s);

// Classical MDS (k_cmds.hip).  out = D^2 V over full rows of Delta (diagonal
// left out) in FP64, V (FP32) and out n x q row-major, q <= kMaxCmdsQ.
// reverse: workgroups take the row blocks last to first (same results).
hipError_t launch_d2v(const float* Delta, int64_t n, int64_t ldd, const float* V, int q, double* out,
                      hipStream_t s, bool reverse = false);
// One subspace step after launch_d2v: from Y = D^2 V and V, the Rayleigh-Ritz
// matrix T = V^T B V (q x q doubles), the map M and mean with which
// Vnext = (Y - 1 mean^T) M = (B V) R^-1 has orthonormal columns (B V = -1/2 H Y,
// R the Cholesky factor of (B V)^T (B V)), and Vnext itself.  `part` holds
// step_part_doubles() doubles; M q*q doubles; mean q doubles.
int64_t step_part_doubles();
// count pseudo-random values in [-1/2, 1/2), a fixed function of the index.
hipError_t launch_start_block(float* V, int64_t count, hipStream_t s);
hipError_t launch_subspace_step(const double* Y, const float* V, int q, int64_t n, double* part, double* T,
                                double* M, double* mean, float* Vnext, hipStream_t s);
// out (qa*qb (hi, lo) pairs) = A^T B over n rows (B == nullptr: column sums
// of A, qb = 1).  `part` holds gram_part_floats() floats.
int64_t gram_part_floats();
hipError_t launch_gram(const float* A, int qa, const float* B, int qb, int64_t n, float* part, float* out,
                       hipStream_t s);
// M (q x q, row-major) such that Y M has orthonormal columns, from the Gram
// matrix g = Y^T Y (launch_gram's (hi, lo) output): Cholesky, then R^-1;
// columns in the span of earlier ones become zero.
hipError_t launch_chol_orth(const float* g, int q, float* M, hipStream_t s);
// out[i, :] = (alpha (A[i, :] - mean)) M; M qa x qb row-major (device),
// mean[c] = (sums[2c] + sums[2c+1]) / n from launch_gram's column sums of A
// (sums may be null: no centring).
hipError_t launch_rowmat(const float* A, int qa, const float* sums, float alpha, const float* M, int qb, int64_t n,
                         float* out, int64_t ldo, hipStream_t s);

// Column standardisation (k_prep.hip): Y = (X - median) / sd per column
// (population sd; a constant column is only centred); stats (2m floats,
// (median, sd) per column) may be null.  Y may alias X only if ldy == ldx.
hipError_t launch_standardise(const float* X, int64_t n, int m, int64_t ldx, float* Y, int64_t ldy, float* stats,
                              hipStream_t s);

// Rows of Delta one stress workgroup streams (a work unit): 64, or 128 for
// p = 3 on tiles of at least 128 columns, where the heavier latent distance
// makes the unit's fixed work (coordinates, partial sums) worth spreading
// over twice the pairs (wider latent spaces would need more registers than
// the longer unit saves).
__host__ __device__ constexpr int unit_rows(int T, int p) { return (p == 3 && T >= 128) ? 128 : 64; }

// Gradient components the stress kernels store per point in the tile
// partials: the p = 2 Gini gradient is (-g, g), so one; p <= 4 has its own
// kernel; larger p runs the kMaxP kernel, which stores kMaxP.
inline int stored_components(int p, int latent) {
    if (p == 2 && latent == 0) return 1;
    return p <= 4 ? p : kMaxP;
}

}  // namespace gmds
