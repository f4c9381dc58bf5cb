// k_stress_sammon.hip -- the Sammon-stress instantiations of the stress
// kernels (templates in stress_impl.hpp), compiled apart from the raw stress
// so that the two sets build in parallel.
#include "stress_impl.hpp"

namespace gmds {

hipError_t launch_units_sammon(const InstDesc* dd, int n_inst, int64_t count, int64_t q_base, int p, int latent,
                               int T, bool grad, hipStream_t s, LaunchTimer tm, bool reverse) {
    return units_dispatch<kLossSammon>(dd, n_inst, count, q_base, p, latent, T, grad, Launch{s, tm, false, reverse});
}

const void* persistent_ptr_sammon(int p, int latent, int T) { return persistent_table<kLossSammon>(p, latent, T); }

}  // namespace gmds
