// common.hpp -- device helpers shared by the Gini MDS kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gmds {

constexpr int kWave = 64;

// Error-free transformation of a + b (Knuth's TwoSum): s + e == a + b exactly.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Compensated accumulator (Neumaier): value = hi + lo.
struct Comp {
    float hi = 0.f, lo = 0.f;
    __device__ __forceinline__ void add(float x) {
        float s, e;
        two_sum(hi, x, s, e);
        hi = s;
        lo += e;
    }
    __device__ __forceinline__ void add(const Comp& o) {
        add(o.hi);
        lo += o.lo;
    }
    __device__ __forceinline__ float value() const { return hi + lo; }
};

// Sum of v over aligned groups of W lanes (W a power of two <= 64); every
// lane of the group receives the total.  The butterfly order is fixed, so the
// result is deterministic.
template <int W>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
    return v;
}

// Triangular tile enumeration: tiles (I, J) with 0 <= I <= J < nb, listed
// row by row; index(I, J) = I*nb - I*(I-1)/2 + (J - I).
__host__ __device__ __forceinline__ int64_t tri_index(int64_t I, int64_t J, int64_t nb) {
    return I * nb - (I * (I - 1)) / 2 + (J - I);
}

__host__ __device__ __forceinline__ int64_t tri_count(int64_t nb) { return nb * (nb + 1) / 2; }

// Inverse of tri_index.
__device__ __forceinline__ void tri_decode(int64_t idx, int64_t nb, int64_t& I, int64_t& J) {
    // Row I starts at I*nb - I*(I-1)/2.  Start from the real root and fix up.
    double b = 2.0 * (double)nb + 1.0;
    double disc = b * b - 8.0 * (double)idx;
    int64_t i = (int64_t)((b - sqrt(disc > 0.0 ? disc : 0.0)) * 0.5);
    if (i < 0) i = 0;
    if (i > nb - 1) i = nb - 1;
    while (i > 0 && tri_index(i, i, nb) > idx) --i;
    while (i + 1 < nb && tri_index(i + 1, i + 1, nb) <= idx) ++i;
    I = i;
    J = i + (idx - tri_index(i, i, nb));
}

}  // namespace gmds
