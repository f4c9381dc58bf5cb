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

// Inverse of tri_index.  Row I is the largest with tri_index(I, I) <= idx,
// the smaller root of I^2 - (2nb+1) I + 2 idx = 0 rounded down.  The
// discriminant is formed exactly in 64-bit integers and only its square root
// is taken in FP32 (within a unit or two of the root for any nb < 2^26); the
// integer fix-up that follows makes the result exact.
__device__ __forceinline__ void tri_decode(int64_t idx, int64_t nb, int64_t& I, int64_t& J) {
    const int64_t b = 2 * nb + 1;
    int64_t disc = b * b - 8 * idx;
    if (disc < 0) disc = 0;
    int64_t i = (b - (int64_t)sqrtf((float)disc)) / 2;
    if (i < 0) i = 0;
    if (i > nb - 1) i = nb - 1;
    while (i > 0 && tri_index(i, i, nb) > idx) --i;
    while (i + 1 < nb && tri_index(i + 1, i + 1, nb) <= idx) ++i;
    I = i;
    J = i + (idx - tri_index(i, i, nb));
}

}  // namespace gmds
