// Device access to the pair-plane state layout described in kgs_internal.h:
// per colour c, the plane of (P, Q) pairs starts at base + 4c*stride and
// the plane of (U, V) pairs at base + (4c + 2)*stride; point t of a pair
// plane occupies elements 2t and 2t + 1.  One vector access moves both
// values of a pair (16 bytes in float64, 8 in float32).
#pragma once

#include <hip/hip_runtime.h>

#include "kgs_internal.h"

namespace kgs {

template <typename T>
struct PairOf;
template <>
struct PairOf<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct PairOf<float> {
    typedef float type __attribute__((ext_vector_type(2)));
};
template <typename T>
using Pair = typename PairOf<T>::type;

enum PairKind { PAIR_PQ = 0, PAIR_UV = 1 };

// The state always lives in device (global) memory.  A state pointer read
// from a descriptor in memory, rather than passed as a kernel argument,
// carries no address space, and accesses through it would compile to FLAT
// instructions, which also count against the LDS wait counter.  Every
// state access below therefore goes through a pointer typed in the global
// address space, which makes the compiler emit global loads and stores.
template <typename T>
using Global = __attribute__((address_space(1))) T;

template <typename T>
__device__ __forceinline__ T ld_global(const T *p)
{
    return *(const Global<T> *)p;
}

// First element of pair plane `pk` (PAIR_PQ or PAIR_UV) of colour c.
template <typename T>
__device__ __forceinline__ T *pair_plane(T *base, int64_t stride, int c, int pk)
{
    return base + static_cast<int64_t>(4 * c + 2 * pk) * stride;
}

template <typename T>
__device__ __forceinline__ const T *pair_plane(const T *base, int64_t stride, int c, int pk)
{
    return base + static_cast<int64_t>(4 * c + 2 * pk) * stride;
}

template <typename T>
__device__ __forceinline__ Pair<T> ld_pair(const T *plane, int64_t t)
{
    return *(const Global<Pair<T>> *)(plane + 2 * t);
}

template <typename T>
__device__ __forceinline__ void st_pair(T *plane, int64_t t, T a, T b)
{
    Pair<T> v;
    v.x = a;
    v.y = b;
    *(Global<Pair<T>> *)(plane + 2 * t) = v;
}

}  // namespace kgs
