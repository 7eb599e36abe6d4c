// Device helpers shared by the sweep kernels: 16-byte vector loads and
// stores, and the tagged 64-bit words through which the members of a
// cluster exchange their partial row products.
//
// A word holds a 32-bit payload and, in its upper half, the tag of the band
// and iteration it belongs to, so a reader validates what it reads without
// fences: it polls (agent-scope relaxed atomic loads) until the tag matches.
// Waits are bounded; at the bound the shared timeout flag is raised and
// every waiter returns.
#pragma once

#include "sfr_internal.hpp"

// 1: non-temporal hints on the sweeps' streams (measured +2-4 % iterations/s
// at 8000^2, r = 10, alternating with 0 on one device)
#ifndef SFR_NT_STREAMS
#define SFR_NT_STREAMS 1
#endif

namespace sfr {

template <typename T> struct Vec;
template <> struct Vec<float> { using t = float4; static constexpr int N = 4; };
template <> struct Vec<double> { using t = double2; static constexpr int N = 2; };

template <typename T>
__device__ __forceinline__ void load_vec(const T* p, T (&v)[Vec<T>::N])
{
    typename Vec<T>::t x = *reinterpret_cast<const typename Vec<T>::t*>(p);
    __builtin_memcpy(v, &x, sizeof(x));
}

template <typename T>
__device__ __forceinline__ void store_vec(T* p, const T (&v)[Vec<T>::N])
{
    typename Vec<T>::t x;
    __builtin_memcpy(&x, v, sizeof(x));
    *reinterpret_cast<typename Vec<T>::t*>(p) = x;
}

// Streaming forms for data touched once per sweep (M, Y_{k-1} read, Y_k
// written): non-temporal hints, so the streams do not displace the cached
// exchange words and factor slices.
template <typename T> struct NtVec;
template <> struct NtVec<float> { typedef float t __attribute__((ext_vector_type(4))); };
template <> struct NtVec<double> { typedef double t __attribute__((ext_vector_type(2))); };

template <typename T>
__device__ __forceinline__ void load_vec_stream(const T* p, T (&v)[Vec<T>::N])
{
#if SFR_NT_STREAMS
    const typename NtVec<T>::t x = __builtin_nontemporal_load(reinterpret_cast<const typename NtVec<T>::t*>(p));
#pragma unroll
    for (int i = 0; i < Vec<T>::N; ++i) v[i] = x[i];
#else
    load_vec<T>(p, v);
#endif
}

template <typename T>
__device__ __forceinline__ void store_vec_stream(T* p, const T (&v)[Vec<T>::N])
{
#if SFR_NT_STREAMS
    typename NtVec<T>::t x;
#pragma unroll
    for (int i = 0; i < Vec<T>::N; ++i) x[i] = v[i];
    __builtin_nontemporal_store(x, reinterpret_cast<typename NtVec<T>::t*>(p));
#else
    store_vec<T>(p, v);
#endif
}

// Number of 32-bit halves per exchanged value.
template <typename T> struct Words { static constexpr int N = sizeof(T) / 4; };

__device__ __forceinline__ unsigned long long spin_word(const unsigned long long* p, uint32_t tag,
                                                        int32_t* timeout_flag)
{
    unsigned long long w = 0;
    uint32_t n = 0;
    for (;;) {
        w = __hip_atomic_load(const_cast<unsigned long long*>(p), __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(w >> 32) == tag) break;
        if (((++n) & 1023u) == 0) {
            if (__hip_atomic_load(timeout_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            if (n >= kSpinLimit) {
                __hip_atomic_store(timeout_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return w;
}

template <typename T>
__device__ __forceinline__ void publish(unsigned long long* dst, T v, uint32_t tag)
{
    if constexpr (sizeof(T) == 4) {
        unsigned long long w = ((unsigned long long)tag << 32) | (unsigned long long)__float_as_uint(v);
        __hip_atomic_store(dst, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        unsigned long long bits = (unsigned long long)__double_as_longlong(v);
        unsigned long long lo = ((unsigned long long)tag << 32) | (bits & 0xffffffffull);
        unsigned long long hi = ((unsigned long long)tag << 32) | (bits >> 32);
        __hip_atomic_store(dst, lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(dst + 1, hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <typename T>
__device__ __forceinline__ T fetch(const unsigned long long* src, uint32_t tag, int32_t* timeout_flag)
{
    if constexpr (sizeof(T) == 4) {
        unsigned long long w = spin_word(src, tag, timeout_flag);
        return __uint_as_float((uint32_t)(w & 0xffffffffull));
    } else {
        unsigned long long lo = spin_word(src, tag, timeout_flag);
        unsigned long long hi = spin_word(src + 1, tag, timeout_flag);
        return __longlong_as_double((long long)((hi << 32) | (lo & 0xffffffffull)));
    }
}

__device__ __forceinline__ unsigned long long peek_word(const unsigned long long* p)
{
    return __hip_atomic_load(const_cast<unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace sfr
