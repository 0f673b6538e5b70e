// Device helpers shared by the HIP translation units (wave64, gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <float.h>
#include <math.h>
#include "concpd_internal.h"

typedef float v4f __attribute__((ext_vector_type(4)));

namespace cpd {

// Global-address-space view of a pointer read from a struct (such pointers
// are generic otherwise, and generic accesses serialise with LDS traffic).
#define CPD_GLOBAL __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ const CPD_GLOBAL T* gptr(const T* p) { return (const CPD_GLOBAL T*)p; }
template <typename T> __device__ __forceinline__ CPD_GLOBAL T* gptr_w(T* p) { return (CPD_GLOBAL T*)p; }

// Orders LDS traffic of one wavefront (lanes of a wave exchanging data
// through LDS without a workgroup barrier).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// max(0, x) that keeps NaN (the projection must not hide a non-finite value).
__device__ __forceinline__ double relu_keep_nan(double x) { return (x > 0.0 || x != x) ? x : 0.0; }

// Acquire-load of a value written by another workgroup of the same launch.
__device__ __forceinline__ double load_agent(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool gated_out(const Ctrl* c, int gate) {
    return c->stop || (gate && !c->redo);
}

// Operand conversion of tensor elements.
template <typename TM> __device__ __forceinline__ float to_f32(TM x);
template <> __device__ __forceinline__ float to_f32<float>(float x) { return x; }
template <> __device__ __forceinline__ float to_f32<__hip_bfloat16>(__hip_bfloat16 x) { return __bfloat162float(x); }
template <> __device__ __forceinline__ float to_f32<__half>(__half x) { return __half2float(x); }

// Extrapolation weight w = min(w_hat, delta_w sqrt(L_prev / L_cur)) (eq.
// eqextrawd / eqextrawu); a negative L_prev marks "no previous constant".
__device__ __forceinline__ double extrap_weight(int extrapolate, double w_hat, double Lp, double Lc, double dw) {
    if (!extrapolate || Lp < 0.0 || !(Lc > 0.0)) return 0.0;
    return fmin(w_hat, dw * sqrt(Lp / Lc));
}

}  // namespace cpd
