// Device helpers shared by the HIP translation units (wave64, gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <float.h>
#include <limits.h>
#include <math.h>
#include "concpd_internal.h"

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));   // one 16-byte load

namespace cpd {

// Global-address-space view of a pointer read from a struct (such pointers
// are generic otherwise, and generic accesses serialise with LDS traffic).
#define CPD_GLOBAL __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ const CPD_GLOBAL T* gptr(const T* p) { return (const CPD_GLOBAL T*)p; }
template <typename T> __device__ __forceinline__ CPD_GLOBAL T* gptr_w(T* p) { return (CPD_GLOBAL T*)p; }

// v_mfma_f64_16x16x4f64: D (16x16) += A (16x4) B (4x16) in FP64.  Lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; register v of lane l holds
// D[4v + l / 16][l % 16].
__device__ __forceinline__ v4d mfma64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

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

// Wavefront min of lo and max of hi in one pass (the two butterflies overlap).
__device__ __forceinline__ void wave_minmax(double& lo, double& hi) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double a = __shfl_xor(lo, o, 64), b = __shfl_xor(hi, o, 64);
        lo = fmin(lo, a);
        hi = fmax(hi, b);
    }
}

// max(0, x) that keeps NaN (the projection must not hide a non-finite value).
__device__ __forceinline__ double relu_keep_nan(double x) { return (x > 0.0 || x != x) ? x : 0.0; }

// A double handed from one workgroup to another of the same launch: the
// writer stores it with an agent-scope atomic store (written through to the
// coherence point shared by all XCDs), waits for the store to complete
// (wait_stores) and only then takes its arrival count; the reader loads it
// with an agent-scope atomic load after seeing the final count.  This orders
// the one value without the device-scope fences, which on this multi-L2 part
// write back and invalidate the whole L2 of the XCD.
__device__ __forceinline__ void store_agent(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_agent(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// s_waitcnt vmcnt(0): every global load and store of the wavefront has
// completed.  The compiler fences on both sides keep the compiler from moving
// a memory access across the wait; the wait itself orders the hardware: an
// agent-scope store has reached the coherence point shared by all XCDs when
// its completion is counted.
__device__ __forceinline__ void wait_stores() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
// Arrival count of a last-workgroup reduction, at agent scope (the counter
// lives at the coherence point; the value returned orders nothing by itself:
// the handed-over data travels by store_agent / wait_stores / load_agent).
__device__ __forceinline__ unsigned arrive_agent(unsigned* counter) {
    return __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// An accepted sweep rotates the slots instead of copying them: logical slot l
// of the factors and lambda (0: x_k being built, 1: x_{k-1}, 2: x_{k-2}) is
// physical slot (rot3 + l) % 3; logical slot l of the Grams and b (0: this
// sweep, 1: x_{k-1}) is physical slot rot2 ^ l.  Kernels remap the pointers of
// their state copy on entry and then address logical slots only.
template <typename T>
__device__ __forceinline__ void apply_rot(StateP<T>& st) {
    const int r3 = st.ctrl->rot3, r2 = st.ctrl->rot2;
    T* u0 = st.U[0];
    T* u1 = st.U[1];
    T* u2 = st.U[2];
    st.U[0] = r3 == 0 ? u0 : (r3 == 1 ? u1 : u2);
    st.U[1] = r3 == 0 ? u1 : (r3 == 1 ? u2 : u0);
    st.U[2] = r3 == 0 ? u2 : (r3 == 1 ? u0 : u1);
    double* l0 = st.lam[0];
    double* l1 = st.lam[1];
    double* l2 = st.lam[2];
    st.lam[0] = r3 == 0 ? l0 : (r3 == 1 ? l1 : l2);
    st.lam[1] = r3 == 0 ? l1 : (r3 == 1 ? l2 : l0);
    st.lam[2] = r3 == 0 ? l2 : (r3 == 1 ? l0 : l1);
    double* v0 = st.V[0];
    double* v1 = st.V[1];
    st.V[0] = r2 ? v1 : v0;
    st.V[1] = r2 ? v0 : v1;
    double* b0 = st.b[0];
    double* b1 = st.b[1];
    st.b[0] = r2 ? b1 : b0;
    st.b[1] = r2 ? b0 : b1;
}

// a[i] for a runtime i without indexing the array (a dynamically indexed
// local copy of the state would be placed in scratch memory).
template <typename P>
__device__ __forceinline__ P pick3(P const (&a)[3], int i) {
    return i == 0 ? a[0] : (i == 1 ? a[1] : a[2]);
}

// Extrapolation is off in the sweep that redoes a rejected one (Algorithm 1).
__device__ __forceinline__ int extrapolating(const Ctrl* c, int extrapolate) { return extrapolate && !c->redo; }

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
