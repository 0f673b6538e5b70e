// Dense MTTKRP of a 3-way block (the data term M_(n) U^{⊙-n} of eq. solapgU,
// operations 6-7 of Table timecomplx) in two passes per sweep:
//
//   pass 1:  Y[i1][i2][r] = sum_i3 M[i1][i2][i3] U3[i3][r]         (M x_3 U^(3))
//            K1 and K2 are contracted from Y by the update kernel;
//   pass 2:  K3[i3][r]    = sum_i1 U1[i1][r] sum_i2 M[i1][i2][i3] U2[i2][r]
//            written as per-chunk partials, reduced in fixed order later.
//
// Under the Gauss-Seidel order, Y (built from the old U^(3)) serves both the
// mode-1 and the mode-2 gradient, so M is streamed twice per sweep.
//
// Matrix core tiling: v_mfma_f32_4x4x1f32 computes 16 independent 4x4 outer
// products per wavefront.  Lane l feeds A = element of output row l of a 64-row
// group and B = U[k][4t + l%4]; the accumulator of lane l holds rows
// 4*(l/4) + v (v = 0..3) of column 4t + l%4.  R is tiled in exact groups of 4
// columns (R = 20, 40 need no padding).  The FP64 path runs the same layout
// with lane shuffles and FP64 FMAs.
#include "dev_common.h"

namespace cpd {

template <typename TA> struct Acc4;
template <> struct Acc4<float> {
    v4f v;
    __device__ void zero() { v = (v4f){0.f, 0.f, 0.f, 0.f}; }
    __device__ void mma(float a, float b) { v = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, v, 0, 0, 0); }
    __device__ float get(int i) const { return v[i]; }
    __device__ void scale(float u) { v *= u; }
};
template <> struct Acc4<double> {
    double v[4];
    __device__ void zero() { v[0] = v[1] = v[2] = v[3] = 0.0; }
    __device__ void mma(double a, double b) {
        const int base = (threadIdx.x & 63) & ~3;
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] += __shfl(a, base + i, 64) * b;
    }
    __device__ double get(int i) const { return v[i]; }
    __device__ void scale(double u) {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] *= u;
    }
};

template <typename TM> struct AccType { typedef float type; };
template <> struct AccType<double> { typedef double type; };

template <typename TA, typename TM> __device__ __forceinline__ TA cvt(TM x);
template <> __device__ __forceinline__ float cvt<float, float>(float x) { return x; }
template <> __device__ __forceinline__ double cvt<double, double>(double x) { return x; }
template <> __device__ __forceinline__ float cvt<float, __hip_bfloat16>(__hip_bfloat16 x) { return __bfloat162float(x); }
template <> __device__ __forceinline__ float cvt<float, __half>(__half x) { return __half2float(x); }

// i3 columns staged per step; the odd LDS row stride keeps column reads
// conflict-free.
template <typename TA> struct P1Shape { static constexpr int KC = 32; static constexpr int STRIDE = 33; };
template <> struct P1Shape<double> { static constexpr int KC = 16; static constexpr int STRIDE = 17; };

// ---------------------------------------------------------------------------
// pass 1: one workgroup per (block, i1 slab, 64-row group of i2); the four
// wavefronts split the i3 range and are summed in LDS.
// ---------------------------------------------------------------------------
template <typename TM, typename T, int RT>
__global__ __launch_bounds__(256) void k_pass1(const Geo* __restrict__ g, StateP<T> st, const ItemP1* __restrict__ items,
                                               int slot, int gate) {
    typedef typename AccType<TM>::type TA;
    if (gated_out(st.ctrl, gate)) return;
    const ItemP1 it = items[blockIdx.x];
    const int s = it.s, i1 = it.i1, row0 = it.rg * 64;
    const int I2 = g->I[s][1], I3 = g->I[s][2], Rq = g->Rq;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nrows = min(64, I2 - row0);
    const TM* __restrict__ Ms = (const TM*)g->M[s] + ((long long)i1 * I2 + row0) * I3;
    const T* __restrict__ U3 = st.U[slot] + g->uoff[2][s];
    extern __shared__ char smraw[];
    TA* sm = (TA*)smraw;
    constexpr int P1_KC = P1Shape<TA>::KC, P1_STRIDE = P1Shape<TA>::STRIDE;
    TA* stage = sm + wave * 64 * P1_STRIDE;

    const int kq = (I3 + 3) / 4;
    const int kb = min(I3, wave * kq), ke = min(I3, kb + kq);
    Acc4<TA> acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t].zero();

    for (int k0 = kb; k0 < ke; k0 += P1_KC) {
        const int kc = min(P1_KC, ke - k0);
        for (int e = lane; e < 64 * P1_KC; e += 64) {
            const int r = e / P1_KC, cc = e % P1_KC;
            TA v = (TA)0;
            if (r < nrows && cc < kc) v = cvt<TA, TM>(Ms[(long long)r * I3 + k0 + cc]);
            stage[r * P1_STRIDE + cc] = v;
        }
        wave_sync();
        const T* __restrict__ urow = U3 + (long long)k0 * Rq + (lane & 3);
        for (int kk = 0; kk < kc; ++kk) {
            const TA a = stage[lane * P1_STRIDE + kk];
#pragma unroll
            for (int t = 0; t < RT; ++t) acc[t].mma(a, (TA)urow[4 * t]);
            urow += Rq;
        }
        wave_sync();
    }
    __syncthreads();
    TA* red = sm;  // [4 waves][64 rows][Rq]
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            red[(wave * 64 + 4 * (lane >> 2) + v) * Rq + 4 * t + (lane & 3)] = acc[t].get(v);
    __syncthreads();
    T* __restrict__ Y = st.Y + g->yoff[s] + ((long long)i1 * I2 + row0) * Rq;
    for (int e = threadIdx.x; e < nrows * Rq; e += 256) {
        const int r = e / Rq, cc = e % Rq;
        const TA v = red[(0 * 64 + r) * Rq + cc] + red[(1 * 64 + r) * Rq + cc] + red[(2 * 64 + r) * Rq + cc] +
                     red[(3 * 64 + r) * Rq + cc];
        Y[(long long)r * Rq + cc] = (T)v;
    }
}

// ---------------------------------------------------------------------------
// pass 2: one workgroup per (block, chunk of 4 i1 slabs, 64 consecutive i3);
// wavefront w takes slab 4*chunk + w.  Lanes run along i3 (the contiguous
// index), so every tensor load is a coalesced 64-element row segment.
// ---------------------------------------------------------------------------
template <typename TM, typename T, int RT>
__global__ __launch_bounds__(256) void k_pass2(const Geo* __restrict__ g, StateP<T> st, const ItemP2* __restrict__ items,
                                               int slot, int gate) {
    typedef typename AccType<TM>::type TA;
    if (gated_out(st.ctrl, gate)) return;
    const ItemP2 it = items[blockIdx.x];
    const int s = it.s, chunk = it.chunk, q0 = it.q0;
    const int I1 = g->I[s][0], I2 = g->I[s][1], I3 = g->I[s][2], Rq = g->Rq;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i1 = chunk * 4 + wave;
    const int i3 = q0 + lane;
    const bool valid = i3 < I3;
    Acc4<TA> z[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) z[t].zero();
    if (i1 < I1) {
        const TM* __restrict__ Mp = (const TM*)g->M[s] + (long long)i1 * I2 * I3 + (valid ? i3 : 0);
        const T* __restrict__ U2 = st.U[slot] + g->uoff[1][s] + (lane & 3);
#pragma unroll 4
        for (int i2 = 0; i2 < I2; ++i2) {
            const TA a = valid ? cvt<TA, TM>(Mp[(long long)i2 * I3]) : (TA)0;
#pragma unroll
            for (int t = 0; t < RT; ++t) z[t].mma(a, (TA)U2[(long long)i2 * Rq + 4 * t]);
        }
        const T* __restrict__ U1 = st.U[slot] + g->uoff[0][s] + (long long)i1 * Rq + (lane & 3);
#pragma unroll
        for (int t = 0; t < RT; ++t) z[t].scale((TA)U1[4 * t]);
    }
    extern __shared__ char smraw[];
    TA* red = (TA*)smraw;  // [4 waves][64][Rq]
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            red[(wave * 64 + 4 * (lane >> 2) + v) * Rq + 4 * t + (lane & 3)] = z[t].get(v);
    __syncthreads();
    const int nq = min(64, I3 - q0);
    T* __restrict__ out = st.part + g->poff[s] + ((long long)chunk * I3 + q0) * Rq;
    for (int e = threadIdx.x; e < nq * Rq; e += 256) {
        const int r = e / Rq, cc = e % Rq;
        const TA v = red[(0 * 64 + r) * Rq + cc] + red[(1 * 64 + r) * Rq + cc] + red[(2 * 64 + r) * Rq + cc] +
                     red[(3 * 64 + r) * Rq + cc];
        out[(long long)r * Rq + cc] = (T)v;
    }
}

// ---------------------------------------------------------------------------
// launchers: dispatch on the tensor operand type and on RT = Rq / 4
// ---------------------------------------------------------------------------
template <typename TM, typename T>
static void pass1_rt(int RT, const Geo* g, const StateP<T>& st, const ItemP1* items, int n, size_t lds, int slot, int gate,
                     hipStream_t q) {
#define CPD_P1(RTV) \
    case RTV: hipLaunchKernelGGL((k_pass1<TM, T, RTV>), dim3(n), dim3(256), lds, q, g, st, items, slot, gate); break;
    switch (RT) {
        CPD_P1(1) CPD_P1(2) CPD_P1(3) CPD_P1(4) CPD_P1(5) CPD_P1(6) CPD_P1(7) CPD_P1(8)
        CPD_P1(9) CPD_P1(10) CPD_P1(11) CPD_P1(12) CPD_P1(13) CPD_P1(14) CPD_P1(15) CPD_P1(16)
        default: break;
    }
#undef CPD_P1
}
template <typename TM, typename T>
static void pass2_rt(int RT, const Geo* g, const StateP<T>& st, const ItemP2* items, int n, size_t lds, int slot, int gate,
                     hipStream_t q) {
#define CPD_P2(RTV) \
    case RTV: hipLaunchKernelGGL((k_pass2<TM, T, RTV>), dim3(n), dim3(256), lds, q, g, st, items, slot, gate); break;
    switch (RT) {
        CPD_P2(1) CPD_P2(2) CPD_P2(3) CPD_P2(4) CPD_P2(5) CPD_P2(6) CPD_P2(7) CPD_P2(8)
        CPD_P2(9) CPD_P2(10) CPD_P2(11) CPD_P2(12) CPD_P2(13) CPD_P2(14) CPD_P2(15) CPD_P2(16)
        default: break;
    }
#undef CPD_P2
}

// The FP64 context only ever sees FP64 tensors; the FP32 context sees
// FP32 / BF16 / FP16 operands.
template <>
void launch_pass1<double>(const Geo* g, const StateP<double>& st, const ItemP1* items, int nitems, int Rq, int slot,
                          int gate, int mdtype, hipStream_t q) {
    (void)mdtype;
    if (nitems <= 0) return;
    size_t lds = sizeof(double) * 4 * 64 * (size_t)P1Shape<double>::STRIDE;
    const size_t lred = sizeof(double) * 4 * 64 * (size_t)Rq;
    if (lred > lds) lds = lred;
    pass1_rt<double, double>(Rq / 4, g, st, items, nitems, lds, slot, gate, q);
}
template <>
void launch_pass2<double>(const Geo* g, const StateP<double>& st, const ItemP2* items, int nitems, int Rq, int slot,
                          int gate, int mdtype, hipStream_t q) {
    (void)mdtype;
    if (nitems <= 0) return;
    pass2_rt<double, double>(Rq / 4, g, st, items, nitems, sizeof(double) * 4 * 64 * (size_t)Rq, slot, gate, q);
}
template <>
void launch_pass1<float>(const Geo* g, const StateP<float>& st, const ItemP1* items, int nitems, int Rq, int slot,
                         int gate, int mdtype, hipStream_t q) {
    if (nitems <= 0) return;
    size_t lds = sizeof(float) * 4 * 64 * (size_t)P1Shape<float>::STRIDE;
    const size_t lred = sizeof(float) * 4 * 64 * (size_t)Rq;
    if (lred > lds) lds = lred;
    if (mdtype == 1) pass1_rt<float, float>(Rq / 4, g, st, items, nitems, lds, slot, gate, q);
    else if (mdtype == 2) pass1_rt<__hip_bfloat16, float>(Rq / 4, g, st, items, nitems, lds, slot, gate, q);
    else pass1_rt<__half, float>(Rq / 4, g, st, items, nitems, lds, slot, gate, q);
}
template <>
void launch_pass2<float>(const Geo* g, const StateP<float>& st, const ItemP2* items, int nitems, int Rq, int slot,
                         int gate, int mdtype, hipStream_t q) {
    if (nitems <= 0) return;
    const size_t lds = sizeof(float) * 4 * 64 * (size_t)Rq;
    if (mdtype == 1) pass2_rt<float, float>(Rq / 4, g, st, items, nitems, lds, slot, gate, q);
    else if (mdtype == 2) pass2_rt<__hip_bfloat16, float>(Rq / 4, g, st, items, nitems, lds, slot, gate, q);
    else pass2_rt<__half, float>(Rq / 4, g, st, items, nitems, lds, slot, gate, q);
}

}  // namespace cpd
