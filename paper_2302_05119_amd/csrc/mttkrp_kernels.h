// Dense MTTKRP of a 3-way block (the data term M_(n) U^{⊙-n} of eq. solapgU,
// operations 6-7 of Table timecomplx) in two passes over M per sweep:
//
//   pass 1:  Y[i1][i2][r] = sum_i3 M[i1][i2][i3] U3[i3][r]        (M x_3 U^(3))
//            K1[i1][r]    = sum_i2 Y[i1][i2][r] U2[i2][r]         (partials per 64 rows)
//   mode 2:  K2[i2][r]    = sum_i1 Y[i1][i2][r] U1[i1][r]         (new U^(1))
//   pass 2:  K3[i3][r]    = sum_i1 U1[i1][r] sum_i2 M[i1][i2][i3] U2[i2][r]
//            (partials per chunk of 4 slabs, reduced in fixed order later)
//
// Under the Gauss-Seidel order Y (built from the old U^(3)) serves the mode-1
// and the mode-2 gradient, so M is streamed twice per sweep.
//
// Matrix cores: v_mfma_f32_4x4x1f32 computes 16 independent 4x4 outer
// products per wavefront.  Lane l feeds A = element of output row l of a
// 64-row group and B = U[k][4t + l%4]; its accumulator holds rows 4*(l/4) + v
// (v = 0..3) of column 4t + l%4.  R is tiled in exact groups of 4 columns
// (R = 20 and 40 need no padding).  The FP64 path runs the same layout with
// lane shuffles and FP64 FMAs.
//
#pragma once
#include <type_traits>
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

// Tensor elements are read through their storage bits (16-bit types as
// unsigned short) and widened to the accumulation type.
template <typename TM> struct Raw { typedef TM type; };
template <> struct Raw<__hip_bfloat16> { typedef unsigned short type; };
template <> struct Raw<__half> { typedef unsigned short type; };
template <typename TA, typename TM> __device__ __forceinline__ TA cvt(typename Raw<TM>::type x);
template <> __device__ __forceinline__ float cvt<float, float>(float x) { return x; }
template <> __device__ __forceinline__ double cvt<double, double>(double x) { return x; }
template <> __device__ __forceinline__ float cvt<float, __hip_bfloat16>(unsigned short x) { return __uint_as_float((unsigned)x << 16); }
template <> __device__ __forceinline__ float cvt<float, __half>(unsigned short x) { return __half2float(__ushort_as_half(x)); }

// i3 columns staged per step; the odd LDS row stride keeps column reads
// conflict-free.
template <typename TA> struct P1Shape { static constexpr int KC = 32, STRIDE = 33; };
template <> struct P1Shape<double> { static constexpr int KC = 16, STRIDE = 17; };

// ---------------------------------------------------------------------------
// pass 1: one workgroup per (block, i1 slab, 64-row group of i2); the four
// wavefronts split the i3 range and are summed in LDS.  Tiles are staged with
// every load of a tile in flight before the first LDS store.
// ---------------------------------------------------------------------------
template <typename TM, typename T, int RT, int GATE>
__global__ __launch_bounds__(256) void k_pass1(const Geo* __restrict__ g, StateP<T> st, const ItemP1* __restrict__ items,
                                               int slot) {
    typedef typename AccType<TM>::type TA;
    if (gated_out(st.ctrl, GATE)) return;
    extern __shared__ char smraw[];
    const ItemP1 it = items[blockIdx.x];
    const int s = it.s, i1 = it.i1, rg = it.rg, row0 = rg * 64;
    const int I2 = g->I[s][1], I3 = g->I[s][2], Rq = g->Rq;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nrows = min(64, I2 - row0);
    typedef typename Raw<TM>::type TR;
    const CPD_GLOBAL TR* __restrict__ Ms = gptr((const TR*)g->M[s] + ((long long)i1 * I2 + row0) * I3);
    const CPD_GLOBAL T* __restrict__ U3 = gptr(st.U[slot] + g->uoff[2][s]);
    TA* sm = (TA*)smraw;
    constexpr int KC = P1Shape<TA>::KC, STRIDE = P1Shape<TA>::STRIDE, RPI = 64 / KC;
    TA* stage = sm + wave * 64 * STRIDE;

    const int kq = (I3 + 3) / 4;
    const int kb = min(I3, wave * kq), ke = min(I3, kb + kq);
    Acc4<TA> acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t].zero();

    const int cc = lane % KC, rsub = lane / KC;
    for (int k0 = kb; k0 < ke; k0 += KC) {
        const int kc = min(KC, ke - k0);
        TA buf[KC];
#pragma unroll
        for (int j = 0; j < KC; ++j) {
            const int r = j * RPI + rsub;
            buf[j] = (r < nrows && cc < kc) ? cvt<TA, TM>(Ms[(long long)r * I3 + k0 + cc]) : (TA)0;
        }
#pragma unroll
        for (int j = 0; j < KC; ++j) stage[(j * RPI + rsub) * STRIDE + cc] = buf[j];
        wave_sync();
        const CPD_GLOBAL T* __restrict__ urow = U3 + (long long)k0 * Rq + (lane & 3);
#pragma unroll 4
        for (int kk = 0; kk < kc; ++kk) {
            const TA a = stage[lane * STRIDE + kk];
            TA bb[RT];
#pragma unroll
            for (int t = 0; t < RT; ++t) bb[t] = (TA)urow[(long long)kk * Rq + 4 * t];
#pragma unroll
            for (int t = 0; t < RT; ++t) acc[t].mma(a, bb[t]);
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
    CPD_GLOBAL T* __restrict__ Y = gptr_w(st.Y + g->yoff[s] + ((long long)i1 * I2 + row0) * Rq);
    for (int e = threadIdx.x; e < nrows * Rq; e += 256) {
        const int r = e / Rq, c = e % Rq;
        const TA v = red[(0 * 64 + r) * Rq + c] + red[(1 * 64 + r) * Rq + c] + red[(2 * 64 + r) * Rq + c] +
                     red[(3 * 64 + r) * Rq + c];
        Y[(long long)r * Rq + c] = (T)v;
        red[r * Rq + c] = (TA)(T)v;
    }
    __syncthreads();
    // mode-1 partial over this row group: sum_r Y[r][c] U2_old[row0 + r][c]
    if (threadIdx.x < Rq) {
        const int c = threadIdx.x;
        const CPD_GLOBAL T* __restrict__ U2 = gptr(st.U[1] + g->uoff[1][s] + (long long)row0 * Rq + c);
        double a = 0.0;
#pragma unroll 8
        for (int r = 0; r < nrows; ++r) a += (double)red[r * Rq + c] * (double)U2[(long long)r * Rq];
        gptr_w(st.K1p)[g->k1off[s] + ((long long)i1 * g->nrg[s] + rg) * Rq + c] = (T)a;
    }
}

// ---------------------------------------------------------------------------
// pass 2: one workgroup per (block, chunk of 4 i1 slabs, 64 consecutive i3);
// wavefront w takes slab 4*chunk + w.  Lanes run along i3 (the contiguous
// index), so every tensor load is a coalesced 64-element row segment; NB rows
// are loaded ahead of the matrix-core work.  U2 is staged in LDS when it fits.
// ---------------------------------------------------------------------------
template <typename TM, typename T, int RT, bool BLDS, int GATE>
__global__ __launch_bounds__(256) void k_pass2(const Geo* __restrict__ g, StateP<T> st, const ItemP2* __restrict__ items,
                                               int slot) {
    typedef typename AccType<TM>::type TA;
    if (gated_out(st.ctrl, GATE)) return;
    extern __shared__ char smraw[];
    const ItemP2 it = items[blockIdx.x];
    const int s = it.s, chunk = it.chunk, q0 = it.q0;
    const int I1 = g->I[s][0], I2 = g->I[s][1], I3 = g->I[s][2], Rq = g->Rq;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i1 = chunk * 4 + wave;
    const int i3 = q0 + lane;
    const bool valid = i3 < I3;
    TA* sm = (TA*)smraw;
    const CPD_GLOBAL T* __restrict__ U2g = gptr(st.U[slot] + g->uoff[1][s]);
    if (BLDS) {
        for (int e = threadIdx.x; e < I2 * Rq; e += 256) sm[e] = (TA)U2g[e];
        __syncthreads();
    }
    Acc4<TA> z[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) z[t].zero();
    constexpr int NB = 16;
    if (i1 < I1) {
        typedef typename Raw<TM>::type TR;
        const CPD_GLOBAL TR* __restrict__ Mp = gptr((const TR*)g->M[s] + (long long)i1 * I2 * I3 + (valid ? i3 : 0));
        TA cur[NB], nxt[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) cur[j] = (valid && j < I2) ? cvt<TA, TM>(Mp[(long long)j * I3]) : (TA)0;
        for (int i2b = 0; i2b < I2; i2b += NB) {
            const int nb2 = i2b + NB;
#pragma unroll
            for (int j = 0; j < NB; ++j) nxt[j] = (valid && nb2 + j < I2) ? cvt<TA, TM>(Mp[(long long)(nb2 + j) * I3]) : (TA)0;
            const int jm = min(NB, I2 - i2b);
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                if (j < jm) {
                    const int i2 = i2b + j;
                    TA bb[RT];
#pragma unroll
                    for (int t = 0; t < RT; ++t)
                        bb[t] = BLDS ? sm[i2 * Rq + 4 * t + (lane & 3)] : (TA)U2g[(long long)i2 * Rq + 4 * t + (lane & 3)];
#pragma unroll
                    for (int t = 0; t < RT; ++t) z[t].mma(cur[j], bb[t]);
                }
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) cur[j] = nxt[j];
        }
        const CPD_GLOBAL T* __restrict__ U1 = gptr(st.U[slot] + g->uoff[0][s] + (long long)i1 * Rq + (lane & 3));
#pragma unroll
        for (int t = 0; t < RT; ++t) z[t].scale((TA)U1[4 * t]);
    }
    if (BLDS) __syncthreads();
    TA* red = sm;  // [4 waves][64][Rq]
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            red[(wave * 64 + 4 * (lane >> 2) + v) * Rq + 4 * t + (lane & 3)] = z[t].get(v);
    __syncthreads();
    const int nq = min(64, I3 - q0);
    CPD_GLOBAL T* __restrict__ out = gptr_w(st.part + g->poff[s] + ((long long)chunk * I3 + q0) * Rq);
    for (int e = threadIdx.x; e < nq * Rq; e += 256) {
        const int r = e / Rq, c = e % Rq;
        const TA v = red[(0 * 64 + r) * Rq + c] + red[(1 * 64 + r) * Rq + c] + red[(2 * 64 + r) * Rq + c] +
                     red[(3 * 64 + r) * Rq + c];
        out[(long long)r * Rq + c] = (T)v;
    }
}

// ---------------------------------------------------------------------------
// mode-2 contraction K2[i2][c] = sum_i1 Y[i1][i2][c] U1[i1][c] (FP64 sums):
// one workgroup per (block, 64 rows of i2).  Four thread groups take
// interleaved quarters of i1 with all their loads in flight, then the
// quarters are added in fixed order.
// ---------------------------------------------------------------------------
template <typename T, int GATE>
__global__ __launch_bounds__(256) void k_k2(const Geo* __restrict__ g, StateP<T> st, const ItemK2* __restrict__ items, int slot) {
    if (gated_out(st.ctrl, GATE)) return;
    __shared__ double part[4][256];
    const ItemK2 it = items[blockIdx.x];
    const int s = it.s, row0 = it.row0;
    const int I1 = g->I[s][0], I2 = g->I[s][1], Rq = g->Rq;
    const int nrows = min(64, I2 - row0);
    const CPD_GLOBAL T* __restrict__ U1 = gptr(st.U[slot] + g->uoff[0][s]);
    const CPD_GLOBAL T* __restrict__ Y = gptr(st.Y + g->yoff[s] + (long long)row0 * Rq);
    const long long ys = (long long)I2 * Rq;
    const int grp = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const int nout = nrows * Rq;
    for (int e0 = 0; e0 < nout; e0 += 64) {
        const int e = e0 + ln;
        const int c = e % Rq;
        double a = 0.0;
        if (e < nout) {
#pragma unroll 8
            for (int i1 = grp; i1 < I1; i1 += 4) a += (double)Y[i1 * ys + e] * (double)U1[(long long)i1 * Rq + c];
        }
        part[grp][ln] = a;
        __syncthreads();
        if (grp == 0 && e < nout)
            gptr_w(st.K2)[g->k2off[s] + (long long)row0 * Rq + e] = (T)(part[0][ln] + part[1][ln] + part[2][ln] + part[3][ln]);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// launch templates: dispatch on the tensor operand type and on RT = Rq / 4.
// GATE = 1 instantiates the kernels of the re-done sweep (distinct symbols,
// built in their own translation unit).
// ---------------------------------------------------------------------------
template <int GATE, typename TM, typename T>
static void pass1_rt(int RT, dim3 grid, size_t lds, hipStream_t q, const Geo* g, const StateP<T>& st, const ItemP1* items,
                     int slot) {
#define CPD_P1(RTV) \
    case RTV: hipLaunchKernelGGL((k_pass1<TM, T, RTV, GATE>), grid, dim3(256), lds, q, g, st, items, slot); break;
    switch (RT) {
        CPD_P1(1) CPD_P1(2) CPD_P1(3) CPD_P1(4) CPD_P1(5) CPD_P1(6) CPD_P1(7) CPD_P1(8)
        CPD_P1(9) CPD_P1(10) CPD_P1(11) CPD_P1(12) CPD_P1(13) CPD_P1(14) CPD_P1(15) CPD_P1(16)
        default: break;
    }
#undef CPD_P1
}
template <int GATE, typename TM, typename T, bool BLDS>
static void pass2_rt(int RT, dim3 grid, size_t lds, hipStream_t q, const Geo* g, const StateP<T>& st, const ItemP2* items,
                     int slot) {
#define CPD_P2(RTV) \
    case RTV: hipLaunchKernelGGL((k_pass2<TM, T, RTV, BLDS, GATE>), grid, dim3(256), lds, q, g, st, items, slot); break;
    switch (RT) {
        CPD_P2(1) CPD_P2(2) CPD_P2(3) CPD_P2(4) CPD_P2(5) CPD_P2(6) CPD_P2(7) CPD_P2(8)
        CPD_P2(9) CPD_P2(10) CPD_P2(11) CPD_P2(12) CPD_P2(13) CPD_P2(14) CPD_P2(15) CPD_P2(16)
        default: break;
    }
#undef CPD_P2
}

template <typename TA>
static size_t pass1_lds(int Rq) {
    size_t a = sizeof(TA) * 4 * 64 * (size_t)P1Shape<TA>::STRIDE, b = sizeof(TA) * 4 * 64 * (size_t)Rq;
    return a > b ? a : b;
}

template <int GATE, typename TM, typename T>
static void pass2_dispatch(int Rq, dim3 grid, int maxI2, hipStream_t q, const Geo* g, const StateP<T>& st,
                           const ItemP2* items, int slot) {
    typedef typename AccType<TM>::type TA;
    const size_t red = sizeof(TA) * 4 * 64 * (size_t)Rq;
    const size_t bst = sizeof(TA) * (size_t)maxI2 * Rq;
    if (bst <= 49152) pass2_rt<GATE, TM, T, true>(Rq / 4, grid, bst > red ? bst : red, q, g, st, items, slot);
    else pass2_rt<GATE, TM, T, false>(Rq / 4, grid, red, q, g, st, items, slot);
}

template <int GATE, typename T>
void pass1_impl(const Geo* g, const StateP<T>& st, const ItemP1* items, int nitems, int Rq, int slot, int mdtype,
                hipStream_t q) {
    if (nitems <= 0) return;
    const dim3 grid(nitems);
    if constexpr (std::is_same<T, double>::value) {
        pass1_rt<GATE, double, double>(Rq / 4, grid, pass1_lds<double>(Rq), q, g, st, items, slot);
    } else {
        const size_t lds = pass1_lds<float>(Rq);
        if (mdtype == 1) pass1_rt<GATE, float, float>(Rq / 4, grid, lds, q, g, st, items, slot);
        else if (mdtype == 2) pass1_rt<GATE, __hip_bfloat16, float>(Rq / 4, grid, lds, q, g, st, items, slot);
        else pass1_rt<GATE, __half, float>(Rq / 4, grid, lds, q, g, st, items, slot);
    }
}

template <int GATE, typename T>
void pass2_impl(const Geo* g, const StateP<T>& st, const ItemP2* items, int nitems, int Rq, int slot, int mdtype, int maxI2,
                hipStream_t q) {
    if (nitems <= 0) return;
    const dim3 grid(nitems);
    if constexpr (std::is_same<T, double>::value) {
        pass2_dispatch<GATE, double, double>(Rq, grid, maxI2, q, g, st, items, slot);
    } else {
        if (mdtype == 1) pass2_dispatch<GATE, float, float>(Rq, grid, maxI2, q, g, st, items, slot);
        else if (mdtype == 2) pass2_dispatch<GATE, __hip_bfloat16, float>(Rq, grid, maxI2, q, g, st, items, slot);
        else pass2_dispatch<GATE, __half, float>(Rq, grid, maxI2, q, g, st, items, slot);
    }
}

template <int GATE, typename T>
void k2_impl(const Geo* g, const StateP<T>& st, const ItemK2* items, int nitems, int slot, hipStream_t q) {
    if (nitems <= 0) return;
    hipLaunchKernelGGL((k_k2<T, GATE>), dim3(nitems), dim3(256), 0, q, g, st, items, slot);
}

#define CPD_MTTKRP_IMPLS(SPEC, G)                                                                                        \
    SPEC void pass1_impl<G, float>(const Geo*, const StateP<float>&, const ItemP1*, int, int, int, int, hipStream_t);      \
    SPEC void pass1_impl<G, double>(const Geo*, const StateP<double>&, const ItemP1*, int, int, int, int, hipStream_t);    \
    SPEC void pass2_impl<G, float>(const Geo*, const StateP<float>&, const ItemP2*, int, int, int, int, int, hipStream_t); \
    SPEC void pass2_impl<G, double>(const Geo*, const StateP<double>&, const ItemP2*, int, int, int, int, int,           \
                                    hipStream_t);                                                                      \
    SPEC void k2_impl<G, float>(const Geo*, const StateP<float>&, const ItemK2*, int, int, hipStream_t);                  \
    SPEC void k2_impl<G, double>(const Geo*, const StateP<double>&, const ItemK2*, int, int, hipStream_t);

}  // namespace cpd
