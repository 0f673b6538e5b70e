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
template <typename TM, typename T, int RT>
__global__ __launch_bounds__(256) void k_pass1(const Geo* __restrict__ g, StateP<T> st, const ItemP1* __restrict__ items,
                                               int slot) {
    typedef typename AccType<TM>::type TA;
    if (st.ctrl->stop) return;
    apply_rot(st);
    extern __shared__ char smraw[];
    const ItemP1 it = items[blockIdx.x];
    const int s = it.s, i1 = it.i1, rg = it.rg, row0 = rg * 64;
    const int I2 = g->I[s][1], I3 = g->I[s][2], Rq = g->Rq;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nrows = min(64, I2 - row0);
    typedef typename Raw<TM>::type TR;
    const CPD_GLOBAL TR* __restrict__ Ms = gptr((const TR*)g->M[s] + ((long long)i1 * I2 + row0) * I3);
    const CPD_GLOBAL T* __restrict__ U3 = gptr(pick3(st.U, slot) + g->uoff[2][s]);
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
template <typename TM, typename T, int RT, bool BLDS>
__global__ __launch_bounds__(256) void k_pass2(const Geo* __restrict__ g, StateP<T> st, const ItemP2* __restrict__ items,
                                               int slot) {
    typedef typename AccType<TM>::type TA;
    if (st.ctrl->stop) return;
    apply_rot(st);
    extern __shared__ char smraw[];
    const ItemP2 it = items[blockIdx.x];
    const int s = it.s, chunk = it.chunk, q0 = it.q0;
    const int I1 = g->I[s][0], I2 = g->I[s][1], I3 = g->I[s][2], Rq = g->Rq;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i1 = chunk * 4 + wave;
    const int i3 = q0 + lane;
    const bool valid = i3 < I3;
    TA* sm = (TA*)smraw;
    const CPD_GLOBAL T* __restrict__ U2g = gptr(pick3(st.U, slot) + g->uoff[1][s]);
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
        const CPD_GLOBAL T* __restrict__ U1 = gptr(pick3(st.U, slot) + g->uoff[0][s] + (long long)i1 * Rq + (lane & 3));
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
// mode 2: K2[i2][r] = sum_i1 Y[i1][i2][r] U1[i1][r] with the new U^(1).  One
// thread per element e = i2*Rq + r of a 256-wide column tile, one workgroup
// per (block, tile, chunk of k2rows rows of i1); every Y load is a
// coalesced row segment.  Chunk partials are summed in fixed order by the
// factor update.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_k2(const Geo* __restrict__ g, StateP<T> st, const ItemK2* __restrict__ items, int slot) {
    if (st.ctrl->stop) return;
    apply_rot(st);
    const ItemK2 it = items[blockIdx.x];
    const int s = it.s, Rq = g->Rq;
    const int I1 = g->I[s][0], I2 = g->I[s][1];
    const long long ys = (long long)I2 * Rq;
    const int e = it.col0 + (int)threadIdx.x;
    if (e >= ys) return;
    const int c = e % Rq;
    const int kr = g->k2rows;
    const int i1a = it.chunk * kr, i1b = min(I1, i1a + kr);
    const CPD_GLOBAL T* __restrict__ Y = gptr(st.Y + g->yoff[s] + e);
    const CPD_GLOBAL T* __restrict__ U1 = gptr(pick3(st.U, slot) + g->uoff[0][s] + c);
    T a0 = 0, a1 = 0;
    int i1 = i1a;
#pragma unroll 4
    for (; i1 + 1 < i1b; i1 += 2) {
        a0 += Y[i1 * ys] * U1[(long long)i1 * Rq];
        a1 += Y[(i1 + 1) * ys] * U1[(long long)(i1 + 1) * Rq];
    }
    if (i1 < i1b) a0 += Y[i1 * ys] * U1[(long long)i1 * Rq];
    gptr_w(st.K2)[g->k2off[s] + (long long)it.chunk * ys + e] = a0 + a1;
}

}  // namespace cpd
