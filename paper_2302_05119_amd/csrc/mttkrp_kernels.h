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
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    const ItemP1 it = items[blockIdx.x];
    const int s = it.s, i1 = it.i1, rg = it.rg, row0 = rg * 64;
    const int I2 = g->I[s][1], I3 = g->I[s][2], Rq = g->Rq;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nrows = min(64, I2 - row0);
    // epilogue mapping (phase, column) and its U2 values, loaded now so their
    // latency overlaps the main loop
    // (Rq = 4 RT, so there are 64 / RT phases and at most EPQ rows per thread)
    constexpr int EPR = 64 / RT, EPQ = (64 + EPR - 1) / EPR;
    const int ep_rp = EPR, ep_j = threadIdx.x / Rq, ep_c = threadIdx.x % Rq;
    const bool ep_on = ep_j < ep_rp;
    T u2v[EPQ];
    double ep_part = 0.0;
    {
        const CPD_GLOBAL T* __restrict__ U2 = gptr(st.U[1] + g->uoff[1][s] + (long long)row0 * Rq);
#pragma unroll
        for (int q = 0; q < EPQ; ++q) {
            const int r = ep_j + q * ep_rp;
            u2v[q] = (ep_on && r < nrows) ? U2[(long long)r * Rq + ep_c] : (T)0;
        }
    }
    typedef typename Raw<TM>::type TR;
    const long long ldm = g->mld[s];   // operand row stride (>= I3)
    const CPD_GLOBAL TR* __restrict__ Ms = gptr((const TR*)g->M[s] + ((long long)i1 * I2 + row0) * ldm);
    const CPD_GLOBAL T* __restrict__ U3 = gptr(pick3(st.U, slot) + g->uoff[2][s]);
    TA* sm = (TA*)smraw;
    constexpr int KC = P1Shape<TA>::KC;
    constexpr int VE = 16 / (int)sizeof(TR);          // tensor elements per 16-byte load
    constexpr int VA = 16 / (int)sizeof(TA);          // operand elements per 16-byte LDS read
    constexpr int RTP = (RT + VA - 1) / VA * VA;      // padded operand run per lane
    constexpr int UPL = (KC * 4 * RT + 63) / 64;      // U3 chunk elements loaded per lane
    // U3 rows of the chunk, transposed so that lane l's operands
    // U3[k][4t + l%4], t < RT, are one contiguous run: [KC][4][RTP]
    TA* ustage = sm + wave * (KC * 4 * RTP);

    // the four wavefronts split i3 at multiples of KC (so chunks stay aligned)
    const int kq = ((I3 + 3) / 4 + KC - 1) / KC * KC;
    const int kb = min(I3, wave * kq), ke = min(I3, kb + kq);
    Acc4<TA> acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t].zero();

    // Lane l owns tensor row l of the row group (rows past the group repeat
    // its last row; their outputs are never stored) and keeps its KC
    // consecutive elements of the chunk in registers as the A operand: 16-byte
    // loads when every row of the block starts 16-byte aligned.  The next
    // chunk is loaded while the current one is consumed.
    const bool vec = g->mvec[s] != 0;
    const CPD_GLOBAL TR* __restrict__ Mrow = Ms + (long long)min(lane, nrows - 1) * ldm;
    TA buf[KC], nbuf[KC], ubuf[UPL], nubuf[UPL];
    auto load_chunk = [&](int k0, TA (&ab)[KC], TA (&ub)[UPL]) {
        const int kc = min(KC, ke - k0);
        if (vec && kc == KC) {
            const CPD_GLOBAL u32x4* vp = (const CPD_GLOBAL u32x4*)(Mrow + k0);
#pragma unroll
            for (int v = 0; v < KC / VE; ++v) {
                const u32x4 w = vp[v];
                const TR* e = (const TR*)&w;
#pragma unroll
                for (int j = 0; j < VE; ++j) ab[v * VE + j] = cvt<TA, TM>(e[j]);
            }
        } else {
#pragma unroll
            for (int j = 0; j < KC; ++j) {
                const TA v = cvt<TA, TM>(Mrow[k0 + min(j, kc - 1)]);
                ab[j] = (j < kc) ? v : (TA)0;
            }
        }
#pragma unroll
        for (int q = 0; q < UPL; ++q) {
            const int e = q * 64 + lane, kk = e / (4 * RT), c = e % (4 * RT);
            const TA v = (TA)U3[(long long)(k0 + min(kk, kc - 1)) * Rq + c];
            ub[q] = (kk < kc) ? v : (TA)0;
        }
    };
    if (kb < ke) load_chunk(kb, buf, ubuf);
    for (int k0 = kb; k0 < ke; k0 += KC) {
#pragma unroll
        for (int q = 0; q < UPL; ++q) {
            const int e = q * 64 + lane, kk = e / (4 * RT), c = e % (4 * RT);
            if (e < KC * 4 * RT) ustage[(kk * 4 + (c & 3)) * RTP + (c >> 2)] = ubuf[q];
        }
        wave_sync();
        if (k0 + KC < ke) load_chunk(k0 + KC, nbuf, nubuf);
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            TA bb[RTP];
            const TA* ur = ustage + (kk * 4 + (lane & 3)) * RTP;
#pragma unroll
            for (int v = 0; v < RTP / VA; ++v) *(u32x4*)&bb[v * VA] = *(const u32x4*)(ur + v * VA);
#pragma unroll
            for (int t = 0; t < RT; ++t) acc[t].mma(buf[kk], bb[t]);
        }
        wave_sync();
#pragma unroll
        for (int j = 0; j < KC; ++j) buf[j] = nbuf[j];
#pragma unroll
        for (int q = 0; q < UPL; ++q) ubuf[q] = nubuf[q];
    }
    __syncthreads();
    TA* red = sm;  // [4 waves][64 rows][Rq]
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            red[(wave * 64 + 4 * (lane >> 2) + v) * Rq + 4 * t + (lane & 3)] = acc[t].get(v);
    __syncthreads();
    // Epilogue: thread (phase j, column c) with Rq * RP <= 256 sums the four
    // wave partials of rows j, j + RP, ..., writes Y, and accumulates the
    // mode-1 partial sum_r Y[r][c] U2_old[row0 + r][c] over its rows (U2
    // prefetched at kernel start); the RP phase sums are added in fixed order.
    CPD_GLOBAL T* __restrict__ Y = gptr_w(st.Y + g->yoff[s] + ((long long)i1 * I2 + row0) * Rq);
    if (ep_on) {
        double a = 0.0;
#pragma unroll
        for (int q = 0; q < EPQ; ++q) {
            const int r = ep_j + q * ep_rp;
            if (r < nrows) {
                const TA v = red[(0 * 64 + r) * Rq + ep_c] + red[(1 * 64 + r) * Rq + ep_c] + red[(2 * 64 + r) * Rq + ep_c] +
                             red[(3 * 64 + r) * Rq + ep_c];
                const T yv = (T)v;
                Y[(long long)r * Rq + ep_c] = yv;
                a += (double)yv * (double)u2v[q];
            }
        }
        ep_part = a;
    }
    __syncthreads();
    double* kp = (double*)smraw;   // [RP][Rq]
    if (ep_on) kp[ep_j * Rq + ep_c] = ep_part;
    __syncthreads();
    if (threadIdx.x < Rq) {
        double a = 0.0;
        for (int j = 0; j < ep_rp; ++j) a += kp[j * Rq + threadIdx.x];
        gptr_w(st.K1p)[g->k1off[s] + ((long long)i1 * g->nrg[s] + rg) * Rq + threadIdx.x] = (T)a;
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
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    const ItemP2 it = items[blockIdx.x];
    const int s = it.s, chunk = it.chunk, q0 = it.q0;
    const int I1 = g->I[s][0], I2 = g->I[s][1], I3 = g->I[s][2], Rq = g->Rq;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i1 = chunk * 4 + wave;
    const int i3 = q0 + lane;
    const bool valid = i3 < I3;
    TA* sm = (TA*)smraw;
    constexpr int VA = 16 / (int)sizeof(TA);          // operand elements per 16-byte LDS read
    constexpr int RTP = (RT + VA - 1) / VA * VA;      // padded operand run per lane
    const CPD_GLOBAL T* __restrict__ U2g = gptr(pick3(st.U, slot) + g->uoff[1][s]);
    // U1 row of this slab (the scale of the mode-3 partial), loaded now
    TA u1v[RT];
    {
        const CPD_GLOBAL T* __restrict__ U1 =
            gptr(pick3(st.U, slot) + g->uoff[0][s] + (long long)min(i1, I1 - 1) * Rq + (lane & 3));
#pragma unroll
        for (int t = 0; t < RT; ++t) u1v[t] = (TA)U1[4 * t];
    }
    if (BLDS) {
        // U2 transposed so that lane l's operands U2[i2][4t + l%4], t < RT,
        // are one contiguous run: [I2][4][RTP]
        for (int e = threadIdx.x; e < I2 * Rq; e += 256) {
            const int i2 = e / Rq, c = e % Rq;
            sm[(i2 * 4 + (c & 3)) * RTP + (c >> 2)] = (TA)U2g[e];
        }
        __syncthreads();
    }
    Acc4<TA> z[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) z[t].zero();
    constexpr int NB = 16;
    if (i1 < I1) {
        typedef typename Raw<TM>::type TR;
        const long long ldm = g->mld[s];   // operand row stride (>= I3)
        const CPD_GLOBAL TR* __restrict__ Mp = gptr((const TR*)g->M[s] + (long long)i1 * I2 * ldm + (valid ? i3 : 0));
        TA cur[NB], nxt[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            // clamped (always valid) address, zero outside: no branch per load
            const TA v = cvt<TA, TM>(Mp[(long long)min(j, I2 - 1) * ldm]);
            cur[j] = (valid && j < I2) ? v : (TA)0;
        }
        for (int i2b = 0; i2b < I2; i2b += NB) {
            const int nb2 = i2b + NB;
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const TA v = cvt<TA, TM>(Mp[(long long)min(nb2 + j, I2 - 1) * ldm]);
                nxt[j] = (valid && nb2 + j < I2) ? v : (TA)0;
            }
            const int jm = min(NB, I2 - i2b);
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                if (j < jm) {
                    const int i2 = i2b + j;
                    TA bb[RTP];
                    if (BLDS) {
                        const TA* ur = sm + (i2 * 4 + (lane & 3)) * RTP;
#pragma unroll
                        for (int v = 0; v < RTP / VA; ++v) *(u32x4*)&bb[v * VA] = *(const u32x4*)(ur + v * VA);
                    } else {
#pragma unroll
                        for (int t = 0; t < RT; ++t) bb[t] = (TA)U2g[(long long)i2 * Rq + 4 * t + (lane & 3)];
                    }
#pragma unroll
                    for (int t = 0; t < RT; ++t) z[t].mma(cur[j], bb[t]);
                }
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) cur[j] = nxt[j];
        }
#pragma unroll
        for (int t = 0; t < RT; ++t) z[t].scale(u1v[t]);
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
