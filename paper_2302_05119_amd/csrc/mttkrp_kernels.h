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
typedef short v4i16 __attribute__((ext_vector_type(4)));   // four BF16 values (raw bits)
template <> struct Acc4<float> {
    v4f v;
    __device__ void zero() { v = (v4f){0.f, 0.f, 0.f, 0.f}; }
    __device__ void mma(float a, float b) { v = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, v, 0, 0, 0); }
    // v_mfma_f32_4x4x4_16b_bf16: block b of 16, lane 4b+i gives four k values
    // of A's row i and lane 4b+j four k values (same k order) of B's column j;
    // the result layout is that of the 4x4x1 form
    __device__ void mma_bf16(v4i16 a, v4i16 b) { v = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(a, b, v, 0, 0, 0); }
    __device__ float get(int i) const { return v[i]; }
    __device__ void scale(float u) { v *= u; }
    __device__ void set(const float (&x)[4]) { v = (v4f){x[0], x[1], x[2], x[3]}; }
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
    __device__ void set(const double (&x)[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = x[i];
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

// An FP32 factor value as the sum of two BF16 values, hi = bf16(u) and
// lo = bf16(u - hi) (round to nearest even), so that two BF16 matrix-core
// products carry it to about 2^-16 relative (the tensor operand is BF16
// storage already).
__device__ __forceinline__ void split_bf16(float u, unsigned short& hi, unsigned short& lo) {
    const __hip_bfloat16 h = __float2bfloat16(u);
    hi = __bfloat16_as_ushort(h);
    lo = __bfloat16_as_ushort(__float2bfloat16(u - __bfloat162float(h)));
}

// ---------------------------------------------------------------------------
// pass 1: one wavefront per (block, i1 slab, 64-row group of i2) item, or P
// wavefronts per item (P = 1, 2 or 4, one value per launch) that split the
// i3 range and add their partial accumulators in LDS in a fixed order.  A
// workgroup holds 4 / P items.  Lane l owns tensor row l of the row group
// (rows past the group repeat its last row; their outputs are never stored)
// and streams it in chunks of 64 bytes (raw storage bits, 16-byte loads when
// every row starts 16-byte aligned), the next chunk in flight while the
// current one is consumed.  The U3 rows of a chunk are staged in the
// wavefront's own LDS area, transposed so that lane l's B operands
// U3[k][4t + l%4], t < RT, are one contiguous run.  No workgroup barrier
// unless P > 1.
// ---------------------------------------------------------------------------
template <typename TA, int RT>
__device__ __forceinline__ void load_run(const TA* __restrict__ p, TA (&bb)[RT]) {
    // RT consecutive operands from LDS with the widest reads
    constexpr int VA = 16 / (int)sizeof(TA);
#pragma unroll
    for (int v = 0; v < RT / VA; ++v) {
        const u32x4 w = *(const u32x4*)(p + v * VA);
#pragma unroll
        for (int j = 0; j < VA; ++j) bb[v * VA + j] = ((const TA*)&w)[j];
    }
    constexpr int R0 = RT / VA * VA;
    if constexpr (RT - R0 >= 2 && sizeof(TA) == 4) {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        const u32x2 w = *(const u32x2*)(p + R0);
        bb[R0] = ((const TA*)&w)[0];
        bb[R0 + 1] = ((const TA*)&w)[1];
        if constexpr (RT - R0 == 3) bb[R0 + 2] = p[R0 + 2];
    } else if constexpr (RT - R0 == 1) {
        bb[R0] = p[R0];
    }
}

template <typename TM, typename T, int RT>
__device__ __forceinline__ void pass1_item(const Geo* __restrict__ g, StateP<T> st, const ItemP1* __restrict__ items,
                                               int nitems, int P, int slot, int bid) {
    typedef typename AccType<TM>::type TA;
    typedef typename Raw<TM>::type TR;
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    constexpr int KC = 64 / (int)sizeof(TR);          // chunk: 64 bytes of a row
    constexpr int NV = 4;                             // 16-byte words per chunk
    constexpr int VA = 16 / (int)sizeof(TA);
    constexpr int RTP = (RT + VA - 1) / VA * VA;      // padded operand run
    constexpr int UPL = (KC * 4 * RT + 63) / 64;      // U3 chunk elements per lane
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ii = bid * (4 / P) + wave / P, part = wave % P;
    const ItemP1 it = items[min(ii, nitems - 1)];
    const bool live = ii < nitems && it.s >= 0;
    const int s = live ? it.s : 0, i1 = it.i1, rg = it.rg, row0 = rg * 64;
    const int I2 = g->I[s][1], I3 = g->I[s][2], Rq = g->Rq;
    const int nrows = min(64, I2 - row0);
    const int myrow = min(lane, nrows - 1);
    // the U2 values of the lane's accumulator rows (mode-1 partial), early
    T u2v[RT][4];
    {
        const CPD_GLOBAL T* __restrict__ U2 = gptr(st.U[1] + g->uoff[1][s] + (long long)row0 * Rq);
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 4 * (lane >> 2) + v;
                const T u = U2[(long long)min(r, nrows - 1) * Rq + 4 * t + (lane & 3)];
                u2v[t][v] = (r < nrows) ? u : (T)0;
            }
    }
    const long long ldm = g->mld[s];   // operand row stride (>= I3)
    const CPD_GLOBAL TR* __restrict__ Mrow = gptr((const TR*)g->M[s] + ((long long)i1 * I2 + row0 + myrow) * ldm);
    const CPD_GLOBAL T* __restrict__ U3 = gptr(pick3(st.U, slot) + g->uoff[2][s]);
    TA* ustage = (TA*)smraw + wave * (KC * 4 * RTP);
    // this wavefront's share of i3, in whole chunks
    const int nck = (I3 + KC - 1) / KC, cpp = (nck + P - 1) / P;
    const int kb = live ? min(I3, part * cpp * KC) : 0, ke = live ? min(I3, kb + cpp * KC) : 0;
    const bool vec = g->mvec[s] != 0;
    Acc4<TA> acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t].zero();
    u32x4 cur[NV], nxt[NV];
    TA ub[UPL], nub[UPL];
    auto load_chunk = [&](int k0, u32x4 (&w)[NV], TA (&u)[UPL]) {
        const int kc = min(KC, ke - k0);
        if (vec && kc == KC) {
            const CPD_GLOBAL u32x4* vp = (const CPD_GLOBAL u32x4*)(Mrow + k0);
#pragma unroll
            for (int v = 0; v < NV; ++v) w[v] = vp[v];
        } else {
            TR e[KC];
#pragma unroll
            for (int j = 0; j < KC; ++j) {
                const TR x = Mrow[k0 + min(j, kc - 1)];
                e[j] = (j < kc) ? x : (TR)0;
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) w[v] = *(const u32x4*)&e[v * (KC / NV)];
        }
#pragma unroll
        for (int q = 0; q < UPL; ++q) {
            const int e = q * 64 + lane, kk = e / (4 * RT), c = e % (4 * RT);
            const TA x = (TA)U3[(long long)(k0 + min(kk, kc - 1)) * Rq + c];
            u[q] = (kk < kc) ? x : (TA)0;
        }
    };
    if (kb < ke) load_chunk(kb, cur, ub);
    for (int k0 = kb; k0 < ke; k0 += KC) {
#pragma unroll
        for (int q = 0; q < UPL; ++q) {
            const int e = q * 64 + lane, kk = e / (4 * RT), c = e % (4 * RT);
            if (e < KC * 4 * RT) ustage[(kk * 4 + (c & 3)) * RTP + (c >> 2)] = ub[q];
        }
        wave_sync();
        if (k0 + KC < ke) load_chunk(k0 + KC, nxt, nub);
        const TR* el = (const TR*)cur;
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            TA bb[RT];
            load_run<TA, RT>(ustage + (kk * 4 + (lane & 3)) * RTP, bb);
            const TA a = cvt<TA, TM>(el[kk]);
#pragma unroll
            for (int t = 0; t < RT; ++t) acc[t].mma(a, bb[t]);
        }
        wave_sync();
#pragma unroll
        for (int v = 0; v < NV; ++v) cur[v] = nxt[v];
#pragma unroll
        for (int q = 0; q < UPL; ++q) ub[q] = nub[q];
    }
    if (P > 1) {
        // partial accumulators of the P wavefronts of an item, added in part order
        TA* red = (TA*)smraw + 4 * (KC * 4 * RTP);   // [4 waves][RT][4][64]
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) red[((wave * RT + t) * 4 + v) * 64 + lane] = acc[t].get(v);
        __syncthreads();
        if (part == 0) {
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                TA x[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    x[v] = red[((wave * RT + t) * 4 + v) * 64 + lane];
                    for (int p = 1; p < P; ++p) x[v] += red[(((wave + p) * RT + t) * 4 + v) * 64 + lane];
                }
                acc[t].set(x);
            }
        }
    }
    if (!live || part != 0) return;
    // Y rows straight from the accumulators (lane: rows 4(l/4)+v, column
    // 4t + l%4), and the mode-1 partial sum_r Y[r][c] U2_old[row0 + r][c]:
    // the lane's four rows, then the sixteen lanes of the column in a fixed
    // butterfly order
    CPD_GLOBAL T* __restrict__ Y = gptr_w(st.Y + g->yoff[s] + ((long long)i1 * I2 + row0) * Rq);
    double kp[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        double a = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 4 * (lane >> 2) + v;
            const T yv = (T)acc[t].get(v);
            if (r < nrows) Y[(long long)r * Rq + 4 * t + (lane & 3)] = yv;
            a += (double)yv * (double)u2v[t][v];
        }
        kp[t] = a;
    }
#pragma unroll
    for (int o = 4; o < 64; o <<= 1)
#pragma unroll
        for (int t = 0; t < RT; ++t) kp[t] += __shfl_xor(kp[t], o, 64);
    if (lane < 4) {
        CPD_GLOBAL T* __restrict__ K1p = gptr_w(st.K1p) + g->k1off[s] + ((long long)i1 * g->nrg[s] + rg) * Rq;
#pragma unroll
        for (int t = 0; t < RT; ++t) K1p[4 * t + lane] = (T)kp[t];
    }
}

template <typename TM, typename T, int RT>
__global__ __launch_bounds__(256) void k_pass1(const Geo* __restrict__ g, StateP<T> st, const ItemP1* __restrict__ items, int nitems, int P, int slot) {
    if (st.ctrl->stop) return;
    apply_rot(st);
    pass1_item<TM, T, RT>(g, st, items, nitems, P, slot, blockIdx.x);
}

// ---------------------------------------------------------------------------
// pass 1 with the tensor streamed straight into LDS (same items, splits and
// outputs as k_pass1; every block's operand rows 16-byte aligned; FP32 or
// 16-bit storage).  A chunk is 16 values of i3 of every row of the item and
// the 16 matching rows of U3.  Both arrive by LDS DMA (global_load_lds: no
// registers), so each wavefront keeps two chunks in flight in a ring of
// three LDS stages: before consuming chunk c it waits for all but the group
// of chunk c+1, then requests chunk c+2 into the stage chunk c-1 used.
// Requests past the end repeat the last chunk (cache hits), which keeps the
// number of groups in flight, and so the wait count, fixed.
//
// Lane l streams tensor row l (16-byte pieces land in lane order); the lane
// class q = l % 4 owns output columns RT q .. RT q + RT - 1, so its B operands
// are one contiguous run of a raw U3 row.
// ---------------------------------------------------------------------------
// One 16-byte LDS DMA: lane l's 16 bytes at g land at LDS byte offset
// lds + 16 l.  The address register is an input only (no register is
// written), M0 holds the LDS offset.
__device__ __forceinline__ void lds_dma16(const void* g, unsigned lds) {
    // lds is the same in every lane of the wavefront
    asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off" ::"s"(__builtin_amdgcn_readfirstlane(lds)), "v"(g)
                 : "memory", "m0");
}
// s_waitcnt vmcnt(N) (N < 64), other counters untouched.
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x70 | 0xF00);
}

// RT consecutive FP32 words at p, where p is 4 RT q words past a 16-byte
// boundary: 16-byte reads when RT is a multiple of 4, 8-byte reads when even.
template <int RT>
__device__ __forceinline__ void load_cols(const float* __restrict__ p, float (&bb)[RT]) {
    if constexpr (RT % 4 == 0) {
#pragma unroll
        for (int v = 0; v < RT / 4; ++v) {
            const v4f w = *(const v4f*)(p + 4 * v);
#pragma unroll
            for (int j = 0; j < 4; ++j) bb[4 * v + j] = w[j];
        }
    } else if constexpr (RT % 2 == 0) {
        typedef float f2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int v = 0; v < RT / 2; ++v) {
            const f2 w = *(const f2*)(p + 2 * v);
            bb[2 * v] = w[0];
            bb[2 * v + 1] = w[1];
        }
    } else {
#pragma unroll
        for (int t = 0; t < RT; ++t) bb[t] = p[t];
    }
}

#ifndef CPD_P1D_NSTG
#define CPD_P1D_NSTG 3   // LDS stages per wavefront (NSTG - 1 chunks in flight)
#endif
template <typename TM, int RT>
struct P1D {
    typedef typename Raw<TM>::type TR;
    static constexpr int NSTG = CPD_P1D_NSTG;
    static constexpr int KC = 16;                                   // i3 values per chunk
    static constexpr int NA = KC * (int)sizeof(TR) / 16;            // tensor DMAs per chunk
    static constexpr int UBY = KC * 4 * RT * 4;                     // U3 bytes per chunk (FP32 factors)
    static constexpr int NUF = UBY / 1024;                          // full U3 DMAs
    static constexpr int NUL = (UBY % 1024) / 16;                   // lanes of the last, partial one
    static constexpr int NU = NUF + (NUL > 0 ? 1 : 0);              // U3 DMAs per chunk
    static constexpr int CBYTES = KC * (int)sizeof(TR);             // bytes of a row per chunk
    static constexpr int ABY = 64 * CBYTES;                         // tensor bytes per chunk
    static constexpr int STG = ABY + UBY;                           // one stage (16-byte multiple)
    static constexpr int RING = NSTG * STG;                         // one wavefront's ring
    static constexpr int WAVE = RING > RT * 1024 ? RING : RT * 1024; // its LDS (ring, or P > 1 partials)
    static constexpr int G = NA + NU;                               // DMAs per chunk
    static_assert(UBY % 16 == 0, "U3 chunk in 16-byte pieces");
};

template <typename TM, int RT>
__device__ __forceinline__ void pass1d_item(const Geo* __restrict__ g, StateP<float> st, const ItemP1* __restrict__ items,
                                                int nitems, int P, int slot, int bid) {
    typedef P1D<TM, RT> D;
    typedef typename D::TR TR;
    constexpr int KC = D::KC, EPP = 16 / (int)sizeof(TR);   // values per 16-byte piece
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63, q = lane & 3;
    const int ii = bid * (4 / P) + wave / P, part = wave % P;
    const ItemP1 it = items[min(ii, nitems - 1)];
    const bool live = ii < nitems && it.s >= 0;
    const int s = live ? it.s : 0, i1 = it.i1, rg = it.rg, row0 = rg * 64;
    const int I2 = g->I[s][1], I3 = g->I[s][2], Rq = g->Rq;
    const int nrows = min(64, I2 - row0);
    const int myrow = min(lane, nrows - 1);
    // U2 values of the lane's accumulator rows (mode-1 partial), early
    float u2v[RT][4];
    {
        const CPD_GLOBAL float* __restrict__ U2 = gptr(st.U[1] + g->uoff[1][s] + (long long)row0 * Rq);
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 4 * (lane >> 2) + v;
                const float u = U2[(long long)min(r, nrows - 1) * Rq + RT * q + t];
                u2v[t][v] = (r < nrows) ? u : 0.f;
            }
    }
    const long long ldm = g->mld[s];
    const TR* Mrow = (const TR*)g->M[s] + ((long long)i1 * I2 + row0 + myrow) * ldm;
    const float* U3 = pick3(st.U, slot) + g->uoff[2][s];
    const long long u3bytes = (long long)I3 * Rq * 4;
    const unsigned ring = (unsigned)(unsigned long long)(__attribute__((address_space(3))) char*)smraw + wave * D::WAVE;
    const char* ringp = smraw + wave * D::WAVE;
    // this wavefront's share of i3, in whole chunks
    const int nck = (I3 + KC - 1) / KC, cpp = (nck + P - 1) / P;
    const int cb = live ? min(nck, part * cpp) : 0, ce = live ? min(nck, cb + cpp) : 0;
    const int cl = max(ce - 1, cb);   // last chunk (requests past the end repeat it)
    // chunks before the last lie wholly inside the row and the factor: plain
    // offsets; the last one clamps every piece into its buffer
    const char* Mlane = (const char*)Mrow;
    const char* Ulane = (const char*)U3 + lane * 16;
    auto request = [&](int c, int stage) {
        const int cc = min(c, cl);
        const unsigned sb = ring + stage * D::STG;
        if (cc < cl) {
            const char* mp = Mlane + (long long)cc * D::CBYTES;
            const char* up = Ulane + (long long)cc * D::UBY;
#pragma unroll
            for (int j = 0; j < D::NA; ++j) lds_dma16(mp + 16 * j, sb + j * 1024);
#pragma unroll
            for (int u = 0; u < D::NU; ++u)
                if (u < D::NUF || lane < D::NUL) lds_dma16(up + 1024 * u, sb + D::ABY + u * 1024);
        } else {
            // a tensor piece past the row end is moved back inside it (its
            // values meet zero rows of U3); U3 bytes past the factor repeat
            // its last 16 bytes (those rows are zeroed before use)
#pragma unroll
            for (int j = 0; j < D::NA; ++j) {
                const long long e = min((long long)cc * KC + j * EPP, ldm - EPP);
                lds_dma16(Mrow + e, sb + j * 1024);
            }
#pragma unroll
            for (int u = 0; u < D::NU; ++u) {
                const long long b = min((long long)cc * D::UBY + u * 1024 + lane * 16, u3bytes - 16);
                if (u < D::NUF || lane < D::NUL) lds_dma16((const char*)U3 + b, sb + D::ABY + u * 1024);
            }
        }
    };
    Acc4<float> acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t].zero();
    if (cb < ce) {
#pragma unroll
        for (int j = 0; j < D::NSTG - 1; ++j) request(cb + j, j);
        int stage = 0;
        for (int c = cb; c < ce; ++c) {
            wait_vm<(D::NSTG - 2) * D::G>();   // chunk c has landed; the next NSTG-2 may be in flight
            const char* sp = ringp + stage * D::STG;
            const float* ur = (const float*)(sp + D::ABY);
            const int kc = min(KC, I3 - c * KC);
            if (kc < KC) {
                // U3 rows past the factor's end read clamped data: zero them
                for (int e = lane; e < (KC - kc) * Rq; e += 64) ((float*)ur)[kc * Rq + e] = 0.f;
            }
            wave_sync();
            request(c + D::NSTG - 1, stage == 0 ? D::NSTG - 1 : stage - 1);
            if constexpr (std::is_same<TM, __hip_bfloat16>::value) {
                // BF16 matrix cores: the stage's U3 rows become hi and lo BF16
                // operands in place, [group of 4 k][lane class j][tile t][4 k]
                // each (a lane's RT operands of a group are one run); the
                // tensor's 16-byte pieces give two 4-k groups of a row per lane
                constexpr int RQ = 4 * RT, NPAIR = (KC / 4) * RQ, NPL = (NPAIR + 63) / 64;
                float uv[NPL][4];
#pragma unroll
                for (int r = 0; r < NPL; ++r) {
                    const int p = min(lane + 64 * r, NPAIR - 1), gk = p / RQ, col = p % RQ;
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) uv[r][kk] = ur[(4 * gk + kk) * RQ + col];
                }
                wave_sync();
                unsigned short* hb = (unsigned short*)ur;
                unsigned short* lb = hb + (KC / 4) * 4 * RT * 4;
#pragma unroll
                for (int r = 0; r < NPL; ++r) {
                    const int p = lane + 64 * r;
                    if (p < NPAIR) {
                        const int gk = p / RQ, col = p % RQ, jc = col / RT, t = col % RT;
                        const int o = ((gk * 4 + jc) * RT + t) * 4;
#pragma unroll
                        for (int kk = 0; kk < 4; ++kk) split_bf16(uv[r][kk], hb[o + kk], lb[o + kk]);
                    }
                }
                wave_sync();
#pragma unroll
                for (int pc = 0; pc < KC / EPP; ++pc) {
                    const u32x4 w = *(const u32x4*)(sp + pc * 1024 + lane * 16);
#pragma unroll
                    for (int h2 = 0; h2 < EPP / 4; ++h2) {
                        const int gk = pc * (EPP / 4) + h2;
                        v4i16 a;
                        *(unsigned long long*)&a = ((unsigned long long)w[2 * h2 + 1] << 32) | w[2 * h2];
                        const v4i16* bh = (const v4i16*)(hb + (gk * 4 + q) * RT * 4);
                        const v4i16* bl = (const v4i16*)(lb + (gk * 4 + q) * RT * 4);
#pragma unroll
                        for (int t = 0; t < RT; ++t) {
                            acc[t].mma_bf16(a, bh[t]);
                            acc[t].mma_bf16(a, bl[t]);
                        }
                    }
                }
            } else {
#pragma unroll
            for (int pc = 0; pc < KC / EPP; ++pc) {
                const u32x4 w = *(const u32x4*)(sp + pc * 1024 + lane * 16);
                const TR* ev = (const TR*)&w;
#pragma unroll
                for (int x = 0; x < EPP; ++x) {
                    const int kk = pc * EPP + x;
                    const float a = cvt<float, TM>(ev[x]);
                    float bb[RT];
                    load_cols<RT>(ur + kk * Rq + RT * q, bb);
#pragma unroll
                    for (int t = 0; t < RT; ++t) acc[t].mma(a, bb[t]);
                }
            }
            }
            // (the wait before the next request also retires this chunk's
            // LDS reads before its stage is overwritten)
            stage = (stage == D::NSTG - 1) ? 0 : stage + 1;
        }
    }
    wait_vm<0>();   // no DMA may still be writing this wavefront's LDS when it leaves
    if (P > 1) {
        // partial accumulators of the P wavefronts of an item, each in its own
        // (drained) ring as [RT][4][64], added in part order
        static_assert(RT * 4 * 64 * 4 <= D::WAVE, "partials fit the wavefront's area");
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) ((float*)ringp)[(t * 4 + v) * 64 + lane] = acc[t].get(v);
        __syncthreads();
        if (part == 0) {
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                float x[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    x[v] = ((const float*)ringp)[(t * 4 + v) * 64 + lane];
                    for (int p = 1; p < P; ++p) x[v] += ((const float*)(ringp + p * D::WAVE))[(t * 4 + v) * 64 + lane];
                }
                acc[t].set(x);
            }
        }
    }
    if (!live || part != 0) return;
    CPD_GLOBAL float* __restrict__ Y = gptr_w(st.Y + g->yoff[s] + ((long long)i1 * I2 + row0) * Rq);
    double kp[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        double a = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 4 * (lane >> 2) + v;
            const float yv = acc[t].get(v);
            if (r < nrows) Y[(long long)r * Rq + RT * q + t] = yv;
            a += (double)yv * (double)u2v[t][v];
        }
        kp[t] = a;
    }
#pragma unroll
    for (int o = 4; o < 64; o <<= 1)
#pragma unroll
        for (int t = 0; t < RT; ++t) kp[t] += __shfl_xor(kp[t], o, 64);
    if (lane < 4) {
        CPD_GLOBAL float* __restrict__ K1p = gptr_w(st.K1p) + g->k1off[s] + ((long long)i1 * g->nrg[s] + rg) * Rq;
#pragma unroll
        for (int t = 0; t < RT; ++t) K1p[RT * lane + t] = (float)kp[t];
    }
}

template <typename TM, int RT>
__global__ __launch_bounds__(256) void k_pass1d(const Geo* __restrict__ g, StateP<float> st, const ItemP1* __restrict__ items, int nitems, int P, int slot) {
    if (st.ctrl->stop) return;
    apply_rot(st);
    pass1d_item<TM, RT>(g, st, items, nitems, P, slot, blockIdx.x);
}

// ---------------------------------------------------------------------------
// pass 2: one workgroup per (block, chunk of 4 i1 slabs, 64 consecutive i3);
// wavefront w takes slab 4*chunk + w.  Lanes run along i3 (the contiguous
// index), so every tensor load is a coalesced 64-element row segment; NB rows
// are loaded ahead of the matrix-core work.  U2 is staged in LDS, whole when it
// fits (BLDS), else in chunks of P2CHR rows shared by the four wavefronts.
// ---------------------------------------------------------------------------
// rows of U2 per staged chunk: a multiple of 16 within 32 KiB of LDS
// (transposed rows of 4 x RTP operands)
template <typename TA, int RT>
constexpr int p2_chunk_rows() {
    constexpr int VA = 16 / (int)sizeof(TA);
    constexpr int RTP = (RT + VA - 1) / VA * VA;
    return (32768 / (4 * RTP * (int)sizeof(TA))) / 16 * 16;
}

template <typename TM, typename T, int RT, bool BLDS, int SPW = 1>
__device__ __forceinline__ void pass2_item(const Geo* __restrict__ g, StateP<T> st, const ItemP2* __restrict__ items,
                                               int slot, int bid) {
    typedef typename AccType<TM>::type TA;
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    const ItemP2 it = items[bid];
    const int s = it.s, chunk = it.chunk, q0 = it.q0;
    const int I1 = g->I[s][0], I2 = g->I[s][1], I3 = g->I[s][2], Rq = g->Rq;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i3 = q0 + lane;
    const bool valid = i3 < I3;
    TA* sm = (TA*)smraw;
    constexpr int VA = 16 / (int)sizeof(TA);          // operand elements per 16-byte LDS read
    constexpr int RTP = (RT + VA - 1) / VA * VA;      // padded operand run per lane
    const CPD_GLOBAL T* __restrict__ U2g = gptr(pick3(st.U, slot) + g->uoff[1][s]);
    typedef typename Raw<TM>::type TR;
    const long long ldm = g->mld[s];   // operand row stride (>= I3)
    // a chunk is 4 SPW slabs of i1 (SPW is the context's p2spw); wavefront w
    // takes slabs 4 (SPW chunk + k) + w, k < SPW, one after another, and adds
    // their scaled partials in k order (U2 is staged once when it fits LDS
    // whole)
    constexpr int spw = SPW;
    Acc4<TA> z[RT];
    TA zt[RT][4];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) zt[t][v] = (TA)0;
    for (int k = 0; k < spw; ++k) {
        const int i1 = (chunk * spw + k) * 4 + wave;
        const bool restage = !BLDS || k == 0;
        // U1 row of this slab (the scale of the mode-3 partial), loaded now
        TA u1v[RT];
        {
            const CPD_GLOBAL T* __restrict__ U1 =
                gptr(pick3(st.U, slot) + g->uoff[0][s] + (long long)min(i1, I1 - 1) * Rq + (lane & 3));
#pragma unroll
            for (int t = 0; t < RT; ++t) u1v[t] = (TA)U1[4 * t];
        }
#pragma unroll
        for (int t = 0; t < RT; ++t) z[t].zero();
        constexpr int NB = 16;
        // the first NB rows of the slab are requested before the U2 staging, so
        // their latency overlaps it (clamped, always valid addresses; zeros
        // outside the slab)
        const bool live = i1 < I1;
        const CPD_GLOBAL TR* __restrict__ Mp =
            gptr((const TR*)g->M[s] + (long long)min(i1, I1 - 1) * I2 * ldm + (valid ? i3 : 0));
        TA cur[NB], nxt[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const TA v = cvt<TA, TM>(Mp[(long long)min(j, I2 - 1) * ldm]);
            cur[j] = (live && valid && j < I2) ? v : (TA)0;
        }
        // U2 rows [c0, c1) transposed into LDS so that lane l's operands
        // U2[i2][4t + l%4], t < RT, are one contiguous run: [rows][4][RTP]
        // (eight loads per thread in flight per step, clamped addresses)
        auto stage_u2 = [&](int c0, int c1) {
            const int nu = (c1 - c0) * Rq;
            const CPD_GLOBAL T* __restrict__ src = U2g + (long long)c0 * Rq;
            for (int e0 = threadIdx.x; e0 < nu; e0 += 256 * 8) {
                T v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = src[min(e0 + 256 * j, nu - 1)];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int e = e0 + 256 * j;
                    if (e < nu) {
                        const int r = e / Rq, c = e % Rq;
                        sm[(r * 4 + (c & 3)) * RTP + (c >> 2)] = (TA)v[j];
                    }
                }
            }
        };
        constexpr int CHR = BLDS ? (1 << 30) : p2_chunk_rows<TA, RT>();
        static_assert(CHR % NB == 0, "U2 chunks must hold whole NB-row groups");
        if constexpr (std::is_same<TM, __hip_bfloat16>::value) {
            // BF16 matrix cores: four consecutive i2 rows of a lane's tensor column
            // form the A operand of v_mfma_f32_4x4x4_16b_bf16; U2 is staged as hi
            // and lo BF16 parts, [group of 4 rows][lane class j][tile t][4 rows]
            // (column 4t + j), rows past I2 zero.  Tensor loads are never masked
            // (clamped addresses, finite values): a row past I2 meets zero U2
            // operands, and a lane past I3 only feeds its own output row, which is
            // never stored
            unsigned short cb[NB], nb[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) cb[j] = Mp[(long long)min(j, I2 - 1) * ldm];
            unsigned short* hb = (unsigned short*)smraw;
            for (int c0 = 0; c0 < I2; c0 += CHR) {
                const int c1 = min(I2, c0 + CHR), nr = c1 - c0, nr4 = (nr + 3) & ~3;
                unsigned short* lb = hb + nr4 * Rq;
                if (restage) {
                    __syncthreads();
                    const int nu = nr4 * Rq;
                    const CPD_GLOBAL T* __restrict__ src = U2g + (long long)c0 * Rq;
                    for (int e0 = threadIdx.x; e0 < nu; e0 += 256 * 8) {
                        T v[8];
#pragma unroll
                        for (int j = 0; j < 8; ++j) v[j] = src[min(e0 + 256 * j, nr * Rq - 1)];
#pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            const int e = e0 + 256 * j;
                            if (e < nu) {
                                const int r = e / Rq, c = e % Rq;
                                const int o = (((r >> 2) * 4 + (c & 3)) * RT + (c >> 2)) * 4 + (r & 3);
                                unsigned short h = 0, l = 0;
                                if (r < nr) split_bf16((float)v[j], h, l);
                                hb[o] = h;
                                lb[o] = l;
                            }
                        }
                    }
                    __syncthreads();
                }
                if (live) {
                    for (int i2b = c0; i2b < c1; i2b += NB) {
                        const int nb2 = i2b + NB;
#pragma unroll
                        for (int j = 0; j < NB; ++j) nb[j] = Mp[(long long)min(nb2 + j, I2 - 1) * ldm];
                        const int jm = min(NB, I2 - i2b);
#pragma unroll
                        for (int gg = 0; gg < NB / 4; ++gg) {
                            if (4 * gg < jm) {
                                v4i16 a;
                                *(unsigned long long*)&a = (unsigned long long)cb[4 * gg] | ((unsigned long long)cb[4 * gg + 1] << 16) |
                                                           ((unsigned long long)cb[4 * gg + 2] << 32) |
                                                           ((unsigned long long)cb[4 * gg + 3] << 48);
                                const int gk = (i2b - c0) / 4 + gg;
                                const v4i16* bh = (const v4i16*)(hb + (gk * 4 + (lane & 3)) * RT * 4);
                                const v4i16* bl = (const v4i16*)(lb + (gk * 4 + (lane & 3)) * RT * 4);
#pragma unroll
                                for (int t = 0; t < RT; ++t) {
                                    z[t].mma_bf16(a, bh[t]);
                                    z[t].mma_bf16(a, bl[t]);
                                }
                            }
                        }
#pragma unroll
                        for (int j = 0; j < NB; ++j) cb[j] = nb[j];
                    }
                }
            }
        } else
        for (int c0 = 0; c0 < I2; c0 += CHR) {
            const int c1 = min(I2, c0 + CHR);
            // every wavefront of the workgroup stages and waits (also those past I1)
            if (restage) {
                __syncthreads();
                stage_u2(c0, c1);
                __syncthreads();
            }
            if (live) {
                for (int i2b = c0; i2b < c1; i2b += NB) {
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
                            const TA* ur = sm + ((i2b - c0 + j) * 4 + (lane & 3)) * RTP;
                            TA bb[RTP];
#pragma unroll
                            for (int v = 0; v < RTP / VA; ++v) *(u32x4*)&bb[v * VA] = *(const u32x4*)(ur + v * VA);
#pragma unroll
                            for (int t = 0; t < RT; ++t) z[t].mma(cur[j], bb[t]);
                        }
                    }
#pragma unroll
                    for (int j = 0; j < NB; ++j) cur[j] = nxt[j];
                }
            }
        }
        if (live) {
#pragma unroll
            for (int t = 0; t < RT; ++t) z[t].scale(u1v[t]);
        }
        if constexpr (SPW > 1) {
#pragma unroll
            for (int t = 0; t < RT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) zt[t][v] += z[t].get(v);
        }
    }
    __syncthreads();
    TA* red = sm;  // [4 waves][64][Rq]
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            red[(wave * 64 + 4 * (lane >> 2) + v) * Rq + 4 * t + (lane & 3)] = SPW > 1 ? zt[t][v] : z[t].get(v);
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

template <typename TM, typename T, int RT, bool BLDS, int SPW>
__global__ __launch_bounds__(256) void k_pass2(const Geo* __restrict__ g, StateP<T> st, const ItemP2* __restrict__ items, int slot) {
    if (st.ctrl->stop) return;
    apply_rot(st);
    pass2_item<TM, T, RT, BLDS, SPW>(g, st, items, slot, blockIdx.x);
}

// ---------------------------------------------------------------------------
// mode 2: K2[i2][r] = sum_i1 Y[i1][i2][r] U1[i1][r] with the new U^(1).  One
// thread per element e = i2*Rq + r of a 256-wide column tile, one workgroup
// per (block, tile, chunk of k2rows rows of i1); every Y load is a
// coalesced row segment.  Chunk partials are summed in fixed order by the
// factor update.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void k2_item(const Geo* __restrict__ g, StateP<T> st, const ItemK2* __restrict__ items, int slot, int bid) {
    const ItemK2 it = items[bid];
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

template <typename T>
__global__ __launch_bounds__(256) void k_k2(const Geo* __restrict__ g, StateP<T> st, const ItemK2* __restrict__ items, int slot) {
    if (st.ctrl->stop) return;
    apply_rot(st);
    k2_item<T>(g, st, items, slot, blockIdx.x);
}

// pass 1 LDS: four staging areas (64-byte chunk x 4 x RTP operands), then,
// when P > 1, the partial accumulators of the four wavefronts (RT x 4 x 64)
template <typename TM>
inline size_t pass1_lds(int RT, int P) {
    typedef typename AccType<TM>::type TA;
    const size_t kc = 64 / sizeof(typename Raw<TM>::type), va = 16 / sizeof(TA), rtp = ((size_t)RT + va - 1) / va * va;
    return sizeof(TA) * (4 * kc * 4 * rtp + (P > 1 ? 4 * (size_t)RT * 4 * 64 : 0));
}

// pass 2 LDS: U2 staged whole when it fits 48 KiB (*whole = true), else in
// chunks of whole 16-row groups within 32 KiB (as p2_chunk_rows); at least
// the partial sums of the four wavefronts
template <typename TM>
inline size_t pass2_lds(int Rq, int maxI2, bool* whole) {
    typedef typename AccType<TM>::type TA;
    const size_t va = 16 / sizeof(TA), rtp = ((size_t)Rq / 4 + va - 1) / va * va;
    const size_t red = sizeof(TA) * 4 * 64 * (size_t)Rq;
    const size_t bst = sizeof(TA) * (size_t)maxI2 * 4 * rtp;   // transposed U2
    const size_t chr = (32768 / (4 * rtp * sizeof(TA))) / 16 * 16;
    const size_t cst = sizeof(TA) * chr * 4 * rtp;
    *whole = bst <= 49152;
    size_t st = *whole ? bst : cst;
    if (std::is_same<TM, __hip_bfloat16>::value && *whole) {
        // hi and lo BF16 parts of the whole U2, rows rounded up to 4
        const size_t hl = 4 * (size_t)Rq * (((size_t)maxI2 + 3) & ~(size_t)3);
        st = st > hl ? st : hl;
    }
    return st > red ? st : red;
}

}  // namespace cpd
