// MTTKRP of an order-N block (N > 3; the data term M_(n) U^{⊙-n} of
// eq. solapgU for the N-way model of Section II-C) by a two-level dimension
// tree, so that M is streamed twice per sweep whatever N is.
//
// M^(s) (C order, last mode fastest) is an A x B matrix: rows a are the
// multi-indices of modes 0..h-1, columns b those of modes h..N-1.  Under the
// Gauss-Seidel order of Algorithm 1:
//
//   pass A:  T_A[a][r] = sum_b M[a][b] KR_B[b][r],  KR_B = Khatri-Rao of the
//            x_{k-1} factors of modes h..N-1 (none of them is updated before
//            the modes 0..h-1 are)
//   mode n < h:   K_n[i][r] = sum_{a : a_n = i} T_A[a][r] prod_{m < h, m != n} U^(m)[a_m][r]
//   pass B:  T_B[b][r] = sum_a M[a][b] KR_A[a][r],  KR_A from the new factors
//            of modes 0..h-1
//   mode n >= h:  K_n[i][r] = sum_{b : b_n = i} T_B[b][r] prod_{m >= h, m != n} U^(m)[b_m][r]
//
// with U^(m) new for m < n and from x_{k-1} for m > n.  The passes split the
// contraction into parts (partial outputs, summed in part order by the mode
// contraction in FP64) so that a launch has enough wavefronts.
//
// Passes run on the matrix cores in the layout of the order-3 pass 1
// (v_mfma_f32_4x4x1f32; FP64 by lane shuffles): lane l of a wavefront owns
// output row o0 + l and feeds the element of that row at the current k; the
// Khatri-Rao rows of a 16-deep chunk are staged in LDS so that lane class
// l % 4 reads its columns 4t + l % 4 as one contiguous run.
#include "mttkrp_kernels.h"
#include "small_dev.h"

namespace cpd {

// Khatri-Rao operand of one half: rows o (multi-index over the half's modes,
// last fastest), columns r < Rq; product of FP64 factor values, rounded once.
// (st remapped; workgroup wg of nwg covers entries wg*256 + t, step nwg*256)
template <typename T>
__device__ __forceinline__ void nw_kr_part(const Geo* __restrict__ g, const StateP<T>& st, int half, int slot, int s, int wg,
                                           int nwg) {
    const int N = g->N, h = g->nh, Rq = g->Rq;
    // half 0: the operand of pass A (modes h..N-1), half 1: of pass B (modes 0..h-1)
    const int m0 = half ? 0 : h, m1 = half ? h : N;
    const long long rows = half ? g->nwA[s] : g->nwB[s];
    const T* U = pick3(st.U, slot);
    T* out = st.part + g->kroff[s];
    for (long long e = wg * 256LL + threadIdx.x; e < rows * Rq; e += (long long)nwg * 256) {
        const int r = (int)(e % Rq);
        long long x = e / Rq;
        double p = 1.0;
        for (int m = m1 - 1; m >= m0; --m) {
            const int Im = g->I[s][m];
            const long long i = x % Im;
            x /= Im;
            p *= (double)U[g->uoff[m][s] + i * Rq + r];
        }
        out[e] = (T)p;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_nw_kr(const Geo* __restrict__ g, StateP<T> st, int half, int slot, int check_stop) {
    if (check_stop && st.ctrl->stop) return;
    apply_rot(st);
    nw_kr_part<T>(g, st, half, slot, blockIdx.y, blockIdx.x, gridDim.x);
}

// One pass (HALF 0: A, HALF 1: B); one wavefront per item (64 outputs of one
// block, one part of the contraction), four items per workgroup.
template <typename T, int RT, int HALF>
__global__ __launch_bounds__(256) void k_nw_pass(const Geo* __restrict__ g, StateP<T> st, const ItemNW* __restrict__ items,
                                                 int nitems, int check_stop) {
    if (check_stop && st.ctrl->stop) return;
    constexpr int KC = 16;                          // contraction chunk
    constexpr int VA = 16 / (int)sizeof(T);
    constexpr int RTP = (RT + VA - 1) / VA * VA;    // padded operand run
    constexpr int UPL = (KC * 4 * RT + 63) / 64;    // operand chunk elements per lane
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ii = blockIdx.x * 4 + wave;
    if (ii >= nitems) return;   // no workgroup barrier below: waves leave independently
    const ItemNW it = items[ii];
    if (it.s < 0) return;
    const int s = it.s, Rq = g->Rq;
    const long long A = g->nwA[s], B = g->nwB[s];
    const long long O = HALF ? B : A, K = HALF ? A : B;
    const long long kper = HALF ? g->kpb[s] : g->kpa[s];
    const long long kb = (long long)it.part * kper, ke = min(K, kb + kper);
    const long long o0 = (long long)it.og * 64;
    const int no = (int)min(64LL, O - o0);
    const long long myo = o0 + min(lane, no - 1);
    const CPD_GLOBAL T* __restrict__ M = gptr((const T*)g->M[s]);
    const CPD_GLOBAL T* __restrict__ KR = gptr(st.part + g->kroff[s]);
    const bool vec = HALF == 0 && g->mvec[s] != 0;
    T* ustage = (T*)smraw + wave * (KC * 4 * RTP);
    Acc4<T> acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t].zero();
    T el[KC], nel[KC], ub[UPL], nub[UPL];
    auto load_chunk = [&](long long k0, T (&e)[KC], T (&u)[UPL]) {
        const int kc = (int)min((long long)KC, ke - k0);
        if (HALF == 0) {
            // 16 consecutive elements of the lane's row
            const CPD_GLOBAL T* row = M + myo * B + k0;
            if (vec && kc == KC) {
                constexpr int NV = KC * (int)sizeof(T) / 16;
                u32x4 w[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) w[v] = ((const CPD_GLOBAL u32x4*)row)[v];
#pragma unroll
                for (int j = 0; j < KC; ++j) e[j] = ((const T*)w)[j];
            } else {
#pragma unroll
                for (int j = 0; j < KC; ++j) {
                    const T x = row[min(j, kc - 1)];
                    e[j] = (j < kc) ? x : (T)0;
                }
            }
        } else {
            // the lane's column in 16 consecutive rows (coalesced across lanes)
#pragma unroll
            for (int j = 0; j < KC; ++j) {
                const T x = M[(k0 + min(j, kc - 1)) * B + myo];
                e[j] = (j < kc) ? x : (T)0;
            }
        }
#pragma unroll
        for (int q = 0; q < UPL; ++q) {
            const int ee = q * 64 + lane, kk = ee / (4 * RT), c = ee % (4 * RT);
            const T x = KR[(k0 + min(kk, kc - 1)) * Rq + c];
            u[q] = (kk < kc) ? x : (T)0;
        }
    };
    if (kb < ke) load_chunk(kb, el, ub);
    for (long long k0 = kb; k0 < ke; k0 += KC) {
#pragma unroll
        for (int q = 0; q < UPL; ++q) {
            const int ee = q * 64 + lane, kk = ee / (4 * RT), c = ee % (4 * RT);
            if (ee < KC * 4 * RT) ustage[(kk * 4 + (c & 3)) * RTP + (c >> 2)] = ub[q];
        }
        wave_sync();
        if (k0 + KC < ke) load_chunk(k0 + KC, nel, nub);
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            T bb[RT];
            load_run<T, RT>(ustage + (kk * 4 + (lane & 3)) * RTP, bb);
#pragma unroll
            for (int t = 0; t < RT; ++t) acc[t].mma(el[kk], bb[t]);
        }
        wave_sync();
#pragma unroll
        for (int j = 0; j < KC; ++j) el[j] = nel[j];
#pragma unroll
        for (int q = 0; q < UPL; ++q) ub[q] = nub[q];
    }
    // accumulator: rows o0 + 4 (l / 4) + v, column 4t + l % 4
    T* out = st.Y + (HALF ? g->tboff[s] + (long long)it.part * B * Rq : g->taoff[s] + (long long)it.part * A * Rq);
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const long long o = o0 + 4 * (lane >> 2) + v;
            if (o < O) out[o * Rq + 4 * t + (lane & 3)] = acc[t].get(v);
        }
}

// K_n of every block from the partials of its half, one workgroup per (i, block):
// thread (j, r) takes the terms q = j, j + J, ... of column r (J = 256 / Rq
// stripes; each term sums the parts in part order and multiplies by the other
// factors of the half), then thread r adds the J stripe sums in stripe order;
// FP64 throughout, rounded once into the plain K buffer.
template <typename T>
__device__ __forceinline__ void nw_contract_row(const Geo* __restrict__ g, const StateP<T>& st, int n, int lo_slot, int s, int i) {
    const int In = g->I[s][n];
    if (i >= In) return;   // uniform over the workgroup
    const int N = g->N, h = g->nh, Rq = g->Rq, R = g->R, tid = threadIdx.x;
    const int J = 256 / Rq, r = tid % Rq, j = tid / Rq;
    const int half = n >= h;
    const int m0 = half ? h : 0, m1 = half ? N : h;
    const long long O = half ? g->nwB[s] : g->nwA[s];
    const int np = half ? g->npb[s] : g->npa[s];
    const T* part = st.Y + (half ? g->tboff[s] : g->taoff[s]) + r;
    const T* Ulo = pick3(st.U, lo_slot);
    const T* Uhi = st.U[1];
    const long long cnt = O / In, pst = O * Rq;
    __shared__ double red[256];
    double acc = 0.0;
    if (j < J && r < R) {
        for (long long q = j; q < cnt; q += J) {
            // q runs over the half's other modes (row-major); mode n is pinned to i
            long long x = q, o = 0, mult = 1;
            double w = 1.0;
            for (int m = m1 - 1; m >= m0; --m) {
                const int Im = g->I[s][m];
                long long im;
                if (m == n) {
                    im = i;
                } else {
                    im = x % Im;
                    x /= Im;
                    w *= (double)(m < n ? Ulo : Uhi)[g->uoff[m][s] + im * Rq + r];
                }
                o += im * mult;
                mult *= Im;
            }
            const T* pp = part + o * Rq;
            double tv = 0.0;
#pragma unroll 4
            for (int p = 0; p < np; ++p) tv += (double)pp[p * pst];
            acc = fma(tv, w, acc);
        }
    }
    red[tid] = acc;
    __syncthreads();
    if (tid < Rq) {
        double sum = 0.0;
        for (int jj = 0; jj < J; ++jj) sum += red[jj * Rq + tid];
        st.K3[g->koff[s] + (long long)i * Rq + tid] = (T)(tid < R ? sum : 0.0);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_nw_contract(const Geo* __restrict__ g, StateP<T> st, int n, int lo_slot,
                                                     int check_stop) {
    if (check_stop && st.ctrl->stop) return;
    apply_rot(st);
    nw_contract_row<T>(g, st, n, lo_slot, blockIdx.y, blockIdx.x);
}

// The sweep's R x R work beside order-N work it does not depend on (the
// first nsmall workgroups, S rounded up to a multiple of 8, take one block
// each; the rest the other kernel's work): the core update beside the
// Khatri-Rao operand of pass A (x_{k-1} factors), the step matrix of mode n
// beside the contraction of mode n (both read the factors updated so far).
template <int NM> struct NwFuseWaves { static constexpr int W = NM <= 32 ? 2 : 1; };

template <typename T, int NM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NwFuseWaves<NM>::W))) void k_nw_core_kr(
    const Geo* __restrict__ g, StateP<T> st, int extrapolate, int S, int nsmall, int krw) {
    if (st.ctrl->stop) return;
    apply_rot(st);
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    const int bid = blockIdx.x;
    if (bid < nsmall) {
        if (bid < S) core_block<T, NM>(g, st, bid, extrapolating(st.ctrl, extrapolate), smraw);
        return;
    }
    const int b = bid - nsmall;
    nw_kr_part<T>(g, st, 0, 1, b / krw, b % krw, krw);
}

template <typename T, int NM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NwFuseWaves<NM>::W))) void k_nw_prep_contract(
    const Geo* __restrict__ g, StateP<T> st, int n, int S, int nsmall, int maxI) {
    if (st.ctrl->stop) return;
    apply_rot(st);
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    const int bid = blockIdx.x;
    if (bid < nsmall) {
        if (bid < S) prep_block<T, NM>(g, st, bid, n, smraw);
        return;
    }
    const int b = bid - nsmall;
    nw_contract_row<T>(g, st, n, 0, b / maxI, b % maxI);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static unsigned grid_x(long long work) {
    long long nb = (work + 255) / 256;
    if (nb > 4096) nb = 4096;
    return (unsigned)(nb < 1 ? 1 : nb);
}

template <typename T>
void launch_nw_kr(const Geo* g, const StateP<T>& st, int S, int half, int slot, long long maxrows, int Rq, int check_stop,
                  hipStream_t q) {
    hipLaunchKernelGGL(k_nw_kr<T>, dim3(grid_x(maxrows * Rq), S), dim3(256), 0, q, g, st, half, slot, check_stop);
}

template <typename T>
void launch_nw_pass(const Geo* g, const StateP<T>& st, const ItemNW* items, int nitems, int half, int Rq, int check_stop,
                    hipStream_t q) {
    if (nitems <= 0) return;
    const int RT = Rq / 4;
    constexpr int VA = 16 / (int)sizeof(T);
    const int RTP = (RT + VA - 1) / VA * VA;
    const size_t lds = sizeof(T) * 4 * 16 * 4 * (size_t)RTP;
    const dim3 grid((nitems + 3) / 4);
#define CPD_NWP(RTV)                                                                                                   \
    case RTV:                                                                                                          \
        if (half) hipLaunchKernelGGL((k_nw_pass<T, RTV, 1>), grid, dim3(256), lds, q, g, st, items, nitems, check_stop); \
        else hipLaunchKernelGGL((k_nw_pass<T, RTV, 0>), grid, dim3(256), lds, q, g, st, items, nitems, check_stop);      \
        break;
    switch (RT) {
        CPD_NWP(1) CPD_NWP(2) CPD_NWP(3) CPD_NWP(4) CPD_NWP(5) CPD_NWP(6) CPD_NWP(7) CPD_NWP(8)
        CPD_NWP(9) CPD_NWP(10) CPD_NWP(11) CPD_NWP(12) CPD_NWP(13) CPD_NWP(14) CPD_NWP(15) CPD_NWP(16)
        default: break;
    }
#undef CPD_NWP
}

template <typename T>
void launch_nw_contract(const Geo* g, const StateP<T>& st, int S, int n, int lo_slot, int maxI, int Rq, int check_stop,
                        hipStream_t q) {
    (void)Rq;
    hipLaunchKernelGGL(k_nw_contract<T>, dim3(maxI, S), dim3(256), 0, q, g, st, n, lo_slot, check_stop);
}

static int nw_small_wgs(int S) { return (S + 7) & ~7; }

template <typename T>
void launch_nw_core_kr(const Geo* g, const StateP<T>& st, int S, int R, int extrap, long long maxB, int Rq, hipStream_t q) {
    const int ns = nw_small_wgs(S);
    const int krw = (int)grid_x(maxB * Rq);
    const dim3 grid(ns + krw * S);
    const size_t lds = eig_lds_bytes(R);
#define CPD_NCK(NMV) hipLaunchKernelGGL((k_nw_core_kr<T, NMV>), grid, dim3(256), lds, q, g, st, extrap, S, ns, krw)
    switch (nmax_class(R)) {
    case 16: CPD_NCK(16); break;
    case 24: CPD_NCK(24); break;
    case 32: CPD_NCK(32); break;
    case 48: CPD_NCK(48); break;
    default: CPD_NCK(64); break;
    }
#undef CPD_NCK
}

template <typename T>
void launch_nw_prep_contract(const Geo* g, const StateP<T>& st, int S, int R, int n, int maxI, int Rq, hipStream_t q) {
    const int ns = nw_small_wgs(S);
    const dim3 grid(ns + maxI * S);
    const size_t lds = prep_lds_bytes<T>(R, Rq);
#define CPD_NPC(NMV) hipLaunchKernelGGL((k_nw_prep_contract<T, NMV>), grid, dim3(256), lds, q, g, st, n, S, ns, maxI)
    switch (nmax_class(R)) {
    case 16: CPD_NPC(16); break;
    case 24: CPD_NPC(24); break;
    case 32: CPD_NPC(32); break;
    case 48: CPD_NPC(48); break;
    default: CPD_NPC(64); break;
    }
#undef CPD_NPC
}

#define CPD_INST_NW(T)                                                                                                    \
    template void launch_nw_kr<T>(const Geo*, const StateP<T>&, int, int, int, long long, int, int, hipStream_t);       \
    template void launch_nw_pass<T>(const Geo*, const StateP<T>&, const ItemNW*, int, int, int, int, hipStream_t);      \
    template void launch_nw_contract<T>(const Geo*, const StateP<T>&, int, int, int, int, int, int, hipStream_t);    \
    template void launch_nw_core_kr<T>(const Geo*, const StateP<T>&, int, int, int, long long, int, hipStream_t);    \
    template void launch_nw_prep_contract<T>(const Geo*, const StateP<T>&, int, int, int, int, int, hipStream_t);
CPD_INST_NW(float)
CPD_INST_NW(double)

}  // namespace cpd
