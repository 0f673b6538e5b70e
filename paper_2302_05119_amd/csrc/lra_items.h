// Work of one workgroup of the lra iteration kernels (Algorithm 2's data
// terms in Tucker form), shared by their own launches and by the launches that
// run them beside the R x R work.
#pragma once
#include "dev_common.h"

namespace cpd {

// W_n^(s)[j][c] = sum_i A_n[i][j] U^(n,s)[i][c] of block s, row j (four row
// phases x 64 columns, eight rows of loads in flight per thread, phases summed
// in fixed order).  st has its slots remapped; wslot is the physical W slot.
template <typename T>
__device__ __forceinline__ void lra_w_item(const Geo* __restrict__ g, const StateP<T>& st, int n, int uslot, int wslot, int s,
                                           int j) {
    const int Jn = g->J[s][n];
    if (j >= Jn) return;
    const int I = g->I[s][n], Rq = g->Rq, R = g->R;
    const double* A = st.lra + g->aoff[n][s];
    const T* U = pick3(st.U, uslot) + g->uoff[n][s];
    __shared__ double part[4][64];
    const int c = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int cc = min(c, R - 1);
    double a0 = 0.0, a1 = 0.0;
    for (int i0 = ph; i0 < I; i0 += 32) {
        double av[8], uv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int i = min(i0 + 4 * q, I - 1);
            av[q] = A[(long long)i * Jn + j];
            uv[q] = (double)U[(long long)i * Rq + cc];
        }
#pragma unroll
        for (int q = 0; q < 8; q += 2) {
            if (i0 + 4 * q < I) a0 = fma(av[q], uv[q], a0);
            if (i0 + 4 * q + 4 < I) a1 = fma(av[q + 1], uv[q + 1], a1);
        }
    }
    part[ph][c] = a0 + a1;
    __syncthreads();
    if (threadIdx.x < Rq) {
        const double v = (c < R) ? ((part[0][c] + part[1][c]) + part[2][c]) + part[3][c] : 0.0;
        st.lra[g->woff[n][s] + (long long)wslot * g->wslot_len + (long long)j * Rq + c] = v;
    }
}

// C_n^(s)[jn][c] = sum_{ja, jb} G_(n)[jn][(ja, jb)] W_a[ja][c] W_b[jb][c], where
// (a, b) are the other two modes (W of modes before n from slot 0, after n
// from slot 1), row jn of block s.  The G slice of jn and both W factors are
// staged in LDS (sm: lra_c_lds_bytes); T = G_slice W_b (Ja x Rq) runs on the
// FP64 matrix cores in 16 x 16 tiles (v_mfma_f64_16x16x4f64, wavefront w
// takes tiles w, w + 4, ...), and C[c] = sum_ja W_a[ja][c] T[ja][c] is formed
// from the accumulators: per lane over its four rows, then over the four lane
// groups and the row tiles in fixed order through LDS.
template <typename T>
__device__ __forceinline__ void lra_c_item(const Geo* __restrict__ g, const StateP<T>& st, int n, int s, int jn, double* sm) {
    const int r2 = st.ctrl->rot2;
    const int J1 = g->J[s][1], J2 = g->J[s][2];
    const int Jn = g->J[s][n];
    if (jn >= Jn) return;
    const int Rq = g->Rq, R = g->R;
    const int ma = (n == 0) ? 1 : 0, mb = (n == 2) ? 1 : 2;
    const int Ja = g->J[s][ma], Jb = g->J[s][mb];
    const long long wl = g->wslot_len;
    const double* Wa = st.lra + g->woff[ma][s] + ((ma < n ? 0 : 1) ^ r2) * wl;
    const double* Wb = st.lra + g->woff[mb][s] + ((mb < n ? 0 : 1) ^ r2) * wl;
    const double* G = st.lra + g->goff[s];
    double* gs = sm;                       // [Ja][Jb]
    double* wa = gs + Ja * Jb;             // [Ja][Rq]
    double* wb = wa + Ja * Rq;             // [Jb][Rq]
    double* part = wb + Jb * Rq;           // [row tile][lane group][64]
    const int tid = threadIdx.x;
    for (int e = tid; e < Ja * Jb; e += 256) {
        const int ja = e / Jb, jb = e % Jb;
        long long gi;
        if (n == 0) gi = ((long long)jn * J1 + ja) * J2 + jb;
        else if (n == 1) gi = ((long long)ja * J1 + jn) * J2 + jb;
        else gi = ((long long)ja * J1 + jb) * J2 + jn;
        gs[e] = G[gi];
    }
    for (int e = tid; e < Ja * Rq; e += 256) wa[e] = Wa[e];
    for (int e = tid; e < Jb * Rq; e += 256) wb[e] = Wb[e];
    __syncthreads();
    const int lane = tid & 63, wv = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int nta = (Ja + 15) >> 4, ntc = (Rq + 15) >> 4;
    for (int tile = wv; tile < nta * ntc; tile += 4) {
        const int ta = tile / ntc, tc = tile % ntc;
        const int row = 16 * ta + li, col = 16 * tc + li;
        v4d acc = (v4d){0.0, 0.0, 0.0, 0.0};
        // lane l: A[l % 16][l / 16] = G_slice[row][k], B[l / 16][l % 16] = W_b[k][col]
        for (int k0 = 0; k0 < Jb; k0 += 4) {
            const int k = k0 + lk;
            const double a = (row < Ja && k < Jb) ? gs[row * Jb + k] : 0.0;
            const double b = (k < Jb && col < Rq) ? wb[k * Rq + col] : 0.0;
            acc = mfma64(a, b, acc);
        }
        // register v holds T[16 ta + 4 v + l / 16][16 tc + l % 16]
        double p = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int ja = 16 * ta + 4 * v + lk;
            if (ja < Ja && col < Rq) p = fma(wa[ja * Rq + col], acc[v], p);
        }
        part[(ta * 4 + lk) * 64 + col] = p;
    }
    __syncthreads();
    if (tid < Rq) {
        double c = 0.0;
        if (tid < R)
            for (int ta = 0; ta < nta; ++ta)
                c += ((part[(ta * 4 + 0) * 64 + tid] + part[(ta * 4 + 1) * 64 + tid]) + part[(ta * 4 + 2) * 64 + tid]) +
                     part[(ta * 4 + 3) * 64 + tid];
        st.lra[g->coff[s] + (long long)jn * Rq + tid] = c;
    }
}

}  // namespace cpd
