// Sources of the MTTKRP result K = M_(n) U^{⊙-n} used by the factor update,
// the statistics and the gradient kernels: the pass partials of the dense
// path (summed in fixed order) or the Tucker form of the lra path.
#pragma once
#include "dev_common.h"

namespace cpd {

enum { KSRC_K1P = 0, KSRC_K2 = 1, KSRC_PART = 2, KSRC_LRA0 = 3, KSRC_LRA1 = 4, KSRC_LRA2 = 5 };

// K[i][col] of block s from the MTTKRP pass outputs (FP64 sums in fixed order).
template <typename T, int KSRC>
__device__ __forceinline__ double k_value(const Geo* __restrict__ g, const StateP<T>& st, int s, int i, int col) {
    const int Rq = g->Rq;
    double acc = 0.0;
    if (KSRC == KSRC_K1P) {
        const int nrg = g->nrg[s];
        const T* p = st.K1p + g->k1off[s] + (long long)i * nrg * Rq + col;
        for (int r = 0; r < nrg; ++r) acc += (double)p[r * Rq];
    } else if (KSRC == KSRC_K2) {
        const int nk = g->nk2[s];
        const long long ps = (long long)g->I[s][1] * Rq;
        const T* p = st.K2 + g->k2off[s] + (long long)i * Rq + col;
        for (int ch = 0; ch < nk; ++ch) acc += (double)p[ch * ps];
    } else if (KSRC >= KSRC_LRA0) {
        // Tucker form: K_n[i][col] = sum_j A_n[i][j] C_n[j][col]
        const int n = KSRC - KSRC_LRA0, Jn = g->J[s][n];
        const double* A = st.lra + g->aoff[n][s] + (long long)i * Jn;
        const double* C = st.lra + g->coff[s] + col;
        double a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int j = 0;
        for (; j + 3 < Jn; j += 4) {
            acc = fma(A[j], C[(long long)j * Rq], acc);
            a1 = fma(A[j + 1], C[(long long)(j + 1) * Rq], a1);
            a2 = fma(A[j + 2], C[(long long)(j + 2) * Rq], a2);
            a3 = fma(A[j + 3], C[(long long)(j + 3) * Rq], a3);
        }
        for (; j < Jn; ++j) acc = fma(A[j], C[(long long)j * Rq], acc);
        acc = (acc + a1) + (a2 + a3);
    } else {
        const int I3 = g->I[s][2], nch = g->nchunk[s];
        const T* p = st.part + g->poff[s] + (long long)i * Rq + col;
        const long long ps = (long long)I3 * Rq;
#pragma unroll 8
        for (int ch = 0; ch < nch; ++ch) acc += (double)p[ch * ps];
    }
    return acc;
}

}  // namespace cpd
