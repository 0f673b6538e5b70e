// Sources of the MTTKRP result K = M_(n) U^{⊙-n} used by the factor update,
// the statistics and the gradient kernels: the pass partials of the dense
// path (summed in fixed order), the Tucker form of the lra path, or the plain
// I_n x Rq buffer that the order-N contraction writes.
#pragma once
#include "dev_common.h"

namespace cpd {

enum { KSRC_K1P = 0, KSRC_K2 = 1, KSRC_PART = 2, KSRC_LRA0 = 3, KSRC_LRA1 = 4, KSRC_LRA2 = 5, KSRC_PLAIN = 6 };

// Sum of n strided values p[0], p[st], ..., p[(n-1) st] in index order, eight
// loads in flight per step (clamped addresses, zeros past n): a loop with one
// load per iteration would wait for each load in turn.
template <typename T>
__device__ __forceinline__ double strided_sum(const T* __restrict__ p, long long st, int n) {
    double acc = 0.0;
    for (int r0 = 0; r0 < n; r0 += 8) {
        T v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = p[min(r0 + j, n - 1) * st];
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (r0 + j < n) acc += (double)v[j];
    }
    return acc;
}

// K[i][col] of block s from the MTTKRP pass outputs (FP64 sums in fixed order).
template <typename T, int KSRC>
__device__ __forceinline__ double k_value(const Geo* __restrict__ g, const StateP<T>& st, int s, int i, int col) {
    const int Rq = g->Rq;
    double acc = 0.0;
    if (KSRC == KSRC_K1P) {
        const int nrg = g->nrg[s];
        acc = strided_sum(st.K1p + g->k1off[s] + (long long)i * nrg * Rq + col, Rq, nrg);
    } else if (KSRC == KSRC_K2) {
        acc = strided_sum(st.K2 + g->k2off[s] + (long long)i * Rq + col, (long long)g->I[s][1] * Rq, g->nk2[s]);
    } else if (KSRC == KSRC_PLAIN) {
        acc = (double)st.K3[g->koff[s] + (long long)i * Rq + col];
    } else if (KSRC >= KSRC_LRA0) {
        // Tucker form: K_n[i][col] = sum_j A_n[i][j] C_n[j][col] (four chains
        // by j mod 4, then the remainder; eight terms in flight per step)
        const int n = KSRC - KSRC_LRA0, Jn = g->J[s][n], J4 = Jn & ~3;
        const double* A = st.lra + g->aoff[n][s] + (long long)i * Jn;
        const double* C = st.lra + g->coff[s] + col;
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        for (int j0 = 0; j0 < Jn; j0 += 8) {
            double av[8], cv[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int j = min(j0 + q, Jn - 1);
                av[q] = A[j];
                cv[q] = C[(long long)j * Rq];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int j = j0 + q;
                if (j < J4) a[q & 3] = fma(av[q], cv[q], a[q & 3]);
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int j = j0 + q;
                if (j >= J4 && j < Jn) a[0] = fma(av[q], cv[q], a[0]);
            }
        }
        acc = (a[0] + a[1]) + (a[2] + a[3]);
    } else {
        acc = strided_sum(st.part + g->poff[s] + (long long)i * Rq + col, (long long)g->I[s][2] * Rq, g->nchunk[s]);
    }
    return acc;
}

}  // namespace cpd
