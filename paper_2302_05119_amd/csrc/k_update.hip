// Factor update of one mode for every block (eq. solUns / solUnC / solUnsI):
//
//   U_hat = U_{k-1} + w (U_{k-1} - U_{k-2})                  (eq. eqextraPU)
//   G     = U_hat P - K diag(lambda),  P = D H_{-n} D        (eq. solapgU)
//   individual columns:  U_I = max(0, U_hat_I - G_I / L_u^(n,s))
//   shared columns:      U_C = max(0, U_hat_C - sum_s G_C^(s) / sum_s L_u^(n,s))
//
// K = M_(n) U^{⊙-n} comes from the MTTKRP kernels: at order 3 the mode-1
// partials of pass 1 (one per 64 rows of i2), the mode-2 contraction, and the
// pass-2 chunk partials for mode 3, each summed here in fixed order; at order
// N > 3 the plain buffer of the dimension-tree contraction.
// All of the small arithmetic is FP64; the new factor is rounded to the
// storage type once.  A workgroup owns a row tile of every block that shares
// the mode's columns, so the coupled sum runs in LDS in block order.
#include "ksource.h"

namespace cpd {

// BS threads per workgroup: 256, or 512 / 1024 when an item holds more
// elements (a row of a coupling group over many blocks), so that each thread
// takes one element and its chain of loads runs once
template <typename T, int KSRC, int BS>
__global__ __launch_bounds__(BS) void k_update(const Geo* __restrict__ g, StateP<T> st, const ItemU* __restrict__ items,
                                                int n, int extrapolate) {
    const Ctrl* c = st.ctrl;
    if (c->stop) return;
    apply_rot(st);
    extrapolate = extrapolating(c, extrapolate);
    const ItemU it = items[blockIdx.x];
    // a coupling-group item (ns < 0) covers the -ns blocks of grp[n]; any other
    // item covers blocks s0.. with every column individual
    const bool cg = it.ns < 0;
    const int s0 = it.s0, ns = cg ? -it.ns : it.ns, row0 = it.row0, nrows = it.nrows;
    const int S = g->S, R = g->R, Rq = g->Rq, RR = R * R, Ln = cg ? g->L[n] : 0;
    const int* blk = cg ? g->grp[n] : nullptr;
    const int tid = threadIdx.x;
    extern __shared__ double sm[];
    double* uh = sm;                       // [ns][nrows][R]
    double* gc = uh + ns * nrows * R;      // [ns][nrows][Ln]
    const int tot = ns * nrows * R;
    const double what = c->w_hat, dw = c->delta_w;
    double LC = 0.0;
    if (Ln > 0)
        for (int k = 0; k < ns; ++k) LC += st.Lu_cur[n * S + blk[k]];
    const double wC = (Ln > 0) ? extrap_weight(extrapolate, what, st.LC_prev[n], LC, dw) : 0.0;

    // extrapolated point
    for (int e = tid; e < tot; e += BS) {
        const int sl = e / (nrows * R), rem = e % (nrows * R), rr = rem / R, col = rem % R;
        const int s = cg ? blk[sl] : s0 + sl;
        const long long off = g->uoff[n][s] + (long long)(row0 + rr) * Rq + col;
        const double x1 = (double)st.U[1][off], x2 = (double)st.U[2][off];
        const double w = (col < Ln) ? wC : extrap_weight(extrapolate, what, st.Lu_prev[n * S + s], st.Lu_cur[n * S + s], dw);
        uh[e] = x1 + w * (x1 - x2);
    }
    __syncthreads();
    // gradient; individual columns are projected here
    for (int e = tid; e < tot; e += BS) {
        const int sl = e / (nrows * R), rem = e % (nrows * R), rr = rem / R, col = rem % R;
        const int s = cg ? blk[sl] : s0 + sl, i = row0 + rr;
        const double* P = st.P + (long long)s * RR;
        const double* u = uh + (sl * nrows + rr) * R;
        // four chains by r mod 4, then the remainder into the first; eight
        // entries of the P column in flight per step
        double ga[4] = {0.0, 0.0, 0.0, 0.0};
        const int R4 = R & ~3;
        for (int r0 = 0; r0 < R; r0 += 8) {
            double pv[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) pv[q] = P[min(r0 + q, R - 1) * R + col];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (r0 + q < R4) ga[q & 3] = fma(u[r0 + q], pv[q], ga[q & 3]);
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (r0 + q >= R4 && r0 + q < R) ga[0] = fma(u[r0 + q], pv[q], ga[0]);
        }
        double gr = (ga[0] + ga[1]) + (ga[2] + ga[3]);
        const double kv = k_value<T, KSRC>(g, st, s, i, col);
        gr -= kv * st.lam[0][s * Rq + col];
        if (KSRC == KSRC_PART || KSRC == KSRC_LRA2) st.K3[g->koff[s] + (long long)i * Rq + col] = (T)kv;
        const long long off = g->uoff[n][s] + (long long)i * Rq + col;
        if (col >= Ln) {
            const double Lu = st.Lu_cur[n * S + s];
            const double un = (Lu > 0.0) ? relu_keep_nan(uh[e] - gr / Lu) : (double)st.U[1][off];
            st.U[0][off] = (T)un;
        } else {
            gc[(sl * nrows + rr) * Ln + col] = gr;
        }
    }
    if (Ln == 0) return;
    __syncthreads();
    // shared columns: sum the block gradients in block order
    for (int e = tid; e < nrows * Ln; e += BS) {
        const int rr = e / Ln, col = e % Ln, i = row0 + rr;
        double gsum = 0.0;
        for (int sl = 0; sl < ns; ++sl) gsum += gc[(sl * nrows + rr) * Ln + col];
        const long long off0 = g->uoff[n][blk[0]] + (long long)i * Rq + col;
        const double un = (LC > 0.0) ? relu_keep_nan(uh[rr * R + col] - gsum / LC) : (double)st.U[1][off0];
        const T ut = (T)un;
        for (int sl = 0; sl < ns; ++sl) st.U[0][g->uoff[n][blk[sl]] + (long long)i * Rq + col] = ut;
    }
}

// K = M_(n) U^{⊙-n} of one block from the pass outputs (computed by the caller
// on the iterate of interest); used at initialisation and by the test hook.
template <typename T, int KSRC>
__global__ __launch_bounds__(256) void k_extract(const Geo* __restrict__ g, StateP<T> st, int s, int I, T* __restrict__ out,
                                                 int ld_out) {
    const int R = g->R;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < (long long)I * R; e += (long long)gridDim.x * 256) {
        const int i = (int)(e / R), col = (int)(e % R);
        out[(long long)i * ld_out + col] = (T)k_value<T, KSRC>(g, st, s, i, col);
    }
}

template <typename T>
void launch_extract_k(const Geo* g, const StateP<T>& st, int s, int n, int I, int R, T* out, int ld_out, int lra, hipStream_t q) {
    long long nb = ((long long)I * R + 255) / 256;
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    if (lra) {
        if (n == 0) hipLaunchKernelGGL((k_extract<T, KSRC_LRA0>), dim3((unsigned)nb), dim3(256), 0, q, g, st, s, I, out, ld_out);
        else if (n == 1) hipLaunchKernelGGL((k_extract<T, KSRC_LRA1>), dim3((unsigned)nb), dim3(256), 0, q, g, st, s, I, out, ld_out);
        else hipLaunchKernelGGL((k_extract<T, KSRC_LRA2>), dim3((unsigned)nb), dim3(256), 0, q, g, st, s, I, out, ld_out);
        return;
    }
    if (n == 0) hipLaunchKernelGGL((k_extract<T, KSRC_K1P>), dim3((unsigned)nb), dim3(256), 0, q, g, st, s, I, out, ld_out);
    else if (n == 1) hipLaunchKernelGGL((k_extract<T, KSRC_K2>), dim3((unsigned)nb), dim3(256), 0, q, g, st, s, I, out, ld_out);
    else hipLaunchKernelGGL((k_extract<T, KSRC_PART>), dim3((unsigned)nb), dim3(256), 0, q, g, st, s, I, out, ld_out);
}
template void launch_extract_k<float>(const Geo*, const StateP<float>&, int, int, int, int, float*, int, int, hipStream_t);
template void launch_extract_k<double>(const Geo*, const StateP<double>&, int, int, int, int, double*, int, int, hipStream_t);

template <typename T>
void launch_update(const Geo* g, const StateP<T>& st, const ItemU* items, int nitems, int n, int R, int extrap, int lds_rows,
                   int ksrc, hipStream_t q) {
    if (nitems <= 0) return;
    // lds_rows = max over items of ns * nrows; the shared-gradient buffer uses at most as much
    const size_t lds = sizeof(double) * (size_t)lds_rows * (size_t)(2 * R);
    const int ks = ksrc == 2 ? KSRC_PLAIN
                             : (ksrc == 1 ? KSRC_LRA0 + n : (n == 0 ? KSRC_K1P : (n == 1 ? KSRC_K2 : KSRC_PART)));
    // lds_rows * R is the largest item's element count
    const long long tot = (long long)lds_rows * R;
    const int bs = tot <= 256 ? 256 : tot <= 512 ? 512 : 1024;
#define CPD_UPD(KS)                                                                                                       \
    case KS:                                                                                                              \
        if (bs == 256) hipLaunchKernelGGL((k_update<T, KS, 256>), dim3(nitems), dim3(256), lds, q, g, st, items, n, extrap);   \
        else if (bs == 512) hipLaunchKernelGGL((k_update<T, KS, 512>), dim3(nitems), dim3(512), lds, q, g, st, items, n, extrap); \
        else hipLaunchKernelGGL((k_update<T, KS, 1024>), dim3(nitems), dim3(1024), lds, q, g, st, items, n, extrap);          \
        break;
    switch (ks) {
        CPD_UPD(KSRC_K1P) CPD_UPD(KSRC_K2) CPD_UPD(KSRC_PART) CPD_UPD(KSRC_LRA0) CPD_UPD(KSRC_LRA1) CPD_UPD(KSRC_LRA2)
        CPD_UPD(KSRC_PLAIN)
        default: break;
    }
#undef CPD_UPD
}
template void launch_update<float>(const Geo*, const StateP<float>&, const ItemU*, int, int, int, int, int, int, hipStream_t);
template void launch_update<double>(const Geo*, const StateP<double>&, const ItemU*, int, int, int, int, int, int, hipStream_t);

}  // namespace cpd
