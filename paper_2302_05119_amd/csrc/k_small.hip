// Small FP64 kernels of the sweep: the core (lambda) update, Grams and step
// matrices with their exact spectral norms, the objective with the restart
// test, and the commit of an accepted iterate.  One workgroup per block for
// the R x R work.
#include "small_kernels.h"

namespace cpd {

CPD_SMALL_IMPLS(extern template, 1)
CPD_SMALL_IMPLS(template, 0)

// Accept the sweep: x_{k-2} <- x_{k-1}, x_{k-1} <- x_k for factors and lambda,
// Grams and b to slot 1.  The last workgroup keeps the Lipschitz constants of
// the accepted sweep, advances k and t and applies the stopping rule.
template <typename T>
__global__ __launch_bounds__(256) void k_commit(const Geo* __restrict__ g, StateP<T> st, long long uslot, long long wlen) {
    Ctrl* c = st.ctrl;
    if (c->stop) return;
    const int S = g->S, R = g->R, Rq = g->Rq;
    const long long nl = (long long)S * Rq, nv = 3LL * S * R * R, nb = (long long)S * Rq;
    const long long total = uslot + nl + nv + nb + wlen;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < total; i += (long long)gridDim.x * 256) {
        if (i < uslot) {
            st.U[2][i] = st.U[1][i];
            st.U[1][i] = st.U[0][i];
        } else if (i < uslot + nl) {
            const long long j = i - uslot;
            st.lam[2][j] = st.lam[1][j];
            st.lam[1][j] = st.lam[0][j];
        } else if (i < uslot + nl + nv) {
            const long long j = i - uslot - nl;
            st.V[1][j] = st.V[0][j];
        } else if (i < uslot + nl + nv + nb) {
            const long long j = i - uslot - nl - nv;
            st.b[1][j] = st.b[0][j];
        } else {
            // Tucker-form W = A^T U (lra): slot 0 -> slot 1
            const long long j = i - uslot - nl - nv - nb;
            st.lra[g->woff[0][0] + g->wslot_len + j] = st.lra[g->woff[0][0] + j];
        }
    }
    __shared__ int last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = (atomicAdd(&c->counter_commit, 1u) == (unsigned)(gridDim.x - 1));
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    const int tid = threadIdx.x;
    __shared__ double lu[3 * CPD_MAXS];
    if (tid < S) st.Ld_prev[tid] = st.Ld_cur[tid];
    if (tid < 3 * S) {
        const double v = st.Lu_cur[tid];
        st.Lu_prev[tid] = v;
        lu[tid] = v;
    }
    __syncthreads();
    if (tid < 3) {
        double LC = 0.0;
        for (int b = 0; b < S; ++b) LC += lu[tid * S + b];
        st.LC_prev[tid] = LC;
    }
    if (tid != 0) return;
    const int redo = c->redo;
    c->restarts += redo;
    c->last_restarted = redo;
    const double rel_old = c->rel_prev;
    c->F_prev = c->F_cur;
    c->rel_prev = c->rel_cur;
    c->k += 1;
    double t_k = 0.5 * (1.0 + sqrt(1.0 + 4.0 * c->t * c->t));
    if (redo && c->reset_t) t_k = 1.0;
    c->t = t_k;
    c->w_hat = (t_k - 1.0) / (0.5 * (1.0 + sqrt(1.0 + 4.0 * t_k * t_k)));
    if (c->tol > 0.0 && fabs(c->rel_cur - rel_old) < c->tol) c->stop = 1;
    c->redo = 0;
    c->counter_commit = 0u;
}

// Iterate in slot 1 (initial or restored): Grams of every factor, b from the
// reduced mode-3 MTTKRP, F and RelErr; sets F_prev / rel_prev.
template <typename T>
__global__ __launch_bounds__(256) void k_init_stats(const Geo* __restrict__ g, StateP<T> st) {
    Ctrl* c = st.ctrl;
    const int s = blockIdx.x, tid = threadIdx.x;
    const int S = g->S, R = g->R, Rq = g->Rq, RR = R * R;
    extern __shared__ char smraw[];
    __shared__ int last;
    __shared__ double fb[CPD_MAXS], nb[CPD_MAXS];
    for (int m = 0; m < 2; ++m)
        block_gram<T>(st.U[1] + g->uoff[m][s], g->I[s][m], R, Rq, st.V[1] + (m * S + s) * RR,
                      (T*)(smraw + ((gram_acc_bytes(R) + 255) & ~(size_t)255)), 128, (double*)smraw);
    double* V2 = st.V[1] + (2 * S + s) * RR;
    double* b = st.b[1] + s * Rq;
    gram_and_b<T>(st.U[1] + g->uoff[2][s], st.K3 + g->koff[s], g->I[s][2], R, Rq, V2, b, smraw);
    __threadfence_block();
    __syncthreads();
    const double F = block_objective(st.lam[1] + s * Rq, st.V[1] + (0 * S + s) * RR, st.V[1] + (1 * S + s) * RR, V2, b,
                                     st.normM2[s], R);
    if (tid == 0) {
        st.Fblk[s] = F;
        __threadfence();
        last = (atomicAdd(&c->counter_aux, 1u) == (unsigned)(gridDim.x - 1));
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    if (tid < S) {
        fb[tid] = load_agent(&st.Fblk[tid]);
        nb[tid] = st.normM2[tid];
    }
    __syncthreads();
    if (tid != 0) return;
    double Fs = 0.0, rel = 0.0;
    for (int q = 0; q < S; ++q) {
        Fs += fb[q];
        rel += sqrt(fmax(0.0, 2.0 * fb[q])) / sqrt(nb[q]);
    }
    c->F_prev = Fs;
    c->F_cur = Fs;
    c->rel_prev = rel / S;
    c->rel_cur = rel / S;
    c->nonfinite = !isfinite(Fs);
    c->counter_aux = 0u;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
void launch_core(const Geo* g, const StateP<T>& st, int S, int R, int extrap, int gate, hipStream_t q) {
    if (gate) core_impl<1, T>(g, st, S, R, extrap, q);
    else core_impl<0, T>(g, st, S, R, extrap, q);
}
template <typename T>
void launch_prep(const Geo* g, const StateP<T>& st, int S, int R, int n, int gate, hipStream_t q) {
    if (gate) prep_impl<1, T>(g, st, S, R, n, q);
    else prep_impl<0, T>(g, st, S, R, n, q);
}
template <typename T>
void launch_finish(const Geo* g, const StateP<T>& st, int S, int R, int first_sweep, int gate, hipStream_t q) {
    if (gate) finish_impl<1, T>(g, st, S, R, first_sweep, q);
    else finish_impl<0, T>(g, st, S, R, first_sweep, q);
}
template <typename T>
void launch_commit(const Geo* g, const StateP<T>& st, long long uslot, int S, int Rq, int R, long long wlen, hipStream_t q) {
    const long long total = uslot + (long long)S * Rq * 2 + 3LL * S * R * R + wlen;
    long long nb = (total + 255) / 256;
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_commit<T>, dim3((unsigned)nb), dim3(256), 0, q, g, st, uslot, wlen);
}
template <typename T>
void launch_init_stats(const Geo* g, const StateP<T>& st, int S, int R, hipStream_t q) {
    const int Rq = (R + 3) / 4 * 4;
    hipLaunchKernelGGL(k_init_stats<T>, dim3(S), dim3(256), gram_lds_bytes<T>(R, Rq, 128), q, g, st);
}

#define CPD_INST_SMALL(T)                                                                                  \
    template void launch_core<T>(const Geo*, const StateP<T>&, int, int, int, int, hipStream_t);          \
    template void launch_prep<T>(const Geo*, const StateP<T>&, int, int, int, int, hipStream_t);          \
    template void launch_finish<T>(const Geo*, const StateP<T>&, int, int, int, int, hipStream_t);        \
    template void launch_commit<T>(const Geo*, const StateP<T>&, long long, int, int, int, long long, hipStream_t); \
    template void launch_init_stats<T>(const Geo*, const StateP<T>&, int, int, hipStream_t);
CPD_INST_SMALL(float)
CPD_INST_SMALL(double)

}  // namespace cpd
