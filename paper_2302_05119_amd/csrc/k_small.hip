// Small FP64 kernels of the sweep: the core (lambda) update, Grams and step
// matrices with their exact spectral norms, the objective with the restart
// test, and the commit of an accepted iterate.  One workgroup per block for
// the R x R work.
#include "small_dev.h"

namespace cpd {

template <typename T, int NMAX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_core(const Geo* __restrict__ g, StateP<T> st, int extrapolate, int gate) {
    if (gated_out(st.ctrl, gate)) return;
    extern __shared__ char smraw[];
    core_block<T, NMAX>(g, st, blockIdx.x, extrapolate, smraw);
}

template <typename T, int NMAX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_prep(const Geo* __restrict__ g, StateP<T> st, int n, int gate) {
    if (gated_out(st.ctrl, gate)) return;
    extern __shared__ char smraw[];
    prep_block<T, NMAX>(g, st, blockIdx.x, n, smraw);
}

// b = colsum(K3 ⊛ U^(3)) and the Gram of U^(3) from LDS-staged rows.
template <typename T>
__device__ __forceinline__ void gram_and_b(const T* __restrict__ U3, const T* __restrict__ K3, int I3, int R, int Rq, double* __restrict__ V,
                           double* __restrict__ b, char* lds) {
    T* tile = (T*)(lds + ((gram_acc_bytes(R) + 255) & ~(size_t)255));
    block_gram<T>(U3, I3, R, Rq, V, tile, 128, (double*)lds);
    // b: 256 threads = 4 row phases x 64 columns; tiles of 64 rows of K3 and U3 in LDS
    __shared__ double bp[4][CPD_MAXR];
    const int tid = threadIdx.x, c = tid & 63, ph = tid >> 6;
    T* tk = tile;
    T* tu = tile + 64 * Rq;
    double acc = 0.0;
    for (int r0 = 0; r0 < I3; r0 += 64) {
        const int nr = min(64, I3 - r0);
        for (int e = tid; e < nr * Rq; e += 256) {
            tk[e] = K3[(long long)r0 * Rq + e];
            tu[e] = U3[(long long)r0 * Rq + e];
        }
        __syncthreads();
        if (c < R)
            for (int i = ph; i < nr; i += 4) acc += (double)tk[i * Rq + c] * (double)tu[i * Rq + c];
        __syncthreads();
    }
    if (c < R) bp[ph][c] = acc;
    __syncthreads();
    if (tid < R) b[tid] = bp[0][tid] + bp[1][tid] + bp[2][tid] + bp[3][tid];
    __syncthreads();
}

// F^(s) = 1/2 (||M||^2 - 2 lam^T b + lam^T H lam), H = V0 ⊛ V1 ⊛ V2 (eq. costfunc
// expanded with the Hadamard-of-Grams identity of Appendix A).
__device__ __forceinline__ double block_objective(const double* lam, const double* V0, const double* V1, const double* V2,
                                  const double* b, double normM2, int R) {
    __shared__ double red[256];
    const int tid = threadIdx.x, RR = R * R;
    double part = 0.0;
    for (int i = tid; i < RR; i += 256) part += lam[i / R] * lam[i % R] * V0[i] * V1[i] * V2[i];
    if (tid < R) part -= 2.0 * lam[tid] * b[tid];
    red[tid] = part;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    return 0.5 * (normM2 + red[0]);
}

// After the mode-3 update: Gram of U^(3), b (the data term (U^⊙)^T vec(M) of
// eq. solapgG, reused by the next core update) and F^(s).  The last workgroup
// sums F over the blocks in block order and, for the extrapolated sweep,
// raises the restart flag when F_k >= F_{k-1} (Algorithm 1).
template <typename T>
__global__ __launch_bounds__(256) void k_finish(const Geo* __restrict__ g, StateP<T> st, int first_sweep, int gate) {
    Ctrl* c = st.ctrl;
    if (gated_out(c, gate)) return;
    const int s = blockIdx.x, tid = threadIdx.x;
    const int S = g->S, R = g->R, Rq = g->Rq, RR = R * R;
    extern __shared__ char smraw[];
    __shared__ int last;
    __shared__ double fb[CPD_MAXS], nb[CPD_MAXS];
    double* V2 = st.V[0] + (2 * S + s) * RR;
    double* b = st.b[0] + s * Rq;
    gram_and_b<T>(st.U[0] + g->uoff[2][s], st.K3 + g->koff[s], g->I[s][2], R, Rq, V2, b, smraw);
    __threadfence_block();
    __syncthreads();
    const double F = block_objective(st.lam[0] + s * Rq, st.V[0] + (0 * S + s) * RR, st.V[0] + (1 * S + s) * RR, V2, b,
                                     st.normM2[s], R);
    if (tid == 0) {
        st.Fblk[s] = F;
        __threadfence();
        last = (atomicAdd(&c->counter_finish, 1u) == (unsigned)(gridDim.x - 1));
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
    rel /= S;
    c->F_cur = Fs;
    c->rel_cur = rel;
    c->nonfinite = !isfinite(Fs);
    if (first_sweep) c->redo = (c->restart_on && Fs >= c->F_prev) ? 1 : 0;
    c->counter_finish = 0u;
}

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
#define CPD_NMAX_DISPATCH(R, CALL) \
    do {                              \
        if ((R) <= 16) { CALL(16); }  \
        else if ((R) <= 32) { CALL(32); } \
        else if ((R) <= 48) { CALL(48); } \
        else { CALL(64); }            \
    } while (0)

template <typename T>
void launch_core(const Geo* g, const StateP<T>& st, int S, int R, int extrap, int gate, hipStream_t q) {
#define CPD_CORE(N) hipLaunchKernelGGL((k_core<T, N>), dim3(S), dim3(256), eig_lds_bytes(R), q, g, st, extrap, gate)
    CPD_NMAX_DISPATCH(R, CPD_CORE);
#undef CPD_CORE
}
template <typename T>
void launch_prep(const Geo* g, const StateP<T>& st, int S, int R, int n, int gate, hipStream_t q) {
    const int Rq = (R + 3) / 4 * 4;
#define CPD_PREP(N) hipLaunchKernelGGL((k_prep<T, N>), dim3(S), dim3(256), prep_lds_bytes<T>(R, Rq), q, g, st, n, gate)
    CPD_NMAX_DISPATCH(R, CPD_PREP);
#undef CPD_PREP
}
template <typename T>
void launch_finish(const Geo* g, const StateP<T>& st, int S, int R, int first_sweep, int gate, hipStream_t q) {
    const int Rq = (R + 3) / 4 * 4;
    hipLaunchKernelGGL(k_finish<T>, dim3(S), dim3(256), gram_lds_bytes<T>(R, Rq, 128), q, g, st, first_sweep, gate);
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
