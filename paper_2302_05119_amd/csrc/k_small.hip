// Small FP64 kernels of the sweep: the core (lambda) update, Grams and step
// matrices with their exact spectral norms, and the objective with the
// restart test and the commit of an accepted iterate.  One workgroup per block for
// the R x R work.
#include "small_dev.h"

namespace cpd {

template <typename T, int NMAX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_core(const Geo* __restrict__ g, StateP<T> st, int extrapolate) {
    if (st.ctrl->stop) return;
    apply_rot(st);
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    core_block<T, NMAX>(g, st, blockIdx.x, extrapolating(st.ctrl, extrapolate), smraw);
}

template <typename T, int NMAX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_prep(const Geo* __restrict__ g, StateP<T> st, int n) {
    if (st.ctrl->stop) return;
    apply_rot(st);
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    prep_block<T, NMAX>(g, st, blockIdx.x, n, smraw);
}


// After the last mode's update: Gram of U^(N), b (the data term (U^⊙)^T vec(M)
// of eq. solapgG, reused by the next core update) and F^(s).  A block whose
// last mode is longer than CPD_FIN_ROWS rows is split over workgroups of that
// many rows: each hands its partial Gram and b to the block's last-arriving
// workgroup (agent-scope stores, completion wait, arrival count), which adds
// them in chunk order.  The last block to finish sums F over the blocks in
// block order, applies the restart test of Algorithm 1 and, for an accepted
// sweep, commits it: Lipschitz constants, k, t, w_hat, the stopping rule and
// the slot rotation.
template <typename T, int NMAX>
__global__ __launch_bounds__(256) void k_finish(const Geo* __restrict__ g, StateP<T> st) {
    Ctrl* c = st.ctrl;
    if (c->stop) return;
    apply_rot(st);
    const int tid = threadIdx.x;
    const int S = g->S, R = g->R, Rq = g->Rq, RR = R * R, N = g->N, NS = N * S;
    // block and chunk of this workgroup (binary search over the chunk offsets)
    int s = 0;
    {
        int lo = 0, hi = S - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (g->fin_c0[mid] <= (int)blockIdx.x) lo = mid;
            else hi = mid - 1;
        }
        s = lo;
    }
    const int nc = g->fin_nc[s], chunk = blockIdx.x - g->fin_c0[s];
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    __shared__ int last;
    __shared__ double fb[CPD_MAXS], nb[CPD_MAXS];
    // what the last workgroup needs, read now so that its latency overlaps the
    // Gram (no workgroup of this launch writes any of it before the last one);
    // N S Lipschitz constants, up to two per thread
    const double nrm = (tid < S) ? st.normM2[tid] : 1.0;
    const double ldc = (tid < S) ? st.Ld_cur[tid] : 0.0;
    const double luc = (tid < NS) ? st.Lu_cur[tid] : 0.0;
    const double luc2 = (tid + 256 < NS) ? st.Lu_cur[tid + 256] : 0.0;
    const int redo0 = c->redo, restart_on = c->restart_on, reset_t = c->reset_t;
    const double F_prev = c->F_prev, rel_old = c->rel_prev, t_old = c->t, tol = c->tol;
    const long long k_old = c->k;
    const long long restarts = c->restarts;
    const int rot3 = c->rot3, rot2 = c->rot2;
    // the objective's other inputs (Grams of the new modes 1 .. N-1, lambda;
    // at order N > 3 v1 carries V_2 * ... * V_{N-1})
    constexpr int EP = (NMAX * NMAX + 255) / 256;
    double v0[EP], v1[EP];
    {
        const double* V0 = st.V[0] + (0 * S + s) * RR;
        const double* V1 = st.V[0] + (1 * S + s) * RR;
#pragma unroll
        for (int q = 0; q < EP; ++q) {
            const int i = min(tid + 256 * q, RR - 1);
            v0[q] = V0[i];
            v1[q] = V1[i];
        }
        for (int m = 2; m < N - 1; ++m) {
            const double* Vx = st.V[0] + (m * S + s) * RR;
#pragma unroll
            for (int q = 0; q < EP; ++q) v1[q] *= Vx[min(tid + 256 * q, RR - 1)];
        }
    }
    __shared__ double lam[64];
    if (tid < 64) lam[tid] = st.lam[0][s * Rq + min(tid, R - 1)];
    const double nrm_s = st.normM2[s];
    double* V2 = st.V[0] + ((N - 1) * S + s) * RR;
    double* b = st.b[0] + s * Rq;
    double* V2l = (double*)(smraw + gram_lds_bytes<T>(Rq, 1));
    double* bl = V2l + RR;
    const int In = g->I[s][N - 1];
    if (nc == 1) {
        block_gram<T, 8>(st.U[0] + g->uoff[N - 1][s], In, R, Rq, V2, st.K3 + g->koff[s], b, smraw, V2l, bl);
    } else {
        // this chunk's rows: partial Gram and b into LDS, then to the block's
        // partial slots
        const int r0 = chunk * CPD_FIN_ROWS, nr = min(CPD_FIN_ROWS, In - r0);
        block_gram<T, 8, 32>(st.U[0] + g->uoff[N - 1][s] + (long long)r0 * Rq, nr, R, Rq, nullptr, st.K3 + g->koff[s] + (long long)r0 * Rq,
                         nullptr, smraw, V2l, bl);
        double* fp = st.fpart + (long long)blockIdx.x * (RR + Rq);
        for (int e = tid; e < RR; e += 256) store_agent(&fp[e], V2l[e]);
        if (tid < R) store_agent(&fp[RR + tid], bl[tid]);
        wait_stores();
        __syncthreads();
        __shared__ int lastblk;
        if (tid == 0) lastblk = (arrive_agent(&c->blkcnt[s]) == (unsigned)(nc - 1));
        __syncthreads();
        if (!lastblk) return;
        if (tid == 0) c->blkcnt[s] = 0u;
        // the block's Gram and b: the chunks' partials added in chunk order,
        // QB chunks of loads in flight per step (clamped addresses); thread e
        // holds Gram entries e, e + 256, ... and entry RR + e of b (e < R)
        const double* fb0 = st.fpart + (long long)g->fin_c0[s] * (RR + Rq);
        constexpr int EG = EP + 1, QB = EP <= 4 ? 8 : 4;
        double a[EG];
#pragma unroll
        for (int p = 0; p < EG; ++p) a[p] = 0.0;
        for (int q0 = 0; q0 < nc; q0 += QB) {
            double v[EG][QB];
#pragma unroll
            for (int p = 0; p < EG; ++p) {
                const int e = (p < EP) ? min(tid + 256 * p, RR - 1) : RR + min(tid, R - 1);
#pragma unroll
                for (int j = 0; j < QB; ++j) v[p][j] = load_agent(&fb0[(long long)min(q0 + j, nc - 1) * (RR + Rq) + e]);
            }
#pragma unroll
            for (int p = 0; p < EG; ++p)
#pragma unroll
                for (int j = 0; j < QB; ++j)
                    if (q0 + j < nc) a[p] += v[p][j];
        }
#pragma unroll
        for (int p = 0; p < EP; ++p) {
            const int e = tid + 256 * p;
            if (e < RR) {
                V2l[e] = a[p];
                V2[e] = a[p];
            }
        }
        if (tid < R) {
            bl[tid] = a[EP];
            b[tid] = a[EP];
        }
        __syncthreads();
    }
    const double F = block_objective_pf<EP>(lam, v0, v1, V2l, bl, nrm_s, R);
    if (tid == 0) {
        store_agent(&st.Fblk[s], F);
        wait_stores();
        last = (arrive_agent(&c->counter_finish) == (unsigned)(S - 1));
    }
    __syncthreads();
    if (!last) return;
    if (tid < S) {
        fb[tid] = load_agent(&st.Fblk[tid]);
        nb[tid] = nrm;
    }
    __syncthreads();
    __shared__ int accept;
    __shared__ double fsum, rsum;
    if (tid == 0) {
        double Fs = 0.0, rel = 0.0;
        for (int q = 0; q < S; ++q) {
            Fs += fb[q];
            rel += sqrt(fmax(0.0, 2.0 * fb[q])) / sqrt(nb[q]);
        }
        rel /= S;
        c->F_cur = Fs;
        c->rel_cur = rel;
        c->nonfinite = !isfinite(Fs);
        // restart test of Algorithm 1: a rejected extrapolated sweep leaves
        // x_{k-1} in place and the next sweep redoes it without extrapolation
        const int reject = !redo0 && restart_on && Fs >= F_prev;
        if (reject) c->redo = 1;
        accept = !reject;
        fsum = Fs;
        rsum = rel;
        c->counter_finish = 0u;
    }
    __syncthreads();
    if (!accept) return;
    // accept: the Lipschitz constants of this sweep become the previous ones
    __shared__ double lu[CPD_MAXN * CPD_MAXS];
    if (tid < S) st.Ld_prev[tid] = ldc;
    if (tid < NS) {
        st.Lu_prev[tid] = luc;
        lu[tid] = luc;
    }
    if (tid + 256 < NS) {
        st.Lu_prev[tid + 256] = luc2;
        lu[tid + 256] = luc2;
    }
    __syncthreads();
    if (tid < N) {
        // L_C over the mode's coupling group (every block when L_n = 0)
        double LC = 0.0;
        for (int k = 0; k < g->ngrp[tid]; ++k) LC += lu[tid * S + g->grp[tid][k]];
        st.LC_prev[tid] = LC;
    }
    if (tid != 0) return;
    c->restarts = restarts + redo0;
    c->last_restarted = redo0;
    c->F_prev = fsum;
    c->rel_prev = rsum;
    c->k = k_old + 1;
    double t_k = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t_old * t_old));
    if (redo0 && reset_t) t_k = 1.0;
    c->t = t_k;
    c->w_hat = (t_k - 1.0) / (0.5 * (1.0 + sqrt(1.0 + 4.0 * t_k * t_k)));
    if (tol > 0.0 && fabs(rsum - rel_old) < tol) c->stop = 1;
    c->redo = 0;
    // x_{k-2} <- x_{k-1} <- x_k by slot rotation
    c->rot3 = (rot3 + 2) % 3;
    c->rot2 = rot2 ^ 1;
}

// Iterate in slot 1 (initial or restored): Grams of every factor, b from the
// reduced MTTKRP of the last mode, F and RelErr; sets F_prev / rel_prev.
template <typename T>
__global__ __launch_bounds__(256) void k_init_stats(const Geo* __restrict__ g, StateP<T> st) {
    Ctrl* c = st.ctrl;
    apply_rot(st);
    const int s = blockIdx.x, tid = threadIdx.x;
    const int S = g->S, R = g->R, Rq = g->Rq, RR = R * R;
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    __shared__ int last;
    __shared__ double fb[CPD_MAXS], nb[CPD_MAXS];
    const int N = g->N;
    for (int m = 0; m < N - 1; ++m)
        block_gram<T, 16>(st.U[1] + g->uoff[m][s], g->I[s][m], R, Rq, st.V[1] + (m * S + s) * RR, nullptr, nullptr, smraw);
    double* V2 = st.V[1] + ((N - 1) * S + s) * RR;
    double* b = st.b[1] + s * Rq;
    block_gram<T, 16>(st.U[1] + g->uoff[N - 1][s], g->I[s][N - 1], R, Rq, V2, st.K3 + g->koff[s], b, smraw);   // once per fit
    __threadfence_block();
    __syncthreads();
    const double F = (N == 3) ? block_objective(st.lam[1] + s * Rq, st.V[1] + (0 * S + s) * RR, st.V[1] + (1 * S + s) * RR, V2,
                                                b, st.normM2[s], R)
                              : block_objective_n(st.lam[1] + s * Rq, st.V[1] + s * RR, (long long)S * RR, N, b, st.normM2[s], R);
    if (tid == 0) {
        store_agent(&st.Fblk[s], F);
        wait_stores();
        last = (arrive_agent(&c->counter_aux) == (unsigned)(gridDim.x - 1));
    }
    __syncthreads();
    if (!last) return;
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

// Spectral norms of `count` symmetric n x n matrices (row-major, packed one
// after another), one workgroup each, by the same device code as the sweep.
template <int NMAX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_spectral_norm(const double* __restrict__ mats, int n,
                                                                                                  double* __restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    double* A = (double*)smraw;
    const int ld = n | 1;
    const double* src = mats + (long long)blockIdx.x * n * n;
    for (int i = threadIdx.x; i < n * n; i += 256) A[(i / n) * ld + i % n] = src[i];
    __syncthreads();
    const double v = wg_lmax_nonneg<NMAX>(A, n, ld, eig_work(A, n));
    if (threadIdx.x == 0) out[blockIdx.x] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define CPD_NMAX_DISPATCH(R, CALL)        \
    do {                                  \
        switch (nmax_class(R)) {          \
        case 16: CALL(16); break;         \
        case 24: CALL(24); break;         \
        case 32: CALL(32); break;         \
        case 48: CALL(48); break;         \
        default: CALL(64); break;         \
        }                                 \
    } while (0)

template <typename T>
void launch_core(const Geo* g, const StateP<T>& st, int S, int R, int extrap, hipStream_t q) {
#define CPD_CORE(N) hipLaunchKernelGGL((k_core<T, N>), dim3(S), dim3(256), eig_lds_bytes(R), q, g, st, extrap)
    CPD_NMAX_DISPATCH(R, CPD_CORE);
#undef CPD_CORE
}
template <typename T>
void launch_prep(const Geo* g, const StateP<T>& st, int S, int R, int n, hipStream_t q) {
    const int Rq = (R + 3) / 4 * 4;
#define CPD_PREP(N) hipLaunchKernelGGL((k_prep<T, N>), dim3(S), dim3(256), prep_lds_bytes<T>(R, Rq), q, g, st, n)
    CPD_NMAX_DISPATCH(R, CPD_PREP);
#undef CPD_PREP
}
template <typename T>
void launch_finish(const Geo* g, const StateP<T>& st, int S, int R, int nwg, hipStream_t q) {
    const int Rq = (R + 3) / 4 * 4;
    (void)S;
#define CPD_FIN(N) hipLaunchKernelGGL((k_finish<T, N>), dim3(nwg), dim3(256), finish_lds_bytes<T>(R, Rq), q, g, st)
    CPD_NMAX_DISPATCH(R, CPD_FIN);
#undef CPD_FIN
}
template <typename T>
void launch_init_stats(const Geo* g, const StateP<T>& st, int S, int R, hipStream_t q) {
    const int Rq = (R + 3) / 4 * 4;
    hipLaunchKernelGGL(k_init_stats<T>, dim3(S), dim3(256), gram_lds_bytes<T>(Rq, 1), q, g, st);
}

void launch_spectral_norm(const double* mats, int n, int count, double* out, hipStream_t q) {
#define CPD_SN(N) hipLaunchKernelGGL((k_spectral_norm<N>), dim3(count), dim3(256), eig_lds_bytes(n), q, mats, n, out)
    CPD_NMAX_DISPATCH(n, CPD_SN);
#undef CPD_SN
}

#define CPD_INST_SMALL(T)                                                                                  \
    template void launch_core<T>(const Geo*, const StateP<T>&, int, int, int, hipStream_t);               \
    template void launch_prep<T>(const Geo*, const StateP<T>&, int, int, int, hipStream_t);               \
    template void launch_finish<T>(const Geo*, const StateP<T>&, int, int, int, hipStream_t);             \
    template void launch_init_stats<T>(const Geo*, const StateP<T>&, int, int, hipStream_t);
CPD_INST_SMALL(float)
CPD_INST_SMALL(double)

}  // namespace cpd
