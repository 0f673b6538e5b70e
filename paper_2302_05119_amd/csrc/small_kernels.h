// Kernels of the sweep's small FP64 work (core update, Grams and step
// matrices with their spectral norms, objective and restart test) and their
// launch templates.  GATE = 1 instantiates the re-done sweep's kernels under
// distinct symbols (k_small_redo.hip).
#pragma once
#include "small_dev.h"

namespace cpd {

template <typename T, int NMAX, int GATE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_core(const Geo* __restrict__ g, StateP<T> st, int extrapolate) {
    if (gated_out(st.ctrl, GATE)) return;
    extern __shared__ char smraw[];
    core_block<T, NMAX>(g, st, blockIdx.x, extrapolate, smraw);
}

template <typename T, int NMAX, int GATE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_prep(const Geo* __restrict__ g, StateP<T> st, int n) {
    if (gated_out(st.ctrl, GATE)) return;
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
template <typename T, int GATE>
__global__ __launch_bounds__(256) void k_finish(const Geo* __restrict__ g, StateP<T> st, int first_sweep) {
    Ctrl* c = st.ctrl;
    if (gated_out(c, GATE)) return;
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

// ---------------------------------------------------------------------------
// launch templates
// ---------------------------------------------------------------------------
#define CPD_NMAX_DISPATCH(R, CALL) \
    do {                              \
        if ((R) <= 16) { CALL(16); }  \
        else if ((R) <= 32) { CALL(32); } \
        else if ((R) <= 48) { CALL(48); } \
        else { CALL(64); }            \
    } while (0)

template <int GATE, typename T>
void core_impl(const Geo* g, const StateP<T>& st, int S, int R, int extrap, hipStream_t q) {
#define CPD_CORE(N) hipLaunchKernelGGL((k_core<T, N, GATE>), dim3(S), dim3(256), eig_lds_bytes(R), q, g, st, extrap)
    CPD_NMAX_DISPATCH(R, CPD_CORE);
#undef CPD_CORE
}
template <int GATE, typename T>
void prep_impl(const Geo* g, const StateP<T>& st, int S, int R, int n, hipStream_t q) {
    const int Rq = (R + 3) / 4 * 4;
#define CPD_PREP(N) hipLaunchKernelGGL((k_prep<T, N, GATE>), dim3(S), dim3(256), prep_lds_bytes<T>(R, Rq), q, g, st, n)
    CPD_NMAX_DISPATCH(R, CPD_PREP);
#undef CPD_PREP
}
template <int GATE, typename T>
void finish_impl(const Geo* g, const StateP<T>& st, int S, int R, int first_sweep, hipStream_t q) {
    const int Rq = (R + 3) / 4 * 4;
    hipLaunchKernelGGL((k_finish<T, GATE>), dim3(S), dim3(256), gram_lds_bytes<T>(R, Rq, 128), q, g, st, first_sweep);
}

#define CPD_SMALL_IMPLS_T(SPEC, G, T)                                                           \
    SPEC void core_impl<G, T>(const Geo*, const StateP<T>&, int, int, int, hipStream_t);        \
    SPEC void prep_impl<G, T>(const Geo*, const StateP<T>&, int, int, int, hipStream_t);        \
    SPEC void finish_impl<G, T>(const Geo*, const StateP<T>&, int, int, int, hipStream_t);
#define CPD_SMALL_IMPLS(SPEC, G) CPD_SMALL_IMPLS_T(SPEC, G, float) CPD_SMALL_IMPLS_T(SPEC, G, double)

}  // namespace cpd
