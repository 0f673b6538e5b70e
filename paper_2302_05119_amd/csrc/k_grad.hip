// Loss F and its partial gradients at an arbitrary point (the autograd form):
//   dF/dlambda^(s) = H lambda - b                    (eq. solbpgG)
//   dF/dU^(n,s)    = U P_n - K_n diag(lambda),  P_n = lambda lambda^T ⊛ H_{-n}
//                                                    (eq. solbpgU)
// with K_n = M_(n) U^{⊙-n} from the dense MTTKRP passes run on the given point
// (every slot of the state copy addresses it), b = colsum(K_3 ⊛ U_3) and
// F = 1/2 (||M||^2 - 2 lambda^T b + lambda^T H lambda) per block.
#include "small_dev.h"
#include "ksource.h"

namespace cpd {

// Per block: Grams of the three factors, b, g_lambda, F, and P_n for n = 0..2.
template <typename T>
__global__ __launch_bounds__(256) void k_grad_block(const Geo* __restrict__ g, StateP<T> st, double* const* __restrict__ glam,
                                                    double* __restrict__ Fblk) {
    const int s = blockIdx.x, tid = threadIdx.x;
    const int S = g->S, R = g->R, Rq = g->Rq, RR = R * R;
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    double* V0 = st.V[0] + (0 * S + s) * RR;
    double* V1 = st.V[0] + (1 * S + s) * RR;
    double* V2 = st.V[0] + (2 * S + s) * RR;
    double* b = st.b[0] + s * Rq;
    block_gram<T>(st.U[0] + g->uoff[0][s], g->I[s][0], R, Rq, V0, nullptr, nullptr, smraw);
    block_gram<T>(st.U[0] + g->uoff[1][s], g->I[s][1], R, Rq, V1, nullptr, nullptr, smraw);
    block_gram<T>(st.U[0] + g->uoff[2][s], g->I[s][2], R, Rq, V2, st.K3 + g->koff[s], b, smraw);
    __threadfence_block();
    __syncthreads();
    const double* lam = st.lam[0] + s * Rq;
    if (tid < R) {
        double h = 0.0;
        for (int r = 0; r < R; ++r) h = fma(V0[tid * R + r] * V1[tid * R + r] * V2[tid * R + r], lam[r], h);
        glam[s][tid] = h - b[tid];
    }
    const double F = block_objective(lam, V0, V1, V2, b, st.normM2[s], R);
    if (tid == 0) Fblk[s] = F;
    for (int i = tid; i < RR; i += 256) {
        const double ll = lam[i / R] * lam[i % R];
        st.P[(0 * S + s) * RR + i] = ll * V1[i] * V2[i];
        st.P[(1 * S + s) * RR + i] = ll * V0[i] * V2[i];
        st.P[(2 * S + s) * RR + i] = ll * V0[i] * V1[i];
    }
}

// Gradient of every factor of mode n: one thread per element (i, c) of one
// block (grid.y = block), written I_n x R row-major to out[s].
template <typename T, int KSRC>
__global__ __launch_bounds__(256) void k_grad_u(const Geo* __restrict__ g, StateP<T> st, int n, T* const* __restrict__ out) {
    const int s = blockIdx.y;
    const int S = g->S, R = g->R, Rq = g->Rq, RR = R * R, I = g->I[s][n];
    const long long e = blockIdx.x * 256LL + threadIdx.x;
    if (e >= (long long)I * R) return;
    const int i = (int)(e / R), c = (int)(e % R);
    const T* u = st.U[0] + g->uoff[n][s] + (long long)i * Rq;
    const double* P = st.P + (long long)(n * S + s) * RR;
    double g0 = 0.0, g1 = 0.0;
    int r = 0;
    for (; r + 1 < R; r += 2) {
        g0 = fma((double)u[r], P[r * R + c], g0);
        g1 = fma((double)u[r + 1], P[(r + 1) * R + c], g1);
    }
    if (r < R) g0 = fma((double)u[r], P[r * R + c], g0);
    const double kv = k_value<T, KSRC>(g, st, s, i, c);
    out[s][e] = (T)((g0 + g1) - kv * st.lam[0][s * Rq + c]);
}

// Shared columns of a coupled mode: the gradient with respect to U_C is the
// sum over the mode's coupling group (block order), written to every member.
template <typename T>
__global__ __launch_bounds__(256) void k_grad_shared(const Geo* __restrict__ g, int n, T* const* __restrict__ out) {
    const int R = g->R, Ln = g->L[n], ng = g->ngrp[n];
    const int* grp = g->grp[n];
    const int I = g->I[grp[0]][n];
    const long long e = blockIdx.x * 256LL + threadIdx.x;
    if (e >= (long long)I * Ln) return;
    const long long o = (e / Ln) * R + e % Ln;
    double acc = 0.0;
    for (int k = 0; k < ng; ++k) acc += (double)out[grp[k]][o];
    for (int k = 0; k < ng; ++k) out[grp[k]][o] = (T)acc;
}

// In: largest I_n over the blocks, per mode.
template <typename T>
void launch_grad(const Geo* g, const StateP<T>& st, int S, int R, int Rq, const int* In, int L0, int L1, int L2,
                 double* const* glam, double* Fblk, T* const* gU0, T* const* gU1, T* const* gU2, int coupled, hipStream_t q) {
    hipLaunchKernelGGL(k_grad_block<T>, dim3(S), dim3(256), gram_lds_bytes<T>(Rq, 1), q, g, st, glam, Fblk);
    T* const* gU[3] = {gU0, gU1, gU2};
    const int L[3] = {L0, L1, L2};
    for (int n = 0; n < 3; ++n) {
        const unsigned nb = (unsigned)((In[n] * (long long)R + 255) / 256);
        if (n == 0) hipLaunchKernelGGL((k_grad_u<T, KSRC_K1P>), dim3(nb, S), dim3(256), 0, q, g, st, n, gU[n]);
        else if (n == 1) hipLaunchKernelGGL((k_grad_u<T, KSRC_K2>), dim3(nb, S), dim3(256), 0, q, g, st, n, gU[n]);
        else hipLaunchKernelGGL((k_grad_u<T, KSRC_PART>), dim3(nb, S), dim3(256), 0, q, g, st, n, gU[n]);
        if (coupled && L[n] > 0) {
            const unsigned nb2 = (unsigned)((In[n] * (long long)L[n] + 255) / 256);
            hipLaunchKernelGGL(k_grad_shared<T>, dim3(nb2), dim3(256), 0, q, g, n, gU[n]);
        }
    }
}
template void launch_grad<float>(const Geo*, const StateP<float>&, int, int, int, const int*, int, int, int, double* const*,
                                 double*, float* const*, float* const*, float* const*, int, hipStream_t);
template void launch_grad<double>(const Geo*, const StateP<double>&, int, int, int, const int*, int, int, int, double* const*,
                                  double*, double* const*, double* const*, double* const*, int, hipStream_t);

}  // namespace cpd
