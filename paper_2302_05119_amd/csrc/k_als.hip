// Unconstrained CPD of every block by alternating least squares: the paper's
// own compression step of Algorithm 2 (Section III-B; ALS with the RelErr
// stopping rule of Section IV).  One ALS iteration updates the three factors
// in turn, each as the least-squares solution with the other two fixed:
//
//   U~^(n) = K_n H_n^{-1},   K_n = M_(n) U~^{⊙-n},   H_n = ⊛_{m≠n} U~^(m)T U~^(m)
//
// K_n comes from the sweep's MTTKRP passes, run on the ALS factors (held in
// the iterate's current slot while the fit runs), in the same dimension-tree
// order: pass 1 gives K_1 and Y = M x_3 U~^(3); K_2 = Y contracted with the
// new U~^(1); pass 2 gives K_3 from the new U~^(1), U~^(2).  The kernels here
// keep the Gram V_m = U~^(m)T U~^(m) of every factor (FP64, refreshed after
// each solve), form H_n from two of them and its Cholesky factor (one
// workgroup per block), solve the I_n right-hand sides (one lane per row), and
// evaluate RelErr through
//
//   ||M - X~||^2 = ||M||^2 - 2 <K_3, U~^(3)> + 1^T (⊛_m U~^(m)T U~^(m)) 1.
//
// Blocks stop independently: a block whose flag is 0 is skipped.  K_3's chunk
// partials are summed once into the K3 buffer (wide launch) before the mode-3
// solve and the fit read it: a lane summing 100+ partials per entry itself
// would wait on each group of loads in turn.
#include "ksource.h"

namespace cpd {

// V_n = U~^(n)T U~^(n) (R x R, FP64) of every active block, at V + (3 s + n) R^2.
// Thread t owns the pairs e = t + 256 j; rows are staged 32 at a time in LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_als_gram(const Geo* __restrict__ g, StateP<T> st, int n, int R,
                                                  const int* __restrict__ act, double* __restrict__ V) {
    apply_rot(st);
    constexpr int CH = 32;
    const int s = blockIdx.x, Rq = g->Rq, tid = threadIdx.x;
    if (!act[s]) return;
    const int Rs = R;                      // the block's stride in V
    R = min(R, g->rk[s]);                  // its CP rank
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    double* stage = (double*)smraw;        // 32 x R
    const int npair = R * R;
    const int I = g->I[s][n];
    const T* U = st.U[1] + g->uoff[n][s];
    double acc[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[j] = 0.0;
    for (int i0 = 0; i0 < I; i0 += CH) {
        const int nr = min(CH, I - i0);
        __syncthreads();
        for (int e = tid; e < CH * R; e += 256) {
            const int rr = e / R, c = e % R;
            stage[e] = rr < nr ? (double)U[(long long)(i0 + rr) * Rq + c] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int e = tid + 256 * j;
            if (e < npair) {
                const int a = e / R, b = e % R;
                double v = acc[j];
                for (int rr = 0; rr < nr; ++rr) v = fma(stage[rr * R + a], stage[rr * R + b], v);
                acc[j] = v;
            }
        }
    }
    double* out = V + (3LL * s + n) * Rs * Rs;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int e = tid + 256 * j;
        if (e < npair) out[e] = acc[j];
    }
}

// H_n = V_a ⊛ V_b (the kept Grams of the other two modes) and its Cholesky
// factor L (lower, row-major R x R) for every active block; bad[s] = 1 if a
// pivot falls below 1e-13 of its starting diagonal entry or is not finite
// (H_n numerically singular).
__global__ __launch_bounds__(256) void k_als_chol(const Geo* __restrict__ g, int n, int R, const int* __restrict__ act,
                                                  const double* __restrict__ V, double* __restrict__ Lout,
                                                  int* __restrict__ bad) {
    const int s = blockIdx.x, tid = threadIdx.x;
    if (!act[s]) return;
    const long long RR = (long long)R * R;  // per-block storage
    R = min(R, g->rk[s]);
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    double* H = (double*)smraw;            // R x R
    __shared__ int flag;
    __shared__ double diag[CPD_MAXR];
    if (tid == 0) flag = 0;
    const int a = n == 0 ? 1 : 0, b = n == 2 ? 1 : 2;
    const double* Va = V + (3LL * s + a) * RR;
    const double* Vb = V + (3LL * s + b) * RR;
    for (int e = tid; e < R * R; e += 256) H[e] = Va[e] * Vb[e];
    __syncthreads();
    for (int j = tid; j < R; j += 256) diag[j] = H[j * R + j];
    __syncthreads();
    // right-looking Cholesky in place (lower triangle); a pivot below 1e-13 of
    // its starting diagonal entry counts as singular (cond(H) beyond ~1e13)
    for (int j = 0; j < R; ++j) {
        if (tid == 0) {
            const double p = H[j * R + j];
            const bool ok = p > 1e-13 * diag[j] && p <= 1.7976931348623157e308;
            if (!ok) flag = 1;
            H[j * R + j] = ok ? sqrt(p) : 1.0;
        }
        __syncthreads();
        const double d = H[j * R + j];
        for (int i = j + 1 + tid; i < R; i += 256) H[i * R + j] /= d;
        __syncthreads();
        const int m = R - j - 1;
        for (int e = tid; e < m * m; e += 256) {
            const int i = j + 1 + e / m, k = j + 1 + e % m;
            if (k <= i) H[i * R + k] = fma(-H[i * R + j], H[k * R + j], H[i * R + k]);
        }
        __syncthreads();
    }
    double* L = Lout + (long long)s * RR;
    for (int e = tid; e < R * R; e += 256) {
        const int i = e / R, k = e % R;
        L[e] = k <= i ? H[e] : 0.0;
    }
    if (tid == 0 && flag) bad[s] = 1;   // sticky over the modes of an iteration
}

// U~^(n) row i = K_n row i times H_n^{-1}: forward then back substitution with
// L, one lane per row, the lane's vector in LDS column-major (col * 64 + lane).
template <typename T, int KSRC>
__global__ __launch_bounds__(64) void k_als_solve(const Geo* __restrict__ g, StateP<T> st, int n, int R,
                                                  const int* __restrict__ act, const double* __restrict__ Lin) {
    apply_rot(st);
    const int s = blockIdx.y, Rq = g->Rq, lane = threadIdx.x;
    if (!act[s]) return;
    const long long RR = (long long)R * R;
    R = min(R, g->rk[s]);
    const int I = g->I[s][n];
    const int row0 = blockIdx.x * 64;
    if (row0 >= I) return;
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    double* L = (double*)smraw;            // R x R
    double* x = L + R * R;                 // R x 64
    const double* Lg = Lin + (long long)s * RR;
    for (int e = lane; e < R * R; e += 64) L[e] = Lg[e];
    const int i = row0 + lane;
    const int ic = min(i, I - 1);
    if (KSRC == KSRC_PART) {
        const T* K3 = st.K3 + g->koff[s] + (long long)ic * Rq;
        for (int c = 0; c < R; ++c) x[c * 64 + lane] = (double)K3[c];
    } else {
        for (int c = 0; c < R; ++c) x[c * 64 + lane] = k_value<T, KSRC>(g, st, s, ic, c);
    }
    __syncthreads();
    for (int j = 0; j < R; ++j) {
        double v = x[j * 64 + lane];
        for (int l = 0; l < j; ++l) v = fma(-L[j * R + l], x[l * 64 + lane], v);
        x[j * 64 + lane] = v / L[j * R + j];
    }
    for (int j = R - 1; j >= 0; --j) {
        double v = x[j * 64 + lane];
        for (int l = j + 1; l < R; ++l) v = fma(-L[l * R + j], x[l * 64 + lane], v);
        x[j * 64 + lane] = v / L[j * R + j];
    }
    if (i < I) {
        T* U = st.U[1] + g->uoff[n][s] + (long long)i * Rq;
        for (int c = 0; c < R; ++c) U[c] = (T)x[c * 64 + lane];
    }
}

// RelErr of every active block after its mode-3 update (K_3, summed into the
// K3 buffer from pass 2 on the new U~^(1), U~^(2)); xx[s] = ||X~||^2.
// Fixed-order tree reductions.
template <typename T>
__global__ __launch_bounds__(256) void k_als_fit(const Geo* __restrict__ g, StateP<T> st, int R,
                                                 const int* __restrict__ act, const double* __restrict__ V,
                                                 double* __restrict__ relerr, double* __restrict__ xx) {
    apply_rot(st);
    const int s = blockIdx.x, Rq = g->Rq, tid = threadIdx.x;
    if (!act[s]) return;
    const long long RR = (long long)R * R;
    R = min(R, g->rk[s]);
    __shared__ double red[2][256];
    const int I3 = g->I[s][2];
    const T* U3 = st.U[1] + g->uoff[2][s];
    const T* K3 = st.K3 + g->koff[s];
    double ip = 0.0;
    for (long long e = tid; e < (long long)I3 * R; e += 256) {
        const long long i = e / R;
        const int c = (int)(e % R);
        ip = fma((double)K3[i * Rq + c], (double)U3[i * Rq + c], ip);
    }
    const double* V0 = V + 3LL * s * RR;
    const double* V1 = V0 + RR;
    const double* V2 = V1 + RR;
    double hs = 0.0;
    for (int e = tid; e < R * R; e += 256) hs += V0[e] * V1[e] * V2[e];
    red[0][tid] = ip;
    red[1][tid] = hs;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            red[0][tid] += red[0][tid + o];
            red[1][tid] += red[1][tid + o];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double nm = st.normM2[s];
        const double r2 = nm - 2.0 * red[0][0] + red[1][0];
        relerr[s] = nm > 0.0 ? sqrt(fmax(r2, 0.0) / nm) : 0.0;
        xx[s] = red[1][0];
    }
}

// The fitted blocks in Tucker form for the lra path: A_n = U~^(n) (FP64,
// I_n x R), G = super-diagonal ones (R x R x R), ||X~||^2 as the block norm.
template <typename T>
__global__ __launch_bounds__(256) void k_als_export(const Geo* __restrict__ g, StateP<T> st, int R,
                                                    const double* __restrict__ xx) {
    apply_rot(st);
    const int s = blockIdx.y, Rq = g->Rq;
    R = min(R, g->rk[s]);
    double* L = st.lra;
    const long long stride = (long long)gridDim.x * 256;
    for (int n = 0; n < 3; ++n) {
        const int I = g->I[s][n];
        const T* U = st.U[1] + g->uoff[n][s];
        double* A = L + g->aoff[n][s];
        for (long long e = blockIdx.x * 256LL + threadIdx.x; e < (long long)I * R; e += stride) {
            const long long i = e / R;
            const int c = (int)(e % R);
            A[e] = (double)U[i * Rq + c];
        }
    }
    double* G = L + g->goff[s];
    const long long R2 = (long long)R * R;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < R2 * R; e += stride) {
        const long long a = e / R2, b = (e / R) % R, c = e % R;
        G[e] = (a == b && b == c) ? 1.0 : 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) st.normM2[s] = xx[s];
}

template <typename T>
void launch_als_gram(const Geo* g, const StateP<T>& st, int S, int R, int n, const int* act, double* V, hipStream_t q) {
    hipLaunchKernelGGL((k_als_gram<T>), dim3(S), dim3(256), sizeof(double) * 32 * (size_t)R, q, g, st, n, R, act, V);
}

void launch_als_chol(const Geo* g, int S, int R, int n, const int* act, const double* V, double* L, int* bad,
                     hipStream_t q) {
    hipLaunchKernelGGL(k_als_chol, dim3(S), dim3(256), sizeof(double) * (size_t)R * R, q, g, n, R, act, V, L, bad);
}

template <typename T>
void launch_als_solve(const Geo* g, const StateP<T>& st, int S, int R, int n, int Imax, const int* act, const double* L,
                      hipStream_t q) {
    const size_t lds = sizeof(double) * ((size_t)R * R + 64 * (size_t)R);
    const dim3 grid((unsigned)((Imax + 63) / 64), (unsigned)S);
    if (n == 0) hipLaunchKernelGGL((k_als_solve<T, KSRC_K1P>), grid, dim3(64), lds, q, g, st, n, R, act, L);
    else if (n == 1) hipLaunchKernelGGL((k_als_solve<T, KSRC_K2>), grid, dim3(64), lds, q, g, st, n, R, act, L);
    else hipLaunchKernelGGL((k_als_solve<T, KSRC_PART>), grid, dim3(64), lds, q, g, st, n, R, act, L);
}

template <typename T>
void launch_als_fit(const Geo* g, const StateP<T>& st, int S, int R, const int* act, const double* V, double* relerr,
                    double* xx, hipStream_t q) {
    hipLaunchKernelGGL((k_als_fit<T>), dim3(S), dim3(256), 0, q, g, st, R, act, V, relerr, xx);
}

template <typename T>
void launch_als_export(const Geo* g, const StateP<T>& st, int S, int R, const double* xx, hipStream_t q) {
    hipLaunchKernelGGL((k_als_export<T>), dim3(64, S), dim3(256), 0, q, g, st, R, xx);
}

#define CPD_ALS_INST(T)                                                                                              \
    template void launch_als_gram<T>(const Geo*, const StateP<T>&, int, int, int, const int*, double*, hipStream_t);    \
    template void launch_als_solve<T>(const Geo*, const StateP<T>&, int, int, int, int, const int*, const double*,      \
                                      hipStream_t);                                                                  \
    template void launch_als_fit<T>(const Geo*, const StateP<T>&, int, int, const int*, const double*, double*, double*, \
                                    hipStream_t);                                                                    \
    template void launch_als_export<T>(const Geo*, const StateP<T>&, int, int, const double*, hipStream_t);
CPD_ALS_INST(float)
CPD_ALS_INST(double)

}  // namespace cpd
