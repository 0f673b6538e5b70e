// Small FP64 kernels of the sweep: Hadamard products of Grams, exact spectral
// norms, the core (lambda) update, the objective / restart test and the
// commit of an accepted iterate.  One workgroup per block for the R x R work.
#include "dev_common.h"

namespace cpd {

// ---------------------------------------------------------------------------
// Largest eigenvalue of a symmetric n x n matrix (n <= 64) held row-major in
// LDS (row stride ld).  Executed by one wavefront: Householder reduction to
// tridiagonal form, then Sturm-count multisection (64 shifts per round) on the
// tridiagonal.  This is the spectral norm of eq. eqLipsLd / eqLipsLu for the
// PSD matrices used there; A is overwritten.  `w` is >= 320 doubles of LDS.
// ---------------------------------------------------------------------------
__device__ double wave_sym_lmax(double* A, int n, int ld, double* w) {
    const int lane = threadIdx.x & 63;
    double* v = w;
    double* q = w + 64;
    double* d = w + 128;
    double* e2 = w + 192;
    double* ea = w + 256;

    int bad = 0;
    for (int i = lane; i < n * n; i += 64) {
        double x = A[(i / n) * ld + (i % n)];
        bad |= !isfinite(x);
    }
    if (__ballot(bad)) return __longlong_as_double(0x7ff8000000000000LL);
    if (n == 1) return A[0];

    for (int k = 0; k + 2 < n; ++k) {
        const double x = (lane > k && lane < n) ? A[lane * ld + k] : 0.0;
        const double sig = wave_sum(x * x);
        const double dk = A[k * ld + k];
        if (sig == 0.0) {
            if (lane == 0) { d[k] = dk; e2[k] = 0.0; ea[k] = 0.0; }
            wave_sync();
            continue;
        }
        const double x0 = __shfl(x, k + 1, 64);
        const double alpha = (x0 >= 0.0) ? -sqrt(sig) : sqrt(sig);
        const double vn = sqrt(2.0 * (sig - alpha * x0));
        const double vi = (x - ((lane == k + 1) ? alpha : 0.0)) / vn;
        v[lane] = vi;
        wave_sync();
        double p = 0.0;
        if (lane > k && lane < n) {
            const double* row = A + lane * ld;
            for (int j = k + 1; j < n; ++j) p += row[j] * v[j];
        }
        const double K = wave_sum(vi * p);
        const double qi = p - K * vi;
        q[lane] = qi;
        wave_sync();
        if (lane > k && lane < n) {
            double* row = A + lane * ld;
            for (int j = k + 1; j < n; ++j) row[j] -= 2.0 * (vi * q[j] + qi * v[j]);
        }
        if (lane == 0) { d[k] = dk; e2[k] = alpha * alpha; ea[k] = fabs(alpha); }
        wave_sync();
    }
    if (lane == 0) {
        d[n - 2] = A[(n - 2) * ld + n - 2];
        d[n - 1] = A[(n - 1) * ld + n - 1];
        const double e = A[(n - 1) * ld + n - 2];
        e2[n - 2] = e * e;
        ea[n - 2] = fabs(e);
    }
    wave_sync();

    // Gershgorin interval of the tridiagonal
    double lo = INFINITY, hi = -INFINITY;
    if (lane < n) {
        const double r = (lane > 0 ? ea[lane - 1] : 0.0) + (lane < n - 1 ? ea[lane] : 0.0);
        lo = d[lane] - r;
        hi = d[lane] + r;
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    for (int it = 0; it < 64; ++it) {
        if (!(hi - lo > 4.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)))) break;
        const double x = lo + (hi - lo) * ((double)(lane + 1) / 65.0);
        // number of eigenvalues below x = negative pivots of T - x I = L D L^T
        double piv = d[0] - x;
        int cnt = piv < 0.0;
        for (int i = 1; i < n; ++i) {
            if (piv == 0.0) piv = -DBL_MIN;
            piv = (d[i] - x) - e2[i - 1] / piv;
            cnt += piv < 0.0;
        }
        const unsigned long long above = __ballot(cnt >= n);
        if (above == 0ull) {
            lo = __shfl(x, 63, 64);
        } else {
            const int f = __ffsll((long long)above) - 1;
            const double xf = __shfl(x, f, 64);
            const double xp = __shfl(x, f > 0 ? f - 1 : 0, 64);
            hi = xf;
            if (f > 0) lo = xp;
        }
    }
    return 0.5 * (lo + hi);
}

// ---------------------------------------------------------------------------
// Core tensor update (eq. solD with the gradient of eq. solapgG at the
// extrapolated point of eq. eqextraPG) and the mode-1 step matrix
// P = D H_{-1} D with its spectral norm.  One 64-thread workgroup per block.
// b (the data term (U^⊙)^T vec(M)) is the value kept from the previous sweep.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void k_core(const Geo* __restrict__ g, StateP<T> st, int extrapolate, int gate) {
    const Ctrl* c = st.ctrl;
    if (gated_out(c, gate)) return;
    const int s = blockIdx.x, lane = threadIdx.x;
    const int S = g->S, R = g->R, Rq = g->Rq, ld = R | 1, RR = R * R;
    extern __shared__ double sm[];
    double* A = sm;
    double* w = A + R * ld;
    double* lh = w + 320;
    double* ln = lh + 64;

    const double* V0 = st.V[1] + (0 * S + s) * RR;
    const double* V1 = st.V[1] + (1 * S + s) * RR;
    const double* V2 = st.V[1] + (2 * S + s) * RR;
    for (int i = lane; i < RR; i += 64) A[(i / R) * ld + i % R] = V0[i] * V1[i] * V2[i];
    wave_sync();
    const double Ld = wave_sym_lmax(A, R, ld, w);

    const double* l1 = st.lam[1] + s * Rq;
    const double* l2 = st.lam[2] + s * Rq;
    const double wd = extrap_weight(extrapolate, c->w_hat, st.Ld_prev[s], Ld, c->delta_w);
    if (lane < R) lh[lane] = l1[lane] + wd * (l1[lane] - l2[lane]);
    wave_sync();
    double nl = (lane < R) ? l1[lane] : 0.0;
    if (g->upd_core && Ld > 0.0 && lane < R) {
        double gr = -st.b[1][s * Rq + lane];
        for (int r = 0; r < R; ++r) {
            const int i = lane * R + r;
            gr += V0[i] * V1[i] * V2[i] * lh[r];
        }
        nl = relu_keep_nan(lh[lane] - gr / Ld);
    }
    if (lane < Rq) st.lam[0][s * Rq + lane] = (lane < R) ? nl : 0.0;
    if (lane < 64) ln[lane] = (lane < R) ? nl : 0.0;
    if (lane == 0) st.Ld_cur[s] = Ld;
    wave_sync();
    for (int i = lane; i < RR; i += 64) {
        const int r = i / R, cc = i % R;
        const double p = ln[r] * ln[cc] * V1[i] * V2[i];
        st.P[s * RR + i] = p;
        A[r * ld + cc] = p;
    }
    wave_sync();
    const double Lu = wave_sym_lmax(A, R, ld, w);
    if (lane == 0) st.Lu_cur[0 * S + s] = Lu;
}

// Gram V = U^T U of one factor (I rows, row stride Rq) into LDS/global, FP64.
template <typename T>
__device__ void block_gram(const T* __restrict__ U, int I, int R, int Rq, double* __restrict__ out) {
    const int npair = R * (R + 1) / 2;
    for (int p = threadIdx.x; p < npair; p += blockDim.x) {
        // (a, b) with a <= b from the packed index
        int a = 0, rem = p;
        while (rem >= R - a) { rem -= R - a; ++a; }
        const int b = a + rem;
        double acc = 0.0;
        for (int i = 0; i < I; ++i) acc += (double)U[(long long)i * Rq + a] * (double)U[(long long)i * Rq + b];
        out[a * R + b] = acc;
        out[b * R + a] = acc;
    }
}

// Gram of the mode just updated, then P = D H_{-n} D and its spectral norm for
// mode n.  Modes before n take slot 0 (this sweep), after n slot 1.
template <typename T>
__global__ __launch_bounds__(256) void k_prep(const Geo* __restrict__ g, StateP<T> st, int n, int gate) {
    const Ctrl* c = st.ctrl;
    if (gated_out(c, gate)) return;
    const int s = blockIdx.x;
    const int S = g->S, R = g->R, Rq = g->Rq, ld = R | 1, RR = R * R;
    extern __shared__ double sm[];
    double* A = sm;
    double* w = A + R * ld;
    const int m = n - 1;
    double* Vm = st.V[0] + (m * S + s) * RR;
    block_gram<T>(st.U[0] + g->uoff[m][s], g->I[s][m], R, Rq, Vm);
    __syncthreads();
    if (threadIdx.x >= 64) return;
    const int lane = threadIdx.x;
    const double* lam = st.lam[0] + s * Rq;
    const double* Va = st.V[0] + (0 * S + s) * RR;           // mode 0: updated
    const double* Vb = (n == 1) ? st.V[1] + (2 * S + s) * RR  // mode 2: not yet
                                : st.V[0] + (1 * S + s) * RR; // mode 1: updated
    for (int i = lane; i < RR; i += 64) {
        const int r = i / R, cc = i % R;
        const double p = lam[r] * lam[cc] * Va[i] * Vb[i];
        st.P[s * RR + i] = p;
        A[r * ld + cc] = p;
    }
    wave_sync();
    const double Lu = wave_sym_lmax(A, R, ld, w);
    if (lane == 0) st.Lu_cur[n * S + s] = Lu;
}

// After the mode-3 update: Gram of U^(3), b = colsum(K3 ⊛ U^(3)) (the data term
// (U^⊙)^T vec(M) of eq. solapgG, reused by the next core update), and
// F^(s) = 1/2 (||M||^2 - 2 lam^T b + lam^T H lam) (eq. costfunc expanded).  The
// last workgroup sums F over the blocks in block order and, for the
// extrapolated sweep, raises the restart flag when F_k >= F_{k-1} (Algorithm 1).
template <typename T>
__global__ __launch_bounds__(256) void k_finish(const Geo* __restrict__ g, StateP<T> st, int first_sweep, int gate) {
    Ctrl* c = st.ctrl;
    if (gated_out(c, gate)) return;
    const int s = blockIdx.x, tid = threadIdx.x;
    const int S = g->S, R = g->R, Rq = g->Rq, RR = R * R;
    __shared__ double bsh[CPD_MAXR];
    __shared__ double red[256];
    __shared__ int last;
    double* V2 = st.V[0] + (2 * S + s) * RR;
    const T* U3 = st.U[0] + g->uoff[2][s];
    const int I3 = g->I[s][2];
    block_gram<T>(U3, I3, R, Rq, V2);
    const T* K3 = st.K3 + g->koff[s];
    if (tid < R) {
        double acc = 0.0;
        for (int i = 0; i < I3; ++i) acc += (double)K3[(long long)i * Rq + tid] * (double)U3[(long long)i * Rq + tid];
        bsh[tid] = acc;
        st.b[0][s * Rq + tid] = acc;
    }
    __syncthreads();
    const double* lam = st.lam[0] + s * Rq;
    const double* V0 = st.V[0] + (0 * S + s) * RR;
    const double* V1 = st.V[0] + (1 * S + s) * RR;
    double part = 0.0;
    for (int i = tid; i < RR; i += 256) part += lam[i / R] * lam[i % R] * V0[i] * V1[i] * V2[i];
    red[tid] = part;
    __syncthreads();
    if (tid == 0) {
        double quad = 0.0;
        for (int i = 0; i < 256; ++i) quad += red[i];
        double lb = 0.0;
        for (int r = 0; r < R; ++r) lb += lam[r] * bsh[r];
        st.Fblk[s] = 0.5 * (st.normM2[s] - 2.0 * lb + quad);
        __threadfence();
        last = (atomicAdd(&c->counter_finish, 1u) == (unsigned)(gridDim.x - 1));
    }
    __syncthreads();
    if (!last || tid != 0) return;
    __threadfence();
    double F = 0.0, rel = 0.0;
    for (int b = 0; b < S; ++b) {
        const double fb = load_agent(&st.Fblk[b]);
        F += fb;
        rel += sqrt(fmax(0.0, 2.0 * fb)) / sqrt(st.normM2[b]);
    }
    rel /= S;
    c->F_cur = F;
    c->rel_cur = rel;
    c->nonfinite = !isfinite(F);
    if (first_sweep) c->redo = (c->restart_on && F >= c->F_prev) ? 1 : 0;
    c->counter_finish = 0u;
}

// Accept the sweep: x_{k-2} <- x_{k-1}, x_{k-1} <- x_k for factors and lambda,
// Grams and b to slot 1.  The last workgroup advances k and t, keeps the
// Lipschitz constants of the accepted sweep and applies the stopping rule.
template <typename T>
__global__ __launch_bounds__(256) void k_commit(const Geo* __restrict__ g, StateP<T> st, long long uslot) {
    Ctrl* c = st.ctrl;
    if (c->stop) return;
    const int S = g->S, R = g->R, Rq = g->Rq;
    const long long nl = (long long)S * Rq, nv = 3LL * S * R * R, nb = (long long)S * Rq;
    const long long total = uslot + nl + nv + nb;
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
        } else {
            const long long j = i - uslot - nl - nv;
            st.b[1][j] = st.b[0][j];
        }
    }
    __shared__ int last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = (atomicAdd(&c->counter_commit, 1u) == (unsigned)(gridDim.x - 1));
    }
    __syncthreads();
    if (!last || threadIdx.x != 0) return;
    __threadfence();
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
    for (int b = 0; b < S; ++b) st.Ld_prev[b] = st.Ld_cur[b];
    for (int n = 0; n < 3; ++n) {
        double LC = 0.0;
        for (int b = 0; b < S; ++b) {
            st.Lu_prev[n * S + b] = st.Lu_cur[n * S + b];
            LC += st.Lu_cur[n * S + b];
        }
        st.LC_prev[n] = LC;
    }
    if (c->tol > 0.0 && fabs(c->rel_cur - rel_old) < c->tol) c->stop = 1;
    c->redo = 0;
    c->counter_commit = 0u;
}

// Initial (or restored) iterate in slot 1: Grams of every factor, b from the
// reduced mode-3 MTTKRP, F and RelErr; sets F_prev / rel_prev.
template <typename T>
__global__ __launch_bounds__(256) void k_init_stats(const Geo* __restrict__ g, StateP<T> st) {
    Ctrl* c = st.ctrl;
    const int s = blockIdx.x, tid = threadIdx.x;
    const int S = g->S, R = g->R, Rq = g->Rq, RR = R * R;
    __shared__ double bsh[CPD_MAXR];
    __shared__ double red[256];
    __shared__ int last;
    for (int m = 0; m < 3; ++m) block_gram<T>(st.U[1] + g->uoff[m][s], g->I[s][m], R, Rq, st.V[1] + (m * S + s) * RR);
    const T* U3 = st.U[1] + g->uoff[2][s];
    const T* K3 = st.K3 + g->koff[s];
    const int I3 = g->I[s][2];
    if (tid < R) {
        double acc = 0.0;
        for (int i = 0; i < I3; ++i) acc += (double)K3[(long long)i * Rq + tid] * (double)U3[(long long)i * Rq + tid];
        bsh[tid] = acc;
        st.b[1][s * Rq + tid] = acc;
    }
    __syncthreads();
    const double* lam = st.lam[1] + s * Rq;
    const double* V0 = st.V[1] + (0 * S + s) * RR;
    const double* V1 = st.V[1] + (1 * S + s) * RR;
    const double* V2 = st.V[1] + (2 * S + s) * RR;
    double part = 0.0;
    for (int i = tid; i < RR; i += 256) part += lam[i / R] * lam[i % R] * V0[i] * V1[i] * V2[i];
    red[tid] = part;
    __syncthreads();
    if (tid == 0) {
        double quad = 0.0;
        for (int i = 0; i < 256; ++i) quad += red[i];
        double lb = 0.0;
        for (int r = 0; r < R; ++r) lb += lam[r] * bsh[r];
        st.Fblk[s] = 0.5 * (st.normM2[s] - 2.0 * lb + quad);
        __threadfence();
        last = (atomicAdd(&c->counter_aux, 1u) == (unsigned)(gridDim.x - 1));
    }
    __syncthreads();
    if (!last || tid != 0) return;
    __threadfence();
    double F = 0.0, rel = 0.0;
    for (int b = 0; b < S; ++b) {
        const double fb = load_agent(&st.Fblk[b]);
        F += fb;
        rel += sqrt(fmax(0.0, 2.0 * fb)) / sqrt(st.normM2[b]);
    }
    c->F_prev = F;
    c->F_cur = F;
    c->rel_prev = rel / S;
    c->rel_cur = rel / S;
    c->nonfinite = !isfinite(F);
    c->counter_aux = 0u;
}


// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static size_t eig_lds(int R) { return sizeof(double) * ((size_t)R * (R | 1) + 320); }

template <typename T>
void launch_core(const Geo* g, const StateP<T>& st, int S, int R, int extrap, int gate, hipStream_t q) {
    const size_t lds = eig_lds(R) + sizeof(double) * 128;
    hipLaunchKernelGGL(k_core<T>, dim3(S), dim3(64), lds, q, g, st, extrap, gate);
}
template <typename T>
void launch_prep(const Geo* g, const StateP<T>& st, int S, int R, int n, int gate, hipStream_t q) {
    hipLaunchKernelGGL(k_prep<T>, dim3(S), dim3(256), eig_lds(R), q, g, st, n, gate);
}
template <typename T>
void launch_finish(const Geo* g, const StateP<T>& st, int S, int R, int first_sweep, int gate, hipStream_t q) {
    (void)R;
    hipLaunchKernelGGL(k_finish<T>, dim3(S), dim3(256), 0, q, g, st, first_sweep, gate);
}
template <typename T>
void launch_commit(const Geo* g, const StateP<T>& st, long long uslot, int S, int Rq, int R, hipStream_t q) {
    const long long total = uslot + (long long)S * Rq * 2 + 3LL * S * R * R;
    long long nb = (total + 255) / 256;
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_commit<T>, dim3((unsigned)nb), dim3(256), 0, q, g, st, uslot);
}
template <typename T>
void launch_init_stats(const Geo* g, const StateP<T>& st, int S, int R, hipStream_t q) {
    (void)R;
    hipLaunchKernelGGL(k_init_stats<T>, dim3(S), dim3(256), 0, q, g, st);
}

#define CPD_INST_SMALL(T)                                                                                  \
    template void launch_core<T>(const Geo*, const StateP<T>&, int, int, int, int, hipStream_t);          \
    template void launch_prep<T>(const Geo*, const StateP<T>&, int, int, int, int, hipStream_t);          \
    template void launch_finish<T>(const Geo*, const StateP<T>&, int, int, int, int, hipStream_t);        \
    template void launch_commit<T>(const Geo*, const StateP<T>&, long long, int, int, int, hipStream_t);  \
    template void launch_init_stats<T>(const Geo*, const StateP<T>&, int, int, hipStream_t);
CPD_INST_SMALL(float)
CPD_INST_SMALL(double)

}  // namespace cpd
