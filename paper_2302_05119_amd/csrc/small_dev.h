// Device functions of the small FP64 work of a sweep, shared by the stand-alone
// kernels and by the launches that run them beside an MTTKRP pass:
//   - the exact largest eigenvalue of an R x R symmetric matrix (the spectral
//     norms of eq. eqLipsLd / eqLipsLu),
//   - Grams V = U^T U staged through LDS,
//   - the core update (eq. solD) and the step matrix P = D H_{-n} D.
#pragma once
#include "dev_common.h"

namespace cpd {

// Sum over the wavefront of one double per lane, returned to every lane:
// each lane posts its value to LDS and all lanes add the posted values in the
// same order (identical results on every lane).  `buf` holds 64 doubles.
template <int NL>
__device__ __forceinline__ double wave_allsum(double x, double* __restrict__ buf) {
    const int lane = threadIdx.x & 63;
    buf[lane] = x;
    wave_sync();
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
    for (int j = 0; j < NL; j += 4) {
        a0 += buf[j];
        a1 += buf[j + 1];
        a2 += buf[j + 2];
        a3 += buf[j + 3];
    }
    wave_sync();
    return (a0 + a1) + (a2 + a3);
}

// Sturm count (eigenvalues below x) of the tridiagonal (d, e2 = squared
// off-diagonal), for two shifts at once: sign changes of p_0 = 1,
// p_1 = d_0 - x, p_{i+1} = (d_i - x) p_i - e2_{i-1} p_{i-1}.  The tridiagonal
// is scaled to unit size and padded to MM rows with d = 4, e2 = 0 (a padded
// row cannot change the count); every 8 steps the pair (p_i, p_{i-1}) is
// renormalised by a power of two.  Branch-free.
template <int MM, typename DA>
__device__ __forceinline__ void sturm2(const DA& d, const DA& e2, double xa, double xb, int& ca, int& cb) {
    double pma = 1.0, pa = d[0] - xa, pmb = 1.0, pb = d[0] - xb;
    bool na = !(pa > 0.0), nb = !(pb > 0.0);
    int ka = na, kb = nb;
#pragma unroll
    for (int i = 1; i < MM; ++i) {
        const double di = d[i], ei = e2[i - 1];
        const double qa = (di - xa) * pa - ei * pma;
        const double qb = (di - xb) * pb - ei * pmb;
        pma = pa;
        pa = qa;
        pmb = pb;
        pb = qb;
        const bool ga = (pa < 0.0) | ((pa == 0.0) & !na);
        const bool gb = (pb < 0.0) | ((pb == 0.0) & !nb);
        ka += (ga != na);
        kb += (gb != nb);
        na = ga;
        nb = gb;
        if ((i & 7) == 7) {
            const int ea = __builtin_amdgcn_frexp_exp(fmax(fabs(pa), fabs(pma)));
            const int eb = __builtin_amdgcn_frexp_exp(fmax(fabs(pb), fabs(pmb)));
            pa = ldexp(pa, -ea);
            pma = ldexp(pma, -ea);
            pb = ldexp(pb, -eb);
            pmb = ldexp(pmb, -eb);
        }
    }
    ca = ka;
    cb = kb;
}

// 128-point multisection for the largest eigenvalue of the (scaled)
// tridiagonal (d, e2) of size m within [lo, hi].
template <int MM, typename DA>
__device__ __forceinline__ double multisect_top(const DA& d, const DA& e2, int m, double lo, double hi) {
    const int lane = threadIdx.x & 63;
    for (int it = 0; it < 48; ++it) {
        if (!(hi - lo > 4.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)))) break;
        const double h = (hi - lo) * (1.0 / 129.0);
        const double xa = lo + h * (double)(2 * lane + 1), xb = lo + h * (double)(2 * lane + 2);
        int ca, cb;
        sturm2<MM, DA>(d, e2, xa, xb, ca, cb);
        // points in increasing order: (lane 0: xa, xb), (lane 1: xa, xb), ...
        const unsigned long long ua = __ballot(ca >= m), ub = __ballot(cb >= m);
        if ((ua | ub) == 0ull) {
            lo = __shfl(xb, 63, 64);
        } else {
            const int fa = ua ? __ffsll((long long)ua) - 1 : 64;
            const int fb = ub ? __ffsll((long long)ub) - 1 : 64;
            if (fa <= fb) {  // first point reaching m is xa of lane fa; xb of lane fa-1 precedes it
                const double xf = __shfl(xa, fa, 64);
                const double xp = __shfl(xb, fa > 0 ? fa - 1 : 0, 64);
                hi = xf;
                if (fa > 0) lo = xp;
            } else {         // it is xb of lane fb; xa of the same lane precedes it
                hi = __shfl(xb, fb, 64);
                lo = __shfl(xa, fb, 64);
            }
        }
    }
    return 0.5 * (lo + hi);
}

// Largest eigenvalue of the symmetric n x n matrix A (n <= NMAX <= 64, held
// row-major in LDS with row stride ld) with nonnegative entries, computed by
// one wavefront.  Lanczos from the all-ones vector (which overlaps the
// Perron vector of a nonnegative matrix) for up to n + 8 steps, stopping on
// breakdown, builds a tridiagonal T whose largest eigenvalue is that of A;
// 128-point multisection with Sturm counts then brackets it to a few ulps.
// Lane i keeps row i of A in registers.  w: >= 448 doubles of LDS.
template <int NMAX>
__device__ __forceinline__ double wave_sym_lmax_t(const double* __restrict__ A, int n, int ld, double* __restrict__ w) {
    constexpr int MM = NMAX + 8;
    const int lane = threadIdx.x & 63;
    double* __restrict__ qb = w;         // broadcast of the Lanczos vector
    double* __restrict__ rb = w + 64;    // reduction buffer
    double* __restrict__ dl = w + 128;   // alpha_k
    double* __restrict__ el = w + 256;   // beta_k^2
    const int mmax = min(n + 8, MM);
    int m = 0;
    double anorm;
    {
        double row[NMAX];
#pragma unroll
        for (int j = 0; j < NMAX; ++j) row[j] = (lane < n && j < n) ? A[lane * ld + j] : 0.0;
        int bad = 0;
        double amax = 0.0;
#pragma unroll
        for (int j = 0; j < NMAX; ++j) {
            bad |= !isfinite(row[j]);
            amax = fmax(amax, fabs(row[j]));
        }
        if (__ballot(bad)) return __longlong_as_double(0x7ff8000000000000LL);
        anorm = wave_max(amax) * n;  // >= ||A||_2
        if (!(anorm > 0.0)) return 0.0;
        double q = (lane < n) ? 1.0 / sqrt((double)n) : 0.0, qprev = 0.0, beta = 0.0;
        for (int k = 0; k < mmax; ++k) {
            if (k > 0 && !(beta > 1e-14 * anorm)) break;
            qb[lane] = q;
            wave_sync();
            double z0 = 0.0, z1 = 0.0, z2 = 0.0, z3 = 0.0;
#pragma unroll
            for (int j = 0; j < NMAX; j += 4) {
                z0 = fma(row[j], qb[j], z0);
                z1 = fma(row[j + 1], qb[j + 1], z1);
                z2 = fma(row[j + 2], qb[j + 2], z2);
                z3 = fma(row[j + 3], qb[j + 3], z3);
            }
            wave_sync();
            double z = ((z0 + z1) + (z2 + z3)) - beta * qprev;
            const double alpha = wave_allsum<NMAX>(z * q, rb);
            z -= alpha * q;
            const double bn = sqrt(wave_allsum<NMAX>(z * z, rb));
            if (lane == 0) {
                dl[k] = alpha;
                el[k] = bn * bn;
            }
            m = k + 1;
            qprev = q;
            q = (bn > 0.0) ? z / bn : 0.0;
            beta = bn;
        }
    }
    wave_sync();
    // Gershgorin interval of T (lanes over rows), then T scaled to unit size
    double lo = INFINITY, hi = -INFINITY;
    if (lane < m) {
        const double r = (lane > 0 ? sqrt(el[lane - 1]) : 0.0) + (lane + 1 < m ? sqrt(el[lane]) : 0.0);
        lo = dl[lane] - r;
        hi = dl[lane] + r;
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    const double sc = fmax(fabs(lo), fabs(hi));
    if (!(sc > 0.0)) return 0.0;
    const int ke = ilogb(sc);
    lo = ldexp(lo, -ke);
    hi = ldexp(hi, -ke);
    if (NMAX <= 48) {
        double d[MM], e2[MM];
#pragma unroll
        for (int i = 0; i < MM; ++i) {
            d[i] = (i < m) ? ldexp(dl[i], -ke) : 4.0;
            e2[i] = (i + 1 < m) ? ldexp(el[i], -2 * ke) : 0.0;
        }
        return ldexp(multisect_top<MM, double[MM]>(d, e2, m, lo, hi), ke);
    } else {
        wave_sync();
        for (int i = lane; i < MM; i += 64) {
            dl[i] = (i < m) ? ldexp(dl[i], -ke) : 4.0;
            el[i] = (i + 1 < m) ? ldexp(el[i], -2 * ke) : 0.0;
        }
        wave_sync();
        const double* dp = dl;
        const double* ep = el;
        return ldexp(multisect_top<MM, const double*>(dp, ep, m, lo, hi), ke);
    }
}

// Largest eigenvalue of an entrywise nonnegative symmetric n x n matrix A
// (LDS, row stride ld), computed by the whole 256-thread workgroup.
// Repeated squaring S <- S^2 (scaled by powers of two) turns
// x = S 1 into the Perron vector of A; the Collatz-Wielandt bounds
//     min_i (A x)_i / x_i  <=  lambda_max(A)  <=  max_i (A x)_i / x_i,
// rigorous for any nonnegative A and positive x, then give lambda_max once
// they agree to 1e-14.  Rows with a zero diagonal are zero rows of the PSD
// matrix and are left out.  When the bounds do not close (tiny eigengap,
// reducible pattern, a negative entry) the first wavefront falls back to
// wave_sym_lmax_t.  Returns the same value to every thread.
// work: 2 * n * ld + 576 doubles of LDS.
template <int NMAX>
__device__ __forceinline__ double wg_lmax_nonneg(const double* __restrict__ A, int n, int ld, double* __restrict__ work) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double* __restrict__ S0 = work;
    double* __restrict__ S1 = work + (NMAX <= 48 ? n * ld : 0);
    double* __restrict__ xv = S1 + (NMAX <= 48 ? n * ld : 0);   // 64
    double* __restrict__ red = xv + 64;       // 4 waves x 4
    double* __restrict__ res = red + 16;      // result broadcast
    double* __restrict__ wl = res + 16;       // fallback work (448)
    // copy, check sign / finiteness, first scale
    double mx = 0.0;
    int bad = 0;
    for (int e = tid; e < n * n; e += 256) {
        const double a = A[(e / n) * ld + e % n];
        bad |= !(a >= 0.0) | !isfinite(a);
        mx = fmax(mx, a);
        if (NMAX <= 48) S0[(e / n) * ld + e % n] = a;
    }
    mx = wave_max(mx);
    const int anybad = __syncthreads_or(bad);
    if (lane == 0) red[wave] = mx;
    __syncthreads();
    mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    double result = 0.0;
    bool done = false;
    if (!anybad && !(mx > 0.0)) {
        result = 0.0;
        done = true;
    }
    if (NMAX <= 48 && !anybad && !done) {
        int es = __builtin_amdgcn_frexp_exp(mx);  // S0 = A; entries scaled by 2^-es on read
        double* Sa = S0;
        double* Sb = S1;
        for (int it = 0; it < 24 && !done; ++it) {
            // Sb = (Sa 2^-es)^2, the next scale exponent from its maximum
            __syncthreads();
            double m2 = 0.0;
            for (int e = tid; e < n * n; e += 256) {
                const int i = e / n, j = e % n;
                if (j < i) continue;
                const double* ri = Sa + i * ld;
                const double* rj = Sa + j * ld;
                double a0 = 0.0, a1 = 0.0;
                int k = 0;
                for (; k + 1 < n; k += 2) {
                    a0 = fma(ri[k], rj[k], a0);
                    a1 = fma(ri[k + 1], rj[k + 1], a1);
                }
                if (k < n) a0 = fma(ri[k], rj[k], a0);
                const double v = ldexp(a0 + a1, -2 * es);
                Sb[i * ld + j] = v;
                Sb[j * ld + i] = v;
                m2 = fmax(m2, v);
            }
            m2 = wave_max(m2);
            if (lane == 0) red[wave] = m2;
            __syncthreads();
            m2 = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
            es = __builtin_amdgcn_frexp_exp(m2);
            double* t = Sa;
            Sa = Sb;
            Sb = t;
            if (it >= 5 && (it & 3) == 1) {
                // x = S 1 over the support, then the two bounds
                if (tid < n) {
                    double x = 0.0;
                    for (int j = 0; j < n; ++j) x += Sa[tid * ld + j];
                    xv[tid] = x;
                }
                __syncthreads();
                double lo = INFINITY, hi = -INFINITY;
                int miss = 0;
                if (tid < n && A[tid * ld + tid] > 0.0) {
                    double y = 0.0;
                    for (int j = 0; j < n; ++j) y = fma(A[tid * ld + j], xv[j], y);
                    const double x = xv[tid];
                    if (x > 0.0) {
                        lo = y / x;
                        hi = lo;
                    } else {
                        miss = 1;
                    }
                }
                lo = wave_min(lo);
                hi = wave_max(hi);
                const int anymiss = __syncthreads_or(miss);
                if (tid == 0) {
                    red[8] = lo;
                    red[9] = hi;
                }
                __syncthreads();
                lo = red[8];
                hi = red[9];
                if (!anymiss && hi >= lo && hi - lo <= 1e-14 * hi) {
                    result = 0.5 * (lo + hi);
                    done = true;
                }
            }
        }
    }
    if (!done) {
        __syncthreads();
        if (wave == 0) {
            const double v = wave_sym_lmax_t<NMAX>(A, n, ld, wl);
            if (lane == 0) res[0] = v;
        }
        __syncthreads();
        result = res[0];
    }
    __syncthreads();
    return result;
}

// Gram V = U^T U (FP64) of an I x R factor with row stride Rq.  Rows are
// staged through LDS in tiles of `tile` rows; the R(R+1)/2 pair sums
// accumulate in LDS (accl), one owner thread per pair.  All threads of the
// workgroup take part.
template <typename T>
__device__ __forceinline__ void block_gram(const T* __restrict__ U, int I, int R, int Rq, double* __restrict__ out, T* __restrict__ tileb,
                           int tile, double* __restrict__ accl) {
    const int npair = R * (R + 1) / 2;
    const int nt = blockDim.x;
    for (int p = threadIdx.x; p < npair; p += nt) accl[p] = 0.0;
    for (int r0 = 0; r0 < I; r0 += tile) {
        const int nr = min(tile, I - r0);
        __syncthreads();
        for (int e = threadIdx.x; e < nr * Rq; e += nt) tileb[e] = U[(long long)r0 * Rq + e];
        __syncthreads();
        for (int p = threadIdx.x; p < npair; p += nt) {
            int a = 0, rem = p;
            while (rem >= R - a) { rem -= R - a; ++a; }
            const T* ca = tileb + a;
            const T* cb = tileb + a + rem;
            double s0 = 0.0, s1 = 0.0;
            int i = 0;
            for (; i + 1 < nr; i += 2) {
                s0 = fma((double)ca[i * Rq], (double)cb[i * Rq], s0);
                s1 = fma((double)ca[(i + 1) * Rq], (double)cb[(i + 1) * Rq], s1);
            }
            if (i < nr) s0 = fma((double)ca[i * Rq], (double)cb[i * Rq], s0);
            accl[p] += s0 + s1;
        }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < npair; p += nt) {
        int a = 0, rem = p;
        while (rem >= R - a) { rem -= R - a; ++a; }
        const int b = a + rem;
        out[a * R + b] = accl[p];
        out[b * R + a] = accl[p];
    }
    __syncthreads();
}

// LDS (bytes) of the eigenvalue work (matrix, three R-vectors, squaring
// buffers and fallback work) and of the Gram (pair accumulators, row tile).
__host__ __device__ inline size_t eig_lds_bytes(int R) {
    const size_t ld = (size_t)(R | 1);
    return sizeof(double) * ((size_t)R * ld + 192 + (R <= 48 ? 2 * (size_t)R * ld : 0) + 576);
}
__host__ __device__ inline size_t gram_acc_bytes(int R) { return sizeof(double) * (size_t)(R * (R + 1) / 2 + 1); }
template <typename T>
__host__ __device__ inline size_t gram_lds_bytes(int R, int Rq, int tile) {
    return ((gram_acc_bytes(R) + 255) & ~(size_t)255) + sizeof(T) * (size_t)tile * Rq;
}
template <typename T>
__host__ __device__ inline size_t prep_lds_bytes(int R, int Rq) {
    const size_t a = eig_lds_bytes(R), b = gram_lds_bytes<T>(R, Rq, 128);
    return a > b ? a : b;
}

// Core tensor update (eq. solD with the gradient of eq. solapgG at the
// extrapolated point of eq. eqextraPG), then P = D H_{-1} D and its spectral
// norm for the mode-1 update.  All 256 threads of the workgroup take part.
template <typename T, int NMAX>
__device__ __forceinline__ void core_block(const Geo* __restrict__ g, const StateP<T>& st, int s, int extrapolate, char* smraw) {
    const Ctrl* c = st.ctrl;
    const int tid = threadIdx.x;
    const int S = g->S, R = g->R, Rq = g->Rq, ld = R | 1, RR = R * R;
    double* A = (double*)smraw;
    double* lv = A + R * ld;   // lambda_{k-1} | lambda_{k-1} - lambda_{k-2} | new lambda
    double* work = lv + 192;
    const double* V0 = st.V[1] + (0 * S + s) * RR;
    const double* V1 = st.V[1] + (1 * S + s) * RR;
    const double* V2 = st.V[1] + (2 * S + s) * RR;
    for (int i = tid; i < RR; i += 256) A[(i / R) * ld + i % R] = V0[i] * V1[i] * V2[i];
    const double* l1 = st.lam[1] + s * Rq;
    const double* l2 = st.lam[2] + s * Rq;
    double lam1 = 0.0, dlam = 0.0;
    if (tid < 64) {
        lam1 = (tid < R) ? l1[tid] : 0.0;
        dlam = (tid < R) ? lam1 - l2[tid] : 0.0;
        lv[tid] = lam1;
        lv[64 + tid] = dlam;
    }
    __syncthreads();
    // H lam_{k-1} and H (lam_{k-1} - lam_{k-2}); the gradient at the
    // extrapolated point combines them once the weight is known
    double h1 = 0.0, h2 = 0.0;
    if (tid < R)
        for (int r = 0; r < R; ++r) {
            const double h = A[tid * ld + r];
            h1 = fma(h, lv[r], h1);
            h2 = fma(h, lv[64 + r], h2);
        }
    const double Ld = wg_lmax_nonneg<NMAX>(A, R, ld, work);
    const double wd = extrap_weight(extrapolate, c->w_hat, st.Ld_prev[s], Ld, c->delta_w);
    double nl = lam1;
    if (g->upd_core && Ld > 0.0 && tid < R) {
        const double lhat = lam1 + wd * dlam;
        const double gr = (h1 + wd * h2) - st.b[1][s * Rq + tid];
        nl = relu_keep_nan(lhat - gr / Ld);
    }
    if (tid < Rq) st.lam[0][s * Rq + tid] = (tid < R) ? nl : 0.0;
    if (tid < 64) lv[128 + tid] = (tid < R) ? nl : 0.0;
    if (tid == 0) st.Ld_cur[s] = Ld;
    __syncthreads();
    for (int i = tid; i < RR; i += 256) {
        const int r = i / R, cc = i % R;
        const double p = lv[128 + r] * lv[128 + cc] * V1[i] * V2[i];
        st.P[s * RR + i] = p;
        A[r * ld + cc] = p;
    }
    __syncthreads();
    const double Lu = wg_lmax_nonneg<NMAX>(A, R, ld, work);
    if (tid == 0) st.Lu_cur[0 * S + s] = Lu;
}

// Gram of mode n-1 (just updated, slot 0), then P = D H_{-n} D and its spectral
// norm for mode n (modes before n from slot 0, after n from slot 1).  All
// threads of the workgroup enter; the eigenvalue runs on the first wavefront.
template <typename T, int NMAX>
__device__ __forceinline__ void prep_block(const Geo* __restrict__ g, const StateP<T>& st, int s, int n, char* smraw) {
    const int S = g->S, R = g->R, Rq = g->Rq, ld = R | 1, RR = R * R;
    const int m = n - 1;
    double* Vm = st.V[0] + (m * S + s) * RR;
    block_gram<T>(st.U[0] + g->uoff[m][s], g->I[s][m], R, Rq, Vm,
                  (T*)(smraw + ((gram_acc_bytes(R) + 255) & ~(size_t)255)), 128, (double*)smraw);
    __threadfence_block();
    __syncthreads();
    const int tid = threadIdx.x;
    double* A = (double*)smraw;
    double* work = A + R * ld + 192;
    const double* lam = st.lam[0] + s * Rq;
    const double* Va = st.V[0] + (0 * S + s) * RR;
    const double* Vb = (n == 1) ? st.V[1] + (2 * S + s) * RR : st.V[0] + (1 * S + s) * RR;
    for (int i = tid; i < RR; i += 256) {
        const int r = i / R, cc = i % R;
        const double p = lam[r] * lam[cc] * Va[i] * Vb[i];
        st.P[s * RR + i] = p;
        A[r * ld + cc] = p;
    }
    __syncthreads();
    const double Lu = wg_lmax_nonneg<NMAX>(A, R, ld, work);
    if (tid == 0) st.Lu_cur[n * S + s] = Lu;
}

}  // namespace cpd
