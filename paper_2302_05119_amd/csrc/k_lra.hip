// Low-rank-approximation path (Algorithm 2, Section III-B).
//
// Compression (once per block): truncated HOSVD
//   Sigma_n = M_(n) M_(n)^T                     (mode Grams, FP64)
//   A_n     = J_n leading eigenvectors of Sigma_n (tridiagonalisation,
//             bisection, inverse iteration)
//   G       = M x_1 A_1^T x_2 A_2^T x_3 A_3^T   (TTM chain, FP64)
// Only the subspace matters: the compressed tensor X~ = G x_n A_n, and with
// it every quantity the iterations use, is invariant to the basis chosen.
//
// Iterations: the data terms of eq. solapgU / solapgG in Tucker form
//   W_m = A_m^T U^(m)                      (J_m x R)
//   C_n = G_(n) (⊙_{m != n} W_m)           (J_n x R)
//   K_n = A_n C_n,  b = colsum(K_3 ⊛ U^(3)) = colsum(C_3 ⊛ W_3)
// (with G super-diagonal of ones and A_n = U~^(n) this is eq. eqlrau /
// eq. eqlrag).  K_n is formed inside the factor-update kernel.
#include "lra_items.h"

namespace cpd {

// ---------------------------------------------------------------------------
// Mode Gram Sigma_n[a][b] = sum_t X_n(a, t) X_n(b, t) of one block, as a tiled
// SYRK on the FP64 matrix cores: a 64 x 64 output tile per workgroup (upper
// triangle of tiles only), a 32 x 32 quarter per wavefront (2 x 2 tiles of
// v_mfma_f64_16x16x4f64), the contraction index t staged through LDS in
// chunks of 32 (the next chunk's loads in flight while the current one is
// consumed).  Products and sums are FP64 (the FP32 inputs convert exactly),
// so the Gram carries no rounding beyond FP64 summation.
// Element (a, t) of the unfolding sits at
//   mode 0: a*I2*I3 + t                        (t = i2*I3 + i3)
//   mode 1: (t / I3)*I2*I3 + a*I3 + t % I3     (t = i1*I3 + i3)
//   mode 2: t*I3 + a                           (t = i1*I2 + i2)
// (every index fits 32 bits: I_n <= 512).  A split-K grid dimension
// (blockIdx.y) writes partial tiles, summed later.
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long unfold_addr(int mode, int a, unsigned t, int I2, int I3) {
    if (mode == 0) return (long long)a * I2 * I3 + t;
    if (mode == 1) return (long long)(t / (unsigned)I3) * I2 * I3 + (long long)a * I3 + (t % (unsigned)I3);
    return (long long)t * I3 + a;
}

__global__ __launch_bounds__(256) void k_mode_gram(const float* __restrict__ X, int mode, int I1, int I2, int I3,
                                                   int ntile, double* __restrict__ part) {
    const int In = mode == 0 ? I1 : (mode == 1 ? I2 : I3);
    const unsigned T = (unsigned)((long long)I1 * I2 * I3 / In);
    // tile pair (ta <= tb) from blockIdx.x
    int ta = 0, rem = blockIdx.x;
    while (rem >= ntile - ta) { rem -= ntile - ta; ++ta; }
    const int tb = ta + rem;
    const int nsplit = gridDim.y, sp = blockIdx.y;
    const unsigned tb0 = (unsigned)((long long)T * sp / nsplit), tb1 = (unsigned)((long long)T * (sp + 1) / nsplit);
    __shared__ double sa[32][66];
    __shared__ double sb[32][66];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;   // the wavefront's quarter of the tile
    const int li = lane & 15, lk = lane >> 4;
    v4d acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};
    // staging: 8 elements of each operand per thread; the fastest-varying
    // thread index follows the contiguous direction
    float na[8], nb[8];
    auto load = [&](unsigned t0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + 256 * q;
            const int r = mode == 2 ? (e & 63) : (e >> 5);
            const int k = mode == 2 ? (e >> 6) : (e & 31);
            const unsigned t = t0 + k;
            const int ra = ta * 64 + r, rb = tb * 64 + r;
            const bool tin = t < tb1;
            na[q] = (ra < In && tin) ? X[unfold_addr(mode, ra, t, I2, I3)] : 0.0f;
            nb[q] = (rb < In && tin) ? X[unfold_addr(mode, rb, t, I2, I3)] : 0.0f;
        }
    };
    if (tb0 < tb1) load(tb0);
    for (unsigned t0 = tb0; t0 < tb1; t0 += 32) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + 256 * q;
            const int r = mode == 2 ? (e & 63) : (e >> 5);
            const int k = mode == 2 ? (e >> 6) : (e & 31);
            sa[k][r] = (double)na[q];
            sb[k][r] = (double)nb[q];
        }
        __syncthreads();
        if (t0 + 32 < tb1) load(t0 + 32);
#pragma unroll
        for (int k0 = 0; k0 < 32; k0 += 4) {
            // lane l: A[l % 16][l / 16] = X_a(row, k0 + l / 16), B likewise
            const double a0 = sa[k0 + lk][wr + li], a1 = sa[k0 + lk][wr + 16 + li];
            const double b0 = sb[k0 + lk][wc + li], b1 = sb[k0 + lk][wc + 16 + li];
            acc[0][0] = mfma64(a0, b0, acc[0][0]);
            acc[0][1] = mfma64(a0, b1, acc[0][1]);
            acc[1][0] = mfma64(a1, b0, acc[1][0]);
            acc[1][1] = mfma64(a1, b1, acc[1][1]);
        }
        __syncthreads();
    }
    // partial tile sp of Sigma (full In x In storage, both triangles; on a
    // diagonal tile the mirrored writes carry identical values).  Register v of
    // lane l holds D[4v + l / 16][l % 16].
    double* out = part + (long long)sp * In * In;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int a = ta * 64 + wr + 16 * i + 4 * v + lk, b = tb * 64 + wc + 16 * j + li;
                if (a < In && b < In) {
                    out[(long long)a * In + b] = acc[i][j][v];
                    out[(long long)b * In + a] = acc[i][j][v];
                }
            }
}

__global__ __launch_bounds__(256) void k_sum_split(const double* __restrict__ part, int nsplit, long long n,
                                                   double* __restrict__ out) {
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        double a = 0.0;
        for (int p = 0; p < nsplit; ++p) a += part[p * n + e];
        out[e] = a;
    }
}

// ---------------------------------------------------------------------------
// J leading eigenvectors of a symmetric n x n matrix (n <= 512, J <= 64), one
// workgroup per matrix, FP64 throughout:
//   1. Householder tridiagonalisation Q^T A Q = T (Golub & Van Loan, Alg.
//      5.1.1 for the reflectors, 8.3.1 for the reduction), in place in A;
//      the reflector vectors are kept below the subdiagonal of A.
//   2. The J largest eigenvalues of T by bisection on Sturm counts.
//   3. Their eigenvectors of T by inverse iteration with a partially pivoted
//      LU of T - lambda I (as in LAPACK's xSTEIN); vectors whose eigenvalues lie
//      within 1e-3 ||T|| of each other are kept orthogonal by Gram-Schmidt.
//   4. Back-transformation by the reflectors, descending-eigenvalue column
//      order, each column signed so its largest-magnitude entry is positive.
// Matrix m = blockIdx.x is block m / 3, mode m % 3; its Gram sits at
// sig + m * sig_stride, its scratch at work + m * work_stride, and the basis
// is written to the block's A_n (I_n x J_n, row-major) in the Tucker storage.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double hash_uniform(unsigned long long k) {
    unsigned long long z = k + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

__device__ __forceinline__ double block_sum256(double v, double* red) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// number of eigenvalues of T (d, e2 = e^2) below x
__device__ __forceinline__ int sturm_count(const double* d, const double* e2, int n, double x, double pivmin) {
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int cnt = q < 0.0;
    for (int i = 1; i < n; ++i) {
        q = (d[i] - x) - e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
    }
    return cnt;
}

// Householder reflector of step k from row k of A (= column k): v (v_0 = 1)
// into sv, beta, mu = ||x||, alpha = x_0; false when the row below the
// diagonal is already zero (no reflection).  Every workgroup that calls it on
// the same row gets the same bits (same loads, same summation order).
__device__ bool tri_reflector(const double* __restrict__ A, int n, int k, double* sv, double* red, double& beta,
                              double& mu, double& alpha) {
    const int tid = threadIdx.x, m = n - k - 1;
    const double* xrow = A + (long long)k * n + k + 1;
    double ss = 0.0;
    for (int i = tid; i < m; i += 256) {
        const double x = xrow[i];
        sv[i] = x;
        if (i > 0) ss = fma(x, x, ss);
    }
    const double sigma = block_sum256(ss, red);
    alpha = sv[0];
    if (!(sigma > 0.0)) {
        __syncthreads();
        return false;
    }
    mu = sqrt(fma(alpha, alpha, sigma));
    const double v1 = alpha <= 0.0 ? alpha - mu : -sigma / (alpha + mu);
    beta = 2.0 * v1 * v1 / (sigma + v1 * v1);
    __syncthreads();
    for (int i = tid; i < m; i += 256) sv[i] = i == 0 ? 1.0 : sv[i] / v1;
    __syncthreads();
    return true;
}

// p[r] = beta (B v)[r] for rows r0 <= r < r1 of the trailing block B of step
// k: four rows per wavefront at a time, the lanes along the rows (coalesced;
// m <= 511, so the eight 64-column pieces of all four rows, 32 loads a lane,
// are in flight together), then wavefront sums in fixed butterfly order.
__device__ void tri_matvec(const double* __restrict__ A, int n, int k, int r0, int r1, double beta, const double* sv,
                           double* p) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, m = n - k - 1;
    const double* B = A + (long long)(k + 1) * n + k + 1;
    for (int rb = r0 + 4 * wv; rb < r1; rb += 16) {
        double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
            const int c = lane + 64 * cc;
            if (64 * cc < m) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int r = min(rb + j, r1 - 1);
                    const double x = B[(long long)r * n + min(c, m - 1)];
                    if (c < m) a[j] = fma(x, sv[c], a[j]);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double t = wave_sum(a[j]);
            if (lane == 0 && rb + j < r1) p[rb + j] = beta * t;
        }
    }
}

// B -= v w^T + w v^T for rows r0 <= r < r1, evaluated in a symmetric order so
// B stays exactly symmetric (four rows per wavefront, loads first).
__device__ void tri_update(double* __restrict__ A, int n, int k, int r0, int r1, const double* sv, const double* sw) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, m = n - k - 1;
    double* Bw = A + (long long)(k + 1) * n + k + 1;
    for (int rb = r0 + 4 * wv; rb < r1; rb += 16) {
        double x[4][8];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int cc = 0; cc < 8; ++cc) {
                const int r = min(rb + j, r1 - 1), c = min(lane + 64 * cc, m - 1);
                x[j][cc] = (64 * cc < m) ? Bw[(long long)r * n + c] : 0.0;
            }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = rb + j;
            if (r >= r1) continue;
            const double vr = sv[r], wr = sw[r];
#pragma unroll
            for (int cc = 0; cc < 8; ++cc) {
                const int c = lane + 64 * cc;
                if (c < m) {
                    const double f = c < r ? fma(sv[c], wr, sw[c] * vr) : fma(vr, sw[c], wr * sv[c]);
                    Bw[(long long)r * n + c] = x[j][cc] - f;
                }
            }
        }
    }
}

// Step k of the tridiagonalisation of every matrix, spread over workgroups of
// TRI_ROWS trailing rows each (grid: row slices x matrices).  k_tri_p writes
// d, e, tau of step k and p = beta B v; k_tri_update forms w = p - K v with
// K = beta p.v / 2 (every workgroup from the whole of p, in the same order),
// updates its rows and stores its part of the reflector below the diagonal.
#define TRI_ROWS 32
__global__ __launch_bounds__(256) void k_tri_p(const Geo* __restrict__ g, double* __restrict__ sig, long long sig_stride,
                                               double* __restrict__ work, long long work_stride, int k) {
    const int mat = blockIdx.y, s = mat / 3, mode = mat % 3;
    const int n = g->I[s][mode];
    if (k + 2 >= n) return;
    const int m = n - k - 1, r0 = blockIdx.x * TRI_ROWS;
    if (r0 >= m) return;
    double* A = sig + (long long)mat * sig_stride;
    double* W = work + (long long)mat * work_stride;
    double* pbuf = W + 4 * n + 64;   // the inverse-iteration factors' space, free until then
    __shared__ double sv[512], red[4];
    double beta, mu, alpha;
    const bool refl = tri_reflector(A, n, k, sv, red, beta, mu, alpha);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        W[k] = A[(long long)k * n + k];         // d
        W[n + k] = refl ? mu : alpha;           // e
        W[3 * n + k] = refl ? beta : 0.0;       // tau
    }
    if (refl) tri_matvec(A, n, k, r0, min(r0 + TRI_ROWS, m), beta, sv, pbuf);
}

__global__ __launch_bounds__(256) void k_tri_update(const Geo* __restrict__ g, double* __restrict__ sig, long long sig_stride,
                                                    double* __restrict__ work, long long work_stride, int k) {
    const int mat = blockIdx.y, s = mat / 3, mode = mat % 3;
    const int n = g->I[s][mode];
    if (k + 2 >= n) return;
    const int m = n - k - 1, r0 = blockIdx.x * TRI_ROWS, r1 = min(r0 + TRI_ROWS, m);
    if (r0 >= m) return;
    double* A = sig + (long long)mat * sig_stride;
    const double* pbuf = work + (long long)mat * work_stride + 4 * n + 64;
    __shared__ double sv[512], sw[512], red[4];
    const int tid = threadIdx.x;
    double beta, mu, alpha;
    if (!tri_reflector(A, n, k, sv, red, beta, mu, alpha)) {
        for (int i = r0 + tid; i < r1; i += 256) A[(long long)(k + 1 + i) * n + k] = 0.0;
        return;
    }
    double pv = 0.0;
    for (int r = tid; r < m; r += 256) {
        const double p = pbuf[r];
        sw[r] = p;
        pv = fma(p, sv[r], pv);
    }
    const double K = 0.5 * beta * block_sum256(pv, red);
    for (int r = tid; r < m; r += 256) sw[r] = fma(-K, sv[r], sw[r]);
    __syncthreads();
    tri_update(A, n, k, r0, r1, sv, sw);
    for (int i = r0 + tid; i < r1; i += 256) A[(long long)(k + 1 + i) * n + k] = sv[i];
}

__global__ __launch_bounds__(256) void k_eig_top(const Geo* __restrict__ g, double* __restrict__ lra,
                                                 double* __restrict__ sig, long long sig_stride,
                                                 double* __restrict__ work, long long work_stride, int tri_done) {
    const int mat = blockIdx.x, s = mat / 3, mode = mat % 3;
    const int n = g->I[s][mode], J = g->J[s][mode];
    double* A = sig + (long long)mat * sig_stride;
    double* W = work + (long long)mat * work_stride;
    double* d = W;
    double* e = W + n;
    double* e2 = W + 2 * n;
    double* tau = W + 3 * n;
    double* ev = W + 4 * n;                 // 64
    double* F = W + 4 * n + 64;             // 5 x n x J factors of T - ev_j I
    double* Z = lra + g->aoff[mode][s];     // n x J output
    __shared__ double sv[512], sw[512], red[4];
    __shared__ double part[4][64];
    __shared__ int cstart[64];
    __shared__ double tinfo[3];
    const int tid = threadIdx.x;

    // ---- 1. tridiagonalisation (done by k_tri_p / k_tri_update, one launch
    // pair per step, when tri_done is set) ---------------------------------
    for (int k = 0; k + 2 < n && !tri_done; ++k) {
        const int m = n - k - 1;
        double beta, mu, alpha;
        const bool refl = tri_reflector(A, n, k, sv, red, beta, mu, alpha);
        if (tid == 0) {
            d[k] = A[(long long)k * n + k];
            e[k] = refl ? mu : alpha;
            tau[k] = refl ? beta : 0.0;
        }
        if (!refl) {
            for (int i = tid; i < m; i += 256) A[(long long)(k + 1 + i) * n + k] = 0.0;
            __syncthreads();
            continue;
        }
        tri_matvec(A, n, k, 0, m, beta, sv, sw);
        __syncthreads();
        double pv = 0.0;
        for (int r = tid; r < m; r += 256) pv = fma(sw[r], sv[r], pv);
        const double K = 0.5 * beta * block_sum256(pv, red);
        for (int r = tid; r < m; r += 256) sw[r] = fma(-K, sv[r], sw[r]);
        __syncthreads();
        tri_update(A, n, k, 0, m, sv, sw);
        // reflector vector below the subdiagonal of column k
        for (int i = tid; i < m; i += 256) A[(long long)(k + 1 + i) * n + k] = sv[i];
        __syncthreads();
    }
    if (tid == 0) {
        if (n >= 2) {
            d[n - 2] = A[(long long)(n - 2) * n + n - 2];
            e[n - 2] = A[(long long)(n - 2) * n + n - 1];
            tau[n - 2] = 0.0;
        }
        d[n - 1] = A[(long long)(n - 1) * n + n - 1];
        tau[n - 1] = 0.0;
        double tn = 0.0, lo = 0.0, hi = 0.0, emax = 0.0;
        for (int i = 0; i < n; ++i) {
            const double el = i > 0 ? fabs(e[i - 1]) : 0.0, er = i + 1 < n ? fabs(e[i]) : 0.0;
            if (i + 1 < n) {
                e2[i] = e[i] * e[i];
                emax = fmax(emax, e2[i]);
            }
            tn = fmax(tn, fabs(d[i]) + el + er);
            lo = i == 0 ? d[i] - el - er : fmin(lo, d[i] - el - er);
            hi = i == 0 ? d[i] + el + er : fmax(hi, d[i] + el + er);
        }
        tinfo[0] = tn;
        tinfo[1] = lo - (2.0 * DBL_EPSILON * n * tn + 1e-300);
        tinfo[2] = hi + (2.0 * DBL_EPSILON * n * tn + 1e-300);
        red[0] = DBL_MIN * fmax(1.0, emax);
    }
    __syncthreads();
    const double tnorm = tinfo[0], pivmin = red[0];
    __syncthreads();

    if (!(tnorm > 0.0)) {
        // zero matrix: any orthonormal basis spans an invariant subspace
        for (long long q = tid; q < (long long)n * J; q += 256) Z[q] = ((int)(q / J) == (int)(q % J)) ? 1.0 : 0.0;
        return;
    }

    // ---- 2. bisection ----------------------------------------------------
    if (tid < J) {
        const int t = n - 1 - tid;   // ascending index of the wanted eigenvalue
        double lo = tinfo[1], hi = tinfo[2];
        const double atol = 2.0 * DBL_EPSILON * tnorm;
        for (int it = 0; it < 200; ++it) {
            if (hi - lo <= fmax(atol, 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)))) break;
            const double mid = 0.5 * (lo + hi);
            if (sturm_count(d, e2, n, mid, pivmin) <= t) lo = mid;
            else hi = mid;
        }
        ev[tid] = 0.5 * (lo + hi);
    }
    __syncthreads();
    if (tid == 0) {
        cstart[0] = 0;
        for (int j = 1; j < J; ++j) cstart[j] = (ev[j - 1] - ev[j] > 1e-3 * tnorm) ? j : cstart[j - 1];
    }

    // ---- 3. inverse iteration -------------------------------------------
    // factors of T - ev_j I: F[(f * n + i) * J + j], f = l, u0, u1, u2, swap
    const double pivtol = DBL_EPSILON * tnorm;
    if (tid < J) {
        const int j = tid;
        const double lam = ev[j];
        double al = d[0] - lam, be = n > 1 ? e[0] : 0.0;
        for (int i = 0; i + 1 < n; ++i) {
            const double c = e[i], an = d[i + 1] - lam, bn = i + 2 < n ? e[i + 1] : 0.0;
            double l, u0, u1, u2, sw_;
            if (fabs(al) >= fabs(c)) {
                l = al != 0.0 ? c / al : 0.0;
                u0 = al; u1 = be; u2 = 0.0; sw_ = 0.0;
                al = an - l * be;
                be = bn;
            } else {
                l = al / c;
                u0 = c; u1 = an; u2 = bn; sw_ = 1.0;
                al = be - l * an;
                be = -l * bn;
            }
            F[(0LL * n + i) * J + j] = l;
            F[(1LL * n + i) * J + j] = u0;
            F[(2LL * n + i) * J + j] = u1;
            F[(3LL * n + i) * J + j] = u2;
            F[(4LL * n + i) * J + j] = sw_;
        }
        F[(1LL * n + n - 1) * J + j] = al;
        for (int i = 0; i < n; ++i)
            Z[(long long)i * J + j] = hash_uniform(((unsigned long long)mat << 40) ^ ((unsigned long long)j << 20) ^ (unsigned long long)i);
    }
    __syncthreads();
    for (int it = 0; it < 5; ++it) {
        if (tid < J) {
            const int j = tid;
            // forward elimination of the right-hand side (in place); the
            // loads of eight steps are issued before the recurrence runs
            // through them (a step writes Z[i] and reads Z[i + 1], so every
            // value read is the one the plain loop would read)
            double rw = Z[j];
            for (int i0 = 0; i0 + 1 < n; i0 += 8) {
                double lv[8], yv[8], sv8[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int i = min(i0 + q, n - 2);
                    lv[q] = F[(0LL * n + i) * J + j];
                    sv8[q] = F[(4LL * n + i) * J + j];
                    yv[q] = Z[(long long)(i + 1) * J + j];
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int i = i0 + q;
                    if (i + 1 < n) {
                        if (sv8[q] == 0.0) {
                            Z[(long long)i * J + j] = rw;
                            rw = yv[q] - lv[q] * rw;
                        } else {
                            Z[(long long)i * J + j] = yv[q];
                            rw = rw - lv[q] * yv[q];
                        }
                    }
                }
            }
            Z[(long long)(n - 1) * J + j] = rw;
            // back substitution, tiny pivots replaced by +-eps ||T|| (eight
            // steps of loads ahead; a step reads and writes only its own Z[i])
            double x1 = 0.0, x2 = 0.0;
            for (int i0 = n - 1; i0 >= 0; i0 -= 8) {
                double u0v[8], u1v[8], u2v[8], zv[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int i = max(i0 - q, 0);
                    u0v[q] = F[(1LL * n + i) * J + j];
                    u1v[q] = F[(2LL * n + i) * J + j];
                    u2v[q] = F[(3LL * n + i) * J + j];
                    zv[q] = Z[(long long)i * J + j];
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int i = i0 - q;
                    if (i >= 0) {
                        double u0 = u0v[q];
                        if (fabs(u0) < pivtol) u0 = u0 < 0.0 ? -pivtol : pivtol;
                        const double x = (zv[q] - u1v[q] * x1 - u2v[q] * x2) / u0;
                        Z[(long long)i * J + j] = x;
                        x2 = x1;
                        x1 = x;
                    }
                }
            }
        }
        __syncthreads();
        // scale every column to unit max-norm (keeps later sums in range)
        {
            const int j = tid & 63, grp = tid >> 6;
            double mx = 0.0;
            if (j < J)
#pragma unroll 8
                for (int i = grp; i < n; i += 4) mx = fmax(mx, fabs(Z[(long long)i * J + j]));
            part[grp][j] = mx;
            __syncthreads();
            if (j < J) {
                const double m = fmax(fmax(part[0][j], part[1][j]), fmax(part[2][j], part[3][j]));
                const double sc = m > 0.0 ? 1.0 / m : 1.0;
                for (int i = grp; i < n; i += 4) Z[(long long)i * J + j] *= sc;
            }
            __syncthreads();
        }
        // Gram-Schmidt (twice) against earlier vectors of the same cluster,
        // then normalisation
        for (int j = 0; j < J; ++j) {
            const int c0 = cstart[j];
            for (int pass = 0; pass < (c0 < j ? 2 : 0); ++pass) {
                // dots with columns c0 .. j-1: column jj = c0 + (tid & 63), 4 row phases
                const int jj = c0 + (tid & 63), grp = tid >> 6;
                double dt = 0.0;
                if (jj < j)
#pragma unroll 8
                    for (int i = grp; i < n; i += 4) dt = fma(Z[(long long)i * J + jj], Z[(long long)i * J + j], dt);
                part[grp][tid & 63] = dt;
                __syncthreads();
                if (tid < 64) sw[tid] = part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
                __syncthreads();
                for (int i = tid; i < n; i += 256) {
                    // the row's earlier columns, eight loads ahead
                    const double* zr = Z + (long long)i * J;
                    double z = zr[j];
                    for (int q0 = c0; q0 < j; q0 += 8) {
                        double zq[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q) zq[q] = zr[min(q0 + q, j - 1)];
#pragma unroll
                        for (int q = 0; q < 8; ++q)
                            if (q0 + q < j) z = fma(-sw[q0 + q - c0], zq[q], z);
                    }
                    Z[(long long)i * J + j] = z;
                }
                __syncthreads();
            }
            double nn = 0.0;
            for (int i = tid; i < n; i += 256) nn = fma(Z[(long long)i * J + j], Z[(long long)i * J + j], nn);
            const double nrm = sqrt(block_sum256(nn, red));
            const double sc = nrm > 0.0 ? 1.0 / nrm : 0.0;
            for (int i = tid; i < n; i += 256) Z[(long long)i * J + j] *= sc;
            __syncthreads();
        }
    }

    // ---- 4. back-transformation y = H_0 H_1 ... H_{n-3} z ------------------
    for (int k = n - 3; k >= 0; --k) {
        const double tk = tau[k];
        if (tk == 0.0) continue;
        const int m = n - k - 1;
        const double* v = A + (long long)(k + 1) * n + k;   // v_i at row k+1+i, v_0 = 1
        for (int i = tid; i < m; i += 256) sv[i] = i == 0 ? 1.0 : v[(long long)i * n];
        __syncthreads();
        const int j = tid & 63, grp = tid >> 6;
        double* Zk = Z + (long long)(k + 1) * J + j;
        double dt = 0.0;
        if (j < J)
            for (int i0 = grp; i0 < m; i0 += 32) {
                double zv[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) zv[q] = Zk[(long long)min(i0 + 4 * q, m - 1) * J];
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (i0 + 4 * q < m) dt = fma(sv[i0 + 4 * q], zv[q], dt);
            }
        part[grp][j] = dt;
        __syncthreads();
        if (j < J) {
            const double f = tk * (part[0][j] + part[1][j] + part[2][j] + part[3][j]);
            for (int i0 = grp; i0 < m; i0 += 32) {
                double zv[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) zv[q] = Zk[(long long)min(i0 + 4 * q, m - 1) * J];
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (i0 + 4 * q < m) Zk[(long long)(i0 + 4 * q) * J] = fma(-f, sv[i0 + 4 * q], zv[q]);
            }
        }
        __syncthreads();
    }

    // ---- sign convention ---------------------------------------------------
    {
        __shared__ double bv[4][64];
        __shared__ int bidx[4][64];
        const int j = tid & 63, grp = tid >> 6;
        double best = -1.0;
        int bi = 0x7fffffff;
        if (j < J)
            for (int i = grp; i < n; i += 4) {
                const double a = fabs(Z[(long long)i * J + j]);
                if (a > best) { best = a; bi = i; }
            }
        bv[grp][j] = best;
        bidx[grp][j] = bi;
        __syncthreads();
        bool neg = false;
        if (j < J) {
            double b = bv[0][j];
            int ib = bidx[0][j];
            for (int q = 1; q < 4; ++q)
                if (bv[q][j] > b || (bv[q][j] == b && bidx[q][j] < ib)) { b = bv[q][j]; ib = bidx[q][j]; }
            neg = Z[(long long)ib * J + j] < 0.0;
        }
        __syncthreads();
        if (neg)
            for (int i = grp; i < n; i += 4) Z[(long long)i * J + j] = -Z[(long long)i * J + j];
    }
}

// ---------------------------------------------------------------------------
// TTM chain for G = M x_1 A_1^T x_2 A_2^T x_3 A_3^T (FP64 accumulation)
//   T1[i1][i2][j3] = sum_i3 M[i1][i2][i3] A3[i3][j3]          (matrix cores, 64 rows per workgroup)
//   T2[i1][j2][j3] = sum_i2 A2[i2][j2] T1[i1][i2][j3]
//   G [j1][j2][j3] = sum_i1 A1[i1][j1] T2[i1][j2][j3]
// ---------------------------------------------------------------------------
// T1 = M_(3) A3 as a GEMM over the rows (i1, i2) of the tensor on the FP64
// matrix cores: a workgroup takes 64 rows, wavefront w rows 16w .. 16w + 15
// and every 16-column tile of J3 (<= 64); the contraction over i3 is staged
// through LDS in chunks of 32 (tensor rows converted to FP64, the matching
// rows of A3), the next chunk's loads in flight while one is consumed.
__global__ __launch_bounds__(256) void k_ttm3(const float* __restrict__ M, long long rows, int I3,
                                              const double* __restrict__ A3, int J3, double* __restrict__ T1) {
    __shared__ double xs[64][33];
    __shared__ double as[32][66];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const long long row0 = (long long)blockIdx.x * 64;
    const int nct = (J3 + 15) >> 4;
    v4d acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = (v4d){0.0, 0.0, 0.0, 0.0};
    float mx[8];
    double ax[8];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + 256 * q;
            const int r = e >> 5, kk = e & 31;                       // tensor: 64 rows x 32 values
            const long long row = row0 + r;
            const int k = k0 + kk;
            mx[q] = (row < rows && k < I3) ? M[row * I3 + k] : 0.0f;
            const int ka = e >> 6, j = e & 63;                       // A3: 32 rows x 64 columns
            ax[q] = (k0 + ka < I3 && j < J3) ? A3[(long long)(k0 + ka) * J3 + j] : 0.0;
        }
    };
    load(0);
    for (int k0 = 0; k0 < I3; k0 += 32) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + 256 * q;
            xs[e >> 5][e & 31] = (double)mx[q];
            as[e >> 6][e & 63] = ax[q];
        }
        __syncthreads();
        if (k0 + 32 < I3) load(k0 + 32);
#pragma unroll
        for (int kk = 0; kk < 32; kk += 4) {
            const double a = xs[16 * wv + li][kk + lk];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (t < nct) acc[t] = mfma64(a, as[kk + lk][16 * t + li], acc[t]);
        }
        __syncthreads();
    }
    // register v of lane l holds D[4v + l / 16][l % 16]
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const long long row = row0 + 16 * wv + 4 * v + lk;
            const int col = 16 * t + li;
            if (t < nct && row < rows && col < J3) T1[row * J3 + col] = acc[t][v];
        }
}

__global__ __launch_bounds__(256) void k_ttm2(const double* __restrict__ T1, int I2, int J3, const double* __restrict__ A2,
                                              int J2, double* __restrict__ T2) {
    const int i1 = blockIdx.x;
    for (int e = threadIdx.x; e < J2 * J3; e += 256) {
        const int j2 = e / J3, j3 = e % J3;
        double a = 0.0;
        for (int i2 = 0; i2 < I2; ++i2) a = fma(A2[(long long)i2 * J2 + j2], T1[((long long)i1 * I2 + i2) * J3 + j3], a);
        T2[((long long)i1 * J2 + j2) * J3 + j3] = a;
    }
}

__global__ __launch_bounds__(256) void k_ttm1(const double* __restrict__ T2, int I1, int J2J3, const double* __restrict__ A1,
                                              int J1, double* __restrict__ G) {
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < (long long)J1 * J2J3; e += (long long)gridDim.x * 256) {
        const int j1 = (int)(e / J2J3), q = (int)(e % J2J3);
        double a = 0.0;
        for (int i1 = 0; i1 < I1; ++i1) a = fma(A1[(long long)i1 * J1 + j1], T2[(long long)i1 * J2J3 + q], a);
        G[e] = a;
    }
}

// ---------------------------------------------------------------------------
// Iteration kernels
// ---------------------------------------------------------------------------
// W_n = A_n^T U^(n) for every block: one workgroup per (row j, block).
template <typename T>
__global__ __launch_bounds__(256) void k_lra_w(const Geo* __restrict__ g, StateP<T> st, int n, int uslot, int wslot) {
    if (st.ctrl->stop) return;
    apply_rot(st);
    lra_w_item<T>(g, st, n, uslot, wslot ^ st.ctrl->rot2, blockIdx.y, blockIdx.x);
}

// C_n = G_(n) (W_b ⊙ W_a) for every block: one workgroup per (row jn, block).
template <typename T>
__global__ __launch_bounds__(256) void k_lra_c(const Geo* __restrict__ g, StateP<T> st, int n) {
    if (st.ctrl->stop) return;
    extern __shared__ double sm[];
    lra_c_item<T>(g, st, n, blockIdx.y, blockIdx.x, sm);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_mode_gram(const float* X, int mode, int I1, int I2, int I3, double* part, int nsplit, hipStream_t q) {
    const int In = mode == 0 ? I1 : (mode == 1 ? I2 : I3);
    const int nt = (In + 63) / 64;
    hipLaunchKernelGGL(k_mode_gram, dim3(nt * (nt + 1) / 2, nsplit), dim3(256), 0, q, X, mode, I1, I2, I3, nt, part);
}
void launch_sum_split(const double* part, int nsplit, long long n, double* out, hipStream_t q) {
    long long nb = (n + 255) / 256;
    if (nb > 2048) nb = 2048;
    hipLaunchKernelGGL(k_sum_split, dim3((unsigned)nb), dim3(256), 0, q, part, nsplit, n, out);
}
void launch_eig_top(const Geo* g, double* lra, double* sig, long long sig_stride, double* work, long long work_stride,
                    int nmat, int nmax, hipStream_t q) {
    // the tridiagonalisation step by step over row slices of every matrix
    // (each step is a pass over an n x n matrix: spread over workgroups, the
    // steps run at the memory system's rate instead of one CU's latency),
    // then the rest of the solver with one workgroup per matrix
    const dim3 grid((unsigned)((nmax + TRI_ROWS - 1) / TRI_ROWS), (unsigned)nmat);
    for (int k = 0; k + 2 < nmax; ++k) {
        hipLaunchKernelGGL(k_tri_p, grid, dim3(256), 0, q, g, sig, sig_stride, work, work_stride, k);
        hipLaunchKernelGGL(k_tri_update, grid, dim3(256), 0, q, g, sig, sig_stride, work, work_stride, k);
    }
    hipLaunchKernelGGL(k_eig_top, dim3(nmat), dim3(256), 0, q, g, lra, sig, sig_stride, work, work_stride, 1);
}
void launch_ttm_chain(const float* M, int I1, int I2, int I3, const double* A1, const double* A2, const double* A3, int J1,
                      int J2, int J3, double* T1, double* T2, double* G, hipStream_t q) {
    const long long rows = (long long)I1 * I2;
    hipLaunchKernelGGL(k_ttm3, dim3((unsigned)((rows + 63) / 64)), dim3(256), 0, q, M, rows, I3, A3, J3, T1);
    hipLaunchKernelGGL(k_ttm2, dim3(I1), dim3(256), 0, q, T1, I2, J3, A2, J2, T2);
    long long nb = ((long long)J1 * J2 * J3 + 255) / 256;
    if (nb > 1024) nb = 1024;
    hipLaunchKernelGGL(k_ttm1, dim3((unsigned)nb), dim3(256), 0, q, T2, I1, J2 * J3, A1, J1, G);
}
template <typename T>
void launch_lra_w(const Geo* g, const StateP<T>& st, int S, int Jmax, int n, int uslot, int wslot, hipStream_t q) {
    hipLaunchKernelGGL(k_lra_w<T>, dim3(Jmax, S), dim3(256), 0, q, g, st, n, uslot, wslot);
}
template <typename T>
void launch_lra_c(const Geo* g, const StateP<T>& st, int S, int Jmax, int Rq, int n, hipStream_t q) {
    const size_t lds = lra_c_lds_bytes(Jmax, Rq);
    hipLaunchKernelGGL(k_lra_c<T>, dim3(Jmax, S), dim3(256), lds, q, g, st, n);
}
template void launch_lra_w<float>(const Geo*, const StateP<float>&, int, int, int, int, int, hipStream_t);
template void launch_lra_w<double>(const Geo*, const StateP<double>&, int, int, int, int, int, hipStream_t);
template void launch_lra_c<float>(const Geo*, const StateP<float>&, int, int, int, int, hipStream_t);
template void launch_lra_c<double>(const Geo*, const StateP<double>&, int, int, int, int, hipStream_t);

}  // namespace cpd
