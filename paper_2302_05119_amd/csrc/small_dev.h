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
    int m = 0, ka = 0;
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
        const double am = wave_max(amax);
        if (!(am > 0.0)) return 0.0;
        // work on A 2^-ka (largest entry in [1/2, 1)) so that no norm of a
        // Lanczos vector overflows or underflows; the result is scaled back
        ka = __builtin_amdgcn_frexp_exp(am);
#pragma unroll
        for (int j = 0; j < NMAX; ++j) row[j] = ldexp(row[j], -ka);
        anorm = ldexp(am, -ka) * n;  // >= ||A 2^-ka||_2
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
    const int kr = ke + ka;   // undoes both scalings
    if (NMAX <= 48) {
        double d[MM], e2[MM];
#pragma unroll
        for (int i = 0; i < MM; ++i) {
            d[i] = (i < m) ? ldexp(dl[i], -ke) : 4.0;
            e2[i] = (i + 1 < m) ? ldexp(el[i], -2 * ke) : 0.0;
        }
        return ldexp(multisect_top<MM, double[MM]>(d, e2, m, lo, hi), kr);
    } else {
        wave_sync();
        for (int i = lane; i < MM; i += 64) {
            dl[i] = (i < m) ? ldexp(dl[i], -ke) : 4.0;
            el[i] = (i + 1 < m) ? ldexp(el[i], -2 * ke) : 0.0;
        }
        wave_sync();
        const double* dp = dl;
        const double* ep = el;
        return ldexp(multisect_top<MM, const double*>(dp, ep, m, lo, hi), kr);
    }
}

// max_i S[i][i] for i < n (n <= NPM), every load in flight: indices past n
// repeat the last diagonal entry.
template <int NPM>
__device__ __forceinline__ double diag_max(const double* __restrict__ S, int n, int ld) {
    double m0 = 0.0, m1 = 0.0;
#pragma unroll
    for (int i = 0; i < NPM; i += 2) {
        m0 = fmax(m0, S[min(i, n - 1) * (ld + 1)]);
        m1 = fmax(m1, S[min(i + 1, n - 1) * (ld + 1)]);
    }
    return fmax(m0, m1);
}

// Squaring buffers of wg_lmax_nonneg: n padded to NP = 16 * ceil(n / 16),
// row stride lp with 2 * lp = 32 (mod 64) dwords, so rows k and k+1 of a
// matrix-core operand load fall in different LDS bank halves.
__host__ __device__ inline int sq_np(int n) { return (n + 15) & ~15; }
__host__ __device__ inline int sq_lp(int n) { return (sq_np(n) & 31) == 16 ? sq_np(n) : sq_np(n) + 16; }

// Size class of the R x R spectral-norm work (the NMAX template argument of
// the small kernels): 16, 24, 32, 48 or 64.
__host__ __device__ constexpr int nmax_class(int R) { return R <= 16 ? 16 : R <= 24 ? 24 : R <= 32 ? 32 : R <= 48 ? 48 : 64; }

// Squaring buffers of the vector-ALU path (n <= NPM <= 32): NPM rows of
// NPM + 2 doubles.  The stride is an odd multiple of four dwords, so the
// 16-byte reads of sixteen consecutive rows fall in distinct bank quads.
__host__ __device__ inline int vsq_doubles(int NPM) { return 2 * NPM * (NPM + 2) + 80; }

// Largest int over the wavefront (uniform result): maxima inside rows of 16
// lanes by row shifts, then across rows by the row broadcasts, so that lane 63
// ends with the maximum of all lanes.
__device__ __forceinline__ int wave_max_i32(int v) {
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x111, 0xf, 0xf, false));   // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x112, 0xf, 0xf, false));   // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x114, 0xf, 0xf, false));   // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x118, 0xf, 0xf, false));   // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x142, 0xa, 0xf, false));   // row_bcast:15
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x143, 0xc, 0xf, false));   // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

// One DPP move of a double (two 32-bit halves); lanes without a source keep `old`.
template <int CTRL, int RMASK>
__device__ __forceinline__ double dpp_f64(double v, double old) {
    const long long b = __double_as_longlong(v), o = __double_as_longlong(old);
    const int l = __builtin_amdgcn_update_dpp((int)o, (int)b, CTRL, RMASK, 0xf, false);
    const int h = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, RMASK, 0xf, false);
    return __longlong_as_double(((long long)h << 32) | (unsigned int)l);
}

// Wavefront min of lo and max of hi (uniform results), by the same DPP
// pattern as wave_max_i32.
__device__ __forceinline__ void wave_minmax_dpp(double& lo, double& hi) {
#define CPD_MM_STEP(C, M)                               \
    lo = fmin(lo, dpp_f64<C, M>(lo, INFINITY));          \
    hi = fmax(hi, dpp_f64<C, M>(hi, -INFINITY));
    CPD_MM_STEP(0x111, 0xf)
    CPD_MM_STEP(0x112, 0xf)
    CPD_MM_STEP(0x114, 0xf)
    CPD_MM_STEP(0x118, 0xf)
    CPD_MM_STEP(0x142, 0xa)
    CPD_MM_STEP(0x143, 0xc)
#undef CPD_MM_STEP
    const long long bl = __double_as_longlong(lo), bh = __double_as_longlong(hi);
    lo = __longlong_as_double(((long long)__builtin_amdgcn_readlane((int)(bl >> 32), 63) << 32) |
                              (unsigned int)__builtin_amdgcn_readlane((int)bl, 63));
    hi = __longlong_as_double(((long long)__builtin_amdgcn_readlane((int)(bh >> 32), 63) << 32) |
                              (unsigned int)__builtin_amdgcn_readlane((int)bh, 63));
}

// Repeated squaring on the vector ALU for n <= NPM (16, 24 or 32).  At these
// sizes an FP64 matrix-core tile is mostly padding and FP64 FMA runs at the
// matrix-core rate, so the squarings are dot products of rows (S is
// symmetric, so a column is a row).  They run on the first wavefront alone,
// with no workgroup barrier between squarings: lane l forms 2 x 2 blocks
// (rows 2a, 2a+1; columns 2b, 2b+1; a <= b) of the upper triangle of S^2 from
// 16-byte row reads (two FMAs per read, eight independent chains), writes
// each block and its mirror (S stays exactly symmetric: the two halves of a
// diagonal block are the same products summed in the same order), and the
// power-of-two rescaling of the next squaring comes from the largest
// diagonal exponent, a DPP maximum over the wavefront.  The stopping test is
// that of wg_lmax_nonneg.  All threads enter; the result is broadcast.
// Returns false (nothing decided) on a negative or non-finite entry, on a
// nonzero matrix with a zero diagonal (not PSD), or when the bounds do not
// meet within 24 squarings.
template <int NPM>
__device__ __forceinline__ bool wg_lmax_vsq(const double* __restrict__ A, int n, int ld, double* __restrict__ work,
                                            double& result) {
    static_assert(NPM == 16 || NPM == 24 || NPM == 32, "vector squaring path");
    constexpr int LP = NPM + 2;
    constexpr int HM = NPM / 2;                              // row pairs
    constexpr int BPL = (HM * (HM + 1) / 2 + 63) / 64;       // blocks per lane
    typedef double d2 __attribute__((ext_vector_type(2)));
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double* __restrict__ S0 = work;
    double* __restrict__ S1 = work + NPM * LP;
    double* __restrict__ dg = S1 + NPM * LP;   // 64: x of the test
    double* __restrict__ red = dg + 64;        // result broadcast
    const int ne = (n + 1) & ~1, h = ne >> 1;
    if (wave == 0) {
        // A (zero-padded to NPM x NPM) into registers: the entry check, the
        // largest diagonal exponent e0, then S0 = A 2^-e0 (largest diagonal
        // entry in [1/2, 1); every entry of a PSD matrix is at most its
        // largest diagonal entry) and S1 = 0 (its padding is never written)
        constexpr int EPT = (NPM * NPM + 63) / 64;
        double av[EPT];
#pragma unroll
        for (int q = 0; q < EPT; ++q) {   // every load in flight (clamped addresses)
            const int e = lane + 64 * q, i = e / NPM, j = e % NPM;
            av[q] = A[min(i, n - 1) * ld + min(j, n - 1)];
        }
        // branch-free tests (bitwise, not short-circuit, so no load waits
        // behind a branch)
        int bad = 0, nz = 0, ex0 = INT_MIN;
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = lane + 64 * q, i = e / NPM, j = e % NPM;
            const double a = av[q];
            const int in = (e < NPM * NPM) & (i < n) & (j < n);
            bad |= in & ((a >= 0.0) ? 0 : 1) | in & (isfinite(a) ? 0 : 1);
            nz |= in & ((a != 0.0) ? 1 : 0);
            const int ea = __builtin_amdgcn_frexp_exp(a);
            ex0 = (in & (i == j) & (a > 0.0)) ? max(ex0, ea) : ex0;
            av[q] = in ? a : 0.0;
        }
        double res = 0.0, ok = 0.0;
        const int e0 = wave_max_i32(ex0);
        if (__any(bad)) {
            ok = 0.0;   // the Lanczos path decides
        } else if (e0 == INT_MIN) {
            ok = __any(nz) ? 0.0 : 1.0;   // zero diagonal: zero if PSD, else not PSD
        } else {
#pragma unroll
            for (int q = 0; q < EPT; ++q) {
                const int e = lane + 64 * q, i = e / NPM, j = e % NPM;
                if (e < NPM * NPM) {
                    S0[i * LP + j] = ldexp(av[q], -e0);
                    S1[i * LP + j] = 0.0;
                }
            }
            // the lane's blocks (a, b), a <= b < h
            const int nblk = h * (h + 1) / 2;
            int ba[BPL], bb[BPL];
            bool bv[BPL];
#pragma unroll
            for (int m = 0; m < BPL; ++m) {
                // block row a: the number of row starts t*h - t(t-1)/2 (t >= 1)
                // not above the block index
                const int bi = lane + 64 * m;
                bv[m] = bi < nblk;
                const int bc = bv[m] ? bi : 0;
                int a = 0;
#pragma unroll
                for (int t = 1; t < HM; ++t) a += (bc >= t * h - t * (t - 1) / 2) & (t < h);
                ba[m] = a;
                bb[m] = a + bc - (a * h - a * (a - 1) / 2);
            }
            wave_sync();
            int es = 0;   // entries of S are read as S * 2^-es
            for (int it = 0; it < 24; ++it) {
                const double* __restrict__ Sa = (it & 1) ? S1 : S0;
                double* __restrict__ Sb = (it & 1) ? S0 : S1;
                int ex = INT_MIN;
#pragma unroll
                for (int m = 0; m < BPL; ++m) {
                    if (64 * m >= nblk) break;   // uniform
                    const int r0 = 2 * ba[m], c0 = 2 * bb[m];
                    const double* x0 = Sa + r0 * LP;
                    const double* x1 = x0 + LP;
                    const double* y0 = Sa + c0 * LP;
                    const double* y1 = y0 + LP;
                    double s00a = 0.0, s00b = 0.0, s01a = 0.0, s01b = 0.0;
                    double s10a = 0.0, s10b = 0.0, s11a = 0.0, s11b = 0.0;
                    // four steps (sixteen row reads) in flight: enough overlap
                    // without hoisting every read into registers
#pragma unroll 4
                    for (int k = 0; k < NPM; k += 2) {
                        const d2 p0 = *(const d2*)(x0 + k), p1 = *(const d2*)(x1 + k);
                        const d2 q0 = *(const d2*)(y0 + k), q1 = *(const d2*)(y1 + k);
                        s00a = fma(p0.x, q0.x, s00a);
                        s00b = fma(p0.y, q0.y, s00b);
                        s01a = fma(p0.x, q1.x, s01a);
                        s01b = fma(p0.y, q1.y, s01b);
                        s10a = fma(p1.x, q0.x, s10a);
                        s10b = fma(p1.y, q0.y, s10b);
                        s11a = fma(p1.x, q1.x, s11a);
                        s11b = fma(p1.y, q1.y, s11b);
                    }
                    const double v00 = ldexp(s00a + s00b, -2 * es), v01 = ldexp(s01a + s01b, -2 * es);
                    const double v10 = ldexp(s10a + s10b, -2 * es), v11 = ldexp(s11a + s11b, -2 * es);
                    if (bv[m]) {
                        *(d2*)(Sb + r0 * LP + c0) = (d2){v00, v01};
                        *(d2*)(Sb + (r0 + 1) * LP + c0) = (d2){v10, v11};
                        *(d2*)(Sb + c0 * LP + r0) = (d2){v00, v10};
                        *(d2*)(Sb + (c0 + 1) * LP + r0) = (d2){v01, v11};
                        if (ba[m] == bb[m]) {
                            if (v00 > 0.0) ex = max(ex, __builtin_amdgcn_frexp_exp(v00));
                            if (v11 > 0.0) ex = max(ex, __builtin_amdgcn_frexp_exp(v11));
                        }
                    }
                }
                es = wave_max_i32(ex);
                if (es == INT_MIN) es = 0;
                wave_sync();
                if (it >= 3 && (it < 8 || (it & 1))) {
                    // x = S 1 (row sums; S is exactly symmetric), y = A x, and
                    // the Collatz-Wielandt bounds over the support
                    const double* rs = Sb + min(lane, NPM - 1) * LP;
                    double xa = 0.0, xb = 0.0;
#pragma unroll
                    for (int k = 0; k < NPM; k += 2) {
                        const d2 v = *(const d2*)(rs + k);
                        xa += v.x;
                        xb += v.y;
                    }
                    const double x = (lane < n) ? xa + xb : 0.0;
                    dg[lane] = x;
                    wave_sync();
                    // dg is zero past n, so the clamped columns add nothing
                    const double* ar = A + min(lane, n - 1) * ld;
                    double ya = 0.0, yb = 0.0;
#pragma unroll
                    for (int j = 0; j < NPM; j += 2) {
                        const d2 xv = *(const d2*)(dg + j);
                        ya = fma(ar[min(j, n - 1)], xv.x, ya);
                        yb = fma(ar[min(j + 1, n - 1)], xv.y, yb);
                    }
                    const double y = ya + yb;
                    double lo = INFINITY, hi = -INFINITY;
                    int miss = 0;
                    if (lane < n && A[lane * ld + lane] > 0.0) {
                        if (x > 0.0) {
                            lo = y / x;
                            hi = lo;
                        } else {
                            miss = 1;
                        }
                    }
                    wave_minmax_dpp(lo, hi);
                    miss = __any(miss);
                    wave_sync();
                    if (!miss && hi >= lo && hi - lo <= 1e-14 * hi) {   // uniform
                        res = 0.5 * (lo + hi);
                        ok = 1.0;
                        break;
                    }
                }
            }
        }
        if (lane == 0) {
            red[0] = res;
            red[1] = ok;
        }
    }
    __syncthreads();
    result = red[0];
    return red[1] != 0.0;
}

// Exact spectral norm of a nonnegative symmetric PSD matrix A (n x n, row
// stride ld, in LDS), whole workgroup.  Repeated squaring S <- S^2 (with a
// power-of-two rescaling from the largest diagonal entry, which bounds every
// entry of a PSD matrix) drives S toward the leading eigenprojection; then
// x = S 1 on the support (the rows with a positive diagonal) gives the
// Collatz-Wielandt bounds min_i (Ax)_i / x_i <= lambda_max <= max_i (Ax)_i / x_i,
// rigorous for a nonnegative matrix and a positive x, accepted once they agree
// to 1e-14 relative.  Up to n = 32 the squarings run on the vector ALU
// (wg_lmax_vsq); above, on the FP64 matrix cores: 16 x 16
// output tiles (upper triangle, mirrored, so S stays exactly symmetric), one
// tile per wavefront.  Negative or non-finite entries, n > 48, or bounds that
// do not meet within 24 squarings go to the single-wave Lanczos + Sturm solver.
// work: 2 * NP * lp + 576 doubles of LDS.
template <int NMAX>
__device__ __forceinline__ double wg_lmax_nonneg(const double* __restrict__ A, int n, int ld, double* __restrict__ work) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if constexpr (NMAX <= 32) {
        double r = 0.0;
        const bool ok = wg_lmax_vsq<NMAX>(A, n, ld, work, r);
        double* __restrict__ wl = work + vsq_doubles(NMAX);   // fallback work (448)
        double* __restrict__ res = wl + 448;
        if (!ok) {
            __syncthreads();
            if (wave == 0) {
                const double v = wave_sym_lmax_t<NMAX>(A, n, ld, wl);
                if (lane == 0) res[0] = v;
            }
            __syncthreads();
            r = res[0];
        }
        __syncthreads();
        return r;
    }
    constexpr int NPM = (NMAX + 15) & ~15;   // largest padded size of this instantiation
    const int NP = sq_np(n), lp = sq_lp(n);
    double* __restrict__ S0 = work;
    double* __restrict__ S1 = work + (NMAX <= 48 ? NP * lp : 0);
    double* __restrict__ xv = S1 + (NMAX <= 48 ? NP * lp : 0);   // 64
    double* __restrict__ red = xv + 64;       // 16
    double* __restrict__ res = red + 16;      // result broadcast
    double* __restrict__ wl = res + 16;       // fallback work (448)
    // S0 = A 2^-e0 with the largest diagonal entry in [1/2, 1): every entry
    // of a PSD matrix is at most its largest diagonal entry, so no product of
    // the first squaring overflows or underflows
    const double dmax = diag_max<NPM>(A, n, ld);
    const int e0 = (dmax > 0.0 && isfinite(dmax)) ? __builtin_amdgcn_frexp_exp(dmax) : 0;
    int bad = 0;
    for (int e = tid; e < NP * NP; e += 256) {
        const int i = e / NP, j = e % NP;
        double v = 0.0;
        if (i < n && j < n) {
            v = A[i * ld + j];
            bad |= !(v >= 0.0) | !isfinite(v);
        }
        if (NMAX <= 48) S0[i * lp + j] = ldexp(v, -e0);
    }
    const int anybad = __syncthreads_or(bad);
    double result = 0.0;
    bool done = false;
    if (!anybad && !(dmax > 0.0)) {
        // a PSD matrix with a zero diagonal is zero
        result = 0.0;
        done = true;
    }
    if (NMAX <= 48 && !anybad && !done) {
        int es = 0;   // entries of Sa are read as Sa * 2^-es
        const int nt = NP >> 4, ntile = nt * (nt + 1) / 2;
        const int li = lane & 15, lk = lane >> 4;
        const int wv = __builtin_amdgcn_readfirstlane(wave);
        double* Sa = S0;
        double* Sb = S1;
        for (int it = 0; it < 24 && !done; ++it) {
            // Sb = (Sa 2^-es)^2, tile (ta, tb) on wavefront p % 4
            for (int p = wv; p < ntile; p += 4) {
                int ta = 0, rem = p;
                while (rem >= nt - ta) {
                    rem -= nt - ta;
                    ++ta;
                }
                const int tb = ta + rem;
                // all operand loads of the tile in flight; rows past NP read
                // row NP-1 and are zeroed.  Four accumulators by k-step mod 4
                // (independent matrix-core chains), added in a fixed order
                v4d ac[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) ac[j] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int k0 = 0; k0 < NPM; k0 += 4) {
                    const double* rk = Sa + min(k0 + lk, NP - 1) * lp;
                    const double a = rk[16 * ta + li], b = rk[16 * tb + li];
                    const bool ok = k0 < NP;
                    ac[(k0 >> 2) & 3] = mfma64(ok ? a : 0.0, ok ? b : 0.0, ac[(k0 >> 2) & 3]);
                }
                const v4d acc = (ac[0] + ac[1]) + (ac[2] + ac[3]);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * ta + 4 * v + lk, c = 16 * tb + li;
                    if (ta < tb || r <= c) {
                        const double val = ldexp(acc[v], -2 * es);
                        Sb[r * lp + c] = val;
                        Sb[c * lp + r] = val;
                    }
                }
            }
            __syncthreads();
            es = __builtin_amdgcn_frexp_exp(diag_max<NPM>(Sb, n, lp));
            double* t = Sa;
            Sa = Sb;
            Sb = t;
            // the bounds after squarings 4..8, then after every second one
            // (the matrices of a sweep have a wide gap above the second
            // eigenvalue, so most pass after four or five squarings)
            if (it >= 3 && (it < 8 || (it & 1))) {
                // x = S 1 (column sums; S is exactly symmetric), y = A x, and
                // the bounds over the support, on the first wavefront
                if (wave == 0) {
                    // column sums over the zero-padded NP rows, 16 loads in flight
                    const int lc = min(lane, NP - 1);
                    double x0 = 0.0, x1 = 0.0, x2 = 0.0, x3 = 0.0;
#pragma unroll
                    for (int j0 = 0; j0 < NPM; j0 += 4) {
                        const bool ok = j0 < NP;
                        const double* c0 = Sa + min(j0, NP - 4) * lp + lc;
                        x0 += ok ? c0[0] : 0.0;
                        x1 += ok ? c0[lp] : 0.0;
                        x2 += ok ? c0[2 * lp] : 0.0;
                        x3 += ok ? c0[3 * lp] : 0.0;
                    }
                    const double x = (lane < n) ? (x0 + x1) + (x2 + x3) : 0.0;
                    xv[lane] = x;
                    wave_sync();
                    // y = A x (xv is zero past n, so clamped rows add nothing)
                    const int la = min(lane, n - 1);
                    double y0 = 0.0, y1 = 0.0;
#pragma unroll
                    for (int j = 0; j < NPM; j += 2) {
                        y0 = fma(A[min(j, n - 1) * ld + la], xv[j], y0);
                        y1 = fma(A[min(j + 1, n - 1) * ld + la], xv[j + 1], y1);
                    }
                    const double y = y0 + y1;
                    double lo = INFINITY, hi = -INFINITY;
                    int miss = 0;
                    if (lane < n && A[lane * ld + lane] > 0.0) {
                        if (x > 0.0) {
                            lo = y / x;
                            hi = lo;
                        } else {
                            miss = 1;
                        }
                    }
                    wave_minmax(lo, hi);
                    miss = __any(miss);
                    if (lane == 0) {
                        red[8] = lo;
                        red[9] = hi;
                        red[10] = (!miss && hi >= lo && hi - lo <= 1e-14 * hi) ? 1.0 : 0.0;
                    }
                }
                __syncthreads();
                if (red[10] != 0.0) {
                    result = 0.5 * (red[8] + red[9]);
                    done = true;
                }
                __syncthreads();
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

// V = U^T U (R x R, FP64, exactly symmetric) of an I x R factor with row
// stride Rq, and, when K != nullptr, bout[a] = sum_i K[i][a] U[i][a] (the core
// term b = colsum(K ⊛ U)).  The Gram runs on the FP64 matrix cores: 16-column
// tiles of U, one 16 x 16 output tile per tile pair (ta <= tb), four rows per
// step; wave w takes the row steps w, w+4, ... and the four partial tiles are
// added in fixed order through LDS (lds: 256 + 256 doubles).  Only the upper
// triangle is formed and mirrored.  lout / lbout (optional, LDS): copies of V
// (row stride R) and b for the caller.
template <typename T, int GB = 8, int BB = (GB >= 16 ? 32 : 8)>
__device__ __forceinline__ void block_gram(const T* __restrict__ U, int I, int R, int Rq, double* __restrict__ out,
                                           const T* __restrict__ K, double* __restrict__ bout, char* lds,
                                           double* __restrict__ lout = nullptr, double* __restrict__ lbout = nullptr) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nt = (R + 15) >> 4;                       // column tiles (<= 4)
    const int li = lane & 15, lk = lane >> 4;
    double* part = (double*)lds;                        // [4 waves][64 lanes][4]
    double* bpart = part + 4 * 256;                     // [4][64]
    v4d acc[10];
#pragma unroll
    for (int p = 0; p < 10; ++p) acc[p] = (v4d){0.0, 0.0, 0.0, 0.0};
    // row steps of 4 rows, wave w takes steps w, w+4, ...; batches of GB steps
    // with every global load of the batch in flight (clamped addresses,
    // zeros outside the factor), held in the storage type; the kernels that
    // run the Gram alone take 16 steps a batch on long factors (beyond 128
    // rows; on short ones the clamped loads past the end would cost more than
    // the round trips they save), those that share registers with other work 8
    const int nsteps = (I + 3) >> 2;
    for (int sb = wv; sb < nsteps; sb += 4 * GB) {
        T u[GB][4];
#pragma unroll
        for (int q = 0; q < GB; ++q) {
            const int row = 4 * (sb + 4 * q) + lk;
            const int rc = min(row, I - 1);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int col = 16 * t + li;
                const T v = U[(long long)rc * Rq + min(col, R - 1)];
                u[q][t] = (t < nt && row < I && col < R) ? v : (T)0;
            }
        }
#pragma unroll
        for (int q = 0; q < GB; ++q) {
            int p = 0;
#pragma unroll
            for (int ta = 0; ta < 4; ++ta)
#pragma unroll
                for (int tb = ta; tb < 4; ++tb, ++p)
                    if (tb < nt) acc[p] = mfma64((double)u[q][ta], (double)u[q][tb], acc[p]);
        }
    }
    // b = colsum(K ⊛ U): column c = lane, rows of phase wave in ascending
    // order, BB rows (2 BB loads) in flight: 32 with the deep batches, else 8
    double bacc = 0.0;
    if (K != nullptr) {
        const int lc = min(lane, R - 1);
        for (int i0 = wv; i0 < I; i0 += 4 * BB) {
            T kv[BB], uv[BB];
#pragma unroll
            for (int q = 0; q < BB; ++q) {
                const long long o = (long long)min(i0 + 4 * q, I - 1) * Rq + lc;
                kv[q] = K[o];
                uv[q] = U[o];
            }
#pragma unroll
            for (int q = 0; q < BB; ++q)
                if (i0 + 4 * q < I) bacc = fma((double)kv[q], (double)uv[q], bacc);
        }
        bpart[wv * 64 + lane] = bacc;
    }
    int p = 0;
#pragma unroll
    for (int ta = 0; ta < 4; ++ta)
#pragma unroll
        for (int tb = ta; tb < 4; ++tb, ++p) {
            if (tb >= nt) continue;
            __syncthreads();
#pragma unroll
            for (int v = 0; v < 4; ++v) part[(wv * 64 + lane) * 4 + v] = acc[p][v];
            __syncthreads();
            // thread e: lane e % 64, register e / 64 of the tile
            const int l2 = tid & 63, v2 = tid >> 6;
            const double d = ((part[(0 * 64 + l2) * 4 + v2] + part[(1 * 64 + l2) * 4 + v2]) + part[(2 * 64 + l2) * 4 + v2]) +
                             part[(3 * 64 + l2) * 4 + v2];
            const int r = 16 * ta + 4 * v2 + (l2 >> 4), c = 16 * tb + (l2 & 15);
            if (r < R && c < R && (ta < tb || r <= c)) {
                if (out) {
                    out[r * R + c] = d;
                    out[c * R + r] = d;
                }
                if (lout) {
                    lout[r * R + c] = d;
                    lout[c * R + r] = d;
                }
            }
        }
    __syncthreads();
    if (K != nullptr && tid < R) {
        const double bb = ((bpart[tid] + bpart[64 + tid]) + bpart[128 + tid]) + bpart[192 + tid];
        if (bout) bout[tid] = bb;
        if (lbout) lbout[tid] = bb;
    }
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

// The objective at order N > 3: H = V_1 * V_2 * ... * V_N (Grams at stride gs).
__device__ __forceinline__ double block_objective_n(const double* lam, const double* V, long long gs, int N, const double* b,
                                                    double normM2, int R) {
    __shared__ double red[256];
    const int tid = threadIdx.x, RR = R * R;
    double part = 0.0;
    for (int i = tid; i < RR; i += 256) {
        double h = lam[i / R] * lam[i % R];
        for (int m = 0; m < N; ++m) h *= V[m * gs + i];
        part += h;
    }
    if (tid < R) part -= 2.0 * lam[tid] * b[tid];
    red[tid] = part;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    return 0.5 * (normM2 + red[0]);
}

// The same objective from values already at hand: V0, V1 entries tid + 256 q
// in registers, lambda, V2 (row stride R) and b in LDS.  Same products and
// the same summation order as block_objective.
template <int EP>
__device__ __forceinline__ double block_objective_pf(const double* lam, const double (&v0)[EP], const double (&v1)[EP],
                                                     const double* V2, const double* b, double normM2, int R) {
    __shared__ double red[256];
    const int tid = threadIdx.x, RR = R * R;
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < EP; ++q) {
        const int i = tid + 256 * q;
        if (i < RR) part += lam[i / R] * lam[i % R] * v0[q] * v1[q] * V2[i];
    }
    if (tid < R) part -= 2.0 * lam[tid] * b[tid];
    red[tid] = part;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    return 0.5 * (normM2 + red[0]);
}

// LDS (bytes) of the eigenvalue work (matrix, three R-vectors, squaring
// buffers and fallback work) and of the Gram (cross-wave partial tiles).
__host__ __device__ inline size_t eig_lds_bytes(int R) {
    const size_t ld = (size_t)(R | 1);
    const int c = nmax_class(R);
    const size_t sq = c <= 32 ? (size_t)vsq_doubles(c) + 456 : (c <= 48 ? 2 * (size_t)sq_np(R) * sq_lp(R) : 0) + 576;
    return sizeof(double) * ((size_t)R * ld + 192 + 2 + sq);
}

// The eigenvalue work area after the matrix and three R-vectors: an even
// offset in doubles, so 16-byte aligned when A is (pointer arithmetic only,
// which keeps the LDS address space visible to the compiler).
__device__ __forceinline__ double* eig_work(double* A, int R) { return A + ((R * (R | 1) + 192 + 1) & ~1); }
template <typename T>
__host__ __device__ inline size_t gram_lds_bytes(int Rq, int with_k) {
    (void)Rq;
    (void)with_k;
    return sizeof(double) * (4 * 256 + 4 * 64);
}
// finish: the Gram's partial tiles, then copies of the new Gram and b
template <typename T>
__host__ __device__ inline size_t finish_lds_bytes(int R, int Rq) {
    return gram_lds_bytes<T>(Rq, 1) + sizeof(double) * ((size_t)R * R + 64);
}
template <typename T>
__host__ __device__ inline size_t prep_lds_bytes(int R, int Rq) {
    // the eigenvalue work (or the Gram's partial tiles), then the new Gram
    const size_t a = eig_lds_bytes(R), b = gram_lds_bytes<T>(Rq, 0);
    return (a > b ? a : b) + sizeof(double) * (size_t)R * R;
}

// Core tensor update (eq. solD with the gradient of eq. solapgG at the
// extrapolated point of eq. eqextraPG), then P = D H_{-1} D and its spectral
// norm for the mode-1 update.  All 256 threads of the workgroup take part.
// H is the Hadamard product of the N Grams of x_{k-1}, taken as
// V_1 * (V_2 * V_3 * ... * V_N).
template <typename T, int NMAX>
__device__ __forceinline__ void core_block(const Geo* __restrict__ g, const StateP<T>& st, int s, int extrapolate, char* smraw) {
    const Ctrl* c = st.ctrl;
    const int tid = threadIdx.x;
    const int S = g->S, R = g->R, Rq = g->Rq, ld = R | 1, RR = R * R;
    double* A = (double*)smraw;
    double* lv = A + R * ld;   // lambda_{k-1} | lambda_{k-1} - lambda_{k-2} | new lambda
    double* work = eig_work(A, R);
    const double* V0 = st.V[1] + (0 * S + s) * RR;
    const double* V1 = st.V[1] + (1 * S + s) * RR;
    const double* V2 = st.V[1] + (2 * S + s) * RR;
    // every global read of the update issued first; V1 * V2 stays in
    // registers for the step matrix of mode 1
    constexpr int EP = (NMAX * NMAX + 255) / 256;
    double v0[EP], v12[EP];
#pragma unroll
    for (int m = 0; m < EP; ++m) {
        const int i = min(tid + 256 * m, RR - 1);
        v0[m] = V0[i];
        v12[m] = V1[i] * V2[i];
    }
    // order N > 3: the Grams of modes 4.. join the product H_{-1}
    for (int mm = 3; mm < g->N; ++mm) {
        const double* Vx = st.V[1] + (mm * S + s) * RR;
#pragma unroll
        for (int m = 0; m < EP; ++m) v12[m] *= Vx[min(tid + 256 * m, RR - 1)];
    }
    const double* l1 = st.lam[1] + s * Rq;
    const double* l2 = st.lam[2] + s * Rq;
    const int tl = min(tid, R - 1);
    const double l1v = l1[tl], l2v = l2[tl], bv = st.b[1][s * Rq + tl];
    const double w_hat = c->w_hat, dw = c->delta_w, Ldp = st.Ld_prev[s];
    const int upd = g->upd_core;
#pragma unroll
    for (int m = 0; m < EP; ++m) {
        const int i = tid + 256 * m;
        if (i < RR) A[(i / R) * ld + i % R] = v0[m] * v12[m];
    }
    const double lam1 = (tid < R) ? l1v : 0.0;
    const double dlam = (tid < R) ? lam1 - l2v : 0.0;
    if (tid < 64) {
        lv[tid] = lam1;
        lv[64 + tid] = dlam;
    }
    __syncthreads();
    // H lam_{k-1} and H (lam_{k-1} - lam_{k-2}); the gradient at the
    // extrapolated point combines them once the weight is known (lv is zero
    // past R, so the clamped columns add nothing)
    double h1 = 0.0, h2 = 0.0;
    {
        const double* ar = A + tl * ld;
#pragma unroll 8
        for (int r = 0; r < NMAX; ++r) {
            const double h = ar[min(r, R - 1)];
            h1 = fma(h, lv[r], h1);
            h2 = fma(h, lv[64 + r], h2);
        }
    }
    const double Ld = wg_lmax_nonneg<NMAX>(A, R, ld, work);
    const double wd = extrap_weight(extrapolate, w_hat, Ldp, Ld, dw);
    double nl = lam1;
    if (upd && Ld > 0.0 && tid < R) {
        const double lhat = lam1 + wd * dlam;
        const double gr = (h1 + wd * h2) - bv;
        nl = relu_keep_nan(lhat - gr / Ld);
    }
    if (tid < Rq) st.lam[0][s * Rq + tid] = (tid < R) ? nl : 0.0;
    if (tid < 64) lv[128 + tid] = (tid < R) ? nl : 0.0;
    if (tid == 0) st.Ld_cur[s] = Ld;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < EP; ++m) {
        const int i = tid + 256 * m;
        if (i < RR) {
            const int r = i / R, cc = i % R;
            const double p = lv[128 + r] * lv[128 + cc] * v12[m];
            st.P[s * RR + i] = p;
            A[r * ld + cc] = p;
        }
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
    const int S = g->S, R = g->R, Rq = g->Rq, ld = R | 1, RR = R * R, N = g->N;
    const int m = n - 1, tid = threadIdx.x;
    double* Vm = st.V[0] + (m * S + s) * RR;
    // the other Grams of the step matrix (every mode but n - 1 and n, in mode
    // order: at order 3 mode 3 of x_{k-1} for n = 1, the new mode 1 for n = 2)
    // and lambda, read before the Gram so their latency overlaps it; the new
    // Gram comes back through LDS
    constexpr int EP = (NMAX * NMAX + 255) / 256;
    double vo[EP];
    {
        const int q0 = (n == 1) ? 2 : 0;
        const double* Vo = (q0 < n ? st.V[0] : st.V[1]) + (q0 * S + s) * RR;
#pragma unroll
        for (int q = 0; q < EP; ++q) vo[q] = Vo[min(tid + 256 * q, RR - 1)];
        for (int mm = q0 + 1; mm < N; ++mm) {
            if (mm == n - 1 || mm == n) continue;
            const double* Vx = (mm < n ? st.V[0] : st.V[1]) + (mm * S + s) * RR;
#pragma unroll
            for (int q = 0; q < EP; ++q) vo[q] *= Vx[min(tid + 256 * q, RR - 1)];
        }
    }
    __shared__ double lam[64];
    if (tid < 64) lam[tid] = st.lam[0][s * Rq + min(tid, R - 1)];
    double* A = (double*)smraw;
    double* Vl = (double*)(smraw + prep_lds_bytes<T>(R, Rq) - sizeof(double) * (size_t)RR);   // new Gram (LDS)
    block_gram<T>(st.U[0] + g->uoff[m][s], g->I[s][m], R, Rq, Vm, nullptr, nullptr, smraw, Vl);
    double* work = eig_work(A, R);
    // P = D (Va * Vb) D: at order 3 Va = Gram of mode 1, Vb = Gram of mode 3
    // (n = 1) or of mode 2 (n = 2)
#pragma unroll
    for (int q = 0; q < EP; ++q) {
        const int i = tid + 256 * q;
        if (i < RR) {
            const int r = i / R, cc = i % R;
            const double p = (n == 1) ? lam[r] * lam[cc] * Vl[i] * vo[q] : lam[r] * lam[cc] * vo[q] * Vl[i];
            st.P[s * RR + i] = p;
            A[r * ld + cc] = p;
        }
    }
    __syncthreads();
    const double Lu = wg_lmax_nonneg<NMAX>(A, R, ld, work);
    if (tid == 0) st.Lu_cur[n * S + s] = Lu;
}

}  // namespace cpd
