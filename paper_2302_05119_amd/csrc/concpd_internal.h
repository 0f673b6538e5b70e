// Internal types shared by the host runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define CPD_MAXS 64   // blocks per context
#define CPD_MAXR 64   // components per block
#define CPD_MAXN 6    // tensor order (CONCPD_MAX_ORDER)

// Device-side control block: scalars of the outer iteration (Algorithm 1).
#define CPD_K2ROWS_DEFAULT 16   // i1 rows per mode-2 contraction chunk
#define CPD_K2ROWS_MIN 8         // smallest chunk the workspace is sized for

struct Ctrl {
    double t;          // t_{k-1} (Appendix A, parameter settings)
    double w_hat;      // w_hat_{k-1} = (t_{k-1} - 1) / t_k for the coming iteration
    double F_prev;     // F_{k-1}
    double F_cur;      // F of the latest sweep
    double rel_prev;   // RelErr_{k-1}
    double rel_cur;
    double tol;        // |dRelErr| threshold (0: never stop)
    double delta_w;
    long long k;
    long long restarts;
    int rot3, rot2;    // slot rotation: factors/lambda (3 slots), Grams/b/W (2 slots)
    int redo;          // set when F_k >= F_{k-1}: the next sweep redoes it from x_{k-1} without extrapolation
    int stop;          // converged: every later kernel is a no-op
    int last_restarted;
    int nonfinite;
    int restart_on;
    int reset_t;
    unsigned int counter_finish;   // arrival counters for last-workgroup reductions
    unsigned int counter_aux;
    int pad;
    unsigned int blkcnt[CPD_MAXS]; // per-block arrival counters of the chunked finish
};

// Per-context geometry, resident in the workspace.
struct Geo {
    int N;                        // tensor order
    int S, R, Rq;                 // Rq = R rounded up to a multiple of 4 (factor row stride)
    int L[CPD_MAXN];
    int rk[CPD_MAXS];             // R^(s): columns in use per block (the rest stay zero)
    int ngrp[CPD_MAXN];           // blocks of mode n's coupling group (L_n > 0), else every block
    int grp[CPD_MAXN][CPD_MAXS];  // their indices, ascending
    int upd_core;
    int lra;                      // 1: gradients from the Tucker form
    int I[CPD_MAXS][CPD_MAXN];
    int J[CPD_MAXS][3];           // Tucker ranks (lra)
    long long uoff[CPD_MAXN][CPD_MAXS];  // element offset of U^(n,s) inside one factor slot
    long long yoff[CPD_MAXS];     // Y^(s) = M^(s) x_3 U^(3,s): I1 x I2 x Rq
    long long koff[CPD_MAXS];     // K^(3,s) buffer (I3 x Rq)
    long long poff[CPD_MAXS];     // mode-3 MTTKRP partials: nchunk x I3 x Rq
    int nchunk[CPD_MAXS];         // ceil(I1 / (4 p2spw))
    int p2spw;                    // i1 slabs per pass-2 wavefront (a chunk is 4 p2spw slabs)
    long long aoff[3][CPD_MAXS];  // Tucker bases A_n^(s): I_n x J_n (double)
    long long goff[CPD_MAXS];     // Tucker cores G^(s): J1 x J2 x J3 (double), i3 fastest
    long long woff[3][CPD_MAXS];  // W_n^(s) = A_n^T U^(n): J_n x Rq (double)
    long long coff[CPD_MAXS];     // C_n^(s) = G_(n) (⊙ W): Jmax x Rq (double)
    long long wslot_len;          // doubles per W slot (slot 1 follows slot 0)
    long long k1off[CPD_MAXS];    // mode-1 MTTKRP partials per 64-row group: I1 x nrg x Rq
    long long k2off[CPD_MAXS];    // mode-2 MTTKRP partials per chunk of k2rows i1 rows: nk2 x I2 x Rq
    int nk2[CPD_MAXS];            // ceil(I1 / k2rows)
    int k2rows;                   // i1 rows per mode-2 contraction chunk
    int mvec[CPD_MAXS];           // 1: every operand row starts 16-byte aligned (vector loads)
    long long mld[CPD_MAXS];      // row stride (elements) of the operand tensor M[s]
    int nrg[CPD_MAXS];            // ceil(I2 / 64)
    const void* M[CPD_MAXS];      // block tensors in the MTTKRP operand type
    int mdtype;                   // operand type of M (concpd_dtype)
    // order N > 3: two-level dimension tree.  M^(s) is viewed as an A x B
    // matrix, A = I_0 ... I_{h-1} rows (modes 0..h-1), B = I_h ... I_{N-1}
    // columns (the rest, contiguous).  Pass A forms T_A = M KR_B (A x Rq), pass
    // B forms T_B = M^T KR_A (B x Rq); each mode's MTTKRP is a short
    // contraction of T_A or T_B with the other factors of its half.
    int nh;                       // h
    long long nwA[CPD_MAXS], nwB[CPD_MAXS];
    int npa[CPD_MAXS], npb[CPD_MAXS];     // contraction parts of pass A / pass B
    long long kpa[CPD_MAXS], kpb[CPD_MAXS];   // contraction length per part (multiple of 16)
    long long taoff[CPD_MAXS];    // pass-A partials: npa x A x Rq (in the Y region)
    long long tboff[CPD_MAXS];    // pass-B partials: npb x B x Rq (in the Y region)
    long long kroff[CPD_MAXS];    // Khatri-Rao operand: max(A, B) x Rq (in the part region)
    // the finish over the last mode in chunks of CPD_FIN_ROWS rows: block s
    // takes workgroups fin_c0[s] .. fin_c0[s] + fin_nc[s] - 1 of the launch
    int fin_nc[CPD_MAXS];
    int fin_c0[CPD_MAXS];
    int fin_nwg;
};
#define CPD_FIN_ROWS 128

// Device pointers of the iterate state.  Slot 0 = x_k being built,
// slot 1 = x_{k-1}, slot 2 = x_{k-2}.
template <typename T>
struct StateP {
    T* U[3];            // factors, one slot = sum_{n,s} I_n * Rq elements
    double* lam[3];     // [S][Rq]
    double* V[2];       // Grams U^T U, [N][S][R*R], slots 0 and 1
    double* b[2];       // core data term (U^⊙)^T vec(M), [S][Rq]
    double* P;          // D H_{-n} D of the mode being updated, [S][R*R]
    double* Ld_cur;     // [S]
    double* Ld_prev;
    double* Lu_cur;     // [N][S]
    double* Lu_prev;
    double* LC_prev;    // [N]
    double* Fblk;       // [S]
    double* normM2;     // [S] ||M^(s)||_F^2 (or ||G^(s)||^2 in lra mode)
    T* Y;               // pass-1 output
    T* K3;              // reduced mode-3 MTTKRP (order N > 3: the MTTKRP of the mode in work)
    T* part;            // mode-3 partials
    T* K1p;             // mode-1 partials
    T* K2;              // mode-2 MTTKRP
    double* lra;        // Tucker storage base (A, G, W, scratch)
    double* fpart;      // partial Grams and data terms of the chunked finish: [chunk][R*R + Rq]
    Ctrl* ctrl;
};

// Work items of the grouped kernels (host-built lists, one entry per workgroup).
struct ItemP1 { int s, i1, rg, pad; };              // pass 1: block (< 0: empty), slab, 64-row group
struct ItemP2 { int s, chunk, q0, pad; };           // pass 2: block, chunk of 4 p2spw slabs, i3 start
// update: rows [row0, row0+nrows) of blocks [s0, s0+ns) (ns > 0, columns
// individual), or of the -ns blocks of the mode's coupling group (ns < 0)
struct ItemU  { int s0, ns, row0, nrows; }; 
struct ItemK2 { int s, col0, chunk, pad; };         // mode-2 contraction: block, column tile start, i1 chunk
struct ItemNW { int s, og, part, pad; };            // order-N pass: block (< 0: empty), 64-output group, contraction part

// Kernel launchers (defined in the .hip files).
namespace cpd {
void launch_spectral_norm(const double* mats, int n, int count, double* out, hipStream_t q);
template <typename T> void launch_core(const Geo* g, const StateP<T>& st, int S, int R, int extrap, hipStream_t q);
// fused launches (R x R work beside independent MTTKRP work); false when R > 32
template <typename T> bool launch_core_pass1(const Geo* g, const StateP<T>& st, const ItemP1* items, int nitems, int P, int R, int slot, int mdtype, int dma, int extrap, int S, hipStream_t q);
template <typename T> bool launch_prep_k2(const Geo* g, const StateP<T>& st, const ItemK2* items, int nitems, int R, int slot, int S, hipStream_t q);
template <typename T> bool launch_prep_pass2(const Geo* g, const StateP<T>& st, const ItemP2* items, int nitems, int R, int slot, int mdtype, int maxI2, int spw, int S, hipStream_t q);
template <typename T> void launch_prep(const Geo* g, const StateP<T>& st, int S, int R, int n, hipStream_t q);
template <typename T> void launch_finish(const Geo* g, const StateP<T>& st, int S, int R, int nwg, hipStream_t q);
template <typename T> void launch_init_stats(const Geo* g, const StateP<T>& st, int S, int R, hipStream_t q);
template <typename T> void launch_pass1(const Geo* g, const StateP<T>& st, const ItemP1* items, int nitems, int P, int Rq, int slot, int mdtype, int dma, hipStream_t q);
template <typename T> void launch_pass2(const Geo* g, const StateP<T>& st, const ItemP2* items, int nitems, int Rq, int slot, int mdtype, int maxI2, int spw, hipStream_t q);
template <typename T> void launch_k2(const Geo* g, const StateP<T>& st, const ItemK2* items, int nitems, int slot, hipStream_t q);
// ksrc: 0 the order-3 pass outputs, 1 the Tucker form, 2 the plain K buffer (order N > 3)
template <typename T> void launch_update(const Geo* g, const StateP<T>& st, const ItemU* items, int nitems, int n, int R, int extrap, int lds_rows, int ksrc, hipStream_t q);
// order N > 3 (dimension tree): Khatri-Rao operand of one half from factor
// slot `slot`, pass A (half = 0) or B (half = 1), and the MTTKRP of mode n
// from that pass's partials (modes before n of its half from slot lo_slot)
// (check_stop: the sweep's launches do nothing once the stopping rule has fired)
template <typename T> void launch_nw_kr(const Geo* g, const StateP<T>& st, int S, int half, int slot, long long maxrows, int Rq, int check_stop, hipStream_t q);
template <typename T> void launch_nw_pass(const Geo* g, const StateP<T>& st, const ItemNW* items, int nitems, int half, int Rq, int check_stop, hipStream_t q);
template <typename T> void launch_nw_contract(const Geo* g, const StateP<T>& st, int S, int n, int lo_slot, int maxI, int Rq, int check_stop, hipStream_t q);
// the order-N sweep's fused launches: core update + pass A's Khatri-Rao
// operand; step matrix of mode n + the contraction of mode n
template <typename T> void launch_nw_core_kr(const Geo* g, const StateP<T>& st, int S, int R, int extrap, long long maxB, int Rq, hipStream_t q);
template <typename T> void launch_nw_prep_contract(const Geo* g, const StateP<T>& st, int S, int R, int n, int maxI, int Rq, hipStream_t q);
template <typename T> void launch_extract_k(const Geo* g, const StateP<T>& st, int s, int n, int I, int R, T* out, int ld_out, int lra, hipStream_t q);
template <typename T> void launch_resid(const Geo* g, const StateP<T>& st, const void* M, int dtype, int s, int I1, double* part, hipStream_t q);
void launch_sqnorm(const void* src, int dtype, long long n, double* out, double* part, int npart, hipStream_t q);
void launch_mode_gram(const float* X, int mode, int I1, int I2, int I3, double* part, int nsplit, hipStream_t q);
void launch_sum_split(const double* part, int nsplit, long long n, double* out, hipStream_t q);
void launch_eig_top(const Geo* g, double* lra, double* sig, long long sig_stride, double* work, long long work_stride, int nmat, int nmax, hipStream_t q);
void launch_ttm_chain(const float* M, int I1, int I2, int I3, const double* A1, const double* A2, const double* A3, int J1, int J2, int J3, double* T1, double* T2, double* G, hipStream_t q);
template <typename T> void launch_lra_w(const Geo* g, const StateP<T>& st, int S, int Jmax, int n, int uslot, int wslot, hipStream_t q);
template <typename T>
void launch_grad(const Geo* g, const StateP<T>& st, int S, int R, int Rq, const int* In, int L0, int L1, int L2,
                 double* const* glam, double* Fblk, T* const* gU0, T* const* gU1, T* const* gU2, int coupled, hipStream_t q);
// LDS of the core-contraction kernel: G slice, two W factors, per-tile partial sums.
inline size_t lra_c_lds_bytes(int Jmax, int Rq) { return sizeof(double) * ((size_t)Jmax * Jmax + 2 * (size_t)Jmax * Rq + 1024); }
template <typename T> void launch_lra_c(const Geo* g, const StateP<T>& st, int S, int Jmax, int Rq, int n, hipStream_t q);
// the compressed sweep's fused launches: core update + C_1; step matrix of
// mode n + the W refresh of mode n - 1
template <typename T> void launch_core_lrac(const Geo* g, const StateP<T>& st, int S, int R, int Jmax, int Rq, int extrap, hipStream_t q);
template <typename T> void launch_prep_lraw(const Geo* g, const StateP<T>& st, int S, int R, int Jmax, int Rq, int n, hipStream_t q);
void launch_sum_parts(const double* part, int np, double* out, hipStream_t q);
void launch_empty(hipStream_t q);
void launch_pad_copy(const void* src, int src_dtype, void* dst, int dst_dtype, long long rows, int I3, int ld, hipStream_t q);
void launch_finite_check(const void* src, int dtype, long long n, int* flag, hipStream_t q);
template <typename T> void launch_als_gram(const Geo* g, const StateP<T>& st, int S, int R, int n, const int* act, double* V, hipStream_t q);
void launch_als_chol(const Geo* g, int S, int R, int n, const int* act, const double* V, double* L, int* bad, hipStream_t q);
template <typename T> void launch_als_solve(const Geo* g, const StateP<T>& st, int S, int R, int n, int Imax, const int* act, const double* L, hipStream_t q);
template <typename T> void launch_als_fit(const Geo* g, const StateP<T>& st, int S, int R, const int* act, const double* V, double* relerr, double* xx, hipStream_t q);
template <typename T> void launch_als_export(const Geo* g, const StateP<T>& st, int S, int R, const double* xx, hipStream_t q);
}  // namespace cpd
