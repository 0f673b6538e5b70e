/*
 * concpd.h - C ABI of the MI355X (gfx950) implementation of CoNCPD-APG and
 * lraCoNCPD-APG: coupled nonnegative CP decomposition of S third-order
 * tensors by alternating proximal gradient with Nesterov extrapolation and
 * restart (Wang, Liu, Cong, "Fast Learnings of Coupled Nonnegative Tensor
 * Decomposition Using Optimal Gradient and Low-rank Approximation",
 * arXiv 2302.05119).
 *
 * Problem (Section II-C, eq. tensormodel and eq. costfunc): given blocks
 * M^(s) (s = 1..S) of size I1 x I2 x I3, find lambda^(s) >= 0 (the
 * super-diagonal of the core D^(s)) and factors U^(n,s) >= 0 of size
 * I_n x R whose first L_n columns are shared by every block (or by a chosen
 * group of blocks per mode, concpd_config.coupled_blocks; each block may have
 * its own rank R^(s) <= R, concpd_config.block_ranks), minimising
 * 1/2 sum_s || M^(s) - [[D^(s); U^(1,s), U^(2,s), U^(3,s)]] ||_F^2.
 *
 * Entry points: configuration and workspace (concpd_query_workspace,
 * concpd_init, concpd_destroy); Algorithm 1 (concpd_step, concpd_fit);
 * Algorithm 2 (lra_compress_cp: the paper's CPD-ALS compression,
 * lra_compress: truncated HOSVD, lra_step, lra_get_tucker); results and
 * checkpoints (concpd_global_fit, concpd_get_factor, concpd_get_lambda,
 * concpd_get_lipschitz, concpd_get_state, concpd_set_state); the autograd
 * form (concpd_loss_grad); launch options and autotuning; measurement and
 * test hooks (concpd_profile*, concpd_launch_floor, concpd_debug_*).
 *
 * Conventions used by every call:
 *  - Tensors are device buffers, C-contiguous (i3 fastest):
 *    element (i1,i2,i3) of block s at offset (i1*I2 + i2)*I3 + i3.
 *  - Host factor arrays are row-major I_n x R doubles (column r fastest).
 *  - Block s, mode n (0-based) is addressed as index N*s + n in [S*N] arrays
 *    (N = 3: index 3*s + n in [S*3] arrays).
 *  - All device work is queued on the stream given to concpd_init.
 *  - Every call returns a concpd_status; no C++ exception crosses the ABI.
 *    On error the context is unchanged and concpd_last_error() returns a
 *    thread-local message describing the first error.
 *  - A context never allocates device memory: the caller passes one
 *    workspace buffer of at least concpd_query_workspace() bytes and keeps it
 *    (and the tensors) alive until concpd_destroy(), or, with
 *    concpd_init_static, the context uses a fixed-size device array that the
 *    library holds on every device it runs on.  (The context-free test hook
 *    concpd_debug_spectral_norm allocates and frees its own device buffers.)
 */
#ifndef CONCPD_H
#define CONCPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum concpd_status {
    CONCPD_OK = 0,
    CONCPD_EINVAL = 1,     /* invalid argument or configuration */
    CONCPD_ENOTSUP = 2,    /* valid but not supported by this build (e.g. lra at order > 3) */
    CONCPD_ENONFINITE = 3, /* NaN or Inf in an input */
    CONCPD_EHIP = 4,       /* a HIP runtime call failed */
    CONCPD_ESTATE = 5      /* call not valid in the context's current state */
} concpd_status;

typedef enum concpd_dtype {
    CONCPD_F64 = 0,
    CONCPD_F32 = 1,
    CONCPD_BF16 = 2,
    CONCPD_F16 = 3
} concpd_dtype;

#define CONCPD_MAX_ORDER 6   /* largest tensor order N */

typedef struct concpd_config {
    int32_t order;          /* N, the tensor order, 3..CONCPD_MAX_ORDER.  Order 3 has every
                               entry point; order N > 3 (the N-way model of Section II-C) has
                               the dense path with FP32 or FP64 compute: concpd_init(_static),
                               concpd_step, concpd_fit, concpd_global_fit, concpd_get_factor,
                               concpd_get_lambda, concpd_get_lipschitz, concpd_get_state,
                               concpd_set_state, concpd_debug_mttkrp, concpd_get_option,
                               concpd_set_option(CONCPD_OPT_GRAPH_SWEEPS), concpd_destroy;
                               the others return ENOTSUP */
    int32_t num_blocks;     /* S >= 1, at most 64 */
    int32_t rank;           /* R, components per block, 1..64 */
    int32_t coupled[CONCPD_MAX_ORDER]; /* L_n for n < N (later entries ignored), 0 <= L_n <= R:
                               the first L_n columns of every mode-n factor are shared by all
                               blocks (Section II-C); a mode with L_n > 0 needs equal I_n in
                               every block */
    const int64_t* dims;    /* [S*N]: I_n of block s at dims[N*s + n], each >= 1; C-contiguous
                               tensors, the last mode fastest */
    int32_t tensor_dtype;   /* element type of the caller's tensors: CONCPD_F64 or CONCPD_F32 */
    int32_t compute_dtype;  /* MTTKRP operand type.  CONCPD_F64 needs F64 tensors and keeps
                               every quantity in FP64.  CONCPD_F32 runs FP32 MFMA.
                               CONCPD_BF16 / CONCPD_F16 keep a 16-bit shadow of the tensors
                               in the workspace.  BF16 runs the MTTKRP passes on the BF16
                               matrix cores (v_mfma_f32_4x4x4_16b_bf16, FP32 accumulation;
                               pass 1 by LDS DMA, the default for 16-bit storage) with each
                               FP32 factor value split into hi + lo BF16 parts, so only the
                               tensor is rounded to 16 bits; FP16 widens its tensor values
                               to FP32 for the FP32 matrix cores.
                               Grams, Lipschitz constants, the core update, the objective
                               and the restart test are FP64 in every mode. */
    int32_t update_core;    /* 1: update D^(s) (CoNCPD-APG); 0: keep lambda fixed, the -NC
                               variant of Section III-C (core tensors removed, i.e. merged
                               into the factors: the seeded initialisation then sets
                               lambda = 1; a caller's init_lambda is kept as given) */
    int32_t restart;        /* 1: restart rule of Algorithm 1 */
    double delta_w;         /* delta_w < 1 of eq. eqextrawd / eqextrawu (paper: 0.9999) */
    double tol;             /* concpd_fit stops when |RelErr_k - RelErr_{k-1}| < tol */
    int32_t max_it;         /* concpd_fit iteration limit (paper: 1000) */
    const int32_t* tucker_ranks; /* [S*3] Tucker ranks J_n <= I_n for lra_compress, or NULL
                               when the context will not be compressed */
    const int32_t* block_ranks;  /* [S] per-block rank R^(s), max(1, L_1, L_2, L_3) <= R^(s) <= R,
                               or NULL for R^(s) = R.  Uneven ranks (the model of Section II-C
                               allows a rank per block) are run as rank R with the columns
                               R^(s)..R-1 of block s held at zero and lambda_r = 0 there, an
                               exact embedding: such columns have zero gradient, zero rows
                               and columns in every Hadamard Gram and leave every
                               Lipschitz constant unchanged.  Host factor and lambda arrays
                               keep the stride R; columns >= R^(s) are ignored on input and
                               read back as zero. */
    const uint64_t* coupled_blocks; /* [N] flexible coupling (Section III-C): bit s of
                               coupled_blocks[n] set = block s shares mode n's first L_n
                               columns; blocks left out keep all R columns of that mode
                               individual.  A mode with L_n > 0 needs at least one bit set
                               (bits >= S must be clear) and equal I_n over its group.
                               NULL: every block shares (the model of Section II-C). */
} concpd_config;

typedef struct concpd_stats {
    int64_t k;              /* accepted outer iterations so far */
    double F;               /* objective F_k (eq. costfunc, or eq. cosfunclra after lra_compress) */
    double relerr;          /* RelErr_k = 1/S sum_s ||M - M^|| / ||M|| */
    double fit;             /* 1 - relerr */
    int64_t restarts;       /* number of restarted iterations so far */
    int32_t restarted_last; /* 1 if the last iteration was restarted */
    int32_t converged;      /* 1 once |dRelErr| < tol was met (further steps are no-ops) */
    int32_t nonfinite;      /* 1 if F_k is not finite */
    int32_t lra;            /* 1 after lra_compress */
} concpd_stats;

typedef struct concpd_ctx_s* concpd_ctx;

/* Thread-local text of the last error (empty string if none). */
const char* concpd_last_error(void);

/* Bytes of device workspace concpd_init needs for cfg (host-only call).
 * Errors: EINVAL/ENOTSUP for an invalid configuration. */
concpd_status concpd_query_workspace(const concpd_config* cfg, size_t* bytes);

/* Create a context: validates cfg, lays out the workspace, uploads the initial
 * iterate and computes its Grams, core data term b, F_0 and RelErr_0 on the
 * device (Algorithm 1, initialisation).
 *   tensors      [S] device pointers to the blocks (borrowed, read-only).
 *   init_U       [S*N] host I_n x R row-major arrays (copied), or NULL for a
 *                seeded U[0,1] draw (SplitMix64, order: n, then s, then row,
 *                then column; shared columns drawn once).  Shared columns are
 *                taken from block 0.
 *   init_lambda  [S] host R-vectors, or NULL for a seeded U[0,1] draw
 *                (all ones when update_core = 0).
 *   workspace    device buffer of ws_bytes >= concpd_query_workspace(cfg).
 *   stream       hipStream_t (NULL = default stream).
 * Errors: EINVAL, ENOTSUP, ENONFINITE (NaN/Inf in init arrays or tensors), EHIP.
 * On error *out is NULL and nothing stays queued that writes the workspace. */
concpd_status concpd_init(const concpd_config* cfg, const void* const* tensors,
                          const double* const* init_U, const double* const* init_lambda,
                          uint64_t seed, void* workspace, size_t ws_bytes, void* stream,
                          concpd_ctx* out);

/* Bytes of the static workspace of concpd_init_static (32 MiB per device). */
#define CONCPD_STATIC_WORKSPACE_BYTES (32u << 20)

/* concpd_init for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same context, but its workspace is a device array of
 * CONCPD_STATIC_WORKSPACE_BYTES that the library holds on each device until
 * the process ends, so neither this call nor the caller allocates.  The
 * context lives on the current device (its stream must belong to it); the
 * other arguments are those of concpd_init, and every other entry point
 * works on the context unchanged.
 * One such context per device at a time: the array is shared by every call
 * on that device and keeps the last context's contents (this call clears
 * what must start at zero).  Contexts on one device would race on it, so a
 * second call while one is alive fails with ESTATE until concpd_destroy of
 * the first.  The optional second stream (CONCPD_OVERLAP) is never created.
 * Errors: those of concpd_init; EINVAL when concpd_query_workspace(cfg)
 * exceeds CONCPD_STATIC_WORKSPACE_BYTES; ESTATE as above; EHIP if the
 * array's device address cannot be obtained. */
concpd_status concpd_init_static(const concpd_config* cfg, const void* const* tensors,
                                 const double* const* init_U, const double* const* init_lambda,
                                 uint64_t seed, void* stream, concpd_ctx* out);

/* Run outer iterations of Algorithm 1 (each: the extrapolated sweep
 * D^(1..S), U^(1,1..S), ..., U^(3,1..S); if F_k >= F_{k-1} and restart is on,
 * the sweep is redone from x_{k-1} with zero extrapolation and accepted).
 * Every decision is taken on the device, so a rejected sweep is simply
 * followed by its redo in the next sweep launched.
 * With out != NULL: exactly n_iter iterations are accepted (fewer once
 * converged); synchronises the stream and fills *out.
 * With out == NULL: asynchronous; queues n_iter sweeps, so each restart in
 * them leaves one iteration fewer accepted (the stats give k).
 * After convergence (concpd_fit) further sweeps are no-ops.
 * In lra mode (after lra_compress) the gradients use the compressed blocks.
 * Errors: EINVAL (n_iter < 0), EHIP. */
concpd_status concpd_step(concpd_ctx ctx, int32_t n_iter, concpd_stats* out);

/* Iterate until |RelErr_k - RelErr_{k-1}| < tol or k = max_it (Section III-C).
 * Reaching max_it is not an error (out->converged = 0).  Synchronises. */
concpd_status concpd_fit(concpd_ctx ctx, concpd_stats* out);

/* Compress every block by truncated HOSVD to the Tucker ranks given in the
 * configuration (ranks == NULL) or in ranks [S*3] (each <= the configured
 * rank for that block/mode): A_n^(s) = J_n leading left singular vectors of
 * M^(s)_(n), G^(s) = M^(s) x_1 A_1^T x_2 A_2^T x_3 A_3^T, then switch the
 * context to lraCoNCPD-APG (Algorithm 2, eq. cosfunclra): F, RelErr and every
 * gradient are taken against the compressed blocks.  The current iterate is
 * kept; its F and b are recomputed.  Synchronises; out may be NULL.
 * The Grams M_(n) M_(n)^T are formed with FP64 products and sums and their
 * leading eigenvectors found by Householder tridiagonalisation, bisection and
 * inverse iteration (descending order; each vector signed so that its
 * largest-magnitude entry is positive).  Limits (checked by concpd_init when
 * tucker_ranks is set): F32 tensors, I_n <= 512, J_n <= 64.
 * Errors: ESTATE (no Tucker ranks configured), EINVAL (J_n > configured), EHIP. */
concpd_status lra_compress(concpd_ctx ctx, const int32_t* ranks, concpd_stats* out);

/* concpd_step in lra mode.  Errors: ESTATE if lra_compress has not run. */
concpd_status lra_step(concpd_ctx ctx, int32_t n_iter, concpd_stats* out);

/* Compress every block by an unconstrained rank-R~ CPD fitted with alternating
 * least squares: the paper's own first step of Algorithm 2 (Section III-B;
 * ALS and its stopping rule per the experiment settings of Section IV: stop
 * once |RelErr_k - RelErr_{k-1}| < eps, or after max_it iterations; the paper
 * uses eps = 1e-4 and max_it = 200).  One ALS iteration sets U~^(1), U~^(2),
 * U~^(3) in turn to K_n H_n^{-1} (K_n the MTTKRP of the block with the latest
 * factors, H_n the Hadamard product of the other two Grams; Cholesky, FP64).
 * RelErr_0 is taken at the starting point; each block stops on its own.
 * Afterwards the context is in lra mode with X~^(s) = [[U~^(1,s), U~^(2,s),
 * U~^(3,s)]] held in Tucker form (A_n = U~^(n,s) as FP64 I_n x R~, G = the
 * super-diagonal core of ones, which lra_get_tucker returns), and lra_step
 * iterates on it (eq. eqlrau / eqlrag).  The APG iterate is left as it was.
 *   cp_rank R~, 1 <= R~ <= R (eq. cosfunclra allows R~ <= R; the paper's
 *           runs use R~ = R), or 0 for R; block s is fitted at rank
 *           R~_s = min(R~, R^(s)).
 *   init    [S*3] host I_n x R~_s row-major starting factors at index 3*s + n
 *           (copied), or NULL for a seeded U[0,1] draw (SplitMix64(seed);
 *           order: n, then s, then row, then column).
 *   iters   [S] ALS iterations run per block, or NULL.
 *   relerr  [S] final ||M - X~|| / ||M|| per block (M: the operand copy the
 *           MTTKRP reads), or NULL.
 * Needs tucker_ranks with every J_n >= R~_s (so R~_s <= I_n; they reserve the compressed form's
 * storage) and a context not yet compressed.
 * Errors: EINVAL, ESTATE, ENOTSUP, ENONFINITE (a Gram H_n that is not
 * positive definite, e.g. a rank-deficient start, or a non-finite fit; the
 * context is then left uncompressed with its iterate intact), EHIP. */
concpd_status lra_compress_cp(concpd_ctx ctx, const double* const* init, uint64_t seed, double eps, int32_t max_it,
                              int32_t cp_rank, int32_t* iters, double* relerr, concpd_stats* out);

/* Copy one part of block s's compressed form to host memory (FP64):
 * n = 0, 1, 2: the basis A_n (I_n x J_n, row-major); n = 3: the core G
 * (J_1 x J_2 x J_3, row-major).  Synchronises.
 * Errors: EINVAL (s or n out of range), ESTATE (before lra_compress), EHIP. */
concpd_status lra_get_tucker(concpd_ctx ctx, int32_t s, int32_t n, double* host_dst);

/* Global fit 1 - 1/S sum_s ||M^(s) - M^^(s)||_F / ||M^(s)||_F against the
 * original tensors, by one direct FP64-accumulated pass (the "final fit").
 * Synchronises. */
concpd_status concpd_global_fit(concpd_ctx ctx, double* fit);

/* Copy U^(n,s) (I_n x R row-major, shared columns included) or lambda^(s) of
 * the current accepted iterate to host doubles.  Synchronises.
 * Errors: EINVAL for n/s out of range. */
concpd_status concpd_get_factor(concpd_ctx ctx, int32_t n, int32_t s, double* host_dst);
concpd_status concpd_get_lambda(concpd_ctx ctx, int32_t s, double* host_dst);

/* Lipschitz constants used by the last accepted sweep (eq. eqLipsLd /
 * eqLipsLu): Ld [S], Lu [S*N] (index N*s + n), LC [N] = sum_s Lu.  Synchronises. */
concpd_status concpd_get_lipschitz(concpd_ctx ctx, double* Ld, double* Lu, double* LC);

/* Read the iterate state for a checkpoint, in the layout concpd_set_state
 * takes back: U, lam = x_{k-1} and U_prev, lam_prev = x_{k-2} ([S*N] host
 * I_n x R arrays at index N*s + n / [S] R-vectors, caller-allocated; any of
 * the four may be NULL to skip it), Ld_prev [S], Lu_prev [S*N], LC_prev [N]
 * (negative = none), t = t_{k-1}, k.  Restoring these into a context of the
 * same configuration continues the run bit for bit (the restart count starts
 * again from 0).  Synchronises.  Errors: EINVAL, EHIP. */
concpd_status concpd_get_state(concpd_ctx ctx, double* const* U, double* const* U_prev, double* const* lam,
                               double* const* lam_prev, double* Ld_prev, double* Lu_prev, double* LC_prev,
                               double* t, int64_t* k);

/* Replace the iterate state (checkpoint restore / teacher forcing):
 *   U, lam          x_{k-1}: [S*N] / [S] host arrays,
 *   U_prev, lam_prev x_{k-2} (NULL: same as x_{k-1}),
 *   Ld_prev [S], Lu_prev [S*N], LC_prev [N]: constants of the previous sweep,
 *                   NULL or negative entries meaning "none" (weight 0),
 *   t               t_{k-1} of eq. eqextrawu (t_0 = 1), k the iteration count.
 * Recomputes Grams, b, F_{k-1}, RelErr_{k-1}; clears the converged flag.
 * Errors: EINVAL, ENONFINITE, EHIP. */
concpd_status concpd_set_state(concpd_ctx ctx, const double* const* U, const double* const* U_prev,
                               const double* const* lam, const double* const* lam_prev,
                               const double* Ld_prev, const double* Lu_prev, const double* LC_prev,
                               double t, int64_t k);

/* Loss F and its partial gradients at an arbitrary point, without touching the
 * iterate (autograd form): dF/dlambda^(s) = H lambda - b (eq. solbpgG) and
 * dF/dU^(n,s) = U D H_{-n} D - M_(n) U^{⊙-n} D (eq. solbpgU), every block at
 * the same point, F = sum_s 1/2 ||M^(s) - [[lambda^(s); U^(.,s)]]||^2.
 *   U_dev      [S*3] device I_n x R row-major arrays (index 3*s + n) in the
 *              context's factor type (double for compute_dtype F64, else float).
 *   lambda_dev [S] device double R-vectors.
 *   coupled    1: the first L_n columns of every mode-n factor of the mode's
 *              coupling group (every block unless coupled_blocks says
 *              otherwise) are the shared U_C, read from the group's first
 *              block, and every member's gU receives the gradient with
 *              respect to U_C (the sum over the group, eq. solbpgUCI);
 *              0: every block's factors are taken as given and gU holds each
 *              block's own gradient (a caller that ties parameters sums them).
 *   gU_dev     [S*3] device outputs shaped like U_dev.
 *   glam_dev   [S] device double outputs.  *loss receives F (host).
 * Inputs and outputs may not overlap.  Synchronises.
 * Errors: EINVAL (NULL pointer), ESTATE (lra mode), EHIP. */
concpd_status concpd_loss_grad(concpd_ctx ctx, const void* const* U_dev, const void* const* lambda_dev, int32_t coupled,
                               double* loss, void* const* gU_dev, void* const* glam_dev);

/* Test hook: K = M^(s)_(n) U^{⊙-n} at the current iterate, I_n x R row-major
 * float (double in F64 mode) written to dev_out, by the launches a sweep uses
 * (at order N > 3 the dimension-tree pass of mode n's half and its
 * contraction, every factor from x_{k-1}).  Synchronises. */
concpd_status concpd_debug_mttkrp(concpd_ctx ctx, int32_t n, int32_t s, void* dev_out);

/* Measurement hook: the launch-latency floor of a sweep of `kernels` kernels,
 * timed with HIP events on a private stream: *us_graph per replay of a
 * captured graph of that many empty one-wavefront kernels, *us_direct per
 * `kernels` direct launches of them (after one untimed pass each).  Compare a
 * latency-bound sweep against it.  Synchronises.  Errors: EINVAL, EHIP. */
concpd_status concpd_launch_floor(int32_t kernels, int32_t reps, double* us_graph, double* us_direct);

/* Test hook: the largest eigenvalue of each of `count` symmetric n x n FP64
 * matrices (host, row-major, packed one after another), computed on the
 * device by the same code that gives the spectral norms of eq. eqLipsLd /
 * eqLipsLu in a sweep: repeated squaring with Collatz-Wielandt bounds for
 * nonnegative matrices, Lanczos with Sturm multisection otherwise.  Results
 * to host_out [count].  1 <= n <= 64, 1 <= count <= 65535.  Needs no context;
 * allocates and synchronises.  Errors: EINVAL, EHIP. */
concpd_status concpd_debug_spectral_norm(const double* host_A, int32_t n, int32_t count, double* host_out);

/* Per-kernel timing of the dense MTTKRP passes (pass 1: M x_3 U^(3); pass 2:
 * the mode-3 MTTKRP) of later concpd_step calls: with enable != 0, every sweep
 * launches each pass 4 times back to back between two HIP events on the
 * context stream (a pass is a pure function of the iterate within a sweep, so
 * the repeats rewrite the same outputs and leave the iterate unchanged).
 * concpd_profile_read synchronises and returns the summed milliseconds and
 * the number of timed launches of each pass, then clears the record.
 * Errors: EHIP. */
concpd_status concpd_profile(concpd_ctx ctx, int32_t enable);
concpd_status concpd_profile_read(concpd_ctx ctx, double* ms_pass1, double* ms_pass2, int64_t* launches);

/* Launch options of a context (batching form).
 *   CONCPD_OPT_GRAPH_SWEEPS  n > 0: concpd_step queues sweeps as replays of one
 *                            captured HIP graph of n sweeps (all decisions are
 *                            taken on the device, so a sweep is a fixed kernel
 *                            sequence); 0 (default): direct kernel launches.
 *   CONCPD_OPT_OVERLAP       1: the small FP64 kernels run on a second stream
 *                            beside the MTTKRP passes (default 0); with graph
 *                            sweeps the two streams become parallel branches
 *                            of the captured graph.
 *   CONCPD_OPT_K2_ROWS       i1 rows per workgroup of the mode-2 contraction
 *                            (8..64, default 16).
 *   CONCPD_OPT_P1_SPLIT      wavefronts that share one 64-row item of pass 1
 *                            (M x_3 U^(3)), splitting its i3 range: 1, 2 or 4;
 *                            0 (default): chosen from the item count (at
 *                            least 1.5 wavefronts per SIMD).  Get returns the
 *                            split in use.
 *   CONCPD_OPT_P1_DMA        1: pass 1 streams the tensor into LDS by DMA,
 *                            two 32-byte chunks of every row in flight per
 *                            wavefront; 0: through registers.  Possible when
 *                            every operand row is 16-byte aligned and the
 *                            compute type is FP32 or 16-bit (EINVAL
 *                            otherwise); default 1 for 16-bit storage.
 *   CONCPD_OPT_FUSE          1: the dense sweep runs its R x R work in the
 *                            launches of the passes it does not depend on
 *                            (core update beside pass 1, the mode-2 and mode-3
 *                            step matrices beside the mode-2 contraction and
 *                            pass 2): three launches fewer per sweep, fewer
 *                            wavefronts per SIMD for those passes.  Results
 *                            are bit-identical to the unfused sweep.  R > 32
 *                            (and the register path of 16-bit storage) runs
 *                            unfused whatever the value; default 1 when pass 1
 *                            has at most two wavefronts per SIMD, else 0.
 *   CONCPD_OPT_FUSE_LRA      1: the compressed sweep (Algorithm 2) runs the
 *                            core update beside C_1 and the step matrix of
 *                            mode n beside the W refresh of mode n - 1 (ten
 *                            launches instead of thirteen); bit-identical to
 *                            the unfused sweep; default 1.
 * Synchronises.  Errors: EINVAL (unknown option or value), EHIP. */
typedef enum concpd_option {
    CONCPD_OPT_GRAPH_SWEEPS = 1,
    CONCPD_OPT_OVERLAP = 2,
    CONCPD_OPT_K2_ROWS = 3,
    CONCPD_OPT_P1_SPLIT = 4,
    CONCPD_OPT_P1_DMA = 5,
    CONCPD_OPT_FUSE = 6,
    CONCPD_OPT_FUSE_LRA = 7
} concpd_option;
concpd_status concpd_set_option(concpd_ctx ctx, int32_t option, int64_t value);
concpd_status concpd_get_option(concpd_ctx ctx, int32_t option, int64_t* value);

typedef struct concpd_tuning {
    int32_t k2_rows;              /* chosen CONCPD_OPT_K2_ROWS */
    int32_t graph_sweeps;         /* chosen CONCPD_OPT_GRAPH_SWEEPS */
    double us_per_sweep;          /* measured time per sweep of the choice */
    double us_per_sweep_default;  /* of the default configuration */
    int32_t candidates;           /* configurations timed */
    int32_t p1_split;             /* chosen CONCPD_OPT_P1_SPLIT (the split in use) */
    int32_t p1_dma;               /* chosen CONCPD_OPT_P1_DMA */
    int32_t overlap;              /* chosen CONCPD_OPT_OVERLAP */
    int32_t fuse;                 /* chosen CONCPD_OPT_FUSE */
} concpd_tuning;

/* Autotuner: times `sweeps` sweeps (HIP events on the context stream) of
 * candidate launch configurations from the same iterate, restoring the
 * iterate after each, and keeps the fastest: first the pass-1 split 1/2/4
 * (x DMA off/on where possible; dense path), then mode-2 chunk rows 8/16/32 x
 * graph sweeps 0/1/4, then (dense path) the second-stream overlap inside
 * graphs of 1 and 4 sweeps, then (dense path, R <= 32) the fused launches
 * (CONCPD_OPT_FUSE) with direct launches and with the best graph length.
 * The iterate is unchanged on return.  Synchronises.
 * Errors: EINVAL (sweeps not in [1, 10000]), ESTATE (converged iterate), EHIP. */
concpd_status concpd_autotune(concpd_ctx ctx, int32_t sweeps, concpd_tuning* out);

/* Release the host context.  Queued work is synchronised first; the workspace
 * and the tensors stay owned by the caller. */
concpd_status concpd_destroy(concpd_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif /* CONCPD_H */
