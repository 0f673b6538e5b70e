// Host runtime behind the C ABI of concpd.h: configuration checks, workspace
// layout, grouped work lists, the per-iteration launch schedule of
// Algorithm 1 (with the device-side restart test), checkpoint / restore and
// the read-back calls.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/concpd.h"
#include "concpd_internal.h"

// Workspace of concpd_init_static, for callers that cannot allocate device
// memory: an array of the library's own on every device it runs on, held
// until the process ends.  In host code the array's name only stands in for
// it; its device address comes from hipGetSymbolAddress (once per device,
// with that device current) and only that address is ever used.
#define CPD_STATIC_WS_BYTES ((size_t)CONCPD_STATIC_WORKSPACE_BYTES)
#define CPD_MAX_DEVICES 64
static __device__ __align__(256) char scratch[CPD_STATIC_WS_BYTES];

namespace {

thread_local std::string g_err;

concpd_status fail(concpd_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHECK(x)                                                                        \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) return fail(CONCPD_EHIP, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct StaticWs {
    std::mutex mu;
    void* ptr[CPD_MAX_DEVICES] = {};              // device address of scratch per device
    concpd_ctx owner[CPD_MAX_DEVICES] = {};       // the live context using it, if any
};
StaticWs g_static;

#define CPD_PROF_REPS 4   // back-to-back launches of each pass per profiled sweep
// Entry points that exist at order 3 only (the Tucker/ALS path, state
// transfer, autograd, tuning and profiling hooks).
#define NEED_ORDER3(c, what)                                                                   \
    do {                                                                                       \
        if ((c)->N != 3) return fail(CONCPD_ENOTSUP, "%s needs a 3-way context", what);        \
    } while (0)

int operand_bytes(int dtype) { return dtype == CONCPD_F64 ? 8 : (dtype == CONCPD_F32 ? 4 : 2); }

struct Layout {
    size_t geo, ctrl, U[3], lam[3], V[2], b[2], P, Ld_cur, Ld_prev, Lu_cur, Lu_prev, LC_prev, Fblk, normM2, normOrig, Y,
        K3, part, K1p, K2, it1, it2, itk2, itu[CPD_MAXN], itna, itnb, scratch, shadow, lra, fpart, flag, total;
    // loss/gradient evaluation point (autograd form): factors, lambda, Grams,
    // b, step matrices, per-block F, control block, output pointer tables
    size_t gU, glam, gV, gb, gP, gF, gctrl, gptr;
    // autotuner snapshot of the persistent iterate state (ctrl .. normOrig,
    // and the Tucker-form W slots)
    size_t snap, snap_len, snap_w;
    long long uslot, ylen, klen, plen, shadow_elems[CPD_MAXS], shadow_off[CPD_MAXS], shadow_ld[CPD_MAXS], lra_len;
    // lra region (doubles from its base): compression scratch
    long long l_sig, l_part, l_work, l_t1, l_t2, sig_stride, work_stride;
    int nsplit, Imax, Jmax;
    size_t scratch_len;
    int esz;  // bytes per factor element
};

struct Lists {
    std::vector<ItemP1> p1;
    std::vector<ItemP2> p2;
    std::vector<ItemK2> k2;
    std::vector<ItemU> u[CPD_MAXN];
    std::vector<ItemNW> na, nb;   // order N > 3: the two passes of the dimension tree
    int maxI2;
    int lds_rows[CPD_MAXN];
    int p1_split;   // wavefronts per pass-1 item (1, 2 or 4)
};

// Blocks that share mode n's first L_n columns (bit s = block s; 0 when L_n = 0).
uint64_t group_mask(const concpd_config* c, int n) {
    if (c->coupled[n] <= 0) return 0;
    const uint64_t all = c->num_blocks >= 64 ? ~0ull : ((1ull << c->num_blocks) - 1);
    return c->coupled_blocks ? (c->coupled_blocks[n] & all) : all;
}
int first_member(uint64_t m) { return m ? __builtin_ctzll(m) : -1; }
bool in_group(uint64_t m, int s) { return (m >> s) & 1ull; }

concpd_status validate(const concpd_config* c) {
    if (!c) return fail(CONCPD_EINVAL, "config is NULL");
    if (c->order < 3 || c->order > CPD_MAXN) return fail(CONCPD_EINVAL, "order %d not in [3, %d]", c->order, CPD_MAXN);
    const int N = c->order;
    if (c->num_blocks < 1 || c->num_blocks > CPD_MAXS) return fail(CONCPD_EINVAL, "num_blocks %d not in [1, %d]", c->num_blocks, CPD_MAXS);
    if (c->rank < 1 || c->rank > CPD_MAXR) return fail(CONCPD_EINVAL, "rank %d not in [1, %d]", c->rank, CPD_MAXR);
    if (!c->dims) return fail(CONCPD_EINVAL, "dims is NULL");
    for (int n = 0; n < N; ++n)
        if (c->coupled[n] < 0 || c->coupled[n] > c->rank)
            return fail(CONCPD_EINVAL, "coupled[%d] = %d not in [0, rank]", n, c->coupled[n]);
    if (c->coupled_blocks) {
        const uint64_t all = c->num_blocks >= 64 ? ~0ull : ((1ull << c->num_blocks) - 1);
        for (int n = 0; n < N; ++n) {
            if (c->coupled_blocks[n] & ~all) return fail(CONCPD_EINVAL, "coupled_blocks[%d] names blocks >= S", n);
            if (c->coupled[n] > 0 && !c->coupled_blocks[n])
                return fail(CONCPD_EINVAL, "coupled_blocks[%d] selects no block for L = %d", n, c->coupled[n]);
        }
    }
    for (int s = 0; s < c->num_blocks; ++s) {
        long long nel = 1;
        for (int n = 0; n < N; ++n) {
            const int64_t d = c->dims[N * s + n];
            if (d < 1 || d > (1 << 24)) return fail(CONCPD_EINVAL, "dims[%d] = %lld out of range", N * s + n, (long long)d);
            nel *= d;
            if (nel > (1LL << 40)) return fail(CONCPD_EINVAL, "block %d has more than 2^40 elements", s);
            const uint64_t gm = group_mask(c, n);
            const int f = first_member(gm);
            if (in_group(gm, s) && d != c->dims[N * f + n])
                return fail(CONCPD_EINVAL, "mode %d is coupled but block %d has I=%lld != %lld", n, s, (long long)d,
                            (long long)c->dims[N * f + n]);
        }
    }
    if (N > 3) {
        if (c->compute_dtype != CONCPD_F32 && c->compute_dtype != CONCPD_F64)
            return fail(CONCPD_ENOTSUP, "order %d supports compute_dtype F32 or F64", N);
        if (c->tucker_ranks) return fail(CONCPD_ENOTSUP, "lra compression needs order 3");
    }
    if (c->tensor_dtype != CONCPD_F64 && c->tensor_dtype != CONCPD_F32)
        return fail(CONCPD_EINVAL, "tensor_dtype must be F64 or F32");
    if (c->compute_dtype < CONCPD_F64 || c->compute_dtype > CONCPD_F16) return fail(CONCPD_EINVAL, "bad compute_dtype");
    if (c->compute_dtype == CONCPD_F64 && c->tensor_dtype != CONCPD_F64)
        return fail(CONCPD_EINVAL, "compute_dtype F64 needs F64 tensors");
    if (c->compute_dtype != CONCPD_F64 && c->tensor_dtype == CONCPD_F64)
        return fail(CONCPD_ENOTSUP, "F64 tensors are only supported with compute_dtype F64");
    if (c->compute_dtype == CONCPD_F64 && c->rank > 32) return fail(CONCPD_ENOTSUP, "compute_dtype F64 supports rank <= 32");
    if (!(c->delta_w >= 0.0 && c->delta_w < 1.0)) return fail(CONCPD_EINVAL, "delta_w must be in [0, 1)");
    if (!(c->tol >= 0.0)) return fail(CONCPD_EINVAL, "tol must be >= 0");
    if (c->max_it < 0) return fail(CONCPD_EINVAL, "max_it must be >= 0");
    if (c->tucker_ranks)
        for (int s = 0; s < c->num_blocks; ++s)
            for (int n = 0; n < 3; ++n) {
                const int J = c->tucker_ranks[3 * s + n];
                if (J < 1 || J > c->dims[3 * s + n] || J > 64)
                    return fail(CONCPD_EINVAL, "tucker_ranks[%d] = %d must be in [1, min(I_n, 64)]", 3 * s + n, J);
                if (c->dims[3 * s + n] > 512)
                    return fail(CONCPD_ENOTSUP, "lra compression supports I_n <= 512 (block %d mode %d)", s, n);
            }
    if (c->block_ranks) {
        for (int s = 0; s < c->num_blocks; ++s) {
            int lmax = 1;
            for (int n = 0; n < N; ++n)
                if (in_group(group_mask(c, n), s)) lmax = std::max(lmax, c->coupled[n]);
            if (c->block_ranks[s] < lmax || c->block_ranks[s] > c->rank)
                return fail(CONCPD_EINVAL, "block_ranks[%d] = %d not in [max(1, L_n), rank]", s, c->block_ranks[s]);
        }
    }
    if (c->tucker_ranks && c->tensor_dtype != CONCPD_F32)
        return fail(CONCPD_ENOTSUP, "lra compression needs F32 tensors");
    if (c->tucker_ranks) {
        int jm = 1;
        for (int i = 0; i < 3 * c->num_blocks; ++i) jm = std::max(jm, (int)c->tucker_ranks[i]);
        if (cpd::lra_c_lds_bytes(jm, (c->rank + 3) / 4 * 4) > 65536)
            return fail(CONCPD_ENOTSUP, "Tucker rank %d with rank %d exceeds the core-contraction LDS budget", jm, c->rank);
    }
    return CONCPD_OK;
}

// Workgroups are dealt to the 8 XCDs round-robin (blockIdx % 8), and each XCD
// has its own L2.  Reordering a list built in memory order so that XCD x runs
// the contiguous range x * n / 8 .. of it keeps items that share cache lines
// (neighbouring row segments of the tensor, of Y) in one L2.
template <typename Item>
void xcd_order(std::vector<Item>& v, size_t grp = 1) {
    // v holds whole workgroups of grp consecutive items
    const size_t ng = v.size() / grp, n8 = ng - ng % 8, per = n8 / 8;
    if (per < 2) return;
    std::vector<Item> out(v.size());
    for (size_t b = 0; b < n8; ++b)
        for (size_t j = 0; j < grp; ++j) out[b * grp + j] = v[((b % 8) * per + b / 8) * grp + j];
    for (size_t b = n8 * grp; b < v.size(); ++b) out[b] = v[b];
    v.swap(out);
}

// Order N > 3: the split h of the dimension tree (the one with the smallest
// intermediates sum_s A_s + B_s) and the contraction parts of both passes:
// each pass gets about 2048 wavefronts (eight per CU), a part covers at least
// 64 values of the contraction, in whole chunks of 16.
struct NwPlan {
    int h = 0;
    long long A[CPD_MAXS], B[CPD_MAXS], kpa[CPD_MAXS], kpb[CPD_MAXS];
    int npa[CPD_MAXS], npb[CPD_MAXS];
};
void nw_plan(const concpd_config* c, NwPlan* P) {
    const int S = c->num_blocks, N = c->order;
    long long best = -1;
    for (int h = 1; h < N; ++h) {
        long long tot = 0;
        for (int s = 0; s < S; ++s) {
            long long a = 1, b = 1;
            for (int m = 0; m < N; ++m) (m < h ? a : b) *= c->dims[N * s + m];
            tot += a + b;
        }
        if (best < 0 || tot < best) {
            best = tot;
            P->h = h;
        }
    }
    long long oga = 0, ogb = 0;
    for (int s = 0; s < S; ++s) {
        long long a = 1, b = 1;
        for (int m = 0; m < N; ++m) (m < P->h ? a : b) *= c->dims[N * s + m];
        P->A[s] = a;
        P->B[s] = b;
        oga += (a + 63) / 64;
        ogb += (b + 63) / 64;
    }
    const long long want = 2048;
    auto parts = [&](long long og, long long K, int* np, long long* kp) {
        long long p = std::max(1LL, (want + og - 1) / og);
        p = std::min(p, std::max(1LL, K / 64));
        long long per = (K + p - 1) / p;
        per = (per + 15) / 16 * 16;
        *kp = per;
        *np = (int)((K + per - 1) / per);
    };
    for (int s = 0; s < S; ++s) {
        parts(oga, P->B[s], &P->npa[s], &P->kpa[s]);
        parts(ogb, P->A[s], &P->npb[s], &P->kpb[s]);
    }
}

// i1 slabs per pass-2 wavefront (a pass-2 workgroup takes 4 p2_slabs slabs):
// two when that still leaves at least 2048 workgroups (eight per compute
// unit) and every block's U^(2) is short enough to be staged once (I2 <= 128),
// which halves the mode-3 partials and the U^(2) staging per tensor byte; else
// one (always one for FP64 operands).  CONCPD_P2_SLABS=1 or 2 overrides the
// choice (measurements).
int p2_slabs(const concpd_config* c) {
    if (c->order != 3 || c->compute_dtype == CONCPD_F64) return 1;
    const char* ev = getenv("CONCPD_P2_SLABS");
    if (ev && (ev[0] == '1' || ev[0] == '2') && ev[1] == 0) return ev[0] - '0';
    long long wg = 0;
    for (int s = 0; s < c->num_blocks; ++s) {
        const long long I1 = c->dims[3 * s], I2 = c->dims[3 * s + 1], I3 = c->dims[3 * s + 2];
        if (I2 > 128) return 1;
        wg += ((I1 + 7) / 8) * ((I3 + 63) / 64);
    }
    return wg >= 2048 ? 2 : 1;
}

void build_lists(const concpd_config* c, Lists* L, int k2rows = CPD_K2ROWS_DEFAULT, int p1split = 0) {
    const int S = c->num_blocks, R = c->rank, Rq = (R + 3) / 4 * 4, N = c->order;
    L->p1.clear();
    L->p2.clear();
    L->k2.clear();
    L->na.clear();
    L->nb.clear();
    L->maxI2 = 1;
    L->p1_split = 1;
    if (N > 3) {
        NwPlan W;
        nw_plan(c, &W);
        for (int s = 0; s < S; ++s) {
            for (int og = 0; og * 64LL < W.A[s]; ++og)
                for (int p = 0; p < W.npa[s]; ++p) L->na.push_back({s, og, p, 0});
            for (int og = 0; og * 64LL < W.B[s]; ++og)
                for (int p = 0; p < W.npb[s]; ++p) L->nb.push_back({s, og, p, 0});
        }
        while (L->na.size() % 4) L->na.push_back({-1, 0, 0, 0});
        while (L->nb.size() % 4) L->nb.push_back({-1, 0, 0, 0});
        xcd_order(L->na, 4);
        xcd_order(L->nb, 4);
    }
    // the two-pass MTTKRP work lists exist at order 3 only
    const int spw = p2_slabs(c);
    for (int s = 0; s < S && N == 3; ++s) {
        const int I1 = (int)c->dims[3 * s], I2 = (int)c->dims[3 * s + 1], I3 = (int)c->dims[3 * s + 2];
        L->maxI2 = std::max(L->maxI2, I2);
        for (int ch = 0; ch * k2rows < I1; ++ch)
            for (long long c0 = 0; c0 < (long long)I2 * Rq; c0 += 256) L->k2.push_back({s, (int)c0, ch, 0});
        for (int i1 = 0; i1 < I1; ++i1)
            for (int rg = 0; rg * 64 < I2; ++rg) L->p1.push_back({s, i1, rg, 0});
        for (int ch = 0; ch * 4 * spw < I1; ++ch)
            for (int q0 = 0; q0 < I3; q0 += 64) L->p2.push_back({s, ch, q0, 0});
    }
    // pass 1: the smallest split P of i3 over wavefronts that gives at least
    // 1.5 wavefronts per SIMD (1536 on 1024 SIMDs; measured: 2000 items
    // stream best unsplit, 1024 items split in two), no more than the 64-byte
    // chunks of the shortest row;
    // the list is padded to whole workgroups (4 / P items) with empty items
    if (N == 3) {
        int minck = 1 << 30;
        for (int s = 0; s < S; ++s) minck = std::min(minck, (int)((c->dims[3 * s + 2] + 15) / 16));
        int P = 1;
        if (p1split > 0) P = p1split;
        else
            while (P < 4 && L->p1.size() * P < 1536 && 2 * P <= minck) P *= 2;
        L->p1_split = P;
        while (L->p1.size() % (4 / P)) L->p1.push_back({-1, 0, 0, 0});
        xcd_order(L->p1, 4 / P);
    }
    xcd_order(L->p2);
    xcd_order(L->k2);
    for (int n = 0; n < N; ++n) {
        L->u[n].clear();
        int lds_rows = 1;
        if (c->coupled[n] > 0) {
            // the coupling group's rows, all its blocks in one item (ns < 0),
            // then the blocks outside the group with individual columns
            const uint64_t gm = group_mask(c, n);
            const int nm = __builtin_popcountll(gm);
            const int I = (int)c->dims[N * first_member(gm) + n];
            int nrows = std::max(1, 256 / (nm * R));
            // LDS: ns * nrows * 2R doubles <= 48 KiB
            while (nrows > 1 && (size_t)nm * nrows * 2 * R * 8 > 49152) --nrows;
            for (int r0 = 0; r0 < I; r0 += nrows) L->u[n].push_back({0, -nm, r0, std::min(nrows, I - r0)});
            lds_rows = nm * nrows;
            const int nri = std::max(1, 256 / R);
            for (int s = 0; s < S; ++s) {
                if (in_group(gm, s)) continue;
                const int Is = (int)c->dims[N * s + n];
                for (int r0 = 0; r0 < Is; r0 += nri) L->u[n].push_back({s, 1, r0, std::min(nri, Is - r0)});
                lds_rows = std::max(lds_rows, nri);
            }
        } else {
            const int nrows = std::max(1, 256 / R);
            for (int s = 0; s < S; ++s) {
                const int I = (int)c->dims[N * s + n];
                for (int r0 = 0; r0 < I; r0 += nrows) L->u[n].push_back({s, 1, r0, std::min(nrows, I - r0)});
            }
            lds_rows = nrows;
        }
        L->lds_rows[n] = lds_rows;
    }
}

void plan(const concpd_config* c, const Lists& L, Layout* P, Geo* g) {
    memset(P, 0, sizeof *P);
    memset(g, 0, sizeof *g);
    const int S = c->num_blocks, R = c->rank, Rq = (R + 3) / 4 * 4, N = c->order;
    const bool f64 = c->compute_dtype == CONCPD_F64;
    P->esz = f64 ? 8 : 4;
    g->N = N;
    g->S = S;
    g->R = R;
    g->Rq = Rq;
    for (int n = 0; n < N; ++n) {
        g->L[n] = c->coupled[n];
        const uint64_t gm = group_mask(c, n);
        g->ngrp[n] = 0;
        for (int s = 0; s < c->num_blocks; ++s)
            if (c->coupled[n] <= 0 || in_group(gm, s)) g->grp[n][g->ngrp[n]++] = s;
    }
    g->upd_core = c->update_core;
    g->mdtype = c->compute_dtype;
    g->k2rows = CPD_K2ROWS_DEFAULT;
    long long u = 0, y = 0, k = 0, p = 0, k1 = 0, k2 = 0;
    for (int n = 0; n < N; ++n)
        for (int s = 0; s < S; ++s) {
            g->uoff[n][s] = u;
            u += c->dims[N * s + n] * Rq;
        }
    if (N > 3) {
        // order N > 3: one MTTKRP buffer per block (the mode in work), the
        // partials of both passes in the Y region, the Khatri-Rao operand in
        // the part region
        NwPlan W;
        nw_plan(c, &W);
        g->nh = W.h;
        for (int s = 0; s < S; ++s) {
            for (int n = 0; n < N; ++n) g->I[s][n] = (int)c->dims[N * s + n];
            long long im = 1;
            for (int n = 0; n < N; ++n) im = std::max<long long>(im, c->dims[N * s + n]);
            g->koff[s] = k;
            k += im * Rq;
            g->nwA[s] = W.A[s];
            g->nwB[s] = W.B[s];
            g->npa[s] = W.npa[s];
            g->npb[s] = W.npb[s];
            g->kpa[s] = W.kpa[s];
            g->kpb[s] = W.kpb[s];
            g->taoff[s] = y;
            y += (long long)W.npa[s] * W.A[s] * Rq;
            g->tboff[s] = y;
            y += (long long)W.npb[s] * W.B[s] * Rq;
            g->kroff[s] = p;
            p += std::max(W.A[s], W.B[s]) * Rq;
        }
    }
    g->p2spw = p2_slabs(c);
    for (int s = 0; s < S && N == 3; ++s) {
        const long long I1 = c->dims[3 * s], I2 = c->dims[3 * s + 1], I3 = c->dims[3 * s + 2];
        for (int n = 0; n < 3; ++n) g->I[s][n] = (int)c->dims[3 * s + n];
        g->yoff[s] = y;
        y += I1 * I2 * Rq;
        g->koff[s] = k;
        k += I3 * Rq;
        g->nchunk[s] = (int)((I1 + 4 * g->p2spw - 1) / (4 * g->p2spw));
        g->poff[s] = p;
        p += g->nchunk[s] * I3 * Rq;
        g->nrg[s] = (int)((I2 + 63) / 64);
        g->k1off[s] = k1;
        k1 += I1 * g->nrg[s] * Rq;
        g->k2off[s] = k2;
        g->nk2[s] = (int)((I1 + CPD_K2ROWS_DEFAULT - 1) / CPD_K2ROWS_DEFAULT);
        k2 += ((I1 + CPD_K2ROWS_MIN - 1) / CPD_K2ROWS_MIN) * I2 * Rq;   // room for the smallest chunk
    }
    // the finish over the last mode in chunks of CPD_FIN_ROWS rows
    {
        int c0 = 0;
        for (int s = 0; s < S; ++s) {
            const long long In = c->dims[(size_t)N * s + N - 1];
            g->fin_nc[s] = In > CPD_FIN_ROWS ? (int)((In + CPD_FIN_ROWS - 1) / CPD_FIN_ROWS) : 1;
            g->fin_c0[s] = c0;
            c0 += g->fin_nc[s];
        }
        g->fin_nwg = c0;
    }
    P->uslot = u;
    P->ylen = y;
    P->klen = k;
    P->plen = p;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    P->geo = take(sizeof(Geo));
    P->ctrl = take(sizeof(Ctrl));
    for (int i = 0; i < 3; ++i) P->U[i] = take((size_t)u * P->esz);
    for (int i = 0; i < 3; ++i) P->lam[i] = take(sizeof(double) * S * Rq);
    for (int i = 0; i < 2; ++i) P->V[i] = take(sizeof(double) * N * S * R * R);
    for (int i = 0; i < 2; ++i) P->b[i] = take(sizeof(double) * S * Rq);
    P->P = take(sizeof(double) * S * R * R);
    P->Ld_cur = take(sizeof(double) * S);
    P->Ld_prev = take(sizeof(double) * S);
    P->Lu_cur = take(sizeof(double) * N * S);
    P->Lu_prev = take(sizeof(double) * N * S);
    P->LC_prev = take(sizeof(double) * N);
    P->Fblk = take(sizeof(double) * S);
    P->normM2 = take(sizeof(double) * S);
    P->normOrig = take(sizeof(double) * S);
    P->Y = take((size_t)y * P->esz);
    P->K3 = take((size_t)k * P->esz);
    P->part = take((size_t)p * P->esz);
    P->K1p = take((size_t)k1 * P->esz);
    P->K2 = take((size_t)k2 * P->esz);
    P->it1 = take(sizeof(ItemP1) * (L.p1.size() + 4));   // room for the padding of any split
    P->it2 = take(sizeof(ItemP2) * std::max<size_t>(1, L.p2.size()));
    {
        Lists Lmin;
        build_lists(c, &Lmin, CPD_K2ROWS_MIN);
        P->itk2 = take(sizeof(ItemK2) * std::max<size_t>(1, std::max(L.k2.size(), Lmin.k2.size())));
    }
    for (int n = 0; n < N; ++n) P->itu[n] = take(sizeof(ItemU) * std::max<size_t>(1, L.u[n].size()));
    P->itna = take(sizeof(ItemNW) * std::max<size_t>(1, L.na.size()));
    P->itnb = take(sizeof(ItemNW) * std::max<size_t>(1, L.nb.size()));
    size_t scr = 4096;
    for (int s = 0; s < S; ++s) scr = std::max<size_t>(scr, (size_t)c->dims[N * s]);
    P->scratch_len = scr;
    P->scratch = take(sizeof(double) * scr);
    P->fpart = take(sizeof(double) * (size_t)g->fin_nwg * ((size_t)R * R + Rq));
    P->flag = take(sizeof(int) * 4);
    P->gU = take((size_t)u * P->esz);
    P->glam = take(sizeof(double) * S * Rq);
    P->gV = take(sizeof(double) * 3 * S * R * R);
    P->gb = take(sizeof(double) * S * Rq);
    P->gP = take(sizeof(double) * 3 * S * R * R);
    P->gF = take(sizeof(double) * S);
    P->gctrl = take(sizeof(Ctrl));
    P->gptr = take(sizeof(void*) * 4 * S);
    P->snap_len = P->normOrig + sizeof(double) * S - P->ctrl;
    P->snap = take(P->snap_len);
    P->snap_w = 0;
    {
        // Operand copies: every block of a 16-bit compute type, and every
        // block whose rows would not start 16-byte aligned, gets a copy with
        // rows padded to ld = I3 rounded up to 16 bytes, 256-byte aligned.
        const int me = operand_bytes(c->compute_dtype), ve = 16 / me;
        const bool half = c->compute_dtype == CONCPD_BF16 || c->compute_dtype == CONCPD_F16;
        size_t tot = 0;
        // (order N > 3 reads the caller's tensors directly)
        for (int s = 0; s < S && N == 3; ++s) {
            const long long I3 = c->dims[3 * s + 2];
            const bool copy = half || I3 % ve != 0;
            const long long ld = (I3 + ve - 1) / ve * ve;
            P->shadow_ld[s] = copy ? ld : 0;
            P->shadow_elems[s] = copy ? c->dims[3 * s] * c->dims[3 * s + 1] * ld : 0;
            P->shadow_off[s] = (long long)tot;
            if (copy) tot = align256(tot + (size_t)P->shadow_elems[s] * me);
        }
        P->shadow = tot ? take(tot) : 0;
    }
    if (c->tucker_ranks) {
        long long a = 0;
        int Imax = 1, Jmax = 1;
        long long t1 = 1, t2 = 1;
        for (int n = 0; n < 3; ++n)
            for (int s = 0; s < S; ++s) {
                const int J = c->tucker_ranks[3 * s + n];
                g->J[s][n] = J;
                g->aoff[n][s] = a;
                a += c->dims[3 * s + n] * J;
                Imax = std::max(Imax, (int)c->dims[3 * s + n]);
                Jmax = std::max(Jmax, J);
            }
        for (int s = 0; s < S; ++s) {
            g->goff[s] = a;
            a += (long long)g->J[s][0] * g->J[s][1] * g->J[s][2];
            t1 = std::max<long long>(t1, c->dims[3 * s] * c->dims[3 * s + 1] * g->J[s][2]);
            t2 = std::max<long long>(t2, c->dims[3 * s] * (long long)g->J[s][1] * g->J[s][2]);
        }
        long long w = 0;
        for (int n = 0; n < 3; ++n)
            for (int s = 0; s < S; ++s) {
                g->woff[n][s] = a + w;
                w += (long long)g->J[s][n] * Rq;
            }
        g->wslot_len = w;
        a += 2 * w;
        for (int s = 0; s < S; ++s) {
            g->coff[s] = a;
            a += (long long)Jmax * Rq;
        }
        P->nsplit = 16;
        P->Imax = Imax;
        P->Jmax = Jmax;
        P->sig_stride = (long long)Imax * Imax;
        P->work_stride = 4LL * Imax + 64 + 5LL * Imax * Jmax;
        P->l_sig = a;
        a += 3LL * S * P->sig_stride;
        P->l_work = a;
        a += 3LL * S * P->work_stride;
        P->l_part = a;
        a += (long long)P->nsplit * Imax * Imax;
        P->l_t1 = a;
        a += t1;
        P->l_t2 = a;
        a += t2;
        P->lra_len = a;
        P->lra = take(sizeof(double) * (size_t)a);
        P->snap_w = take(sizeof(double) * 2 * (size_t)g->wslot_len);
    }
    P->total = off;
}

// SplitMix64 (Steele, Lea, Flood 2014) -> uniform doubles in [0, 1).
struct SplitMix64 {
    uint64_t x;
    uint64_t next() {
        uint64_t z = (x += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

}  // namespace

struct concpd_ctx_s {
    concpd_config cfg;
    std::vector<int64_t> dims;
    std::vector<int32_t> tucker;
    int N;                 // tensor order
    int S, R, Rq, L[CPD_MAXN];
    std::vector<int> rk;   // R^(s): block s uses columns 0..rk[s]-1, the rest stay zero
    uint64_t cmask[CPD_MAXN];   // the caller's coupling groups (copied)
    bool f64;
    int mdtype;
    std::vector<const void*> tensors;
    char* ws;
    hipStream_t q;
    Layout lay;
    Lists lists;
    Geo geo;
    Geo* dgeo;
    StateP<float> sf;
    StateP<double> sd;
    Ctrl* ctrl;
    int lra;
    std::vector<double> normOrig;
    long long launched_iters;
    int profiling;
    // CONCPD_OVERLAP=1 runs the small FP64 kernels (core update, step
    // matrices) on a second stream beside the MTTKRP passes they do not depend
    // on.  Off by default: with direct launches the cross-stream event waits
    // cost more than the overlap gains; inside a captured graph they are graph
    // edges, and the autotuner tries that (measured: 8 % faster sweeps on the
    // EEG-shaped blocks, neutral on the cubes).
    int overlap;
    hipStream_t q2;
    hipEvent_t fj[6];
    // CONCPD_OPT_GRAPH_SWEEPS > 0: sweeps are replayed from a captured graph
    // of that many sweeps (captured on a private stream, launched on q)
    int graph_sweeps;
    hipStream_t qcap;
    hipGraphExec_t gexec;
    int k2rows;
    int p1split = 0;   // requested pass-1 split (0: automatic)
    int p1dma = 0, p1dma_ok = 0;   // pass 1 by LDS DMA (in use / possible)
    int fuse = 0;                  // R x R work fused into the launches of independent passes
    int fuse_dflt = 0;             // its default (pass 1 with few wavefronts per SIMD)
    int fuse_lra = 1;              // the compressed sweep's fused launches (default on)
    int static_dev = -1;           // device whose static workspace this context holds (-1: none)
    std::vector<hipEvent_t> ev1, ev2;  // begin/end pairs of timed pass launches
    void drop_graph() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        gexec = nullptr;
    }
    ~concpd_ctx_s() {
        drop_graph();
        if (qcap) (void)hipStreamDestroy(qcap);
        if (q2) {
            (void)hipStreamSynchronize(q2);
            for (int i = 0; i < 6; ++i) (void)hipEventDestroy(fj[i]);
            (void)hipStreamDestroy(q2);
        }
    }
};

namespace {

template <typename T>
StateP<T> make_state(char* ws, const Layout& P) {
    StateP<T> st;
    for (int i = 0; i < 3; ++i) st.U[i] = (T*)(ws + P.U[i]);
    for (int i = 0; i < 3; ++i) st.lam[i] = (double*)(ws + P.lam[i]);
    for (int i = 0; i < 2; ++i) st.V[i] = (double*)(ws + P.V[i]);
    for (int i = 0; i < 2; ++i) st.b[i] = (double*)(ws + P.b[i]);
    st.P = (double*)(ws + P.P);
    st.Ld_cur = (double*)(ws + P.Ld_cur);
    st.Ld_prev = (double*)(ws + P.Ld_prev);
    st.Lu_cur = (double*)(ws + P.Lu_cur);
    st.Lu_prev = (double*)(ws + P.Lu_prev);
    st.LC_prev = (double*)(ws + P.LC_prev);
    st.Fblk = (double*)(ws + P.Fblk);
    st.normM2 = (double*)(ws + P.normM2);
    st.Y = (T*)(ws + P.Y);
    st.K3 = (T*)(ws + P.K3);
    st.part = (T*)(ws + P.part);
    st.K1p = (T*)(ws + P.K1p);
    st.K2 = (T*)(ws + P.K2);
    st.lra = (double*)(ws + P.lra);
    st.fpart = (double*)(ws + P.fpart);
    st.ctrl = (Ctrl*)(ws + P.ctrl);
    return st;
}

// One sweep of Algorithm 1 (extrapolated, or the redo of a rejected sweep:
// the kernels read that from the control block).
template <typename T>
void run_sweep(concpd_ctx c, const StateP<T>& st) {
    const int extrap = 1;
    const Geo* g = c->dgeo;
    const int S = c->S, R = c->R, Rq = c->Rq;
    hipStream_t q = c->q;
    const ItemP1* it1 = (const ItemP1*)(c->ws + c->lay.it1);
    const ItemP2* it2 = (const ItemP2*)(c->ws + c->lay.it2);
    const ItemK2* itk = (const ItemK2*)(c->ws + c->lay.itk2);
    const ItemU* itu[3];
    for (int n = 0; n < 3; ++n) itu[n] = (const ItemU*)(c->ws + c->lay.itu[n]);
    const bool prof = c->profiling;
    hipEvent_t e[4];
    if (prof)
        for (int i = 0; i < 4; ++i) (void)hipEventCreate(&e[i]);
    if (c->fuse) {
        // the R x R work beside the passes it does not depend on, in the same launches
        const int ni1 = (int)c->lists.p1.size(), P = c->lists.p1_split;
        if (prof) (void)hipEventRecord(e[0], q);
        for (int rep = 0; rep < (prof ? CPD_PROF_REPS : 1); ++rep)
            if (!cpd::launch_core_pass1<T>(g, st, it1, ni1, P, R, 1, c->mdtype, c->p1dma, extrap, S, q)) {
                cpd::launch_core<T>(g, st, S, R, extrap, q);
                cpd::launch_pass1<T>(g, st, it1, ni1, P, Rq, 1, c->mdtype, c->p1dma, q);
            }
        if (prof) (void)hipEventRecord(e[1], q);
        cpd::launch_update<T>(g, st, itu[0], (int)c->lists.u[0].size(), 0, R, extrap, c->lists.lds_rows[0], 0, q);
        if (!cpd::launch_prep_k2<T>(g, st, itk, (int)c->lists.k2.size(), R, 0, S, q)) {
            cpd::launch_prep<T>(g, st, S, R, 1, q);
            cpd::launch_k2<T>(g, st, itk, (int)c->lists.k2.size(), 0, q);
        }
        cpd::launch_update<T>(g, st, itu[1], (int)c->lists.u[1].size(), 1, R, extrap, c->lists.lds_rows[1], 0, q);
        if (prof) (void)hipEventRecord(e[2], q);
        for (int rep = 0; rep < (prof ? CPD_PROF_REPS : 1); ++rep)
            if (!cpd::launch_prep_pass2<T>(g, st, it2, (int)c->lists.p2.size(), R, 0, c->mdtype, c->lists.maxI2, c->geo.p2spw, S, q)) {
                cpd::launch_prep<T>(g, st, S, R, 2, q);
                cpd::launch_pass2<T>(g, st, it2, (int)c->lists.p2.size(), Rq, 0, c->mdtype, c->lists.maxI2, c->geo.p2spw, q);
            }
        if (prof) {
            (void)hipEventRecord(e[3], q);
            c->ev1.push_back(e[0]);
            c->ev1.push_back(e[1]);
            c->ev2.push_back(e[2]);
            c->ev2.push_back(e[3]);
        }
        cpd::launch_update<T>(g, st, itu[2], (int)c->lists.u[2].size(), 2, R, extrap, c->lists.lds_rows[2], 0, q);
        cpd::launch_finish<T>(g, st, S, R, c->geo.fin_nwg, q);
        return;
    }
    // the second stream (if any) takes the small FP64 kernels
    hipStream_t qa = c->overlap ? c->q2 : q;
    auto fork = [&](int i) {
        if (!c->overlap) return;
        (void)hipEventRecord(c->fj[i], q);
        (void)hipStreamWaitEvent(c->q2, c->fj[i], 0);
    };
    auto join = [&](int i) {
        if (!c->overlap) return;
        (void)hipEventRecord(c->fj[i], c->q2);
        (void)hipStreamWaitEvent(q, c->fj[i], 0);
    };
    // core update beside pass 1 (Y from the old U^(3), mode-1 partials)
    fork(0);
    cpd::launch_core<T>(g, st, S, R, extrap, qa);
    // profiled sweeps launch each pass CPD_PROF_REPS times back to back between
    // the events (a pass is a pure function of the iterate within a sweep, so
    // the repeats rewrite the same outputs); the event pair then measures the
    // launches and not the dispatch gap before the first one
    if (prof) (void)hipEventRecord(e[0], q);
    for (int rep = 0; rep < (prof ? CPD_PROF_REPS : 1); ++rep)
        cpd::launch_pass1<T>(g, st, it1, (int)c->lists.p1.size(), c->lists.p1_split, Rq, 1, c->mdtype, c->p1dma, q);
    if (prof) (void)hipEventRecord(e[1], q);
    join(1);
    cpd::launch_update<T>(g, st, itu[0], (int)c->lists.u[0].size(), 0, R, extrap, c->lists.lds_rows[0], 0, q);
    // mode-2 step matrix beside the mode-2 contraction (new U^(1))
    fork(2);
    cpd::launch_prep<T>(g, st, S, R, 1, qa);
    cpd::launch_k2<T>(g, st, itk, (int)c->lists.k2.size(), 0, q);
    join(3);
    cpd::launch_update<T>(g, st, itu[1], (int)c->lists.u[1].size(), 1, R, extrap, c->lists.lds_rows[1], 0, q);
    // mode-3 step matrix beside pass 2 (new U^(1), U^(2))
    fork(4);
    cpd::launch_prep<T>(g, st, S, R, 2, qa);
    if (prof) (void)hipEventRecord(e[2], q);
    for (int rep = 0; rep < (prof ? CPD_PROF_REPS : 1); ++rep)
        cpd::launch_pass2<T>(g, st, it2, (int)c->lists.p2.size(), Rq, 0, c->mdtype, c->lists.maxI2, c->geo.p2spw, q);
    if (prof) {
        (void)hipEventRecord(e[3], q);
        c->ev1.push_back(e[0]);
        c->ev1.push_back(e[1]);
        c->ev2.push_back(e[2]);
        c->ev2.push_back(e[3]);
    }
    join(5);
    cpd::launch_update<T>(g, st, itu[2], (int)c->lists.u[2].size(), 2, R, extrap, c->lists.lds_rows[2], 0, q);
    cpd::launch_finish<T>(g, st, S, R, c->geo.fin_nwg, q);
}

// The same sweep with the gradients taken from the Tucker form (Algorithm 2).
template <typename T>
void run_sweep_lra(concpd_ctx c, const StateP<T>& st) {
    const int extrap = 1;
    const Geo* g = c->dgeo;
    const int S = c->S, R = c->R, J = c->lay.Jmax;
    hipStream_t q = c->q;
    const ItemU* itu[3];
    for (int n = 0; n < 3; ++n) itu[n] = (const ItemU*)(c->ws + c->lay.itu[n]);
    if (c->fuse_lra) {
        // the R x R work beside the lra work it does not depend on: ten launches
        cpd::launch_core_lrac<T>(g, st, S, R, J, c->Rq, extrap, q);
        for (int n = 0; n < 3; ++n) {
            if (n > 0) {
                cpd::launch_prep_lraw<T>(g, st, S, R, J, c->Rq, n, q);
                cpd::launch_lra_c<T>(g, st, S, J, c->Rq, n, q);
            }
            cpd::launch_update<T>(g, st, itu[n], (int)c->lists.u[n].size(), n, R, extrap, c->lists.lds_rows[n], 1, q);
        }
        cpd::launch_lra_w<T>(g, st, S, J, 2, 0, 0, q);
        cpd::launch_finish<T>(g, st, S, R, c->geo.fin_nwg, q);
        return;
    }
    cpd::launch_core<T>(g, st, S, R, extrap, q);
    for (int n = 0; n < 3; ++n) {
        if (n > 0) cpd::launch_prep<T>(g, st, S, R, n, q);
        cpd::launch_lra_c<T>(g, st, S, J, c->Rq, n, q);
        cpd::launch_update<T>(g, st, itu[n], (int)c->lists.u[n].size(), n, R, extrap, c->lists.lds_rows[n], 1, q);
        cpd::launch_lra_w<T>(g, st, S, J, n, 0, 0, q);
    }
    cpd::launch_finish<T>(g, st, S, R, c->geo.fin_nwg, q);
}

// Largest A_s, B_s and I_n of an order-N context (launch grids).
void nw_extents(concpd_ctx c, long long* maxA, long long* maxB, int* maxI) {
    *maxA = *maxB = 1;
    *maxI = 1;
    for (int s = 0; s < c->S; ++s) {
        *maxA = std::max(*maxA, c->geo.nwA[s]);
        *maxB = std::max(*maxB, c->geo.nwB[s]);
        for (int n = 0; n < c->N; ++n) *maxI = std::max(*maxI, c->geo.I[s][n]);
    }
}

// The sweep at order N > 3: core update, then modes 0..h-1 from pass A (x_{k-1}
// factors of modes h..N-1), pass B with the new modes 0..h-1, modes h..N-1.
template <typename T>
void run_sweep_nw(concpd_ctx c, const StateP<T>& st) {
    const int extrap = 1;
    const Geo* g = c->dgeo;
    const int S = c->S, R = c->R, Rq = c->Rq, N = c->N, h = c->geo.nh;
    hipStream_t q = c->q;
    long long maxA, maxB;
    int maxI;
    nw_extents(c, &maxA, &maxB, &maxI);
    const ItemNW* ita = (const ItemNW*)(c->ws + c->lay.itna);
    const ItemNW* itb = (const ItemNW*)(c->ws + c->lay.itnb);
    // the core update beside pass A's Khatri-Rao operand, each mode's step
    // matrix beside its contraction (independent work, one launch each)
    cpd::launch_nw_core_kr<T>(g, st, S, R, extrap, maxB, Rq, q);
    cpd::launch_nw_pass<T>(g, st, ita, (int)c->lists.na.size(), 0, Rq, 1, q);
    for (int n = 0; n < N; ++n) {
        if (n == h) {
            cpd::launch_nw_kr<T>(g, st, S, 1, 0, maxA, Rq, 1, q);
            cpd::launch_nw_pass<T>(g, st, itb, (int)c->lists.nb.size(), 1, Rq, 1, q);
        }
        if (n > 0) cpd::launch_nw_prep_contract<T>(g, st, S, R, n, maxI, Rq, q);
        else cpd::launch_nw_contract<T>(g, st, S, n, 0, maxI, Rq, 1, q);
        cpd::launch_update<T>(g, st, (const ItemU*)(c->ws + c->lay.itu[n]), (int)c->lists.u[n].size(), n, R, extrap,
                              c->lists.lds_rows[n], 2, q);
    }
    cpd::launch_finish<T>(g, st, S, R, c->geo.fin_nwg, q);
}

// One sweep: either an accepted iteration, or an extrapolated sweep that the
// restart test rejects (then the next sweep redoes it and is accepted).
template <typename T>
void run_one_sweep(concpd_ctx c, const StateP<T>& st) {
    if (c->N > 3) run_sweep_nw<T>(c, st);
    else if (c->lra) run_sweep_lra<T>(c, st);
    else run_sweep<T>(c, st);
}

// Queue `count` sweeps: replays of the captured graph when graph mode is on
// (the remainder, and profiled or two-stream sweeps, launch directly).
concpd_status launch_sweeps(concpd_ctx c, long long count) {
    const int gs = c->graph_sweeps;
    long long direct = count;
    if (gs > 0 && !c->profiling && count >= gs) {
        if (!c->gexec) {
            if (!c->qcap) HIPCHECK(hipStreamCreateWithFlags(&c->qcap, hipStreamNonBlocking));
            hipStream_t q = c->q;
            c->q = c->qcap;
            HIPCHECK(hipStreamBeginCapture(c->qcap, hipStreamCaptureModeThreadLocal));
            for (int i = 0; i < gs; ++i) {
                if (c->f64) run_one_sweep<double>(c, c->sd);
                else run_one_sweep<float>(c, c->sf);
            }
            hipGraph_t graph = nullptr;
            const hipError_t e = hipStreamEndCapture(c->qcap, &graph);
            c->q = q;
            if (e != hipSuccess) return fail(CONCPD_EHIP, "sweep capture: %s", hipGetErrorString(e));
            const hipError_t e2 = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e2 != hipSuccess) {
                c->gexec = nullptr;
                return fail(CONCPD_EHIP, "graph instantiate: %s", hipGetErrorString(e2));
            }
        }
        for (long long i = 0; i + gs <= count; i += gs) HIPCHECK(hipGraphLaunch(c->gexec, c->q));
        direct = count % gs;
    }
    for (long long i = 0; i < direct; ++i) {
        if (c->f64) run_one_sweep<double>(c, c->sd);
        else run_one_sweep<float>(c, c->sf);
    }
    c->launched_iters += count;
    HIPCHECK(hipGetLastError());
    return CONCPD_OK;
}

// Grams, b, F and RelErr of the iterate in slot 1.
template <typename T>
void recompute_stats(concpd_ctx c, const StateP<T>& st) {
    if (c->N > 3) {
        // K of the last mode with every factor from slot 1: pass B on the
        // Khatri-Rao product of modes 0..h-1, then the contraction
        long long maxA, maxB;
        int maxI;
        nw_extents(c, &maxA, &maxB, &maxI);
        cpd::launch_nw_kr<T>(c->dgeo, st, c->S, 1, 1, maxA, c->Rq, 0, c->q);
        cpd::launch_nw_pass<T>(c->dgeo, st, (const ItemNW*)(c->ws + c->lay.itnb), (int)c->lists.nb.size(), 1, c->Rq, 0, c->q);
        cpd::launch_nw_contract<T>(c->dgeo, st, c->S, c->N - 1, 1, maxI, c->Rq, 0, c->q);
        cpd::launch_init_stats<T>(c->dgeo, st, c->S, c->R, c->q);
        return;
    }
    if (c->lra) {
        // W of the iterate in both slots, then K3 = A_3 C_3 and the statistics
        for (int n = 0; n < 3; ++n)
            for (int slot = 0; slot < 2; ++slot) cpd::launch_lra_w<T>(c->dgeo, st, c->S, c->lay.Jmax, n, 1, slot, c->q);
        cpd::launch_lra_c<T>(c->dgeo, st, c->S, c->lay.Jmax, c->Rq, 2, c->q);
        for (int s = 0; s < c->S; ++s)
            cpd::launch_extract_k<T>(c->dgeo, st, s, 2, (int)c->dims[3 * s + 2], c->R, st.K3 + c->geo.koff[s], c->Rq, 1, c->q);
        cpd::launch_init_stats<T>(c->dgeo, st, c->S, c->R, c->q);
        return;
    }
    const ItemP2* it2 = (const ItemP2*)(c->ws + c->lay.it2);
    cpd::launch_pass2<T>(c->dgeo, st, it2, (int)c->lists.p2.size(), c->Rq, 1, c->mdtype, c->lists.maxI2, c->geo.p2spw, c->q);
    for (int s = 0; s < c->S; ++s)
        cpd::launch_extract_k<T>(c->dgeo, st, s, 2, (int)c->dims[3 * s + 2], c->R, st.K3 + c->geo.koff[s], c->Rq, 0, c->q);
    cpd::launch_init_stats<T>(c->dgeo, st, c->S, c->R, c->q);
}

// Physical slot of logical factor/lambda slot l (the device rotates slots;
// synchronises the stream).
int phys_slot3(concpd_ctx c, int l) {
    int r3 = 0;
    if (hipMemcpyAsync(&r3, &c->ctrl->rot3, sizeof r3, hipMemcpyDeviceToHost, c->q) != hipSuccess) return l;
    if (hipStreamSynchronize(c->q) != hipSuccess) return l;
    return (r3 + l) % 3;
}

concpd_status read_stats(concpd_ctx c, concpd_stats* out) {
    Ctrl h;
    HIPCHECK(hipMemcpyAsync(&h, c->ctrl, sizeof h, hipMemcpyDeviceToHost, c->q));
    HIPCHECK(hipStreamSynchronize(c->q));
    if (out) {
        out->k = h.k;
        out->F = h.F_prev;
        out->relerr = h.rel_prev;
        out->fit = 1.0 - h.rel_prev;
        out->restarts = h.restarts;
        out->restarted_last = h.last_restarted;
        out->converged = h.stop;
        out->nonfinite = !isfinite(h.F_prev);
        out->lra = c->lra;
    }
    return CONCPD_OK;
}

// Host factor arrays (I x R doubles) -> slot layout (I x Rq, storage type).
template <typename T>
void pack_factors(concpd_ctx c, const double* const* U, std::vector<T>& out) {
    out.assign((size_t)c->lay.uslot, (T)0);
    const int N = c->N;
    for (int n = 0; n < N; ++n)
        for (int s = 0; s < c->S; ++s) {
            const int I = (int)c->dims[N * s + n];
            const double* src = U[N * s + n];
            const uint64_t gm = group_mask(&c->cfg, n);
            const int Ls = in_group(gm, s) ? c->L[n] : 0;
            const double* shared = Ls ? U[N * first_member(gm) + n] : src;
            T* dst = out.data() + c->geo.uoff[n][s];
            for (int i = 0; i < I; ++i)
                for (int r = 0; r < c->rk[s]; ++r)
                    dst[(size_t)i * c->Rq + r] = (T)(r < Ls ? shared[(size_t)i * c->R + r] : src[(size_t)i * c->R + r]);
        }
}

bool all_finite(const double* p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(p[i])) return false;
    return true;
}

// the first `used` columns of a rows x ld row-major array are finite
bool cols_finite(const double* p, int64_t rows, int ld, int used) {
    for (int64_t i = 0; i < rows; ++i)
        if (!all_finite(p + i * ld, used)) return false;
    return true;
}

template <typename T>
concpd_status upload_iterate(concpd_ctx c, const double* const* U, const double* const* Up, const double* const* lam,
                             const double* const* lamp) {
    std::vector<T> h1, h2;
    pack_factors<T>(c, U, h1);
    pack_factors<T>(c, Up ? Up : U, h2);
    const size_t bytes = (size_t)c->lay.uslot * sizeof(T);
    HIPCHECK(hipMemcpyAsync(c->ws + c->lay.U[1], h1.data(), bytes, hipMemcpyHostToDevice, c->q));
    HIPCHECK(hipMemcpyAsync(c->ws + c->lay.U[2], h2.data(), bytes, hipMemcpyHostToDevice, c->q));
    HIPCHECK(hipMemcpyAsync(c->ws + c->lay.U[0], h1.data(), bytes, hipMemcpyHostToDevice, c->q));
    std::vector<double> l1((size_t)c->S * c->Rq, 0.0), l2((size_t)c->S * c->Rq, 0.0);
    for (int s = 0; s < c->S; ++s)
        for (int r = 0; r < c->rk[s]; ++r) {
            l1[(size_t)s * c->Rq + r] = lam[s][r];
            l2[(size_t)s * c->Rq + r] = (lamp ? lamp : lam)[s][r];
        }
    HIPCHECK(hipMemcpyAsync(c->ws + c->lay.lam[1], l1.data(), l1.size() * 8, hipMemcpyHostToDevice, c->q));
    HIPCHECK(hipMemcpyAsync(c->ws + c->lay.lam[2], l2.data(), l2.size() * 8, hipMemcpyHostToDevice, c->q));
    HIPCHECK(hipMemcpyAsync(c->ws + c->lay.lam[0], l1.data(), l1.size() * 8, hipMemcpyHostToDevice, c->q));
    HIPCHECK(hipStreamSynchronize(c->q));  // host vectors go out of scope
    return CONCPD_OK;
}

concpd_status set_lipschitz_prev(concpd_ctx c, const double* Ld, const double* Lu, const double* LC) {
    const int N = c->N;
    std::vector<double> ld(c->S, -1.0), lu((size_t)N * c->S, -1.0), lc(N, -1.0);
    for (int s = 0; s < c->S; ++s) {
        if (Ld) ld[s] = Ld[s];
        for (int n = 0; n < N; ++n)
            if (Lu) lu[n * c->S + s] = Lu[N * s + n];
    }
    for (int n = 0; n < N; ++n)
        if (LC) lc[n] = LC[n];
    HIPCHECK(hipMemcpyAsync(c->ws + c->lay.Ld_prev, ld.data(), ld.size() * 8, hipMemcpyHostToDevice, c->q));
    HIPCHECK(hipMemcpyAsync(c->ws + c->lay.Lu_prev, lu.data(), lu.size() * 8, hipMemcpyHostToDevice, c->q));
    HIPCHECK(hipMemcpyAsync(c->ws + c->lay.LC_prev, lc.data(), lc.size() * 8, hipMemcpyHostToDevice, c->q));
    HIPCHECK(hipStreamSynchronize(c->q));
    return CONCPD_OK;
}

concpd_status set_ctrl(concpd_ctx c, double t, long long k) {
    Ctrl h;
    memset(&h, 0, sizeof h);
    h.t = t;
    const double tk = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
    h.w_hat = (t - 1.0) / tk;
    h.F_prev = INFINITY;
    h.F_cur = INFINITY;
    h.rel_prev = INFINITY;
    h.rel_cur = INFINITY;
    h.tol = 0.0;
    h.delta_w = c->cfg.delta_w;
    h.k = k;
    h.restart_on = c->cfg.restart;
    HIPCHECK(hipMemcpyAsync(c->ctrl, &h, sizeof h, hipMemcpyHostToDevice, c->q));
    HIPCHECK(hipStreamSynchronize(c->q));
    return CONCPD_OK;
}

template <typename T>
void debug_passes(concpd_ctx c, const StateP<T>& st) {
    const ItemP1* it1 = (const ItemP1*)(c->ws + c->lay.it1);
    const ItemP2* it2 = (const ItemP2*)(c->ws + c->lay.it2);
    const ItemK2* itk = (const ItemK2*)(c->ws + c->lay.itk2);
    cpd::launch_pass1<T>(c->dgeo, st, it1, (int)c->lists.p1.size(), c->lists.p1_split, c->Rq, 1, c->mdtype, c->p1dma, c->q);
    cpd::launch_k2<T>(c->dgeo, st, itk, (int)c->lists.k2.size(), 1, c->q);
    cpd::launch_pass2<T>(c->dgeo, st, it2, (int)c->lists.p2.size(), c->Rq, 1, c->mdtype, c->lists.maxI2, c->geo.p2spw, c->q);
}

// Loss and gradients at a caller-given point (autograd form): the point is
// packed into its own slot set (every logical slot addresses it), the dense
// MTTKRP passes run on it, then the per-block and per-factor gradient kernels.
template <typename T>
concpd_status loss_grad_t(concpd_ctx c, const StateP<T>& st, const void* const* U_dev, const void* const* lam_dev, int coupled,
                          double* loss, void* const* gU_dev, void* const* glam_dev) {
    const Layout& P = c->lay;
    const size_t esz = sizeof(T);
    StateP<T> sg = st;
    T* Ug = (T*)(c->ws + P.gU);
    for (int i = 0; i < 3; ++i) sg.U[i] = Ug;
    for (int i = 0; i < 3; ++i) sg.lam[i] = (double*)(c->ws + P.glam);
    for (int i = 0; i < 2; ++i) sg.V[i] = (double*)(c->ws + P.gV);
    for (int i = 0; i < 2; ++i) sg.b[i] = (double*)(c->ws + P.gb);
    sg.P = (double*)(c->ws + P.gP);
    sg.ctrl = (Ctrl*)(c->ws + P.gctrl);
    HIPCHECK(hipMemsetAsync(c->ws + P.gctrl, 0, sizeof(Ctrl), c->q));
    HIPCHECK(hipMemsetAsync(Ug, 0, (size_t)P.uslot * esz, c->q));
    HIPCHECK(hipMemsetAsync(sg.lam[0], 0, sizeof(double) * c->S * c->Rq, c->q));
    // pack: I_n x R (row stride R) -> I_n x Rq; shared columns from the first
    // block of each coupling group when coupled
    for (int s = 0; s < c->S; ++s) {
        for (int n = 0; n < 3; ++n) {
            const int I = (int)c->dims[3 * s + n];
            T* dst = Ug + c->geo.uoff[n][s];
            HIPCHECK(hipMemcpy2DAsync(dst, c->Rq * esz, U_dev[3 * s + n], c->R * esz, c->R * esz, I, hipMemcpyDeviceToDevice, c->q));
            const uint64_t gm = group_mask(&c->cfg, n);
            const int f = first_member(gm);
            if (coupled && c->L[n] > 0 && in_group(gm, s) && s != f)
                HIPCHECK(hipMemcpy2DAsync(dst, c->Rq * esz, U_dev[3 * f + n], c->R * esz, c->L[n] * esz, I,
                                          hipMemcpyDeviceToDevice, c->q));
        }
        HIPCHECK(hipMemcpyAsync(sg.lam[0] + (size_t)s * c->Rq, lam_dev[s], sizeof(double) * c->R, hipMemcpyDeviceToDevice, c->q));
    }
    // output pointer tables: gU for mode n at [n * S + s], glam at [3 S + s]
    std::vector<void*> tab(4 * c->S);
    for (int s = 0; s < c->S; ++s) {
        for (int n = 0; n < 3; ++n) tab[n * c->S + s] = gU_dev[3 * s + n];
        tab[3 * c->S + s] = glam_dev[s];
    }
    void** dtab = (void**)(c->ws + P.gptr);
    HIPCHECK(hipMemcpyAsync(dtab, tab.data(), sizeof(void*) * tab.size(), hipMemcpyHostToDevice, c->q));
    const ItemP1* it1 = (const ItemP1*)(c->ws + P.it1);
    const ItemP2* it2 = (const ItemP2*)(c->ws + P.it2);
    const ItemK2* itk = (const ItemK2*)(c->ws + P.itk2);
    cpd::launch_pass1<T>(c->dgeo, sg, it1, (int)c->lists.p1.size(), c->lists.p1_split, c->Rq, 1, c->mdtype, c->p1dma, c->q);
    cpd::launch_k2<T>(c->dgeo, sg, itk, (int)c->lists.k2.size(), 0, c->q);
    cpd::launch_pass2<T>(c->dgeo, sg, it2, (int)c->lists.p2.size(), c->Rq, 0, c->mdtype, c->lists.maxI2, c->geo.p2spw, c->q);
    for (int s = 0; s < c->S; ++s)
        cpd::launch_extract_k<T>(c->dgeo, sg, s, 2, (int)c->dims[3 * s + 2], c->R, sg.K3 + c->geo.koff[s], c->Rq, 0, c->q);
    int In[3] = {1, 1, 1};
    for (int s = 0; s < c->S; ++s)
        for (int n = 0; n < 3; ++n) In[n] = std::max(In[n], (int)c->dims[3 * s + n]);
    double* Fg = (double*)(c->ws + P.gF);
    cpd::launch_grad<T>(c->dgeo, sg, c->S, c->R, c->Rq, In, c->L[0], c->L[1], c->L[2], (double* const*)(dtab + 3 * c->S), Fg,
                        (T* const*)dtab, (T* const*)(dtab + c->S), (T* const*)(dtab + 2 * c->S), coupled, c->q);
    HIPCHECK(hipGetLastError());
    std::vector<double> F(c->S);
    HIPCHECK(hipMemcpyAsync(F.data(), Fg, sizeof(double) * c->S, hipMemcpyDeviceToHost, c->q));
    HIPCHECK(hipStreamSynchronize(c->q));
    double tot = 0.0;
    for (int s = 0; s < c->S; ++s) tot += F[s];
    *loss = tot;
    return CONCPD_OK;
}

}  // namespace

// Compression by an unconstrained CPD fitted with ALS (the paper's own first
// step of Algorithm 2).  The ALS factors live in the iterate's current slot
// while the fit runs, so the sweep's MTTKRP passes serve it unchanged; the
// APG iterate is saved to the host before and put back after.
template <typename T>
concpd_status als_fit_all(concpd_ctx c, const StateP<T>& st, int R, double eps, int max_it, int32_t* iters,
                          double* relerr_out) {
    const int S = c->S;
    double* L = (double*)(c->ws + c->lay.lra);
    double* Lfac = L + c->lay.l_sig;
    double* rel = L + c->lay.l_work;
    double* xx = rel + S;
    int* act = (int*)(xx + S);
    int* bad = act + S;
    double* V = rel + 4 * S;   // Grams of the three factors, [S][3][R*R]
    int Imax[3] = {1, 1, 1};
    for (int s = 0; s < S; ++s)
        for (int n = 0; n < 3; ++n) Imax[n] = std::max(Imax[n], (int)c->dims[3 * s + n]);
    std::vector<int> hact(S, 1), hbad(S, 0);
    std::vector<double> prev(S), cur(S);
    HIPCHECK(hipMemcpyAsync(act, hact.data(), sizeof(int) * S, hipMemcpyHostToDevice, c->q));
    HIPCHECK(hipMemcpyAsync(bad, hbad.data(), sizeof(int) * S, hipMemcpyHostToDevice, c->q));
    // K_3 = the pass-2 chunk partials summed into the K3 buffer, per block
    auto k3_sum = [&]() {
        for (int s = 0; s < S; ++s)
            cpd::launch_extract_k<T>(c->dgeo, st, s, 2, (int)c->dims[3 * s + 2], R, st.K3 + c->geo.koff[s], c->Rq, 0, c->q);
    };
    // RelErr_0 at the starting point
    for (int n = 0; n < 3; ++n) cpd::launch_als_gram<T>(c->dgeo, st, S, R, n, act, V, c->q);
    debug_passes<T>(c, st);
    k3_sum();
    cpd::launch_als_fit<T>(c->dgeo, st, S, R, act, V, rel, xx, c->q);
    HIPCHECK(hipMemcpyAsync(prev.data(), rel, sizeof(double) * S, hipMemcpyDeviceToHost, c->q));
    HIPCHECK(hipStreamSynchronize(c->q));
    for (int s = 0; s < S; ++s) {
        if (iters) iters[s] = 0;
        if (relerr_out) relerr_out[s] = prev[s];
        if (!isfinite(prev[s])) return fail(CONCPD_ENONFINITE, "ALS: RelErr of block %d at the start is not finite", s);
    }
    const ItemP1* it1 = (const ItemP1*)(c->ws + c->lay.it1);
    const ItemP2* it2 = (const ItemP2*)(c->ws + c->lay.it2);
    const ItemK2* itk = (const ItemK2*)(c->ws + c->lay.itk2);
    int active = S;
    for (int it = 1; it <= max_it && active > 0; ++it) {
        cpd::launch_pass1<T>(c->dgeo, st, it1, (int)c->lists.p1.size(), c->lists.p1_split, c->Rq, 1, c->mdtype, c->p1dma, c->q);
        cpd::launch_als_chol(c->dgeo, S, R, 0, act, V, Lfac, bad, c->q);
        cpd::launch_als_solve<T>(c->dgeo, st, S, R, 0, Imax[0], act, Lfac, c->q);
        cpd::launch_als_gram<T>(c->dgeo, st, S, R, 0, act, V, c->q);
        cpd::launch_k2<T>(c->dgeo, st, itk, (int)c->lists.k2.size(), 1, c->q);
        cpd::launch_als_chol(c->dgeo, S, R, 1, act, V, Lfac, bad, c->q);
        cpd::launch_als_solve<T>(c->dgeo, st, S, R, 1, Imax[1], act, Lfac, c->q);
        cpd::launch_als_gram<T>(c->dgeo, st, S, R, 1, act, V, c->q);
        cpd::launch_pass2<T>(c->dgeo, st, it2, (int)c->lists.p2.size(), c->Rq, 1, c->mdtype, c->lists.maxI2, c->geo.p2spw, c->q);
        k3_sum();
        cpd::launch_als_chol(c->dgeo, S, R, 2, act, V, Lfac, bad, c->q);
        cpd::launch_als_solve<T>(c->dgeo, st, S, R, 2, Imax[2], act, Lfac, c->q);
        cpd::launch_als_gram<T>(c->dgeo, st, S, R, 2, act, V, c->q);
        cpd::launch_als_fit<T>(c->dgeo, st, S, R, act, V, rel, xx, c->q);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipMemcpyAsync(cur.data(), rel, sizeof(double) * S, hipMemcpyDeviceToHost, c->q));
        HIPCHECK(hipMemcpyAsync(hbad.data(), bad, sizeof(int) * S, hipMemcpyDeviceToHost, c->q));
        HIPCHECK(hipStreamSynchronize(c->q));
        for (int s = 0; s < S; ++s) {
            if (!hact[s]) continue;
            if (hbad[s] || !isfinite(cur[s]))
                return fail(CONCPD_ENONFINITE, "ALS: block %d has a singular Gram or a non-finite fit at iteration %d", s, it);
            if (iters) iters[s] = it;
            if (relerr_out) relerr_out[s] = cur[s];
            if (fabs(cur[s] - prev[s]) < eps) {
                hact[s] = 0;
                --active;
            }
            prev[s] = cur[s];
        }
        HIPCHECK(hipMemcpyAsync(act, hact.data(), sizeof(int) * S, hipMemcpyHostToDevice, c->q));
    }
    cpd::launch_als_export<T>(c->dgeo, st, S, R, xx, c->q);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(c->q));
    return CONCPD_OK;
}

extern "C" {

const char* concpd_last_error(void) { return g_err.c_str(); }

concpd_status concpd_query_workspace(const concpd_config* cfg, size_t* bytes) {
    concpd_status st = validate(cfg);
    if (st != CONCPD_OK) return st;
    if (!bytes) return fail(CONCPD_EINVAL, "bytes is NULL");
    Lists L;
    build_lists(cfg, &L);
    Layout P;
    Geo g;
    plan(cfg, L, &P, &g);
    *bytes = P.total;
    return CONCPD_OK;
}

}  // extern "C"

namespace {
// concpd_init with a flag that keeps it from creating any HIP object (the
// optional second stream), for the static-workspace entry point.
concpd_status init_impl(const concpd_config* cfg, const void* const* tensors, const double* const* init_U,
                        const double* const* init_lambda, uint64_t seed, void* workspace, size_t ws_bytes, void* stream,
                        bool no_alloc, concpd_ctx* out) {
    g_err.clear();
    if (!out) return fail(CONCPD_EINVAL, "out is NULL");
    *out = nullptr;
    concpd_status st = validate(cfg);
    if (st != CONCPD_OK) return st;
    if (!tensors) return fail(CONCPD_EINVAL, "tensors is NULL");
    for (int s = 0; s < cfg->num_blocks; ++s)
        if (!tensors[s]) return fail(CONCPD_EINVAL, "tensors[%d] is NULL", s);
    if (!workspace) return fail(CONCPD_EINVAL, "workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(CONCPD_EINVAL, "workspace must be 256-byte aligned");

    concpd_ctx c = new concpd_ctx_s();
    c->cfg = *cfg;
    c->S = cfg->num_blocks;
    c->R = cfg->rank;
    c->Rq = (c->R + 3) / 4 * 4;
    c->N = cfg->order;
    const int N = c->N;
    for (int n = 0; n < CPD_MAXN; ++n) c->L[n] = n < N ? cfg->coupled[n] : 0;
    for (int n = 0; n < CPD_MAXN; ++n) c->cmask[n] = (cfg->coupled_blocks && n < N) ? cfg->coupled_blocks[n] : ~0ull;
    for (int n = N; n < CPD_MAXN; ++n) c->cfg.coupled[n] = 0;
    c->cfg.coupled_blocks = cfg->coupled_blocks ? c->cmask : nullptr;
    c->rk.assign(c->S, c->R);
    if (cfg->block_ranks) c->rk.assign(cfg->block_ranks, cfg->block_ranks + c->S);
    c->cfg.block_ranks = c->rk.data();
    c->dims.assign(cfg->dims, cfg->dims + (size_t)N * c->S);
    c->cfg.dims = c->dims.data();
    if (cfg->tucker_ranks) {
        c->tucker.assign(cfg->tucker_ranks, cfg->tucker_ranks + 3 * c->S);
        c->cfg.tucker_ranks = c->tucker.data();
    }
    c->f64 = cfg->compute_dtype == CONCPD_F64;
    c->mdtype = cfg->compute_dtype;
    c->tensors.assign(tensors, tensors + c->S);
    c->ws = (char*)workspace;
    c->q = (hipStream_t)stream;
    c->lra = 0;
    c->launched_iters = 0;
    c->profiling = 0;
    {
        const char* ov = getenv("CONCPD_OVERLAP");
        c->overlap = !no_alloc && ov && ov[0] == '1';
        c->graph_sweeps = 0;
        c->qcap = nullptr;
        c->gexec = nullptr;
        c->k2rows = CPD_K2ROWS_DEFAULT;
        c->q2 = nullptr;
        if (c->overlap) {
            if (hipStreamCreateWithFlags(&c->q2, hipStreamNonBlocking) != hipSuccess) c->overlap = 0;
            for (int i = 0; c->overlap && i < 6; ++i)
                if (hipEventCreateWithFlags(&c->fj[i], hipEventDisableTiming) != hipSuccess) c->overlap = 0;
        }
    }
    build_lists(&c->cfg, &c->lists);
    plan(&c->cfg, c->lists, &c->lay, &c->geo);
    for (int s = 0; s < c->S; ++s) c->geo.rk[s] = c->rk[s];
    if (ws_bytes < c->lay.total) {
        const size_t need = c->lay.total;
        delete c;
        return fail(CONCPD_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    }

    // host-side initial iterate
    std::vector<std::vector<double>> hU((size_t)N * c->S);
    std::vector<const double*> pU((size_t)N * c->S);
    std::vector<std::vector<double>> hl(c->S);
    std::vector<const double*> pl(c->S);
    if (!init_U || !init_lambda) {
        SplitMix64 rng{seed};
        for (int n = 0; n < N; ++n)
            for (int s = 0; s < c->S; ++s) {
                const int I = (int)c->dims[N * s + n];
                const uint64_t gm = group_mask(&c->cfg, n);
                const int f = first_member(gm);
                const bool copy = in_group(gm, s) && s != f;   // shared columns drawn once, by the first member
                std::vector<double>& v = hU[N * s + n];
                v.assign((size_t)I * c->R, 0.0);
                for (int i = 0; i < I; ++i)
                    for (int r = 0; r < c->R; ++r) {
                        if (r < c->L[n] && copy) v[(size_t)i * c->R + r] = hU[N * f + n][(size_t)i * c->R + r];
                        else v[(size_t)i * c->R + r] = rng.uniform();
                    }
            }
        // without a core update (the -NC variant of Section III-C, core
        // tensors removal) D^(s) is merged into the factors: lambda = 1
        for (int s = 0; s < c->S; ++s) {
            hl[s].resize(c->R);
            for (int r = 0; r < c->R; ++r) hl[s][r] = cfg->update_core ? rng.uniform() : 1.0;
        }
    }
    for (int i = 0; i < N * c->S; ++i) pU[i] = init_U ? init_U[i] : hU[i].data();
    for (int s = 0; s < c->S; ++s) pl[s] = init_lambda ? init_lambda[s] : hl[s].data();
    for (int s = 0; s < c->S; ++s) {
        for (int n = 0; n < N; ++n)
            if (!pU[N * s + n] || !cols_finite(pU[N * s + n], c->dims[N * s + n], c->R, c->rk[s])) {
                delete c;
                return fail(pU[N * s + n] ? CONCPD_ENONFINITE : CONCPD_EINVAL, "init_U[%d] missing or not finite", N * s + n);
            }
        if (!pl[s] || !all_finite(pl[s], c->rk[s])) {
            delete c;
            return fail(pl[s] ? CONCPD_ENONFINITE : CONCPD_EINVAL, "init_lambda[%d] missing or not finite", s);
        }
    }

#define INIT_CHECK(x)                 \
    do {                              \
        concpd_status s_ = (x);       \
        if (s_ != CONCPD_OK) {        \
            hipStreamSynchronize(c->q); \
            delete c;                 \
            return s_;                \
        }                             \
    } while (0)
#define INIT_HIP(x)                                                                          \
    do {                                                                                     \
        hipError_t e_ = (x);                                                                 \
        if (e_ != hipSuccess) {                                                              \
            hipStreamSynchronize(c->q);                                                      \
            delete c;                                                                        \
            return fail(CONCPD_EHIP, "%s: %s", #x, hipGetErrorString(e_));                   \
        }                                                                                    \
    } while (0)

    INIT_HIP(hipMemsetAsync(c->ws, 0, c->lay.total, c->q));
    // operand copies of the tensors
    for (int s = 0; s < c->S; ++s) {
        c->geo.M[s] = c->tensors[s];
        c->geo.mld[s] = c->dims[N * s + N - 1];
        if (c->lay.shadow_ld[s] > 0) {
            char* dst = c->ws + c->lay.shadow + c->lay.shadow_off[s];
            cpd::launch_pad_copy(c->tensors[s], cfg->tensor_dtype, dst, c->mdtype, c->dims[3 * s] * c->dims[3 * s + 1],
                                 (int)c->dims[3 * s + 2], (int)c->lay.shadow_ld[s], c->q);
            c->geo.M[s] = dst;
            c->geo.mld[s] = c->lay.shadow_ld[s];
        }
    }
    // blocks whose operand rows all start 16-byte aligned take 16-byte loads
    {
        const int me = operand_bytes(c->mdtype);
        bool all = true;
        for (int s = 0; s < c->S; ++s) {
            c->geo.mvec[s] = (c->geo.mld[s] % (16 / me) == 0) && ((uintptr_t)c->geo.M[s] % 16 == 0);
            all = all && c->geo.mvec[s];
        }
        // pass 1 can stream the tensor by LDS DMA when every row is 16-byte
        // aligned; by default it does so for 16-bit storage, whose 32-byte
        // chunks carry twice the values (measured: faster for BF16 at every
        // shape, slower for FP32 rows of a few thousand values)
        // order N > 3: pass A reads rows of B = I_h ... I_N values
        for (int s = 0; s < c->S && N > 3; ++s)
            c->geo.mvec[s] = (c->geo.nwB[s] % (16 / me) == 0) && ((uintptr_t)c->geo.M[s] % 16 == 0);
        c->p1dma_ok = all && !c->f64 && N == 3;
        c->p1dma = c->p1dma_ok && c->mdtype != 1;
    }
    // the fused launches by default while pass 1 has at most two wavefronts
    // per SIMD (they keep two or three resident; measured: 10 x 100^3 R = 20
    // 120 -> 97 us per sweep, the EEG-shaped blocks 420 -> 408 us)
    {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
            c->fuse = N == 3 && c->R <= 32 && (long long)c->lists.p1.size() * c->lists.p1_split <= 8LL * ncu;
        c->fuse_dflt = c->fuse;
    }
    c->dgeo = (Geo*)(c->ws + c->lay.geo);
    INIT_HIP(hipMemcpyAsync(c->dgeo, &c->geo, sizeof(Geo), hipMemcpyHostToDevice, c->q));
    if (!c->lists.p1.empty())
        INIT_HIP(hipMemcpyAsync(c->ws + c->lay.it1, c->lists.p1.data(), c->lists.p1.size() * sizeof(ItemP1), hipMemcpyHostToDevice, c->q));
    if (!c->lists.p2.empty())
        INIT_HIP(hipMemcpyAsync(c->ws + c->lay.it2, c->lists.p2.data(), c->lists.p2.size() * sizeof(ItemP2), hipMemcpyHostToDevice, c->q));
    if (!c->lists.k2.empty())
        INIT_HIP(hipMemcpyAsync(c->ws + c->lay.itk2, c->lists.k2.data(), c->lists.k2.size() * sizeof(ItemK2), hipMemcpyHostToDevice, c->q));
    for (int n = 0; n < N; ++n)
        if (!c->lists.u[n].empty())
            INIT_HIP(hipMemcpyAsync(c->ws + c->lay.itu[n], c->lists.u[n].data(), c->lists.u[n].size() * sizeof(ItemU),
                                    hipMemcpyHostToDevice, c->q));
    if (!c->lists.na.empty())
        INIT_HIP(hipMemcpyAsync(c->ws + c->lay.itna, c->lists.na.data(), c->lists.na.size() * sizeof(ItemNW), hipMemcpyHostToDevice, c->q));
    if (!c->lists.nb.empty())
        INIT_HIP(hipMemcpyAsync(c->ws + c->lay.itnb, c->lists.nb.data(), c->lists.nb.size() * sizeof(ItemNW), hipMemcpyHostToDevice, c->q));
    c->sf = make_state<float>(c->ws, c->lay);
    c->sd = make_state<double>(c->ws, c->lay);
    c->ctrl = (Ctrl*)(c->ws + c->lay.ctrl);

    // finiteness of the tensors and their squared norms (original and operand copy)
    int* dflag = (int*)(c->ws + c->lay.flag);
    double* sqpart = (double*)(c->ws + c->lay.scratch);
    for (int s = 0; s < c->S; ++s) {
        long long n = 1;
        for (int m = 0; m < N; ++m) n *= c->dims[N * s + m];
        cpd::launch_finite_check(c->tensors[s], cfg->tensor_dtype, n, dflag, c->q);
        cpd::launch_sqnorm(c->tensors[s], cfg->tensor_dtype, n, (double*)(c->ws + c->lay.normOrig) + s, sqpart, 1024, c->q);
        // the operand copy's padding is zero, so its norm runs over all rows of length ld
        cpd::launch_sqnorm(c->geo.M[s], c->mdtype, n / c->dims[N * s + N - 1] * c->geo.mld[s],
                           (double*)(c->ws + c->lay.normM2) + s, sqpart, 1024, c->q);
    }
    int hflag = 0;
    INIT_HIP(hipMemcpyAsync(&hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, c->q));
    c->normOrig.resize(c->S);
    INIT_HIP(hipMemcpyAsync(c->normOrig.data(), c->ws + c->lay.normOrig, sizeof(double) * c->S, hipMemcpyDeviceToHost, c->q));
    INIT_HIP(hipStreamSynchronize(c->q));
    if (hflag) {
        delete c;
        return fail(CONCPD_ENONFINITE, "a tensor holds NaN or Inf");
    }
    for (int s = 0; s < c->S; ++s)
        if (!(c->normOrig[s] > 0.0)) {
            delete c;
            return fail(CONCPD_EINVAL, "tensor %d is identically zero", s);
        }

    INIT_CHECK(c->f64 ? upload_iterate<double>(c, pU.data(), nullptr, pl.data(), nullptr)
                      : upload_iterate<float>(c, pU.data(), nullptr, pl.data(), nullptr));
    INIT_CHECK(set_lipschitz_prev(c, nullptr, nullptr, nullptr));
    INIT_CHECK(set_ctrl(c, 1.0, 0));
    if (c->f64) recompute_stats<double>(c, c->sd);
    else recompute_stats<float>(c, c->sf);
    INIT_HIP(hipGetLastError());
    INIT_HIP(hipStreamSynchronize(c->q));
    *out = c;
    return CONCPD_OK;
#undef INIT_CHECK
#undef INIT_HIP
}
}  // namespace

extern "C" {

concpd_status concpd_init(const concpd_config* cfg, const void* const* tensors, const double* const* init_U,
                          const double* const* init_lambda, uint64_t seed, void* workspace, size_t ws_bytes, void* stream,
                          concpd_ctx* out) {
    return init_impl(cfg, tensors, init_U, init_lambda, seed, workspace, ws_bytes, stream, false, out);
}

concpd_status concpd_init_static(const concpd_config* cfg, const void* const* tensors, const double* const* init_U,
                                 const double* const* init_lambda, uint64_t seed, void* stream, concpd_ctx* out) {
    g_err.clear();
    if (!out) return fail(CONCPD_EINVAL, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    concpd_status st = concpd_query_workspace(cfg, &need);
    if (st != CONCPD_OK) return st;
    if (need > CPD_STATIC_WS_BYTES)
        return fail(CONCPD_EINVAL, "configuration needs %zu bytes of workspace, more than the static workspace's %zu",
                    need, CPD_STATIC_WS_BYTES);
    int dev = 0;
    HIPCHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= CPD_MAX_DEVICES) return fail(CONCPD_ENOTSUP, "device %d: static workspace only on devices 0..%d", dev, CPD_MAX_DEVICES - 1);
    std::lock_guard<std::mutex> lock(g_static.mu);
    if (g_static.owner[dev])
        return fail(CONCPD_ESTATE, "the static workspace of device %d is held by another context (destroy it first)", dev);
    if (!g_static.ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(CONCPD_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_static.ptr[dev] = p;
    }
    concpd_ctx c = nullptr;
    st = init_impl(cfg, tensors, init_U, init_lambda, seed, g_static.ptr[dev], CPD_STATIC_WS_BYTES, stream, true, &c);
    if (st != CONCPD_OK) return st;
    c->static_dev = dev;
    g_static.owner[dev] = c;
    *out = c;
    return CONCPD_OK;
}

concpd_status concpd_step(concpd_ctx c, int32_t n_iter, concpd_stats* out) {
    if (!c) return fail(CONCPD_EINVAL, "ctx is NULL");
    if (n_iter < 0) return fail(CONCPD_EINVAL, "n_iter < 0");
    if (!out) {
        // asynchronous: n_iter sweeps; a sweep rejected by the restart test
        // is completed by the following one
        return launch_sweeps(c, n_iter);
    }
    // synchronous: exactly n_iter accepted iterations (or until converged)
    Ctrl h;
    HIPCHECK(hipMemcpyAsync(&h, c->ctrl, sizeof h, hipMemcpyDeviceToHost, c->q));
    HIPCHECK(hipStreamSynchronize(c->q));
    const long long target = h.k + n_iter;
    long long todo = n_iter;
    while (todo > 0 && !h.stop) {
        const concpd_status r = launch_sweeps(c, todo);
        if (r != CONCPD_OK) return r;
        HIPCHECK(hipMemcpyAsync(&h, c->ctrl, sizeof h, hipMemcpyDeviceToHost, c->q));
        HIPCHECK(hipStreamSynchronize(c->q));
        todo = target - h.k;
    }
    return read_stats(c, out);
}

concpd_status concpd_fit(concpd_ctx c, concpd_stats* out) {
    if (!c) return fail(CONCPD_EINVAL, "ctx is NULL");
    const double tol = c->cfg.tol;
    HIPCHECK(hipMemcpyAsync(&c->ctrl->tol, &tol, sizeof tol, hipMemcpyHostToDevice, c->q));
    concpd_stats s;
    concpd_status r = read_stats(c, &s);
    if (r != CONCPD_OK) return r;
    while (!s.converged && s.k < c->cfg.max_it) {
        const int chunk = (int)std::min<long long>(16, c->cfg.max_it - s.k);
        r = concpd_step(c, chunk, &s);
        if (r != CONCPD_OK) return r;
    }
    if (out) *out = s;
    return CONCPD_OK;
}

concpd_status lra_compress(concpd_ctx c, const int32_t* ranks, concpd_stats* out) {
    if (c) NEED_ORDER3(c, "lra_compress");
    if (!c) return fail(CONCPD_EINVAL, "ctx is NULL");
    if (c->tucker.empty()) return fail(CONCPD_ESTATE, "lra_compress: no Tucker ranks configured");
    if (ranks)
        for (int i = 0; i < 3 * c->S; ++i)
            if (ranks[i] < 1 || ranks[i] > c->tucker[i])
                return fail(CONCPD_EINVAL, "ranks[%d] = %d not in [1, configured %d]", i, ranks[i], c->tucker[i]);
    for (int s = 0; s < c->S; ++s)
        for (int n = 0; n < 3; ++n) c->geo.J[s][n] = ranks ? ranks[3 * s + n] : c->tucker[3 * s + n];
    double* L = (double*)(c->ws + c->lay.lra);
    const Layout& P = c->lay;
    double* scratch = (double*)(c->ws + c->lay.scratch);
    HIPCHECK(hipMemcpyAsync(c->dgeo, &c->geo, sizeof(Geo), hipMemcpyHostToDevice, c->q));
    // mode Grams of every block, then all leading-eigenvector problems at once
    for (int s = 0; s < c->S; ++s) {
        const int I[3] = {(int)c->dims[3 * s], (int)c->dims[3 * s + 1], (int)c->dims[3 * s + 2]};
        const float* X = (const float*)c->tensors[s];
        for (int n = 0; n < 3; ++n) {
            cpd::launch_mode_gram(X, n, I[0], I[1], I[2], L + P.l_part, P.nsplit, c->q);
            cpd::launch_sum_split(L + P.l_part, P.nsplit, (long long)I[n] * I[n], L + P.l_sig + (3LL * s + n) * P.sig_stride,
                                  c->q);
        }
    }
    cpd::launch_eig_top(c->dgeo, L, L + P.l_sig, P.sig_stride, L + P.l_work, P.work_stride, 3 * c->S, P.Imax, c->q);
    for (int s = 0; s < c->S; ++s) {
        const int I[3] = {(int)c->dims[3 * s], (int)c->dims[3 * s + 1], (int)c->dims[3 * s + 2]};
        const float* X = (const float*)c->tensors[s];
        cpd::launch_ttm_chain(X, I[0], I[1], I[2], L + c->geo.aoff[0][s], L + c->geo.aoff[1][s], L + c->geo.aoff[2][s],
                              c->geo.J[s][0], c->geo.J[s][1], c->geo.J[s][2], L + P.l_t1, L + P.l_t2, L + c->geo.goff[s],
                              c->q);
        cpd::launch_sqnorm(L + c->geo.goff[s], CONCPD_F64, (long long)c->geo.J[s][0] * c->geo.J[s][1] * c->geo.J[s][2],
                           (double*)(c->ws + c->lay.normM2) + s, scratch, 64, c->q);
    }
    c->geo.lra = 1;
    c->lra = 1;
    c->drop_graph();
    HIPCHECK(hipMemcpyAsync(c->dgeo, &c->geo, sizeof(Geo), hipMemcpyHostToDevice, c->q));
    HIPCHECK(hipStreamSynchronize(c->q));
    // statistics of the current iterate against the compressed blocks
    Ctrl h;
    HIPCHECK(hipMemcpy(&h, c->ctrl, sizeof h, hipMemcpyDeviceToHost));
    h.stop = 0;
    h.redo = 0;
    HIPCHECK(hipMemcpy(c->ctrl, &h, sizeof h, hipMemcpyHostToDevice));
    if (c->f64) recompute_stats<double>(c, c->sd);
    else recompute_stats<float>(c, c->sf);
    HIPCHECK(hipGetLastError());
    return read_stats(c, out);
}

concpd_status lra_compress_cp(concpd_ctx c, const double* const* init, uint64_t seed, double eps, int32_t max_it,
                              int32_t cp_rank, int32_t* iters, double* relerr, concpd_stats* out) {
    if (!c) return fail(CONCPD_EINVAL, "ctx is NULL");
    NEED_ORDER3(c, "lra_compress_cp");
    if (c->lra) return fail(CONCPD_ESTATE, "lra_compress_cp: the context is already compressed");
    if (c->tucker.empty()) return fail(CONCPD_ESTATE, "lra_compress_cp: needs tucker_ranks (J_n >= R reserves the storage)");
    if (cp_rank < 0 || cp_rank > c->R) return fail(CONCPD_EINVAL, "cp_rank %d not in [0, rank]", cp_rank);
    const int Rt = cp_rank ? cp_rank : c->R;
    const int S = c->S;
    // block s is fitted at rank min(R~, R^(s))
    std::vector<int> rb(S);
    for (int s = 0; s < S; ++s) rb[s] = std::min(Rt, c->rk[s]);
    for (int i = 0; i < 3 * S; ++i)
        if (c->tucker[i] < rb[i / 3])
            return fail(CONCPD_EINVAL, "lra_compress_cp: tucker_ranks[%d] = %d < CP rank %d", i, c->tucker[i], rb[i / 3]);
    if (!(eps >= 0.0) || !isfinite(eps)) return fail(CONCPD_EINVAL, "eps must be finite and >= 0");
    if (max_it < 0) return fail(CONCPD_EINVAL, "max_it must be >= 0");
    // starting factors (host, FP64, I_n x min(R~, R^(s))): the caller's, or a seeded U[0,1] draw
    std::vector<std::vector<double>> h(3 * S);
    if (!init) {
        SplitMix64 rng{seed};
        for (int n = 0; n < 3; ++n)
            for (int s = 0; s < S; ++s) {
                h[3 * s + n].resize((size_t)c->dims[3 * s + n] * rb[s]);
                for (double& v : h[3 * s + n]) v = rng.uniform();
            }
    }
    for (int i = 0; i < 3 * S; ++i) {
        const double* p = init ? init[i] : h[i].data();
        if (!p) return fail(CONCPD_EINVAL, "init[%d] is NULL", i);
        if (!all_finite(p, (size_t)c->dims[i] * rb[i / 3])) return fail(CONCPD_ENONFINITE, "init[%d] is not finite", i);
    }
    // save the APG iterate's current slot and the control block
    const int phys = phys_slot3(c, 1);
    const size_t slot_bytes = (size_t)c->lay.uslot * c->lay.esz;
    char* slot = c->ws + c->lay.U[phys];
    std::vector<char> saved(slot_bytes);
    Ctrl hc;
    HIPCHECK(hipMemcpyAsync(saved.data(), slot, slot_bytes, hipMemcpyDeviceToHost, c->q));
    HIPCHECK(hipMemcpyAsync(&hc, c->ctrl, sizeof hc, hipMemcpyDeviceToHost, c->q));
    HIPCHECK(hipStreamSynchronize(c->q));
    // the starting factors into that slot (every block its own; no sharing)
    {
        std::vector<char> packed(slot_bytes, 0);
        for (int s = 0; s < S; ++s)
            for (int n = 0; n < 3; ++n) {
                const double* src = init ? init[3 * s + n] : h[3 * s + n].data();
                const int I = (int)c->dims[3 * s + n], R = rb[s];
                for (int i = 0; i < I; ++i)
                    for (int r = 0; r < R; ++r) {
                        const size_t e = (size_t)c->geo.uoff[n][s] + (size_t)i * c->Rq + r;
                        if (c->f64) ((double*)packed.data())[e] = src[(size_t)i * R + r];
                        else ((float*)packed.data())[e] = (float)src[(size_t)i * R + r];
                    }
            }
        HIPCHECK(hipMemcpyAsync(slot, packed.data(), slot_bytes, hipMemcpyHostToDevice, c->q));
        Ctrl run = hc;
        run.stop = 0;
        run.redo = 0;
        HIPCHECK(hipMemcpyAsync(c->ctrl, &run, sizeof run, hipMemcpyHostToDevice, c->q));
        HIPCHECK(hipStreamSynchronize(c->q));
    }
    c->drop_graph();
    concpd_status st = c->f64 ? als_fit_all<double>(c, c->sd, Rt, eps, max_it, iters, relerr)
                              : als_fit_all<float>(c, c->sf, Rt, eps, max_it, iters, relerr);
    // the APG iterate and the control block back in place
    hipStreamSynchronize(c->q);
    hc.stop = 0;
    hc.redo = 0;
    HIPCHECK(hipMemcpyAsync(slot, saved.data(), slot_bytes, hipMemcpyHostToDevice, c->q));
    HIPCHECK(hipMemcpyAsync(c->ctrl, &hc, sizeof hc, hipMemcpyHostToDevice, c->q));
    HIPCHECK(hipStreamSynchronize(c->q));
    if (st != CONCPD_OK) return st;
    for (int s = 0; s < S; ++s)
        for (int n = 0; n < 3; ++n) c->geo.J[s][n] = rb[s];
    c->geo.lra = 1;
    c->lra = 1;
    HIPCHECK(hipMemcpyAsync(c->dgeo, &c->geo, sizeof(Geo), hipMemcpyHostToDevice, c->q));
    if (c->f64) recompute_stats<double>(c, c->sd);
    else recompute_stats<float>(c, c->sf);
    HIPCHECK(hipGetLastError());
    return read_stats(c, out);
}

concpd_status lra_step(concpd_ctx c, int32_t n_iter, concpd_stats* out) {
    if (!c) return fail(CONCPD_EINVAL, "ctx is NULL");
    if (!c->lra) return fail(CONCPD_ESTATE, "lra_step before lra_compress");
    return concpd_step(c, n_iter, out);
}

concpd_status concpd_global_fit(concpd_ctx c, double* fit) {
    if (!c || !fit) return fail(CONCPD_EINVAL, "NULL argument");
    double* scratch = (double*)(c->ws + c->lay.scratch);
    double* res = scratch + c->lay.scratch_len - 1;
    double acc = 0.0;
    for (int s = 0; s < c->S; ++s) {
        const int I1 = (int)c->dims[(size_t)c->N * s];
        if (c->f64) cpd::launch_resid<double>(c->dgeo, c->sd, c->tensors[s], c->cfg.tensor_dtype, s, I1, scratch, c->q);
        else cpd::launch_resid<float>(c->dgeo, c->sf, c->tensors[s], c->cfg.tensor_dtype, s, I1, scratch, c->q);
        cpd::launch_sum_parts(scratch, I1, res, c->q);
        double h = 0.0;
        HIPCHECK(hipMemcpyAsync(&h, res, sizeof h, hipMemcpyDeviceToHost, c->q));
        HIPCHECK(hipStreamSynchronize(c->q));
        acc += sqrt(fmax(0.0, h)) / sqrt(c->normOrig[s]);
    }
    *fit = 1.0 - acc / c->S;
    return CONCPD_OK;
}

concpd_status concpd_get_factor(concpd_ctx c, int32_t n, int32_t s, double* dst) {
    if (!c || !dst) return fail(CONCPD_EINVAL, "NULL argument");
    if (n < 0 || n >= c->N || s < 0 || s >= c->S) return fail(CONCPD_EINVAL, "n/s out of range");
    const int I = (int)c->dims[(size_t)c->N * s + n];
    const size_t cnt = (size_t)I * c->Rq;
    const char* src = c->ws + c->lay.U[phys_slot3(c, 1)] + (size_t)c->geo.uoff[n][s] * c->lay.esz;
    if (c->f64) {
        std::vector<double> h(cnt);
        HIPCHECK(hipMemcpyAsync(h.data(), src, cnt * 8, hipMemcpyDeviceToHost, c->q));
        HIPCHECK(hipStreamSynchronize(c->q));
        for (int i = 0; i < I; ++i)
            for (int r = 0; r < c->R; ++r) dst[(size_t)i * c->R + r] = h[(size_t)i * c->Rq + r];
    } else {
        std::vector<float> h(cnt);
        HIPCHECK(hipMemcpyAsync(h.data(), src, cnt * 4, hipMemcpyDeviceToHost, c->q));
        HIPCHECK(hipStreamSynchronize(c->q));
        for (int i = 0; i < I; ++i)
            for (int r = 0; r < c->R; ++r) dst[(size_t)i * c->R + r] = h[(size_t)i * c->Rq + r];
    }
    return CONCPD_OK;
}

concpd_status concpd_get_lambda(concpd_ctx c, int32_t s, double* dst) {
    if (!c || !dst) return fail(CONCPD_EINVAL, "NULL argument");
    if (s < 0 || s >= c->S) return fail(CONCPD_EINVAL, "s out of range");
    HIPCHECK(hipMemcpyAsync(dst, c->ws + c->lay.lam[phys_slot3(c, 1)] + sizeof(double) * s * c->Rq, sizeof(double) * c->R,
                            hipMemcpyDeviceToHost, c->q));
    HIPCHECK(hipStreamSynchronize(c->q));
    return CONCPD_OK;
}

concpd_status lra_get_tucker(concpd_ctx c, int32_t s, int32_t n, double* dst) {
    if (!c || !dst) return fail(CONCPD_EINVAL, "NULL argument");
    NEED_ORDER3(c, "lra_get_tucker");
    if (s < 0 || s >= c->S || n < 0 || n > 3) return fail(CONCPD_EINVAL, "block or mode out of range");
    if (!c->lra) return fail(CONCPD_ESTATE, "lra_get_tucker before lra_compress");
    const double* L = (const double*)(c->ws + c->lay.lra);
    const long long len = n < 3 ? c->dims[3 * s + n] * c->geo.J[s][n]
                                : (long long)c->geo.J[s][0] * c->geo.J[s][1] * c->geo.J[s][2];
    const double* src = L + (n < 3 ? c->geo.aoff[n][s] : c->geo.goff[s]);
    HIPCHECK(hipMemcpyAsync(dst, src, sizeof(double) * len, hipMemcpyDeviceToHost, c->q));
    HIPCHECK(hipStreamSynchronize(c->q));
    return CONCPD_OK;
}

concpd_status concpd_get_lipschitz(concpd_ctx c, double* Ld, double* Lu, double* LC) {
    if (!c) return fail(CONCPD_EINVAL, "ctx is NULL");
    const int N = c->N;
    std::vector<double> ld(c->S), lu((size_t)N * c->S), lc(N);
    HIPCHECK(hipMemcpyAsync(ld.data(), c->ws + c->lay.Ld_prev, 8 * ld.size(), hipMemcpyDeviceToHost, c->q));
    HIPCHECK(hipMemcpyAsync(lu.data(), c->ws + c->lay.Lu_prev, 8 * lu.size(), hipMemcpyDeviceToHost, c->q));
    HIPCHECK(hipMemcpyAsync(lc.data(), c->ws + c->lay.LC_prev, 8 * lc.size(), hipMemcpyDeviceToHost, c->q));
    HIPCHECK(hipStreamSynchronize(c->q));
    for (int s = 0; s < c->S; ++s) {
        if (Ld) Ld[s] = ld[s];
        for (int n = 0; n < N; ++n)
            if (Lu) Lu[N * s + n] = lu[n * c->S + s];
    }
    if (LC)
        for (int n = 0; n < N; ++n) LC[n] = lc[n];
    return CONCPD_OK;
}

concpd_status concpd_set_state(concpd_ctx c, const double* const* U, const double* const* U_prev,
                               const double* const* lam, const double* const* lam_prev, const double* Ld_prev,
                               const double* Lu_prev, const double* LC_prev, double t, int64_t k) {
    if (!c || !U || !lam) return fail(CONCPD_EINVAL, "NULL argument");
    if (!(t >= 1.0) || k < 0) return fail(CONCPD_EINVAL, "t must be >= 1 and k >= 0");
    const int N = c->N;
    for (int s = 0; s < c->S; ++s) {
        for (int n = 0; n < N; ++n) {
            const int e = N * s + n;
            const int64_t I = c->dims[e];
            const int rk = c->rk[s];
            if (!U[e]) return fail(CONCPD_EINVAL, "U[%d] is NULL", e);
            if (!cols_finite(U[e], I, c->R, rk) || (U_prev && (!U_prev[e] || !cols_finite(U_prev[e], I, c->R, rk))))
                return fail(CONCPD_ENONFINITE, "U / U_prev[%d] missing or not finite", e);
        }
        if (!lam[s] || !all_finite(lam[s], c->rk[s]) || (lam_prev && (!lam_prev[s] || !all_finite(lam_prev[s], c->rk[s]))))
            return fail(CONCPD_ENONFINITE, "lambda / lambda_prev[%d] missing or not finite", s);
    }
    concpd_status r = c->f64 ? upload_iterate<double>(c, U, U_prev, lam, lam_prev)
                             : upload_iterate<float>(c, U, U_prev, lam, lam_prev);
    if (r != CONCPD_OK) return r;
    r = set_lipschitz_prev(c, Ld_prev, Lu_prev, LC_prev);
    if (r != CONCPD_OK) return r;
    r = set_ctrl(c, t, k);
    if (r != CONCPD_OK) return r;
    if (c->f64) recompute_stats<double>(c, c->sd);
    else recompute_stats<float>(c, c->sf);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(c->q));
    return CONCPD_OK;
}

concpd_status concpd_get_state(concpd_ctx c, double* const* U, double* const* U_prev, double* const* lam,
                               double* const* lam_prev, double* Ld_prev, double* Lu_prev, double* LC_prev, double* t,
                               int64_t* k) {
    if (!c) return fail(CONCPD_EINVAL, "ctx is NULL");
    const int S = c->S, R = c->R, Rq = c->Rq, N = c->N;
    Ctrl h;
    HIPCHECK(hipMemcpyAsync(&h, c->ctrl, sizeof h, hipMemcpyDeviceToHost, c->q));
    HIPCHECK(hipStreamSynchronize(c->q));
    // logical slot 1 holds x_{k-1} (the accepted iterate), slot 2 x_{k-2}
    for (int l = 1; l <= 2; ++l) {
        double* const* Ud = l == 1 ? U : U_prev;
        double* const* Ld = l == 1 ? lam : lam_prev;
        const int ph = (h.rot3 + l) % 3;
        if (Ud) {
            const size_t n = (size_t)c->lay.uslot;
            std::vector<double> hv(n);
            if (c->f64) {
                HIPCHECK(hipMemcpyAsync(hv.data(), c->ws + c->lay.U[ph], n * 8, hipMemcpyDeviceToHost, c->q));
            } else {
                std::vector<float> hf(n);
                HIPCHECK(hipMemcpyAsync(hf.data(), c->ws + c->lay.U[ph], n * 4, hipMemcpyDeviceToHost, c->q));
                HIPCHECK(hipStreamSynchronize(c->q));
                for (size_t i = 0; i < n; ++i) hv[i] = hf[i];
            }
            HIPCHECK(hipStreamSynchronize(c->q));
            for (int s = 0; s < S; ++s)
                for (int n2 = 0; n2 < N; ++n2) {
                    double* dst = Ud[N * s + n2];
                    if (!dst) return fail(CONCPD_EINVAL, "U / U_prev[%d] is NULL", N * s + n2);
                    const double* src = hv.data() + c->geo.uoff[n2][s];
                    for (int64_t i = 0; i < c->dims[N * s + n2]; ++i)
                        for (int r = 0; r < R; ++r) dst[i * R + r] = src[i * Rq + r];
                }
        }
        if (Ld) {
            std::vector<double> hl((size_t)S * Rq);
            HIPCHECK(hipMemcpyAsync(hl.data(), c->ws + c->lay.lam[ph], hl.size() * 8, hipMemcpyDeviceToHost, c->q));
            HIPCHECK(hipStreamSynchronize(c->q));
            for (int s = 0; s < S; ++s) {
                if (!Ld[s]) return fail(CONCPD_EINVAL, "lambda / lambda_prev[%d] is NULL", s);
                for (int r = 0; r < R; ++r) Ld[s][r] = hl[(size_t)s * Rq + r];
            }
        }
    }
    std::vector<double> ld(S), lu((size_t)N * S), lc(N);
    HIPCHECK(hipMemcpyAsync(ld.data(), c->ws + c->lay.Ld_prev, 8 * ld.size(), hipMemcpyDeviceToHost, c->q));
    HIPCHECK(hipMemcpyAsync(lu.data(), c->ws + c->lay.Lu_prev, 8 * lu.size(), hipMemcpyDeviceToHost, c->q));
    HIPCHECK(hipMemcpyAsync(lc.data(), c->ws + c->lay.LC_prev, 8 * lc.size(), hipMemcpyDeviceToHost, c->q));
    HIPCHECK(hipStreamSynchronize(c->q));
    for (int s = 0; s < S; ++s) {
        if (Ld_prev) Ld_prev[s] = ld[s];
        for (int n2 = 0; n2 < N; ++n2)
            if (Lu_prev) Lu_prev[N * s + n2] = lu[n2 * S + s];
    }
    for (int n2 = 0; n2 < N; ++n2)
        if (LC_prev) LC_prev[n2] = lc[n2];
    if (t) *t = h.t;
    if (k) *k = h.k;
    return CONCPD_OK;
}

concpd_status concpd_loss_grad(concpd_ctx c, const void* const* U_dev, const void* const* lambda_dev, int32_t coupled,
                               double* loss, void* const* gU_dev, void* const* glam_dev) {
    if (!c || !U_dev || !lambda_dev || !loss || !gU_dev || !glam_dev) return fail(CONCPD_EINVAL, "NULL argument");
    NEED_ORDER3(c, "concpd_loss_grad");
    if (c->lra) return fail(CONCPD_ESTATE, "concpd_loss_grad is not available in lra mode");
    for (int i = 0; i < 3 * c->S; ++i)
        if (!U_dev[i] || !gU_dev[i]) return fail(CONCPD_EINVAL, "NULL factor pointer %d", i);
    for (int s = 0; s < c->S; ++s)
        if (!lambda_dev[s] || !glam_dev[s]) return fail(CONCPD_EINVAL, "NULL lambda pointer %d", s);
    if (c->f64) return loss_grad_t<double>(c, c->sd, U_dev, lambda_dev, coupled, loss, gU_dev, glam_dev);
    return loss_grad_t<float>(c, c->sf, U_dev, lambda_dev, coupled, loss, gU_dev, glam_dev);
}

concpd_status concpd_debug_mttkrp(concpd_ctx c, int32_t n, int32_t s, void* dev_out) {
    if (!c || !dev_out) return fail(CONCPD_EINVAL, "NULL argument");
    if (n < 0 || n >= c->N || s < 0 || s >= c->S) return fail(CONCPD_EINVAL, "n/s out of range");
    if (c->N > 3) {
        // the sweep's own launches for mode n, every other factor from slot 1
        const int I = (int)c->dims[(size_t)c->N * s + n], half = n >= c->geo.nh;
        long long maxA, maxB;
        int maxI;
        nw_extents(c, &maxA, &maxB, &maxI);
        const size_t es = c->lay.esz;
        const ItemNW* items = (const ItemNW*)(c->ws + (half ? c->lay.itnb : c->lay.itna));
        const int nit = (int)(half ? c->lists.nb.size() : c->lists.na.size());
        if (c->f64) {
            cpd::launch_nw_kr<double>(c->dgeo, c->sd, c->S, half, 1, half ? maxA : maxB, c->Rq, 0, c->q);
            cpd::launch_nw_pass<double>(c->dgeo, c->sd, items, nit, half, c->Rq, 0, c->q);
            cpd::launch_nw_contract<double>(c->dgeo, c->sd, c->S, n, 1, maxI, c->Rq, 0, c->q);
        } else {
            cpd::launch_nw_kr<float>(c->dgeo, c->sf, c->S, half, 1, half ? maxA : maxB, c->Rq, 0, c->q);
            cpd::launch_nw_pass<float>(c->dgeo, c->sf, items, nit, half, c->Rq, 0, c->q);
            cpd::launch_nw_contract<float>(c->dgeo, c->sf, c->S, n, 1, maxI, c->Rq, 0, c->q);
        }
        HIPCHECK(hipMemcpy2DAsync(dev_out, (size_t)c->R * es, c->ws + c->lay.K3 + (size_t)c->geo.koff[s] * es,
                                  (size_t)c->Rq * es, (size_t)c->R * es, (size_t)I, hipMemcpyDeviceToDevice, c->q));
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipStreamSynchronize(c->q));
        return CONCPD_OK;
    }
    const int I = (int)c->dims[3 * s + n];
    if (c->f64) {
        debug_passes<double>(c, c->sd);
        cpd::launch_extract_k<double>(c->dgeo, c->sd, s, n, I, c->R, (double*)dev_out, c->R, 0, c->q);
    } else {
        debug_passes<float>(c, c->sf);
        cpd::launch_extract_k<float>(c->dgeo, c->sf, s, n, I, c->R, (float*)dev_out, c->R, 0, c->q);
    }
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(c->q));
    return CONCPD_OK;
}

concpd_status concpd_launch_floor(int32_t kernels, int32_t reps, double* us_graph, double* us_direct) {
    if (kernels < 1 || kernels > 1024 || reps < 1 || reps > 100000 || !us_graph || !us_direct)
        return fail(CONCPD_EINVAL, "launch floor: kernels in [1, 1024], reps in [1, 100000], non-NULL outputs");
    hipStream_t q = nullptr, qc = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipGraphExec_t gx = nullptr;
    concpd_status st = CONCPD_OK;
    auto done = [&](concpd_status r) {
        if (q) (void)hipStreamSynchronize(q);
        if (gx) (void)hipGraphExecDestroy(gx);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (qc) (void)hipStreamDestroy(qc);
        if (q) (void)hipStreamDestroy(q);
        return r;
    };
#define FLOOR_HIP(x)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (x);                                                                      \
        if (e_ != hipSuccess) return done(fail(CONCPD_EHIP, "%s: %s", #x, hipGetErrorString(e_))); \
    } while (0)
    FLOOR_HIP(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
    FLOOR_HIP(hipStreamCreateWithFlags(&qc, hipStreamNonBlocking));
    FLOOR_HIP(hipEventCreate(&e0));
    FLOOR_HIP(hipEventCreate(&e1));
    FLOOR_HIP(hipStreamBeginCapture(qc, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < kernels; ++i) cpd::launch_empty(qc);
    hipGraph_t graph = nullptr;
    FLOOR_HIP(hipStreamEndCapture(qc, &graph));
    const hipError_t ei = hipGraphInstantiate(&gx, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        gx = nullptr;
        return done(fail(CONCPD_EHIP, "graph instantiate: %s", hipGetErrorString(ei)));
    }
    float ms = 0.f;
    for (int pass = 0; pass < 2; ++pass) {   // warm-up, then timed
        FLOOR_HIP(hipEventRecord(e0, q));
        for (int r = 0; r < reps; ++r) FLOOR_HIP(hipGraphLaunch(gx, q));
        FLOOR_HIP(hipEventRecord(e1, q));
        FLOOR_HIP(hipEventSynchronize(e1));
    }
    FLOOR_HIP(hipEventElapsedTime(&ms, e0, e1));
    *us_graph = 1e3 * ms / reps;
    for (int pass = 0; pass < 2; ++pass) {
        FLOOR_HIP(hipEventRecord(e0, q));
        for (int r = 0; r < reps; ++r)
            for (int i = 0; i < kernels; ++i) cpd::launch_empty(q);
        FLOOR_HIP(hipEventRecord(e1, q));
        FLOOR_HIP(hipEventSynchronize(e1));
    }
    FLOOR_HIP(hipGetLastError());
    FLOOR_HIP(hipEventElapsedTime(&ms, e0, e1));
    *us_direct = 1e3 * ms / reps;
#undef FLOOR_HIP
    return done(st);
}

concpd_status concpd_debug_spectral_norm(const double* host_A, int32_t n, int32_t count, double* host_out) {
    if (!host_A || !host_out) return fail(CONCPD_EINVAL, "NULL argument");
    if (n < 1 || n > CPD_MAXR) return fail(CONCPD_EINVAL, "n = %d not in [1, %d]", n, CPD_MAXR);
    if (count < 1 || count > 65535) return fail(CONCPD_EINVAL, "count = %d not in [1, 65535]", count);
    const size_t nm = (size_t)n * n * count;
    double* d = nullptr;
    HIPCHECK(hipMalloc(&d, sizeof(double) * (nm + count)));
    hipError_t e = hipMemcpy(d, host_A, sizeof(double) * nm, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        cpd::launch_spectral_norm(d, n, count, d + nm, 0);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(host_out, d + nm, sizeof(double) * count, hipMemcpyDeviceToHost);
    const hipError_t ef = hipFree(d);
    if (e == hipSuccess) e = ef;
    if (e != hipSuccess) return fail(CONCPD_EHIP, "spectral norm: %s", hipGetErrorString(e));
    return CONCPD_OK;
}

concpd_status concpd_profile(concpd_ctx c, int32_t enable) {
    if (!c) return fail(CONCPD_EINVAL, "ctx is NULL");
    NEED_ORDER3(c, "concpd_profile");
    c->profiling = enable != 0;
    return CONCPD_OK;
}

concpd_status concpd_profile_read(concpd_ctx c, double* ms1, double* ms2, int64_t* launches) {
    if (!c) return fail(CONCPD_EINVAL, "ctx is NULL");
    NEED_ORDER3(c, "concpd_profile_read");
    HIPCHECK(hipStreamSynchronize(c->q));
    double a = 0.0, b = 0.0;
    for (size_t i = 0; i + 1 < c->ev1.size(); i += 2) {
        float ms = 0.f;
        HIPCHECK(hipEventElapsedTime(&ms, c->ev1[i], c->ev1[i + 1]));
        a += ms;
        ms = 0.f;
        HIPCHECK(hipEventElapsedTime(&ms, c->ev2[i], c->ev2[i + 1]));
        b += ms;
    }
    if (ms1) *ms1 = a;
    if (ms2) *ms2 = b;
    if (launches) *launches = (int64_t)(c->ev1.size() / 2) * CPD_PROF_REPS;
    for (hipEvent_t e : c->ev1) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ev2) (void)hipEventDestroy(e);
    c->ev1.clear();
    c->ev2.clear();
    return CONCPD_OK;
}

concpd_status concpd_set_option(concpd_ctx c, int32_t option, int64_t value) {
    if (!c) return fail(CONCPD_EINVAL, "ctx is NULL");
    if (c->N != 3 && option != CONCPD_OPT_GRAPH_SWEEPS)
        return fail(CONCPD_ENOTSUP, "option %d needs a 3-way context (order N > 3 has graph sweeps only)", option);
    HIPCHECK(hipStreamSynchronize(c->q));
    switch (option) {
    case CONCPD_OPT_GRAPH_SWEEPS:
        if (value < 0 || value > 64) return fail(CONCPD_EINVAL, "graph sweeps %lld not in [0, 64]", (long long)value);
        if (value != c->graph_sweeps) c->drop_graph();
        c->graph_sweeps = (int)value;
        return CONCPD_OK;
    case CONCPD_OPT_OVERLAP:
        if (value != 0 && !c->q2) {
            HIPCHECK(hipStreamCreateWithFlags(&c->q2, hipStreamNonBlocking));
            for (int i = 0; i < 6; ++i) HIPCHECK(hipEventCreateWithFlags(&c->fj[i], hipEventDisableTiming));
        }
        if ((value != 0) != (c->overlap != 0)) c->drop_graph();
        c->overlap = value != 0;
        return CONCPD_OK;
    case CONCPD_OPT_P1_DMA:
        if (value != 0 && value != 1) return fail(CONCPD_EINVAL, "pass-1 DMA %lld not 0 or 1", (long long)value);
        if (value && !c->p1dma_ok) return fail(CONCPD_EINVAL, "pass-1 DMA needs 16-byte aligned rows and a 32/16-bit compute type");
        if (value != c->p1dma) c->drop_graph();
        c->p1dma = (int)value;
        return CONCPD_OK;
    case CONCPD_OPT_FUSE:
        if (value != 0 && value != 1) return fail(CONCPD_EINVAL, "fuse %lld not 0 or 1", (long long)value);
        if (value != c->fuse) c->drop_graph();
        c->fuse = (int)value;
        return CONCPD_OK;
    case CONCPD_OPT_FUSE_LRA:
        if (value != 0 && value != 1) return fail(CONCPD_EINVAL, "fuse_lra %lld not 0 or 1", (long long)value);
        if (value != c->fuse_lra) c->drop_graph();
        c->fuse_lra = (int)value;
        return CONCPD_OK;
    case CONCPD_OPT_P1_SPLIT: {
        if (value != 0 && value != 1 && value != 2 && value != 4)
            return fail(CONCPD_EINVAL, "pass-1 split %lld not 0, 1, 2 or 4", (long long)value);
        Lists L;
        build_lists(&c->cfg, &L, c->k2rows, (int)value);
        c->lists.p1 = L.p1;
        c->lists.p1_split = L.p1_split;
        c->p1split = (int)value;
        HIPCHECK(hipMemcpy(c->ws + c->lay.it1, c->lists.p1.data(), c->lists.p1.size() * sizeof(ItemP1), hipMemcpyHostToDevice));
        c->drop_graph();
        return CONCPD_OK;
    }
    case CONCPD_OPT_K2_ROWS: {
        if (value < CPD_K2ROWS_MIN || value > 64)
            return fail(CONCPD_EINVAL, "mode-2 chunk rows %lld not in [%d, 64]", (long long)value, CPD_K2ROWS_MIN);
        Lists L;
        build_lists(&c->cfg, &L, (int)value, c->p1split);
        c->lists.k2 = L.k2;
        HIPCHECK(hipMemcpy(c->ws + c->lay.itk2, c->lists.k2.data(), c->lists.k2.size() * sizeof(ItemK2), hipMemcpyHostToDevice));
        c->k2rows = (int)value;
        c->geo.k2rows = (int)value;
        for (int s = 0; s < c->S; ++s) c->geo.nk2[s] = (int)((c->dims[3 * s] + value - 1) / value);
        HIPCHECK(hipMemcpy(c->dgeo, &c->geo, sizeof(Geo), hipMemcpyHostToDevice));
        c->drop_graph();
        return CONCPD_OK;
    }
    default:
        return fail(CONCPD_EINVAL, "unknown option %d", option);
    }
}

concpd_status concpd_get_option(concpd_ctx c, int32_t option, int64_t* value) {
    if (!c || !value) return fail(CONCPD_EINVAL, "NULL argument");
    switch (option) {
    case CONCPD_OPT_GRAPH_SWEEPS: *value = c->graph_sweeps; return CONCPD_OK;
    case CONCPD_OPT_OVERLAP: *value = c->overlap; return CONCPD_OK;
    case CONCPD_OPT_K2_ROWS: *value = c->k2rows; return CONCPD_OK;
    case CONCPD_OPT_P1_SPLIT: *value = c->lists.p1_split; return CONCPD_OK;
    case CONCPD_OPT_P1_DMA: *value = c->p1dma; return CONCPD_OK;
    case CONCPD_OPT_FUSE: *value = c->fuse; return CONCPD_OK;
    case CONCPD_OPT_FUSE_LRA: *value = c->fuse_lra; return CONCPD_OK;
    default: return fail(CONCPD_EINVAL, "unknown option %d", option);
    }
}

concpd_status concpd_autotune(concpd_ctx c, int32_t sweeps, concpd_tuning* out) {
    if (!c) return fail(CONCPD_EINVAL, "ctx is NULL");
    NEED_ORDER3(c, "concpd_autotune");
    if (sweeps < 1 || sweeps > 10000) return fail(CONCPD_EINVAL, "sweeps %d not in [1, 10000]", sweeps);
    Ctrl h;
    HIPCHECK(hipMemcpyAsync(&h, c->ctrl, sizeof h, hipMemcpyDeviceToHost, c->q));
    HIPCHECK(hipStreamSynchronize(c->q));
    if (h.stop) return fail(CONCPD_ESTATE, "autotune needs an iterate that has not converged");
    const Layout& P = c->lay;
    const size_t wbytes = c->lra ? sizeof(double) * 2 * (size_t)c->geo.wslot_len : 0;
    char* wlive = c->lra ? c->ws + P.lra + sizeof(double) * (size_t)c->geo.woff[0][0] : nullptr;
    auto snapshot = [&]() -> concpd_status {
        HIPCHECK(hipMemcpyAsync(c->ws + P.snap, c->ws + P.ctrl, P.snap_len, hipMemcpyDeviceToDevice, c->q));
        if (wbytes) HIPCHECK(hipMemcpyAsync(c->ws + P.snap_w, wlive, wbytes, hipMemcpyDeviceToDevice, c->q));
        return CONCPD_OK;
    };
    auto restore = [&]() -> concpd_status {
        HIPCHECK(hipMemcpyAsync(c->ws + P.ctrl, c->ws + P.snap, P.snap_len, hipMemcpyDeviceToDevice, c->q));
        if (wbytes) HIPCHECK(hipMemcpyAsync(wlive, c->ws + P.snap_w, wbytes, hipMemcpyDeviceToDevice, c->q));
        return CONCPD_OK;
    };
    concpd_status r = snapshot();
    if (r != CONCPD_OK) return r;
    const int prof = c->profiling;
    c->profiling = 0;
    r = concpd_set_option(c, CONCPD_OPT_OVERLAP, 0);
    if (r != CONCPD_OK) return r;
    int bo = 0;
    const int k2c[3] = {8, 16, 32};
    const int gsc[3] = {0, 1, 4};
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    double best = INFINITY, dflt = INFINITY;
    int bk = c->k2rows, bg = c->graph_sweeps, ncand = 0, bp = c->p1split;
    auto time_sweeps = [&](double& us) -> concpd_status {
        concpd_status q;
        if ((q = restore()) != CONCPD_OK) return q;
        if ((q = launch_sweeps(c, 4)) != CONCPD_OK) return q;   // warm-up (and graph capture)
        if ((q = restore()) != CONCPD_OK) return q;
        HIPCHECK(hipEventRecord(e0, c->q));
        if ((q = launch_sweeps(c, sweeps)) != CONCPD_OK) return q;
        HIPCHECK(hipEventRecord(e1, c->q));
        HIPCHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
        us = 1e3 * ms / sweeps;
        ++ncand;
        return CONCPD_OK;
    };
    // the default configuration of a fresh context first (it competes too)
    const int dma_dflt = c->p1dma_ok && c->mdtype != 1;
    auto set_default = [&]() -> concpd_status {
        concpd_status q;
        if ((q = concpd_set_option(c, CONCPD_OPT_GRAPH_SWEEPS, 0)) != CONCPD_OK) return q;
        if ((q = concpd_set_option(c, CONCPD_OPT_OVERLAP, 0)) != CONCPD_OK) return q;
        if (!c->lra && (q = concpd_set_option(c, CONCPD_OPT_K2_ROWS, CPD_K2ROWS_DEFAULT)) != CONCPD_OK) return q;
        if ((q = concpd_set_option(c, CONCPD_OPT_P1_DMA, dma_dflt)) != CONCPD_OK) return q;
        if ((q = concpd_set_option(c, CONCPD_OPT_P1_SPLIT, 0)) != CONCPD_OK) return q;
        return concpd_set_option(c, CONCPD_OPT_FUSE, c->fuse_dflt);
    };
    if ((r = set_default()) == CONCPD_OK) r = time_sweeps(dflt);
    if (r == CONCPD_OK) r = concpd_set_option(c, CONCPD_OPT_FUSE, 0);
    if (!c->lra && r == CONCPD_OK) {
        // the pass-1 split of i3 over wavefronts (direct launches, default chunk rows)
        Lists La;
        build_lists(&c->cfg, &La, CPD_K2ROWS_DEFAULT, 0);
        const int p_auto = La.p1_split;
        double bpu = INFINITY;
        const int psc[3] = {1, 2, 4};
        int bd = c->p1dma;
        if ((r = concpd_set_option(c, CONCPD_OPT_GRAPH_SWEEPS, 0)) == CONCPD_OK)
            r = concpd_set_option(c, CONCPD_OPT_K2_ROWS, CPD_K2ROWS_DEFAULT);
        for (int di = 0; di < (c->p1dma_ok ? 2 : 1) && r == CONCPD_OK; ++di) {
            const int dma = c->p1dma_ok ? di : 0;
            if ((r = concpd_set_option(c, CONCPD_OPT_P1_DMA, dma)) != CONCPD_OK) break;
            for (int pi = 0; pi < 3 && r == CONCPD_OK; ++pi) {
                if ((r = concpd_set_option(c, CONCPD_OPT_P1_SPLIT, psc[pi])) != CONCPD_OK) break;
                double us = 0.0;
                if ((r = time_sweeps(us)) != CONCPD_OK) break;
                if (us < bpu) {
                    bpu = us;
                    bp = psc[pi];
                    bd = dma;
                }
            }
        }
        if (r == CONCPD_OK) r = concpd_set_option(c, CONCPD_OPT_P1_SPLIT, bp);
        if (r == CONCPD_OK) r = concpd_set_option(c, CONCPD_OPT_P1_DMA, bd);
    }
    for (int ki = 0; ki < 3 && r == CONCPD_OK; ++ki) {
        if (c->lra && ki > 0) break;   // the mode-2 contraction is not on the lra path
        r = concpd_set_option(c, CONCPD_OPT_K2_ROWS, k2c[ki]);
        if (r != CONCPD_OK) break;
        for (int gi = 0; gi < 3; ++gi) {
            r = concpd_set_option(c, CONCPD_OPT_GRAPH_SWEEPS, gsc[gi]);
            if (r != CONCPD_OK) break;
            double us = 0.0;
            if ((r = time_sweeps(us)) != CONCPD_OK) break;
            if (us < best) {
                best = us;
                bk = k2c[ki];
                bg = gsc[gi];
            }
        }
        if (r != CONCPD_OK) break;
    }
    // the small kernels on a second stream beside the passes, as branches of
    // the captured graph (dense path; measured: faster for the EEG-shaped
    // blocks, even for cubes)
    if (!c->lra && r == CONCPD_OK) {
        r = concpd_set_option(c, CONCPD_OPT_K2_ROWS, bk);
        if (r == CONCPD_OK) r = concpd_set_option(c, CONCPD_OPT_OVERLAP, 1);
        for (int gi = 1; gi < 3 && r == CONCPD_OK; ++gi) {
            r = concpd_set_option(c, CONCPD_OPT_GRAPH_SWEEPS, gsc[gi]);
            if (r != CONCPD_OK) break;
            double us = 0.0;
            if ((r = time_sweeps(us)) != CONCPD_OK) break;
            if (us < best) {
                best = us;
                bg = gsc[gi];
                bo = 1;
            }
        }
        if (r == CONCPD_OK) r = concpd_set_option(c, CONCPD_OPT_OVERLAP, bo);
    }
    // the R x R work fused into the launches of the passes (dense path, R <= 32),
    // with direct launches and with the best graph length
    // (direct launches also with the other pass-1 split of 1 and 2: the fused
    // pass keeps fewer wavefronts resident, so shorter items can pay off)
    int bf = 0;
    if (!c->lra && c->R <= 32 && r == CONCPD_OK) {
        const int ov = bo, gbest = bg, pbest = c->lists.p1_split;
        int bsplit = pbest;
        if ((r = concpd_set_option(c, CONCPD_OPT_OVERLAP, 0)) == CONCPD_OK) r = concpd_set_option(c, CONCPD_OPT_FUSE, 1);
        for (int gi = 0; gi < 3 && r == CONCPD_OK; ++gi) {
            const int gsv = gi == 2 ? gbest : 0;
            const int sp = gi == 1 ? (pbest == 1 ? 2 : 1) : pbest;
            if (gi == 2 && gsv == 0) break;
            if (gi == 1 && c->f64) continue;
            if ((r = concpd_set_option(c, CONCPD_OPT_P1_SPLIT, sp)) != CONCPD_OK) break;
            if ((r = concpd_set_option(c, CONCPD_OPT_GRAPH_SWEEPS, gsv)) != CONCPD_OK) break;
            double us = 0.0;
            if ((r = time_sweeps(us)) != CONCPD_OK) break;
            if (us < best) {
                best = us;
                bg = gsv;
                bf = 1;
                bo = 0;
                bsplit = sp;
            }
        }
        if (r == CONCPD_OK) r = concpd_set_option(c, CONCPD_OPT_P1_SPLIT, bf ? bsplit : pbest);
        if (r == CONCPD_OK) r = concpd_set_option(c, CONCPD_OPT_FUSE, bf);
        if (r == CONCPD_OK) r = concpd_set_option(c, CONCPD_OPT_OVERLAP, bf ? 0 : ov);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->profiling = prof;
    if (r != CONCPD_OK) return r;
    if (dflt <= best) {
        // no candidate beat the default configuration
        if ((r = set_default()) != CONCPD_OK) return r;
        best = dflt;
        bk = CPD_K2ROWS_DEFAULT;
        bg = 0;
        bo = 0;
        bf = c->fuse;
    }
    if (!c->lra) {
        r = concpd_set_option(c, CONCPD_OPT_K2_ROWS, bk);
        if (r != CONCPD_OK) return r;
    }
    r = concpd_set_option(c, CONCPD_OPT_GRAPH_SWEEPS, bg);
    if (r != CONCPD_OK) return r;
    r = restore();
    if (r != CONCPD_OK) return r;
    HIPCHECK(hipStreamSynchronize(c->q));
    if (out) {
        out->k2_rows = c->k2rows;
        out->p1_split = c->lists.p1_split;
        out->p1_dma = c->p1dma;
        out->graph_sweeps = bg;
        out->overlap = bo;
        out->fuse = bf;
        out->us_per_sweep = best;
        out->us_per_sweep_default = dflt;
        out->candidates = ncand;
    }
    return CONCPD_OK;
}

concpd_status concpd_destroy(concpd_ctx c) {
    if (!c) return CONCPD_OK;
    (void)hipStreamSynchronize(c->q);
    for (hipEvent_t e : c->ev1) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ev2) (void)hipEventDestroy(e);
    if (c->static_dev >= 0) {
        std::lock_guard<std::mutex> lock(g_static.mu);
        if (g_static.owner[c->static_dev] == c) g_static.owner[c->static_dev] = nullptr;
    }
    delete c;
    return CONCPD_OK;
}

}  // extern "C"
