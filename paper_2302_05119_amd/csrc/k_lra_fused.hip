// Launches of the compressed sweep (Algorithm 2) that run the small FP64
// work beside lra work it does not depend on (Algorithm 1's order is
// unchanged; only independent steps share a launch):
//   - the core update and the mode-1 step matrix (both from x_{k-1}) beside
//     C_1 = G_(1) (W_3 ⊙ W_2), which reads the W of x_{k-1} only,
//   - the step matrix of mode n (Gram of the new U^(n-1)) beside the refresh
//     W_{n-1} = A_{n-1}^T U^(n-1), which reads the same new factor.
// The first nsmall workgroups (S rounded up to a multiple of 8) do one
// block's R x R work each and leave; the rest take the lra rows (row j of
// block s at j + Jmax s).  A compressed sweep then has ten launches instead of
// thirteen.
#include "lra_items.h"
#include "small_dev.h"

namespace cpd {

// Wavefronts per SIMD the launch is compiled for: the R x R code of size
// class NM keeps two up to R = 32 (as the dense fused launches), one above.
template <int NM> struct LraFuseWaves { static constexpr int W = NM <= 32 ? 2 : 1; };

template <typename T, int NM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LraFuseWaves<NM>::W))) void k_core_lrac(
    const Geo* __restrict__ g, StateP<T> st, int extrapolate, int S, int nsmall, int Jmax) {
    if (st.ctrl->stop) return;
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    const int bid = blockIdx.x;
    if (bid < nsmall) {
        if (bid < S) {
            apply_rot(st);
            core_block<T, NM>(g, st, bid, extrapolating(st.ctrl, extrapolate), smraw);
        }
        return;
    }
    const int b = bid - nsmall;
    lra_c_item<T>(g, st, 0, b / Jmax, b % Jmax, (double*)smraw);
}

template <typename T, int NM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LraFuseWaves<NM>::W))) void k_prep_lraw(
    const Geo* __restrict__ g, StateP<T> st, int n, int S, int nsmall, int Jmax) {
    if (st.ctrl->stop) return;
    apply_rot(st);
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    const int bid = blockIdx.x;
    if (bid < nsmall) {
        if (bid < S) prep_block<T, NM>(g, st, bid, n, smraw);
        return;
    }
    const int b = bid - nsmall;
    // W of the mode just updated, logical slot 0
    lra_w_item<T>(g, st, n - 1, 0, st.ctrl->rot2, b / Jmax, b % Jmax);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int lra_small_wgs(int S) { return (S + 7) & ~7; }

template <typename T>
void launch_core_lrac(const Geo* g, const StateP<T>& st, int S, int R, int Jmax, int Rq, int extrap, hipStream_t q) {
    const int ns = lra_small_wgs(S);
    const dim3 grid(ns + Jmax * S);
    const size_t a = eig_lds_bytes(R), b = lra_c_lds_bytes(Jmax, Rq);
    const size_t lds = a > b ? a : b;
#define CPD_CL(NMV) hipLaunchKernelGGL((k_core_lrac<T, NMV>), grid, dim3(256), lds, q, g, st, extrap, S, ns, Jmax)
    switch (nmax_class(R)) {
    case 16: CPD_CL(16); break;
    case 24: CPD_CL(24); break;
    case 32: CPD_CL(32); break;
    case 48: CPD_CL(48); break;
    default: CPD_CL(64); break;
    }
#undef CPD_CL
}

template <typename T>
void launch_prep_lraw(const Geo* g, const StateP<T>& st, int S, int R, int Jmax, int Rq, int n, hipStream_t q) {
    const int ns = lra_small_wgs(S);
    const dim3 grid(ns + Jmax * S);
    const size_t lds = prep_lds_bytes<T>(R, Rq);
#define CPD_PW(NMV) hipLaunchKernelGGL((k_prep_lraw<T, NMV>), grid, dim3(256), lds, q, g, st, n, S, ns, Jmax)
    switch (nmax_class(R)) {
    case 16: CPD_PW(16); break;
    case 24: CPD_PW(24); break;
    case 32: CPD_PW(32); break;
    case 48: CPD_PW(48); break;
    default: CPD_PW(64); break;
    }
#undef CPD_PW
}

#define CPD_INST_LRA_FUSED(T)                                                                                 \
    template void launch_core_lrac<T>(const Geo*, const StateP<T>&, int, int, int, int, int, hipStream_t);   \
    template void launch_prep_lraw<T>(const Geo*, const StateP<T>&, int, int, int, int, int, hipStream_t);
CPD_INST_LRA_FUSED(float)
CPD_INST_LRA_FUSED(double)

}  // namespace cpd
