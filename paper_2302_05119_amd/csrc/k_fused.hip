// Launches that run the small FP64 work of a sweep beside the MTTKRP work it
// does not depend on (Algorithm 1's order is unchanged; only independent
// steps share a launch):
//   - the core update and the mode-1 step matrix (both need only x_{k-1})
//     beside pass 1 (Y = M x_3 U^(3) and the mode-1 partials),
//   - the mode-2 step matrix (Gram of the new U^(1)) beside the mode-2
//     contraction, which also reads the new U^(1),
//   - the mode-3 step matrix (Gram of the new U^(2)) beside pass 2.
// The first nsmall workgroups (S rounded up to a multiple of 8, so the pass
// items keep their XCD placement) do one block's R x R work each and leave;
// the rest run the pass items.  The latency-bound R x R chains then hide
// under the streaming work, and a sweep has three launch boundaries fewer.
// The R x R code needs more registers than the passes, so these launches
// keep fewer wavefronts per SIMD; the context option selects them (they pay
// off while a pass has few items per SIMD).
#include "mttkrp_kernels.h"
#include "small_dev.h"

namespace cpd {

// Wavefronts per SIMD a fused launch is compiled for: the register budget of
// the R x R code of size class NM beside the pass code (chosen so that
// nothing spills): the core update with pass 1 keeps two, a step matrix with
// an FP32 pass three, with an FP64 pass two.
template <typename T, int NM> struct FuseWaves { static constexpr int W = 2; };
template <> struct FuseWaves<float, 16> { static constexpr int W = 3; };
template <> struct FuseWaves<float, 24> { static constexpr int W = 3; };

template <int RT> struct FuseNM { static constexpr int NM = nmax_class(4 * RT); };

// Wavefronts per SIMD of the core update + pass 1 launch: the core code sets
// the register count, and with it the occupancy of the pass wavefronts.  Up to
// R = 20 on an FP32 tensor three fit, with a few core values spilled (C2's
// fused launch: 28 -> 24.5 us); wider tiles, FP64 and the 16-bit DMA path
// (its BF16 operand split) keep two.
template <typename TM, int RT> struct FusePass1Waves {
    static constexpr int W = (std::is_same<TM, float>::value && RT <= 5) ? 3 : 2;
};

template <typename TM, typename T, int RT, int DMA>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FusePass1Waves<TM, RT>::W))) void k_core_pass1(
    const Geo* __restrict__ g, StateP<T> st, const ItemP1* __restrict__ items, int nitems, int P, int slot, int extrapolate,
    int S, int nsmall) {
    if (st.ctrl->stop) return;
    apply_rot(st);
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    const int bid = blockIdx.x;
    if (bid < nsmall) {
        if (bid < S) core_block<T, FuseNM<RT>::NM>(g, st, bid, extrapolating(st.ctrl, extrapolate), smraw);
        return;
    }
    if constexpr (DMA) pass1d_item<TM, RT>(g, st, items, nitems, P, slot, bid - nsmall);
    else pass1_item<TM, T, RT>(g, st, items, nitems, P, slot, bid - nsmall);
}

template <typename T, int NM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FuseWaves<T, NM>::W))) void k_prep_k2(
    const Geo* __restrict__ g, StateP<T> st, const ItemK2* __restrict__ items, int slot, int S, int nsmall) {
    if (st.ctrl->stop) return;
    apply_rot(st);
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    const int bid = blockIdx.x;
    if (bid < nsmall) {
        if (bid < S) prep_block<T, NM>(g, st, bid, 1, smraw);
        return;
    }
    k2_item<T>(g, st, items, slot, bid - nsmall);
}

template <typename TM, typename T, int RT, bool BLDS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FuseWaves<T, FuseNM<RT>::NM>::W))) void k_prep_pass2(
    const Geo* __restrict__ g, StateP<T> st, const ItemP2* __restrict__ items, int slot, int S, int nsmall) {
    if (st.ctrl->stop) return;
    apply_rot(st);
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    const int bid = blockIdx.x;
    if (bid < nsmall) {
        if (bid < S) prep_block<T, FuseNM<RT>::NM>(g, st, bid, 2, smraw);
        return;
    }
    pass2_item<TM, T, RT, BLDS>(g, st, items, slot, bid - nsmall);
}

// ---------------------------------------------------------------------------
// launchers (R <= 32: the vector-ALU spectral-norm classes)
// ---------------------------------------------------------------------------
static int small_wgs(int S) { return (S + 7) & ~7; }

template <typename TM, typename T, int DMA>
static void core_pass1_rt(int RT, dim3 grid, size_t lds, hipStream_t q, const Geo* g, const StateP<T>& st, const ItemP1* items,
                          int nitems, int P, int slot, int extrap, int S, int ns) {
#define CPD_FC1(RTV)                                                                                                  \
    case RTV:                                                                                                         \
        hipLaunchKernelGGL((k_core_pass1<TM, T, RTV, DMA>), grid, dim3(256), lds, q, g, st, items, nitems, P, slot, extrap, \
                           S, ns);                                                                                    \
        break;
    switch (RT) {
        CPD_FC1(1) CPD_FC1(2) CPD_FC1(3) CPD_FC1(4) CPD_FC1(5) CPD_FC1(6) CPD_FC1(7) CPD_FC1(8)
        default: break;
    }
#undef CPD_FC1
}

template <typename T>
bool launch_core_pass1(const Geo* g, const StateP<T>& st, const ItemP1* items, int nitems, int P, int R, int slot, int mdtype,
                       int dma, int extrap, int S, hipStream_t q) {
    const int Rq = (R + 3) / 4 * 4, RT = Rq / 4;
    if (R > 32 || nitems <= 0) return false;
    const int ns = small_wgs(S);
    const dim3 grid(ns + (nitems * P + 3) / 4);
    const size_t eig = eig_lds_bytes(R);
    if constexpr (std::is_same<T, double>::value) {
        const size_t p = pass1_lds<double>(RT, P);
        core_pass1_rt<double, double, 0>(RT, grid, p > eig ? p : eig, q, g, st, items, nitems, P, slot, extrap, S, ns);
    } else if (dma) {
#define CPD_FD(TMV)                                                                                                   \
    {                                                                                                                  \
        size_t p = 0;                                                                                                  \
        switch (RT) {                                                                                                  \
        case 1: p = 4 * (size_t)P1D<TMV, 1>::WAVE; break;                                                              \
        case 2: p = 4 * (size_t)P1D<TMV, 2>::WAVE; break;                                                              \
        case 3: p = 4 * (size_t)P1D<TMV, 3>::WAVE; break;                                                              \
        case 4: p = 4 * (size_t)P1D<TMV, 4>::WAVE; break;                                                              \
        case 5: p = 4 * (size_t)P1D<TMV, 5>::WAVE; break;                                                              \
        case 6: p = 4 * (size_t)P1D<TMV, 6>::WAVE; break;                                                              \
        case 7: p = 4 * (size_t)P1D<TMV, 7>::WAVE; break;                                                              \
        default: p = 4 * (size_t)P1D<TMV, 8>::WAVE; break;                                                             \
        }                                                                                                              \
        core_pass1_rt<TMV, float, 1>(RT, grid, p > eig ? p : eig, q, g, st, items, nitems, P, slot, extrap, S, ns);   \
    }
        if (mdtype == 1) CPD_FD(float)
        else if (mdtype == 2) CPD_FD(__hip_bfloat16)
        else CPD_FD(__half)
#undef CPD_FD
    } else {
        // the register path of 16-bit storage would spill beside the core
        // update: it runs unfused
        if (mdtype != 1) return false;
        const size_t p = pass1_lds<float>(RT, P);
        core_pass1_rt<float, float, 0>(RT, grid, p > eig ? p : eig, q, g, st, items, nitems, P, slot, extrap, S, ns);
    }
    return true;
}

template <typename T>
bool launch_prep_k2(const Geo* g, const StateP<T>& st, const ItemK2* items, int nitems, int R, int slot, int S, hipStream_t q) {
    const int Rq = (R + 3) / 4 * 4;
    if (R > 32 || nitems <= 0) return false;
    const int ns = small_wgs(S);
    const dim3 grid(ns + nitems);
    const size_t lds = prep_lds_bytes<T>(R, Rq);
    switch (nmax_class(R)) {
    case 16: hipLaunchKernelGGL((k_prep_k2<T, 16>), grid, dim3(256), lds, q, g, st, items, slot, S, ns); break;
    case 24: hipLaunchKernelGGL((k_prep_k2<T, 24>), grid, dim3(256), lds, q, g, st, items, slot, S, ns); break;
    default: hipLaunchKernelGGL((k_prep_k2<T, 32>), grid, dim3(256), lds, q, g, st, items, slot, S, ns); break;
    }
    return true;
}

template <typename TM, typename T>
static void prep_pass2_disp(int R, int maxI2, dim3 grid, hipStream_t q, const Geo* g, const StateP<T>& st, const ItemP2* items,
                            int slot, int S, int ns) {
    const int Rq = (R + 3) / 4 * 4, RT = Rq / 4;
    bool whole = true;
    const size_t p = pass2_lds<TM>(Rq, maxI2, &whole), e = prep_lds_bytes<T>(R, Rq);
    const size_t lds = p > e ? p : e;
#define CPD_FP2(RTV)                                                                                                 \
    case RTV:                                                                                                        \
        if (whole) hipLaunchKernelGGL((k_prep_pass2<TM, T, RTV, true>), grid, dim3(256), lds, q, g, st, items, slot, S, ns); \
        else hipLaunchKernelGGL((k_prep_pass2<TM, T, RTV, false>), grid, dim3(256), lds, q, g, st, items, slot, S, ns);     \
        break;
    switch (RT) {
        CPD_FP2(1) CPD_FP2(2) CPD_FP2(3) CPD_FP2(4) CPD_FP2(5) CPD_FP2(6) CPD_FP2(7) CPD_FP2(8)
        default: break;
    }
#undef CPD_FP2
}

template <typename T>
bool launch_prep_pass2(const Geo* g, const StateP<T>& st, const ItemP2* items, int nitems, int R, int slot, int mdtype, int maxI2,
                       int spw, int S, hipStream_t q) {
    // one i1 slab per wavefront only (the fused launch shares its registers)
    if (R > 32 || nitems <= 0 || spw != 1) return false;
    const int ns = small_wgs(S);
    const dim3 grid(ns + nitems);
    if constexpr (std::is_same<T, double>::value) {
        prep_pass2_disp<double, double>(R, maxI2, grid, q, g, st, items, slot, S, ns);
    } else {
        if (mdtype == 1) prep_pass2_disp<float, float>(R, maxI2, grid, q, g, st, items, slot, S, ns);
        else if (mdtype == 2) prep_pass2_disp<__hip_bfloat16, float>(R, maxI2, grid, q, g, st, items, slot, S, ns);
        else prep_pass2_disp<__half, float>(R, maxI2, grid, q, g, st, items, slot, S, ns);
    }
    return true;
}

#define CPD_INST_FUSED(T)                                                                                                  \
    template bool launch_core_pass1<T>(const Geo*, const StateP<T>&, const ItemP1*, int, int, int, int, int, int, int, int, \
                                       hipStream_t);                                                                       \
    template bool launch_prep_k2<T>(const Geo*, const StateP<T>&, const ItemK2*, int, int, int, int, hipStream_t);          \
    template bool launch_prep_pass2<T>(const Geo*, const StateP<T>&, const ItemP2*, int, int, int, int, int, int, int, hipStream_t);
CPD_INST_FUSED(float)
CPD_INST_FUSED(double)

}  // namespace cpd
