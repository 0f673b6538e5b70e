// Launchers of the dense MTTKRP passes (kernels in mttkrp_kernels.h):
// dispatch on the tensor operand type and on RT = Rq / 4.
#include "mttkrp_kernels.h"

namespace cpd {

template <typename TM, typename T>
static void pass1_rt(int RT, dim3 grid, size_t lds, hipStream_t q, const Geo* g, const StateP<T>& st, const ItemP1* items,
                     int nitems, int P, int slot) {
#define CPD_P1(RTV) \
    case RTV: hipLaunchKernelGGL((k_pass1<TM, T, RTV>), grid, dim3(256), lds, q, g, st, items, nitems, P, slot); break;
    switch (RT) {
        CPD_P1(1) CPD_P1(2) CPD_P1(3) CPD_P1(4) CPD_P1(5) CPD_P1(6) CPD_P1(7) CPD_P1(8)
        CPD_P1(9) CPD_P1(10) CPD_P1(11) CPD_P1(12) CPD_P1(13) CPD_P1(14) CPD_P1(15) CPD_P1(16)
        default: break;
    }
#undef CPD_P1
}
template <typename TM>
static void pass1d_rt(int RT, dim3 grid, hipStream_t q, const Geo* g, const StateP<float>& st, const ItemP1* items, int nitems,
                      int P, int slot) {
#define CPD_P1D(RTV)                                                                                        \
    case RTV: {                                                                                             \
        const size_t lds = 4 * (size_t)P1D<TM, RTV>::WAVE;                                                  \
        hipLaunchKernelGGL((k_pass1d<TM, RTV>), grid, dim3(256), lds, q, g, st, items, nitems, P, slot);    \
        break;                                                                                              \
    }
    switch (RT) {
        CPD_P1D(1) CPD_P1D(2) CPD_P1D(3) CPD_P1D(4) CPD_P1D(5) CPD_P1D(6) CPD_P1D(7) CPD_P1D(8)
        CPD_P1D(9) CPD_P1D(10) CPD_P1D(11) CPD_P1D(12) CPD_P1D(13) CPD_P1D(14) CPD_P1D(15) CPD_P1D(16)
        default: break;
    }
#undef CPD_P1D
}
template <typename TM, typename T, bool BLDS, int SPW>
static void pass2_rt(int RT, dim3 grid, size_t lds, hipStream_t q, const Geo* g, const StateP<T>& st, const ItemP2* items,
                     int slot) {
#define CPD_P2(RTV) \
    case RTV: hipLaunchKernelGGL((k_pass2<TM, T, RTV, BLDS, SPW>), grid, dim3(256), lds, q, g, st, items, slot); break;
    switch (RT) {
        CPD_P2(1) CPD_P2(2) CPD_P2(3) CPD_P2(4) CPD_P2(5) CPD_P2(6) CPD_P2(7) CPD_P2(8)
        CPD_P2(9) CPD_P2(10) CPD_P2(11) CPD_P2(12) CPD_P2(13) CPD_P2(14) CPD_P2(15) CPD_P2(16)
        default: break;
    }
#undef CPD_P2
}

// spw: i1 slabs per wavefront, as the context's work list was built (two
// only on FP32/16-bit tensors)
template <typename TM, typename T>
static void pass2_dispatch(int Rq, dim3 grid, int maxI2, int spw, hipStream_t q, const Geo* g, const StateP<T>& st,
                           const ItemP2* items, int slot) {
    bool blds = true;
    const size_t lds = pass2_lds<TM>(Rq, maxI2, &blds);
    if constexpr (!std::is_same<T, double>::value) {
        if (spw == 2) {
            if (blds) pass2_rt<TM, T, true, 2>(Rq / 4, grid, lds, q, g, st, items, slot);
            else pass2_rt<TM, T, false, 2>(Rq / 4, grid, lds, q, g, st, items, slot);
            return;
        }
    }
    if (blds) pass2_rt<TM, T, true, 1>(Rq / 4, grid, lds, q, g, st, items, slot);
    else pass2_rt<TM, T, false, 1>(Rq / 4, grid, lds, q, g, st, items, slot);
}

template <typename T>
void launch_pass1(const Geo* g, const StateP<T>& st, const ItemP1* items, int nitems, int P, int Rq, int slot, int mdtype,
                  int dma, hipStream_t q) {
    if (nitems <= 0) return;
    const dim3 grid((nitems * P + 3) / 4);
    const int RT = Rq / 4;
    if constexpr (std::is_same<T, double>::value) {
        (void)dma;
        pass1_rt<double, double>(RT, grid, pass1_lds<double>(RT, P), q, g, st, items, nitems, P, slot);
    } else if (dma) {
        // every block's operand rows 16-byte aligned: the LDS-DMA stream
        if (mdtype == 1) pass1d_rt<float>(RT, grid, q, g, st, items, nitems, P, slot);
        else if (mdtype == 2) pass1d_rt<__hip_bfloat16>(RT, grid, q, g, st, items, nitems, P, slot);
        else pass1d_rt<__half>(RT, grid, q, g, st, items, nitems, P, slot);
    } else {
        if (mdtype == 1) pass1_rt<float, float>(RT, grid, pass1_lds<float>(RT, P), q, g, st, items, nitems, P, slot);
        else if (mdtype == 2)
            pass1_rt<__hip_bfloat16, float>(RT, grid, pass1_lds<__hip_bfloat16>(RT, P), q, g, st, items, nitems, P, slot);
        else pass1_rt<__half, float>(RT, grid, pass1_lds<__half>(RT, P), q, g, st, items, nitems, P, slot);
    }
}

template <typename T>
void launch_pass2(const Geo* g, const StateP<T>& st, const ItemP2* items, int nitems, int Rq, int slot, int mdtype, int maxI2,
                  int spw, hipStream_t q) {
    if (nitems <= 0) return;
    const dim3 grid(nitems);
    if constexpr (std::is_same<T, double>::value) {
        pass2_dispatch<double, double>(Rq, grid, maxI2, spw, q, g, st, items, slot);
    } else {
        if (mdtype == 1) pass2_dispatch<float, float>(Rq, grid, maxI2, spw, q, g, st, items, slot);
        else if (mdtype == 2) pass2_dispatch<__hip_bfloat16, float>(Rq, grid, maxI2, spw, q, g, st, items, slot);
        else pass2_dispatch<__half, float>(Rq, grid, maxI2, spw, q, g, st, items, slot);
    }
}

template <typename T>
void launch_k2(const Geo* g, const StateP<T>& st, const ItemK2* items, int nitems, int slot, hipStream_t q) {
    if (nitems <= 0) return;
    hipLaunchKernelGGL(k_k2<T>, dim3(nitems), dim3(256), 0, q, g, st, items, slot);
}

template void launch_pass1<float>(const Geo*, const StateP<float>&, const ItemP1*, int, int, int, int, int, int, hipStream_t);
template void launch_pass1<double>(const Geo*, const StateP<double>&, const ItemP1*, int, int, int, int, int, int, hipStream_t);
template void launch_pass2<float>(const Geo*, const StateP<float>&, const ItemP2*, int, int, int, int, int, int, hipStream_t);
template void launch_pass2<double>(const Geo*, const StateP<double>&, const ItemP2*, int, int, int, int, int, int, hipStream_t);
template void launch_k2<float>(const Geo*, const StateP<float>&, const ItemK2*, int, int, hipStream_t);
template void launch_k2<double>(const Geo*, const StateP<double>&, const ItemK2*, int, int, hipStream_t);

}  // namespace cpd
