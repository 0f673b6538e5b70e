// Launchers of the dense MTTKRP passes (kernels in mttkrp_kernels.h).  The
// re-done sweep's instantiations (GATE = 1) live in k_mttkrp_redo.hip.
#include "mttkrp_kernels.h"

namespace cpd {

CPD_MTTKRP_IMPLS(extern template, 1)
CPD_MTTKRP_IMPLS(template, 0)

template <typename T>
void launch_pass1(const Geo* g, const StateP<T>& st, const ItemP1* items, int nitems, int Rq, int slot, int gate, int mdtype,
                  hipStream_t q) {
    if (gate) pass1_impl<1, T>(g, st, items, nitems, Rq, slot, mdtype, q);
    else pass1_impl<0, T>(g, st, items, nitems, Rq, slot, mdtype, q);
}
template <typename T>
void launch_pass2(const Geo* g, const StateP<T>& st, const ItemP2* items, int nitems, int Rq, int slot, int gate, int mdtype,
                  int maxI2, hipStream_t q) {
    if (gate) pass2_impl<1, T>(g, st, items, nitems, Rq, slot, mdtype, maxI2, q);
    else pass2_impl<0, T>(g, st, items, nitems, Rq, slot, mdtype, maxI2, q);
}
template <typename T>
void launch_k2(const Geo* g, const StateP<T>& st, const ItemK2* items, int nitems, int slot, int gate, hipStream_t q) {
    if (gate) k2_impl<1, T>(g, st, items, nitems, slot, q);
    else k2_impl<0, T>(g, st, items, nitems, slot, q);
}
template void launch_pass1<float>(const Geo*, const StateP<float>&, const ItemP1*, int, int, int, int, int, hipStream_t);
template void launch_pass1<double>(const Geo*, const StateP<double>&, const ItemP1*, int, int, int, int, int, hipStream_t);
template void launch_pass2<float>(const Geo*, const StateP<float>&, const ItemP2*, int, int, int, int, int, int, hipStream_t);
template void launch_pass2<double>(const Geo*, const StateP<double>&, const ItemP2*, int, int, int, int, int, int, hipStream_t);
template void launch_k2<float>(const Geo*, const StateP<float>&, const ItemK2*, int, int, int, hipStream_t);
template void launch_k2<double>(const Geo*, const StateP<double>&, const ItemK2*, int, int, int, hipStream_t);

}  // namespace cpd
