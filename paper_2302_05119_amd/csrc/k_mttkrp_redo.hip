// Instantiations of the MTTKRP passes for the re-done sweep (GATE = 1): the
// same kernels under distinct symbols, compiled in parallel with the others.
#include "mttkrp_kernels.h"

namespace cpd {
CPD_MTTKRP_IMPLS(template, 1)
}  // namespace cpd
