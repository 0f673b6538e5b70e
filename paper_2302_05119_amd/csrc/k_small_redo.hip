// Instantiations of the small sweep kernels for the re-done sweep (GATE = 1):
// the same kernels under distinct symbols, compiled in parallel with the others.
#include "small_kernels.h"

namespace cpd {
CPD_SMALL_IMPLS(template, 1)
}  // namespace cpd
