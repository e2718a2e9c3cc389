// The mixed-precision form of the persistent integral kernel (shgo_integrals_kernel.h): the
// product-rule and shift coupling of every primitive pair in binary32 with error-free
// transformations; the nucleus sums, the Boys function, the exp(-mu R^2) and contraction
// prefactors and the accumulation over primitive pairs stay binary64.
#include "shgo_integrals_kernel.h"

namespace shgo_impl {

void launch_integrals_mixed(const shgo_plan* p, double* out, hipStream_t st) { launch_integrals_impl<true>(p, out, st); }

hipError_t integrals_setup_mixed(int* per_cu, std::string* why) { return integrals_setup_impl<true>(per_cu, why); }

}  // namespace shgo_impl
