// The binary64 form of the persistent integral kernel (shgo_integrals_kernel.h).
#include "shgo_integrals_kernel.h"

namespace shgo_impl {

void launch_integrals_fp64(const shgo_plan* p, double* out, hipStream_t st) { launch_integrals_impl<false>(p, out, st); }

hipError_t integrals_setup_fp64(int* per_cu, std::string* why) { return integrals_setup_impl<false>(per_cu, why); }

}  // namespace shgo_impl
