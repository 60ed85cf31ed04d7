// Instantiations of the register-state LB_Improved kernel for p = infinity, half-widths 0..kLbiRegMaxW.
#include "lbi_reg.h"

namespace lbimp {

hipError_t launch_lbi_reg_pinf(int w, int num_cu, const LbiArgs &a, hipStream_t s) {
    static const auto table = lbi_reg_table<kPInf>(std::make_integer_sequence<int, kLbiRegMaxW + 1>{});
    if (w < 0 || w > kLbiRegMaxW) return hipErrorInvalidValue;
    table[w](num_cu, a, s);
    return hipGetLastError();
}

}  // namespace lbimp
