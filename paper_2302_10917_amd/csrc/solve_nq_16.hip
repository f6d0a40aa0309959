// Explicit instances of the per-macro solve for NQ in {16}
// (register blocks of 64 local unknowns), with the default register
// budget and with the budgets of 6, 5 and 4 resident wavefronts per SIMD
// (8, 8, 12 and 16 column chunks per load group).
#include "macro_solve.h"

namespace mhdg {
template void macro_solve_launch<double, 16>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_launch<float, 16>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_t_launch<16>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
#define MSO_INST(T_, W_, LG_)                                                                 \
  template void macro_solve_launch<T_, 16, W_, LG_>(int, const void*, const MacroInfo*,          \
                                                    const int32_t*, int64_t, int64_t, size_t,    \
                                                    const int32_t*, const double*,               \
                                                    const Templates&, const int32_t*, double,    \
                                                    const double*, const double*, double*,       \
                                                    double*, hipStream_t);
MSO_INST(double, 6, 8) MSO_INST(double, 5, 8) MSO_INST(double, 5, 12) MSO_INST(double, 4, 16)
MSO_INST(float, 6, 8) MSO_INST(float, 5, 8) MSO_INST(float, 5, 12) MSO_INST(float, 4, 16)
#undef MSO_INST
template void macro_solve_launch<bf16_t, 16>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
}  // namespace mhdg
