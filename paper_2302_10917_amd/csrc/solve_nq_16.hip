// Explicit instances of the per-macro solve for NQ in {16}
// (register blocks of 64 local unknowns).
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
template void macro_solve_launch<bf16_t, 16>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
}  // namespace mhdg
