// Explicit instances of the per-macro solve for NQ in {1, 2, 3, 5, 8}
// (register blocks of 64 local unknowns).
#include "macro_solve.h"

namespace mhdg {
template void macro_solve_launch<double, 1>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_launch<float, 1>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_launch<double, 2>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_launch<float, 2>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_launch<double, 3>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_launch<float, 3>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_launch<double, 5>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_launch<float, 5>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_launch<double, 8>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_launch<float, 8>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_t_launch<1>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_t_launch<2>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_t_launch<3>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_t_launch<5>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_t_launch<8>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_launch<bf16_t, 1>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_launch<bf16_t, 2>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_launch<bf16_t, 3>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_launch<bf16_t, 5>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_launch<bf16_t, 8>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
}  // namespace mhdg
