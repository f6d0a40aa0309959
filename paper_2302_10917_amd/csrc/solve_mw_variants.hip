// Explicit instances of the multi-wavefront per-macro solve with 8 wavefronts
// per macro (NQ 27 and 58) and with 4 wavefronts for NQ 16: autotuner
// candidates next to the default shapes.
#include "macro_solve.h"

namespace mhdg {
template void macro_solve_mw_launch<double, 27, 8>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_mw_launch<double, 58, 8>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_mw_launch<double, 16, 4>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_mw_launch<float, 27, 8>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_mw_launch<float, 58, 8>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
template void macro_solve_mw_launch<float, 16, 4>(int, const void*, const MacroInfo*, const int32_t*, int64_t, int64_t, size_t,
    const int32_t*, const double*, const Templates&, const int32_t*, double, const double*,
    const double*, double*, double*, hipStream_t);
}  // namespace mhdg
