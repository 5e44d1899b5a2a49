// Entry points whose kernels are not built yet: they refuse every call.
#include "common.hpp"

extern "C" harp_status reduced_factor_ws(int32_t, int32_t, harp_dtype, size_t*) { return HARP_E_ARG; }
extern "C" harp_status reduced_factor(int32_t, int32_t, harp_dtype, void*, int64_t, int64_t, int32_t*, int32_t*,
                                      void*, size_t, hipStream_t) { return HARP_E_ARG; }
extern "C" harp_status reduced_solve_ws(int32_t, int32_t, int32_t, harp_dtype, int32_t, size_t*) { return HARP_E_ARG; }
extern "C" harp_status reduced_solve(int32_t, int32_t, int32_t, harp_dtype, const void*, int64_t, int64_t,
                                     const int32_t*, const void*, int64_t, int64_t, void*, int64_t, int64_t,
                                     const harp_refine*, harp_refine_report*, void*, size_t, hipStream_t) {
    return HARP_E_ARG;
}
extern "C" harp_status embedded_patterns(const void*, int32_t, const double*, const double*, int32_t, const void*,
                                         int64_t, int32_t, const double*, const double*, int32_t, void*,
                                         hipStream_t) { return HARP_E_ARG; }
