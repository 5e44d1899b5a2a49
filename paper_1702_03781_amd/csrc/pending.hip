// Entry points whose kernels are not built yet: they refuse every call.
#include "common.hpp"

extern "C" harp_status embedded_patterns(const void*, int32_t, const double*, const double*, int32_t, const void*,
                                         int64_t, int32_t, const double*, const double*, int32_t, void*,
                                         hipStream_t) { return HARP_E_ARG; }
