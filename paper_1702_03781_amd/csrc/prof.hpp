// Kernel-class event timers (see include/harp_prof.h).
#pragma once

#include "common.hpp"
#include "../../include/harp_prof.h"

namespace harp {
namespace prof {

bool enabled();
// Record a start event on `stream` for class `cls`; returns a token (-1 when
// profiling is off).
int begin(int cls, hipStream_t stream);
// Record the matching stop event and the launch's algorithmic work.
void end(int token, hipStream_t stream, double flops, double bytes);

}  // namespace prof
}  // namespace harp

// Launch `...` bracketed by the class timers (no-op when profiling is off).
#define HARP_PROF_LAUNCH(cls, stream, flops, bytes, ...)                  \
    do {                                                                  \
        const int harp_prof_tok_ = ::harp::prof::begin((cls), (stream));  \
        __VA_ARGS__;                                                      \
        ::harp::prof::end(harp_prof_tok_, (stream), (flops), (bytes));    \
    } while (0)
