// Kernel-class event timers (see include/harp_prof.h).
#pragma once

#include <hip/hip_ext.h>

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
// Kernel-attached timers: *start / *stop receive events (null when profiling
// is off) that the caller hands to hipExtLaunchKernelGGL, which stamps them at
// the dispatch's own start and end, so the time is the kernel's alone.
int begin_ext(int cls, hipEvent_t* start, hipEvent_t* stop);
void end_ext(int token, double flops, double bytes);

}  // namespace prof
}  // namespace harp

// Launch `...` bracketed by the class timers (no-op when profiling is off).
#define HARP_PROF_LAUNCH(cls, stream, flops, bytes, ...)                  \
    do {                                                                  \
        const int harp_prof_tok_ = ::harp::prof::begin((cls), (stream));  \
        __VA_ARGS__;                                                      \
        ::harp::prof::end(harp_prof_tok_, (stream), (flops), (bytes));    \
    } while (0)

// Launch kernel<<<grid, block, shmem, stream>>>(args...) with the class's
// kernel-attached timers; a plain launch when profiling is off (so the
// launch can be captured in a HIP graph).
#define HARP_PROF_EXT_LAUNCH(cls, stream, flops, bytes, kernel, grid, block, shmem, ...)                  \
    do {                                                                                                \
        if (!::harp::prof::enabled()) {                                                                 \
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                        \
        } else {                                                                                        \
            hipEvent_t harp_prof_s_ = nullptr, harp_prof_e_ = nullptr;                                  \
            const int harp_prof_tok_ = ::harp::prof::begin_ext((cls), &harp_prof_s_, &harp_prof_e_);    \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, harp_prof_s_, harp_prof_e_, 0u,   \
                                  __VA_ARGS__);                                                         \
            ::harp::prof::end_ext(harp_prof_tok_, (flops), (bytes));                                    \
        }                                                                                               \
    } while (0)
