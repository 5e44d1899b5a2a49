// Shared device/host helpers of libharp (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/harp.h"

namespace harp {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;
constexpr double kC0 = 299792458.0;          // speed of light, m/s
constexpr double kMu0 = 4.0e-7 * kPi;        // vacuum permeability, H/m
constexpr uint32_t kModelMagic = 0x50524148u;
constexpr uint32_t kModelVersion = 1u;
constexpr int kSampleFields = 8;             // x, y, z, ux, uy, uz, a_re, a_im

// Model blob header; the layout is part of the C ABI (see harp.h).
struct alignas(256) ModelHeader {
    uint32_t magic;
    uint32_t version;
    int32_t n_mbf, n_samp, P, Q, n_alpha, n_t;
    double freq_hz, k, omega_mu, r_min, wire_radius;
    int64_t off_coef, off_coef32, off_self, off_port, off_samples, total_bytes;
};
static_assert(sizeof(ModelHeader) == 256, "model header is 256 bytes");

__host__ __device__ inline int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }

struct ModelLayout {
    int64_t off_coef, off_coef32, off_self, off_port, off_samples, total;
};

__host__ __device__ inline ModelLayout model_layout(int n_mbf, int n_samp, int P, int Q) {
    ModelLayout L;
    const int64_t ncoef = int64_t(n_mbf) * n_mbf * (2 * P + 1) * (Q + 1);
    L.off_coef = 256;
    L.off_coef32 = L.off_coef + align256(ncoef * 16);
    L.off_self = L.off_coef32 + align256(ncoef * 8);
    L.off_port = L.off_self + align256(int64_t(n_mbf) * n_mbf * 16);
    L.off_samples = L.off_port + align256(int64_t(n_mbf) * 16);
    L.total = L.off_samples + align256(int64_t(n_mbf) * n_samp * kSampleFields * 8);
    return L;
}

// Minimal complex arithmetic on (re, im) pairs.
template <typename R> struct cpx {
    R re, im;
};
template <typename R> __host__ __device__ inline cpx<R> cmul(cpx<R> a, cpx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R> __host__ __device__ inline cpx<R> cadd(cpx<R> a, cpx<R> b) {
    return {a.re + b.re, a.im + b.im};
}

}  // namespace harp

#define HARP_LAUNCH_CHECK()                                        \
    do {                                                           \
        if (hipGetLastError() != hipSuccess) return HARP_E_HIP;    \
    } while (0)

#define HARP_HIP_CHECK(call)                                       \
    do {                                                           \
        if ((call) != hipSuccess) return HARP_E_HIP;               \
    } while (0)
