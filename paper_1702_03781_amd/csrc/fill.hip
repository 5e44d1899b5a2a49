// Reduced-matrix fill from the HARP model (Eq. 4, Section II-A).
//
// For an ordered antenna pair (testing m, source n) with R = (x_m - x_n,
// y_m - y_n), r = |R|, w = e^{j alpha} = R / r and t = r_min / r (the modified
// coordinate 1/r of Section II-B, normalised), every MBF pair (T, S) takes
//
//   Z_TS = e^{-jkr} sum_{p=-P..P} w^p H_p(t),   H_p(t) = sum_{q=0..Q} C_pq t^q
//        = e^{-jkr} w^{-P} sum_{p'=0..2P} w^{p'} H_{p'-P}(t).
//
// The kernel evaluates the last form as a two-level Horner scheme: Horner in t
// for H_p (2Q real FMA per p: complex coefficient times real t), then Horner
// in w over p' (4 real FMA per p), and one complex product with the pair phase
// e^{-jkr} w^{-P}, whose angle -k r - P alpha is formed and reduced modulo
// 2 pi in FP64 (k r reaches ~300 rad at 350 MHz across a 38 m station, far
// beyond what an FP32 argument can carry).  Cost: (2P+1)(2Q+4) real FMA per
// entry, 8 (complex64) or 16 (complex128) bytes written: the fill is bound by
// the vector ALU, not by HBM.
//
// Mapping: a 256-thread workgroup owns 64 testing antennas (one per lane) x
// 16 source antennas (4 waves x G = 4 per thread).  All lanes of a wave walk
// the same (T, S, p, q) sequence, so the coefficient stream is wave-uniform
// and is read through the scalar cache; per-pair geometry lives in VGPRs and
// is reused for all N_m^2 entries of the block.  Lanes hold consecutive m, so
// for each (S, T) a wave writes a 64-row strided column segment; the eight T
// values of one column complete the 512-byte runs in L2 before eviction.
#include <math.h>

#include "common.hpp"
#include "prof.hpp"

namespace harp {
namespace {

constexpr int kTileM = 64;   // testing antennas per workgroup (lanes)
constexpr int kG = 4;        // source antennas per thread
constexpr int kTileN = 4 * kG;

struct FillArgs {
    const char* models;
    int64_t model_stride;
    int n_freq, n_mbf, Q, p_max, n_ant;  // n_freq: matrices; n_ant: antennas of the (padded) order
    const double* x;
    const double* y;
    double ri;
    void* Z;
    int64_t ldz, stride_z;
    float* Z32;
    int64_t ld32, stride32;
    int32_t* info;
    // batch of unequal layouts (nullptr: matrix f uses model f, all n_ant antennas at x[0..))
    const harp_system* sys;
    int n_models;
    int64_t n_pos;
};

__global__ void fill_info_init(int32_t* info, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) info[i] = 0;
}

template <typename R> struct FillTraits;
template <> struct FillTraits<float> {
    using store_t = float2;
    __device__ static const float* coef(const char* m, const ModelHeader* h) {
        return reinterpret_cast<const float*>(m + h->off_coef32);
    }
};
template <> struct FillTraits<double> {
    using store_t = double2;
    __device__ static const double* coef(const char* m, const ModelHeader* h) {
        return reinterpret_cast<const double*>(m + h->off_coef);
    }
};

// kPad: identity block of a padding antenna (unit diagonal, zeros elsewhere)
enum PairKind : int { kSkip = 0, kHarp = 1, kSelf = 2, kZero = 3, kPad = 4 };

// The pointers are separate __restrict__ parameters (not struct members) so
// that the compiler may read the model through the scalar cache.
template <typename R, int Q, bool DUAL>
__global__ void __launch_bounds__(256)
    fill_kernel(FillArgs a, const char* __restrict__ models, const double* __restrict__ px,
                const double* __restrict__ py, void* __restrict__ Zout, float* __restrict__ Z32out) {
    const int f = blockIdx.y;
    // antennas of this system (ns <= a.n_ant; the rest of the order is padding)
    int mi = f, ns = a.n_ant;
    if (a.sys) {
        const harp_system d = a.sys[f];
        if (d.model < 0 || d.model >= a.n_models || d.n_ant < 1 || d.n_ant > a.n_ant || d.pos < 0 ||
            d.pos > a.n_pos - d.n_ant) {
            if (blockIdx.x == 0 && threadIdx.x == 0) atomicExch(a.info + f, -2);
            return;
        }
        mi = d.model;
        ns = d.n_ant;
        px += d.pos;
        py += d.pos;
    }
    const char* model = models + size_t(mi) * a.model_stride;
    const ModelHeader* h = reinterpret_cast<const ModelHeader*>(model);
    const int P = h->P;
    if (h->magic != kModelMagic || h->n_mbf != a.n_mbf || h->Q != Q || P > a.p_max || P < 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicExch(a.info + f, -1);
        return;
    }
    const int nm = a.n_mbf;
    const int np = 2 * P + 1;
    const double k = h->k, r_min = h->r_min;

    const int tiles_m = (a.n_ant + kTileM - 1) / kTileM;
    const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int m = tm * kTileM + lane;

    int kind[kG];
    R t[kG];
    cpx<R> w[kG], ph[kG];
    int n_below = 0;
    const double xm = m < ns ? px[m] : 0.0;
    const double ym = m < ns ? py[m] : 0.0;
#pragma unroll
    for (int g = 0; g < kG; ++g) {
        const int n = tn * kTileN + wave * kG + g;
        kind[g] = kSkip;
        t[g] = R(0);
        w[g] = cpx<R>{R(1), R(0)};
        ph[g] = cpx<R>{R(0), R(0)};
        if (m >= a.n_ant || n >= a.n_ant) continue;
        if (m >= ns || n >= ns) {
            kind[g] = m == n ? kPad : kZero;
            continue;
        }
        if (m == n) {
            kind[g] = kSelf;
            continue;
        }
        const double dx = xm - px[n], dy = ym - py[n];
        const double r = sqrt(dx * dx + dy * dy);
        if (a.ri > 0.0 && r > a.ri) {
            kind[g] = kZero;
            continue;
        }
        kind[g] = kHarp;
        if (r < r_min * (1.0 - 1e-12)) ++n_below;
        const double ir = 1.0 / r;
        t[g] = R(r_min * ir);
        w[g] = cpx<R>{R(dx * ir), R(dy * ir)};
        // phase angle -k r - P alpha, reduced to [-pi, pi] in FP64
        double th = -k * r - double(P) * atan2(dy, dx);
        th -= kTwoPi * rint(th * (1.0 / kTwoPi));
        R s, c;
        if constexpr (sizeof(R) == 4) {
            sincosf(float(th), &s, &c);
        } else {
            sincos(th, &s, &c);
        }
        ph[g] = cpx<R>{c, s};
    }
    // domain count: one atomic per wave
    {
        int cnt = n_below;
        for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off, 64);
        if (lane == 0 && cnt) atomicAdd(a.info + f, cnt);
    }
    bool any_harp_lane = false;
#pragma unroll
    for (int g = 0; g < kG; ++g) any_harp_lane |= (kind[g] == kHarp);
    const bool wave_harp = __ballot(any_harp_lane) != 0;

    const R* coef = FillTraits<R>::coef(model, h);
    const double* zself = reinterpret_cast<const double*>(model + h->off_self);
    using store_t = typename FillTraits<R>::store_t;
    store_t* Zf = reinterpret_cast<store_t*>(Zout) + size_t(f) * a.stride_z;
    float2* Z32f = DUAL ? reinterpret_cast<float2*>(Z32out) + size_t(f) * a.stride32 : nullptr;

    for (int S = 0; S < nm; ++S) {
        for (int T = 0; T < nm; ++T) {
            const int ts = T * nm + S;
            cpx<R> acc[kG];
#pragma unroll
            for (int g = 0; g < kG; ++g) acc[g] = cpx<R>{R(0), R(0)};
            if (wave_harp) {
                const R* cts = coef + size_t(ts) * np * (Q + 1) * 2;
                for (int pp = np - 1; pp >= 0; --pp) {
                    const R* cq = cts + pp * (Q + 1) * 2;
                    R cr[Q + 1], ci[Q + 1];
#pragma unroll
                    for (int q = 0; q <= Q; ++q) {
                        cr[q] = cq[2 * q];
                        ci[q] = cq[2 * q + 1];
                    }
#pragma unroll
                    for (int g = 0; g < kG; ++g) {
                        R hr = cr[Q], hi = ci[Q];
#pragma unroll
                        for (int q = Q - 1; q >= 0; --q) {
                            hr = fma(hr, t[g], cr[q]);
                            hi = fma(hi, t[g], ci[q]);
                        }
                        // acc = acc * w + h
                        const R nr = fma(acc[g].re, w[g].re, fma(-acc[g].im, w[g].im, hr));
                        const R ni = fma(acc[g].re, w[g].im, fma(acc[g].im, w[g].re, hi));
                        acc[g].re = nr;
                        acc[g].im = ni;
                    }
                }
            }
            const double sr = zself[2 * ts], si = zself[2 * ts + 1];
#pragma unroll
            for (int g = 0; g < kG; ++g) {
                if (kind[g] == kSkip) continue;
                const int n = tn * kTileN + wave * kG + g;
                cpx<R> z;
                if (kind[g] == kHarp) {
                    z = cmul(acc[g], ph[g]);
                } else if (kind[g] == kSelf) {
                    z = cpx<R>{R(sr), R(si)};
                } else if (kind[g] == kPad) {
                    z = cpx<R>{R(T == S ? 1 : 0), R(0)};
                } else {
                    z = cpx<R>{R(0), R(0)};
                }
                const size_t row = size_t(m) * nm + T;
                const size_t col = size_t(n) * nm + S;
                store_t v;
                v.x = z.re;
                v.y = z.im;
                Zf[col * a.ldz + row] = v;
                if constexpr (DUAL) {
                    float2 v32;
                    v32.x = float(z.re);
                    v32.y = float(z.im);
                    Z32f[col * a.ld32 + row] = v32;
                }
            }
        }
    }
}

template <typename R, bool DUAL>
harp_status launch_fill_q(const FillArgs& a, dim3 grid, hipStream_t stream) {
    switch (a.Q) {
#define HARP_FILL_CASE(QQ)                                                                 \
    case QQ:                                                                               \
        HARP_PROF_EXT_LAUNCH(HARP_K_FILL, stream, 0.0,                                     \
                             double(a.n_freq) * double(a.n_ant) * a.n_mbf * double(a.n_ant) * \
                                 a.n_mbf * (DUAL ? 24.0 : double(2 * sizeof(R))),          \
                             (fill_kernel<R, QQ, DUAL>), grid, dim3(256), 0, a, a.models,  \
                             a.x, a.y, a.Z, a.Z32);                                        \
        break;
        HARP_FILL_CASE(2)
        HARP_FILL_CASE(3)
        HARP_FILL_CASE(4)
        HARP_FILL_CASE(5)
        HARP_FILL_CASE(6)
        HARP_FILL_CASE(7)
        HARP_FILL_CASE(8)
#undef HARP_FILL_CASE
        default:
            return HARP_E_ARG;
    }
    HARP_LAUNCH_CHECK();
    return HARP_OK;
}

harp_status fill_launch(FillArgs& a, harp_dtype dtype, hipStream_t stream) {
    if (!a.models || !a.x || !a.y || !a.Z || !a.info) return HARP_E_ARG;
    if (a.n_freq <= 0 || a.n_mbf <= 0 || a.n_ant <= 0 || a.Q < 2 || a.Q > 8 || a.p_max < 0) return HARP_E_ARG;
    if (a.n_freq > 65535) return HARP_E_ARG;
    if (dtype != HARP_C64 && dtype != HARP_C128) return HARP_E_ARG;
    if (!isfinite(a.ri)) return HARP_E_ARG;
    const int64_t n = int64_t(a.n_ant) * a.n_mbf;
    if (a.ldz < n || (a.n_freq > 1 && a.stride_z < a.ldz * n)) return HARP_E_ARG;
    if (a.model_stride < 256 || (a.model_stride % 256) != 0) return HARP_E_ARG;
    if (a.Z32) {
        if (dtype != HARP_C128) return HARP_E_ARG;
        if (a.ld32 < n || (a.n_freq > 1 && a.stride32 < a.ld32 * n)) return HARP_E_ARG;
    }
    HARP_PROF_LAUNCH(HARP_K_AUX, stream, 0.0, 0.0,
                     hipLaunchKernelGGL(fill_info_init, dim3((a.n_freq + 255) / 256), dim3(256), 0, stream, a.info,
                                        a.n_freq));
    HARP_LAUNCH_CHECK();
    const int tiles = ((a.n_ant + kTileM - 1) / kTileM) * ((a.n_ant + kTileN - 1) / kTileN);
    const dim3 grid{unsigned(tiles), unsigned(a.n_freq), 1u};
    if (dtype == HARP_C64) return launch_fill_q<float, false>(a, grid, stream);
    if (a.Z32) return launch_fill_q<double, true>(a, grid, stream);
    return launch_fill_q<double, false>(a, grid, stream);
}

FillArgs fill_args(const void* d_models, int64_t model_stride, int32_t n_mat, int32_t n_mbf, int32_t Q,
                   int32_t p_max, const double* d_x, const double* d_y, int32_t n_ant, double ri, void* d_Z,
                   int64_t ldz, int64_t stride_z, void* d_Z32, int64_t ld32, int64_t stride32, int32_t* d_info) {
    FillArgs a{};
    a.models = static_cast<const char*>(d_models);
    a.model_stride = model_stride;
    a.n_freq = n_mat;
    a.n_mbf = n_mbf;
    a.Q = Q;
    a.p_max = p_max;
    a.n_ant = n_ant;
    a.x = d_x;
    a.y = d_y;
    a.ri = ri;
    a.Z = d_Z;
    a.ldz = ldz;
    a.stride_z = stride_z;
    a.Z32 = static_cast<float*>(d_Z32);
    a.ld32 = ld32;
    a.stride32 = stride32;
    a.info = d_info;
    return a;
}

}  // namespace
}  // namespace harp

using namespace harp;

extern "C" harp_status harp_fill(const void* d_models, int64_t model_stride, int32_t n_freq, int32_t n_mbf,
                                 int32_t Q, int32_t p_max, const double* d_x, const double* d_y,
                                 int32_t n_ant, double ri, harp_dtype dtype, void* d_Z, int64_t ldz,
                                 int64_t stride_z, void* d_Z32, int64_t ld32, int64_t stride32,
                                 int32_t* d_info, hipStream_t stream) {
    FillArgs a = fill_args(d_models, model_stride, n_freq, n_mbf, Q, p_max, d_x, d_y, n_ant, ri, d_Z, ldz, stride_z,
                           d_Z32, ld32, stride32, d_info);
    return fill_launch(a, dtype, stream);
}

extern "C" harp_status harp_fill_systems(const void* d_models, int64_t model_stride, int32_t n_models,
                                         int32_t n_mbf, int32_t Q, int32_t p_max, const double* d_x,
                                         const double* d_y, int64_t n_pos, const harp_system* d_sys,
                                         int32_t n_sys, int32_t n_ant_pad, double ri, harp_dtype dtype, void* d_Z,
                                         int64_t ldz, int64_t stride_z, void* d_Z32, int64_t ld32,
                                         int64_t stride32, int32_t* d_info, hipStream_t stream) {
    if (!d_sys || n_models <= 0 || n_pos <= 0) return HARP_E_ARG;
    FillArgs a = fill_args(d_models, model_stride, n_sys, n_mbf, Q, p_max, d_x, d_y, n_ant_pad, ri, d_Z, ldz,
                           stride_z, d_Z32, ld32, stride32, d_info);
    a.sys = d_sys;
    a.n_models = n_models;
    a.n_pos = n_pos;
    return fill_launch(a, dtype, stream);
}
