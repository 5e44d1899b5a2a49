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
// Mapping.  The reduced matrix is column-major with the MBF index fastest
// (row m N_m + T), so a run of consecutive rows is (antenna, testing MBF)
// with T fastest.  A lane therefore owns one testing antenna m and one
// testing MBF T (lane = N_m i + T, i < 64 / N_m, at most 16 antennas), and
// G = 4 source antennas; the four waves of a 256-thread workgroup take
// 4 x G = 16 consecutive source antennas.  For each source MBF S a store
// instruction then writes 64 consecutive rows of one column (1 KB of
// complex128): every store is a full, contiguous run.  Because the
// coefficients C^{TS} now differ across the lanes of a wave (by T), the
// coefficients of the current S for every T are staged in LDS as [p][T][q]
// (a lane reads the Q + 1 coefficients of its (p, T) from one base address
// with constant offsets; the N_m distinct runs of a wave fall in distinct
// banks) and shared by the G source antennas of a lane.  The pair
// geometry (t, w, phase, block kind) is computed once per pair into LDS.
#include <math.h>

#include "common.hpp"
#include "prof.hpp"

namespace harp {
namespace {

constexpr int kWaves = 4;
constexpr int kG = 4;                  // source antennas per lane
constexpr int kTileN = kWaves * kG;    // source antennas per workgroup
constexpr int kMaxPPW = 16;            // testing antennas per workgroup (cap)
constexpr int kMaxPairs = kMaxPPW * kTileN;
constexpr int kMaxMbf = 64;            // one testing antenna needs N_m lanes
constexpr int kMaxCoefLds = 65536;     // bytes of the staged coefficients of one S

// testing antennas per workgroup: N_m lanes each, at most 64 lanes and kMaxPPW
__host__ __device__ inline int fill_ppw(int n_mbf) { return 64 / n_mbf < kMaxPPW ? 64 / n_mbf : kMaxPPW; }

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

template <typename R> struct alignas(16) PairGeo {
    R t[kMaxPairs];
    R wr[kMaxPairs], wi[kMaxPairs];
    R pr[kMaxPairs], pi[kMaxPairs];
    int kind[kMaxPairs];
};

// The pointers are separate __restrict__ parameters (not struct members) so
// that the compiler may keep the model reads in the scalar cache.
template <typename R, int Q, bool DUAL>
__global__ void __launch_bounds__(256)
    fill_kernel(FillArgs a, const char* __restrict__ models, const double* __restrict__ px,
                const double* __restrict__ py, void* __restrict__ Zout, float* __restrict__ Z32out) {
    static_assert(Q >= 1, "Horner start");
    extern __shared__ __attribute__((aligned(16))) char fill_smem[];   // [np][N_m][Q+1] complex R
    __shared__ PairGeo<R> geo;
    const int f = blockIdx.y;
    // antennas of this system (ns <= a.n_ant; the rest of the order is padding)
    int mi_model = f, ns = a.n_ant;
    if (a.sys) {
        const harp_system d = a.sys[f];
        if (d.model < 0 || d.model >= a.n_models || d.n_ant < 1 || d.n_ant > a.n_ant || d.pos < 0 ||
            d.pos > a.n_pos - d.n_ant) {
            if (blockIdx.x == 0 && threadIdx.x == 0) atomicExch(a.info + f, -2);
            return;
        }
        mi_model = d.model;
        ns = d.n_ant;
        px += d.pos;
        py += d.pos;
    }
    const char* model = models + size_t(mi_model) * a.model_stride;
    const ModelHeader* h = reinterpret_cast<const ModelHeader*>(model);
    const int P = h->P;
    if (h->magic != kModelMagic || h->n_mbf != a.n_mbf || h->Q != Q || P > a.p_max || P < 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicExch(a.info + f, -1);
        return;
    }
    const int nm = a.n_mbf;
    const int np = 2 * P + 1;
    const double k = h->k, r_min = h->r_min;
    const int ppw = fill_ppw(nm);
    const int tiles_m = (a.n_ant + ppw - 1) / ppw;
    const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
    const int m0 = tm * ppw, n0 = tn * kTileN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    // 1. geometry of the workgroup's pairs, one thread per pair
    int n_below = 0;
    for (int e = tid; e < ppw * kTileN; e += 256) {
        const int ii = e % ppw, jj = e / ppw;
        const int m = m0 + ii, n = n0 + jj;
        int kind = kSkip;
        R t = R(0), wr = R(1), wi = R(0), pr = R(0), pim = R(0);
        if (m < a.n_ant && n < a.n_ant) {
            if (m >= ns || n >= ns) {
                kind = m == n ? kPad : kZero;
            } else if (m == n) {
                kind = kSelf;
            } else {
                const double dx = px[m] - px[n], dy = py[m] - py[n];
                const double r = sqrt(dx * dx + dy * dy);
                if (a.ri > 0.0 && r > a.ri) {
                    kind = kZero;
                } else {
                    kind = kHarp;
                    if (r < r_min * (1.0 - 1e-12)) ++n_below;
                    const double ir = 1.0 / r;
                    t = R(r_min * ir);
                    wr = R(dx * ir);
                    wi = R(dy * ir);
                    // phase angle -k r - P alpha, reduced to [-pi, pi] in FP64
                    double th = -k * r - double(P) * atan2(dy, dx);
                    th -= kTwoPi * rint(th * (1.0 / kTwoPi));
                    if constexpr (sizeof(R) == 4) {
                        sincosf(float(th), &pim, &pr);
                    } else {
                        sincos(th, &pim, &pr);
                    }
                }
            }
        }
        geo.t[e] = t;
        geo.wr[e] = wr;
        geo.wi[e] = wi;
        geo.pr[e] = pr;
        geo.pi[e] = pim;
        geo.kind[e] = kind;
    }
    // domain count: one atomic per wave
    {
        int cnt = n_below;
        for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off, 64);
        if (lane == 0 && cnt) atomicAdd(a.info + f, cnt);
    }
    __syncthreads();

    // 2. this lane: testing antenna m = m0 + mi, testing MBF T, G source antennas
    const int mi = lane / nm, T = lane % nm;
    const bool lane_on = mi < ppw;
    const int m = m0 + mi;
    int kind[kG];
    R t[kG];
    cpx<R> w[kG], ph[kG];
    bool any_harp = false;
#pragma unroll
    for (int g = 0; g < kG; ++g) {
        const int e = (wave * kG + g) * ppw + (lane_on ? mi : 0);
        kind[g] = lane_on ? geo.kind[e] : int(kSkip);
        t[g] = geo.t[e];
        w[g] = cpx<R>{geo.wr[e], geo.wi[e]};
        ph[g] = cpx<R>{geo.pr[e], geo.pi[e]};
        any_harp |= (kind[g] == kHarp);
    }
    const bool wave_harp = __ballot(any_harp) != 0;

    const R* coef = FillTraits<R>::coef(model, h);         // [T][S][p][q] complex
    const double* zself = reinterpret_cast<const double*>(model + h->off_self);
    R* cf = reinterpret_cast<R*>(fill_smem);                // [p][T][q] complex
    const int npq = np * (Q + 1);
    using store_t = typename FillTraits<R>::store_t;
    store_t* Zf = reinterpret_cast<store_t*>(Zout) + size_t(f) * a.stride_z;
    float2* Z32f = DUAL ? reinterpret_cast<float2*>(Z32out) + size_t(f) * a.stride32 : nullptr;

    for (int S = 0; S < nm; ++S) {
        // 3. stage C^{TS}_{pq} of every T for this S
        __syncthreads();
        for (int e = tid; e < nm * npq; e += 256) {
            const int Tc = e / npq, pq = e % npq;
            const R* src = coef + 2 * (size_t(Tc * nm + S) * npq + pq);
            const int pp = pq / (Q + 1), q = pq % (Q + 1);
            R* dst = cf + 2 * ((pp * nm + Tc) * (Q + 1) + q);
            dst[0] = src[0];
            dst[1] = src[1];
        }
        __syncthreads();
        // 4. two-level Horner for the lane's G source antennas
        cpx<R> acc[kG];
#pragma unroll
        for (int g = 0; g < kG; ++g) acc[g] = cpx<R>{R(0), R(0)};
        if (wave_harp) {
#pragma unroll 2
            for (int pp = np - 1; pp >= 0; --pp) {
                R cr[Q + 1], ci[Q + 1];
#pragma unroll
                for (int q = 0; q <= Q; ++q) {
                    const R* c = cf + 2 * ((pp * nm + T) * (Q + 1) + q);
                    cr[q] = c[0];
                    ci[q] = c[1];
                }
#pragma unroll
                for (int g = 0; g < kG; ++g) {
                    // the first step takes C_pQ as an operand (no copy into the accumulators)
                    R hr = fma(cr[Q], t[g], cr[Q - 1]), hi = fma(ci[Q], t[g], ci[Q - 1]);
#pragma unroll
                    for (int q = Q - 2; q >= 0; --q) {
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
        // 5. entries (m, T; n, S): consecutive lanes write consecutive rows
        const double sr = zself[2 * (T * nm + S)], si = zself[2 * (T * nm + S) + 1];
        const size_t row = size_t(m) * nm + T;
#pragma unroll
        for (int g = 0; g < kG; ++g) {
            if (kind[g] == kSkip) continue;
            const int n = n0 + wave * kG + g;
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

// bytes of the staged coefficients of one source MBF
inline size_t fill_lds_bytes(const FillArgs& a, size_t real_bytes) {
    return size_t(2 * a.p_max + 1) * (a.Q + 1) * a.n_mbf * 2 * real_bytes;
}

template <typename R, bool DUAL>
harp_status launch_fill_q(const FillArgs& a, dim3 grid, hipStream_t stream) {
    const size_t lds = fill_lds_bytes(a, sizeof(R));
    switch (a.Q) {
#define HARP_FILL_CASE(QQ)                                                                 \
    case QQ:                                                                               \
        HARP_PROF_EXT_LAUNCH(HARP_K_FILL, stream, 0.0,                                     \
                             double(a.n_freq) * double(a.n_ant) * a.n_mbf * double(a.n_ant) * \
                                 a.n_mbf * (double(2 * sizeof(R)) + (DUAL ? 8.0 : 0.0)),   \
                             (fill_kernel<R, QQ, DUAL>), grid, dim3(256), lds, a, a.models, \
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
    if (a.n_freq <= 0 || a.n_mbf <= 0 || a.n_mbf > kMaxMbf || a.n_ant <= 0 || a.Q < 2 || a.Q > 8 || a.p_max < 0)
        return HARP_E_ARG;
    if (a.n_freq > 65535) return HARP_E_ARG;
    if (dtype != HARP_C64 && dtype != HARP_C128) return HARP_E_ARG;
    if (!isfinite(a.ri)) return HARP_E_ARG;
    const int64_t n = int64_t(a.n_ant) * a.n_mbf;
    if (a.ldz < n || (a.n_freq > 1 && a.stride_z < a.ldz * n)) return HARP_E_ARG;
    if (a.model_stride < 256 || (a.model_stride % 256) != 0) return HARP_E_ARG;
    if (a.Z32) {
        if (a.ld32 < n || (a.n_freq > 1 && a.stride32 < a.ld32 * n)) return HARP_E_ARG;
    }
    if (fill_lds_bytes(a, dtype == HARP_C64 ? 4 : 8) > size_t(kMaxCoefLds)) return HARP_E_ARG;
    HARP_PROF_LAUNCH(HARP_K_AUX, stream, 0.0, 0.0,
                     hipLaunchKernelGGL(fill_info_init, dim3((a.n_freq + 255) / 256), dim3(256), 0, stream, a.info,
                                        a.n_freq));
    HARP_LAUNCH_CHECK();
    const int ppw = fill_ppw(a.n_mbf);
    const int tiles = ((a.n_ant + ppw - 1) / ppw) * ((a.n_ant + kTileN - 1) / kTileN);
    const dim3 grid{unsigned(tiles), unsigned(a.n_freq), 1u};
    if (dtype == HARP_C64)
        return a.Z32 ? launch_fill_q<float, true>(a, grid, stream) : launch_fill_q<float, false>(a, grid, stream);
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
