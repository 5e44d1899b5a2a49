// HARP model construction on the GPU (Section II-A/B, Eqs. 1-3), FP64.
//
// The model build samples the exact interaction of every ordered MBF pair on a
// polar grid, subtracts the far field of Eq. (1), removes the e^{-jkr} phase
// (Eq. 2) and fits Eq. (3) in the modified variable t = r_min / r (the 1/r
// change of variables of Section II-B): a DFT over the angle, then least
// squares over t.  Off the timed path: it runs once per element type and
// frequency and the model is reused for every layout (Section III-C).
//
// Kernels:
//   farfield_kernel    radiation vectors F^-_T, F^+_S and G_ff(alpha_i)
//   reaction_kernel    exact reactions on the grid (and the self block), one
//                      workgroup per (grid point, T, S), block reduction
//   projector_kernel   Householder QR of the Vandermonde matrix in t, giving
//                      the least-squares projector R^-1 Q^T
//   table_kernel       DFT over alpha, projector, far-field fold-in
//   finish_kernel      header, port weights, copy of the samples
#include <math.h>

#include "common.hpp"

namespace harp {
namespace {

constexpr int kMaxMbf = 64;
constexpr int kMaxLs = 64;      // n_t + 1
constexpr int kMaxQ1 = 16;      // Q + 1

struct FitArgs {
    const double* samples;
    int n_mbf, n_samp, P, Q, n_alpha, n_t;
    double freq, k, omega_mu, r_min, wire_radius;
    char* model;
    // workspace sections
    double* B;      // [n_alpha][n_t][T][S][2]   remainder at t_1..t_nt
    double* Gff;    // [n_alpha][T][S][2]
    double* pinv;   // [Q+1][n_t+1]
};

// u1 . G(d) . u2 with the free-space dyadic Green's function; reg > 0 takes the
// thin-wire reduced kernel (|d| -> sqrt(|d|^2 + reg^2)).
__device__ inline cpx<double> dyad(double k, double dx, double dy, double dz, const double* u1,
                                   const double* u2, double reg) {
    const double s2 = dx * dx + dy * dy + dz * dz + reg * reg;
    const double s = sqrt(s2);
    const double x = k * s;
    const double ix = 1.0 / x;
    double sn, cs;
    sincos(x, &sn, &cs);
    const double gs = 1.0 / (4.0 * kPi * s);
    // g = (cos x - j sin x) / (4 pi s)
    const cpx<double> g{cs * gs, -sn * gs};
    const cpx<double> A{1.0 - ix * ix, -ix};
    const cpx<double> Bc{-1.0 + 3.0 * ix * ix, 3.0 * ix};
    const double uu = u1[0] * u2[0] + u1[1] * u2[1] + u1[2] * u2[2];
    const double ud = (u1[0] * dx + u1[1] * dy + u1[2] * dz) * (u2[0] * dx + u2[1] * dy + u2[2] * dz) / s2;
    const cpx<double> bracket{A.re * uu + Bc.re * ud, A.im * uu + Bc.im * ud};
    return cmul(g, bracket);
}

// One workgroup per (point, T, S).  Points 0..n_alpha*n_t-1 are the polar grid
// (alpha index major, radial index minor); point n_alpha*n_t is the self block.
__global__ void __launch_bounds__(256) reaction_kernel(FitArgs a) {
    const int ts = blockIdx.y;
    const int T = ts / a.n_mbf, S = ts % a.n_mbf;
    const int pt = blockIdx.x;
    const int n_grid = a.n_alpha * a.n_t;
    const bool self = pt == n_grid;
    double Rx = 0.0, Ry = 0.0, r = 0.0, reg = a.wire_radius;
    if (!self) {
        const int i = pt / a.n_t, l = pt % a.n_t + 1;
        r = a.r_min * double(a.n_t) / double(l);
        double sa, ca;
        sincospi(2.0 * double(i) / double(a.n_alpha), &sa, &ca);
        Rx = r * ca;
        Ry = r * sa;
        reg = 0.0;
    }
    const double* sT = a.samples + size_t(T) * a.n_samp * kSampleFields;
    const double* sS = a.samples + size_t(S) * a.n_samp * kSampleFields;
    cpx<double> acc{0.0, 0.0};
    const int npair = a.n_samp * a.n_samp;
    for (int e = threadIdx.x; e < npair; e += blockDim.x) {
        const double* tp = sT + (e / a.n_samp) * kSampleFields;
        const double* sp = sS + (e % a.n_samp) * kSampleFields;
        const cpx<double> G = dyad(a.k, Rx + tp[0] - sp[0], Ry + tp[1] - sp[1], tp[2] - sp[2], tp + 3,
                                   sp + 3, reg);
        const cpx<double> aa = cmul(cpx<double>{tp[6], tp[7]}, cpx<double>{sp[6], sp[7]});
        acc = cadd(acc, cmul(aa, G));
    }
    // block reduction: wave shuffles, then across the 4 waves through LDS
    for (int off = 32; off > 0; off >>= 1) {
        acc.re += __shfl_down(acc.re, off, 64);
        acc.im += __shfl_down(acc.im, off, 64);
    }
    __shared__ double red[2][8];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0) {
        red[0][wave] = acc.re;
        red[1][wave] = acc.im;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    cpx<double> z{0.0, 0.0};
    for (int w = 0; w < int(blockDim.x / 64); ++w) {
        z.re += red[0][w];
        z.im += red[1][w];
    }
    // -j omega mu0 (Galerkin reaction, Eq. 1 normalisation)
    z = cpx<double>{a.omega_mu * z.im, -a.omega_mu * z.re};
    if (self) {
        const ModelLayout L = model_layout(a.n_mbf, a.n_samp, a.P, a.Q);
        double* out = reinterpret_cast<double*>(a.model + L.off_self) + 2 * ts;
        out[0] = z.re;
        out[1] = z.im;
        return;
    }
    // Eq. (2): B = (Z_exact - G_ff e^{-jkr} / r) e^{+jkr} = Z_exact e^{jkr} - G_ff / r
    const int i = pt / a.n_t;
    const double* g = a.Gff + 2 * (size_t(i) * a.n_mbf * a.n_mbf + ts);
    double sn, cs;
    sincos(a.k * r, &sn, &cs);
    const cpx<double> e{cs, sn};
    const cpx<double> zb = cmul(z, e);
    double* out = a.B + 2 * (size_t(pt) * a.n_mbf * a.n_mbf + ts);
    out[0] = zb.re - g[0] / r;
    out[1] = zb.im - g[1] / r;
}

// One workgroup per alpha_i: transverse radiation vectors toward alpha-hat and
// G_ff = -(j omega mu0 / 4 pi) F^-_T . F^+_S (Eq. 1; F^- is the testing
// pattern, taken toward -alpha-hat in phase).
__global__ void __launch_bounds__(256) farfield_kernel(FitArgs a) {
    __shared__ double Fm[kMaxMbf][3][2];
    __shared__ double Fp[kMaxMbf][3][2];
    const int i = blockIdx.x;
    double sa, ca;
    sincospi(2.0 * double(i) / double(a.n_alpha), &sa, &ca);
    for (int T = threadIdx.x; T < a.n_mbf; T += blockDim.x) {
        double m[3][2] = {{0, 0}, {0, 0}, {0, 0}}, p[3][2] = {{0, 0}, {0, 0}, {0, 0}};
        for (int s = 0; s < a.n_samp; ++s) {
            const double* sp = a.samples + (size_t(T) * a.n_samp + s) * kSampleFields;
            const double ua = ca * sp[3] + sa * sp[4];
            const double perp[3] = {sp[3] - ua * ca, sp[4] - ua * sa, sp[5]};
            double sn, cs;
            sincos(a.k * (ca * sp[0] + sa * sp[1]), &sn, &cs);
            // a e^{+j phi} and a e^{-j phi}
            const cpx<double> am{sp[6], sp[7]};
            const cpx<double> ep = cmul(am, cpx<double>{cs, sn});
            const cpx<double> em = cmul(am, cpx<double>{cs, -sn});
            for (int c = 0; c < 3; ++c) {
                p[c][0] += ep.re * perp[c];
                p[c][1] += ep.im * perp[c];
                m[c][0] += em.re * perp[c];
                m[c][1] += em.im * perp[c];
            }
        }
        for (int c = 0; c < 3; ++c) {
            Fm[T][c][0] = m[c][0];
            Fm[T][c][1] = m[c][1];
            Fp[T][c][0] = p[c][0];
            Fp[T][c][1] = p[c][1];
        }
    }
    __syncthreads();
    const double pref = a.omega_mu / (4.0 * kPi);
    for (int ts = threadIdx.x; ts < a.n_mbf * a.n_mbf; ts += blockDim.x) {
        const int T = ts / a.n_mbf, S = ts % a.n_mbf;
        cpx<double> d{0.0, 0.0};
        for (int c = 0; c < 3; ++c)
            d = cadd(d, cmul(cpx<double>{Fm[T][c][0], Fm[T][c][1]}, cpx<double>{Fp[S][c][0], Fp[S][c][1]}));
        // -j pref d
        double* out = a.Gff + 2 * (size_t(i) * a.n_mbf * a.n_mbf + ts);
        out[0] = pref * d.im;
        out[1] = -pref * d.re;
    }
}

// Least-squares projector for sum_q c_q t^q over t_l = l / n_t, l = 0..n_t:
// Householder QR V = Q R, projector = R^-1 Q^T restricted to the first Q+1
// rows.  One thread; the matrices live in LDS.
__global__ void projector_kernel(FitArgs a) {
    __shared__ double V[kMaxLs][kMaxQ1];
    __shared__ double beta[kMaxQ1];
    __shared__ double y[kMaxLs];
    if (threadIdx.x != 0) return;
    const int L = a.n_t + 1, N = a.Q + 1;
    for (int l = 0; l < L; ++l) {
        const double t = double(l) / double(a.n_t);
        double v = 1.0;
        for (int q = 0; q < N; ++q) {
            V[l][q] = v;
            v *= t;
        }
    }
    // Householder: column j reflector v (v_j = 1 implicit in storage below
    // the diagonal), H = I - beta v v^T; R on and above the diagonal.
    for (int j = 0; j < N; ++j) {
        double nrm = 0.0;
        for (int l = j; l < L; ++l) nrm += V[l][j] * V[l][j];
        nrm = sqrt(nrm);
        const double x0 = V[j][j];
        const double alpha = x0 >= 0.0 ? -nrm : nrm;
        const double v0 = x0 - alpha;
        // v = (1, V[j+1:, j] / v0), beta = -v0 / alpha
        double b = (alpha != 0.0) ? -v0 / alpha : 0.0;
        for (int l = j + 1; l < L; ++l) V[l][j] = (v0 != 0.0) ? V[l][j] / v0 : 0.0;
        V[j][j] = alpha;
        beta[j] = b;
        for (int c = j + 1; c < N; ++c) {
            double s = V[j][c];
            for (int l = j + 1; l < L; ++l) s += V[l][j] * V[l][c];
            s *= b;
            V[j][c] -= s;
            for (int l = j + 1; l < L; ++l) V[l][c] -= s * V[l][j];
        }
    }
    // projector column for each unit vector e_m: y = Q^T e_m, solve R c = y[0:N]
    for (int m = 0; m < L; ++m) {
        for (int l = 0; l < L; ++l) y[l] = (l == m) ? 1.0 : 0.0;
        for (int j = 0; j < N; ++j) {
            double s = y[j];
            for (int l = j + 1; l < L; ++l) s += V[l][j] * y[l];
            s *= beta[j];
            y[j] -= s;
            for (int l = j + 1; l < L; ++l) y[l] -= s * V[l][j];
        }
        for (int q = N - 1; q >= 0; --q) {
            double s = y[q];
            for (int c = q + 1; c < N; ++c) s -= V[q][c] * y[c];
            y[q] = s / V[q][q];
        }
        for (int q = 0; q < N; ++q) a.pinv[q * L + m] = y[q];
    }
}

// One thread per (T, S, p): DFT over alpha of the remainder (l = 1..n_t; the
// t = 0 sample is zero), least squares over t, far-field fold-in at q = 1.
__global__ void __launch_bounds__(256) table_kernel(FitArgs a) {
    const int np = 2 * a.P + 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int nts = a.n_mbf * a.n_mbf;
    if (idx >= nts * np) return;
    const int ts = idx / np, pp = idx % np, p = pp - a.P;
    const int L = a.n_t + 1, N = a.Q + 1;
    const double inv_na = 1.0 / double(a.n_alpha);
    cpx<double> c[kMaxQ1];
    for (int q = 0; q < N; ++q) c[q] = cpx<double>{0.0, 0.0};
    cpx<double> f{0.0, 0.0};
    for (int l = 1; l < L; ++l) {
        cpx<double> b{0.0, 0.0};
        for (int i = 0; i < a.n_alpha; ++i) {
            // e^{-j p alpha_i}, alpha_i = 2 pi i / n_alpha, argument reduced exactly
            long long pi_mod = ((long long)p * i) % a.n_alpha;
            if (pi_mod < 0) pi_mod += a.n_alpha;
            double sn, cs;
            sincospi(2.0 * double(pi_mod) * inv_na, &sn, &cs);
            const double* Bv = a.B + 2 * ((size_t(i) * a.n_t + (l - 1)) * nts + ts);
            b = cadd(b, cmul(cpx<double>{Bv[0], Bv[1]}, cpx<double>{cs, -sn}));
        }
        b.re *= inv_na;
        b.im *= inv_na;
        for (int q = 0; q < N; ++q) {
            const double w = a.pinv[q * L + l];
            c[q].re += w * b.re;
            c[q].im += w * b.im;
        }
    }
    for (int i = 0; i < a.n_alpha; ++i) {
        long long pi_mod = ((long long)p * i) % a.n_alpha;
        if (pi_mod < 0) pi_mod += a.n_alpha;
        double sn, cs;
        sincospi(2.0 * double(pi_mod) * inv_na, &sn, &cs);
        const double* g = a.Gff + 2 * (size_t(i) * nts + ts);
        f = cadd(f, cmul(cpx<double>{g[0], g[1]}, cpx<double>{cs, -sn}));
    }
    f.re *= inv_na;
    f.im *= inv_na;
    if (N > 1) {
        c[1].re += f.re / a.r_min;
        c[1].im += f.im / a.r_min;
    }
    const ModelLayout Lm = model_layout(a.n_mbf, a.n_samp, a.P, a.Q);
    double* C64 = reinterpret_cast<double*>(a.model + Lm.off_coef);
    float* C32 = reinterpret_cast<float*>(a.model + Lm.off_coef32);
    const size_t base = (size_t(ts) * np + pp) * N;
    for (int q = 0; q < N; ++q) {
        C64[2 * (base + q)] = c[q].re;
        C64[2 * (base + q) + 1] = c[q].im;
        C32[2 * (base + q)] = float(c[q].re);
        C32[2 * (base + q) + 1] = float(c[q].im);
    }
}

__global__ void finish_kernel(FitArgs a) {
    const ModelLayout L = model_layout(a.n_mbf, a.n_samp, a.P, a.Q);
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nsv = a.n_mbf * a.n_samp * kSampleFields;
    double* smp = reinterpret_cast<double*>(a.model + L.off_samples);
    for (int e = tid; e < nsv; e += gridDim.x * blockDim.x) smp[e] = a.samples[e];
    double* w = reinterpret_cast<double*>(a.model + L.off_port);
    for (int T = tid; T < a.n_mbf; T += gridDim.x * blockDim.x) {
        const double* s0 = a.samples + size_t(T) * a.n_samp * kSampleFields;
        w[2 * T] = s0[6];
        w[2 * T + 1] = s0[7];
    }
    if (tid == 0) {
        ModelHeader* h = reinterpret_cast<ModelHeader*>(a.model);
        h->magic = kModelMagic;
        h->version = kModelVersion;
        h->n_mbf = a.n_mbf;
        h->n_samp = a.n_samp;
        h->P = a.P;
        h->Q = a.Q;
        h->n_alpha = a.n_alpha;
        h->n_t = a.n_t;
        h->freq_hz = a.freq;
        h->k = a.k;
        h->omega_mu = a.omega_mu;
        h->r_min = a.r_min;
        h->wire_radius = a.wire_radius;
        h->off_coef = L.off_coef;
        h->off_coef32 = L.off_coef32;
        h->off_self = L.off_self;
        h->off_port = L.off_port;
        h->off_samples = L.off_samples;
        h->total_bytes = L.total;
    }
}

size_t fit_ws_bytes(int n_mbf, int P, int Q, int n_alpha, int n_t) {
    (void)P;
    const int64_t nts = int64_t(n_mbf) * n_mbf;
    return size_t(align256(int64_t(n_alpha) * n_t * nts * 16) + align256(int64_t(n_alpha) * nts * 16) +
                  align256(int64_t(Q + 1) * (n_t + 1) * 8));
}

}  // namespace
}  // namespace harp

using namespace harp;

extern "C" size_t harp_model_bytes(int32_t n_mbf, int32_t n_samp, int32_t P, int32_t Q) {
    if (n_mbf <= 0 || n_samp <= 0 || P < 0 || Q < 0) return 0;
    return size_t(model_layout(n_mbf, n_samp, P, Q).total);
}

extern "C" harp_status harp_fit_ws(int32_t n_mbf, int32_t n_samp, int32_t P, int32_t Q, int32_t n_alpha,
                                   int32_t n_t, size_t* bytes) {
    if (!bytes || n_mbf <= 0 || n_samp <= 0 || P < 0 || Q < 0 || n_alpha <= 0 || n_t <= 0)
        return HARP_E_ARG;
    *bytes = fit_ws_bytes(n_mbf, P, Q, n_alpha, n_t);
    return HARP_OK;
}

extern "C" harp_status harp_fit(const harp_element* elem, double freq_hz, int32_t P, int32_t Q, double r_min,
                                int32_t n_alpha, int32_t n_t, void* d_model, size_t model_bytes, void* d_ws,
                                size_t ws_bytes, hipStream_t stream) {
    if (!elem || !elem->d_samples || !d_model) return HARP_E_ARG;
    const int n_mbf = elem->n_mbf, n_samp = elem->n_samp;
    if (n_mbf <= 0 || n_mbf > kMaxMbf || n_samp <= 0 || P < 0 || Q < 0 || Q + 1 > kMaxQ1) return HARP_E_ARG;
    if (n_alpha < 2 * P + 1 || (n_alpha % 2) != 0 || n_t < Q || n_t + 1 > kMaxLs) return HARP_E_ARG;
    if (!(freq_hz > 0.0) || !(r_min > 0.0) || !isfinite(freq_hz) || !isfinite(r_min)) return HARP_E_ARG;
    if (!(elem->wire_radius > 0.0) || !isfinite(elem->wire_radius)) return HARP_E_ARG;
    if (model_bytes < harp_model_bytes(n_mbf, n_samp, P, Q)) return HARP_E_ARG;
    const size_t need = fit_ws_bytes(n_mbf, P, Q, n_alpha, n_t);
    if (!d_ws || ws_bytes < need) return HARP_E_WORKSPACE;

    FitArgs a;
    a.samples = elem->d_samples;
    a.n_mbf = n_mbf;
    a.n_samp = n_samp;
    a.P = P;
    a.Q = Q;
    a.n_alpha = n_alpha;
    a.n_t = n_t;
    a.freq = freq_hz;
    a.omega_mu = 2.0 * kPi * freq_hz * kMu0;
    a.k = 2.0 * kPi * freq_hz / kC0;
    a.r_min = r_min;
    a.wire_radius = elem->wire_radius;
    a.model = static_cast<char*>(d_model);
    const int64_t nts = int64_t(n_mbf) * n_mbf;
    char* ws = static_cast<char*>(d_ws);
    a.B = reinterpret_cast<double*>(ws);
    ws += align256(int64_t(n_alpha) * n_t * nts * 16);
    a.Gff = reinterpret_cast<double*>(ws);
    ws += align256(int64_t(n_alpha) * nts * 16);
    a.pinv = reinterpret_cast<double*>(ws);

    hipLaunchKernelGGL(farfield_kernel, dim3(n_alpha), dim3(256), 0, stream, a);
    HARP_LAUNCH_CHECK();
    hipLaunchKernelGGL(projector_kernel, dim3(1), dim3(64), 0, stream, a);
    HARP_LAUNCH_CHECK();
    hipLaunchKernelGGL(reaction_kernel, dim3(n_alpha * n_t + 1, unsigned(nts)), dim3(256), 0, stream, a);
    HARP_LAUNCH_CHECK();
    const int nthreads = int(nts) * (2 * P + 1);
    hipLaunchKernelGGL(table_kernel, dim3((nthreads + 255) / 256), dim3(256), 0, stream, a);
    HARP_LAUNCH_CHECK();
    hipLaunchKernelGGL(finish_kernel, dim3(64), dim3(256), 0, stream, a);
    HARP_LAUNCH_CHECK();
    return HARP_OK;
}
