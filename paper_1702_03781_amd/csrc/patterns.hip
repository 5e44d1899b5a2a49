// Embedded element patterns (Eqs. 5-6, Section II-C).
//
// With one MBF set shared by all identical elements, the pattern radiated by
// the coefficient column X[:, p] (the currents for an excitation of port p) is
//   E_c(u) = -(j omega mu0 / 4 pi) sum_T F_T,c(u) sum_i X[i N_m + T, p] e^{jk(u_x x_i + u_y y_i)}
// for the components c = theta, phi.  Written as one dense product
//   E[(2d + c), p] = sum_(i,T) A[(2d + c), (i,T)] X[(i,T), p],
//   A[(2d + c), (i,T)] = -(j omega mu0 / 4 pi) F_T,c(u_d) e^{jk(u_x x_i + u_y y_i)},
// it runs on the FP64 matrix cores (cgemm); the column-major product with
// leading dimension 2 n_dir is exactly the [port][dir][theta/phi] output.
// The MBF radiation vectors F_T(u) = sum_s a_s s_hat e^{+jk u . rho_s}
// (projected on theta-hat, phi-hat) are formed first, one thread per
// (direction, MBF).
#include <math.h>

#include <algorithm>

#include "cgemm.hpp"
#include "common.hpp"
#include "prof.hpp"

namespace harp {
namespace {

__global__ void __launch_bounds__(256)
    mbf_pattern_kernel(const char* __restrict__ model, const double* __restrict__ theta,
                       const double* __restrict__ phi, int n_dir, int n_mbf, double2* __restrict__ F) {
    const ModelHeader* h = reinterpret_cast<const ModelHeader*>(model);
    const double* smp = reinterpret_cast<const double*>(model + h->off_samples);
    const int n_samp = h->n_samp;
    const double k = h->k;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_dir * n_mbf) return;
    const int d = e / n_mbf, T = e % n_mbf;
    double st, ct, sp, cp;
    sincos(theta[d], &st, &ct);
    sincos(phi[d], &sp, &cp);
    const double ux = st * cp, uy = st * sp, uz = ct;
    const double eth[3] = {ct * cp, ct * sp, -st};
    const double eph[3] = {-sp, cp, 0.0};
    double fr[2] = {0.0, 0.0}, fi[2] = {0.0, 0.0};
    for (int s = 0; s < n_samp; ++s) {
        const double* q = smp + (size_t(T) * n_samp + s) * kSampleFields;
        double sn, cs;
        sincos(k * (ux * q[0] + uy * q[1] + uz * q[2]), &sn, &cs);
        // a e^{+j phase}
        const double ar = q[6] * cs - q[7] * sn, ai = q[6] * sn + q[7] * cs;
        const double pt = q[3] * eth[0] + q[4] * eth[1] + q[5] * eth[2];
        const double pp = q[3] * eph[0] + q[4] * eph[1] + q[5] * eph[2];
        fr[0] += ar * pt;
        fi[0] += ai * pt;
        fr[1] += ar * pp;
        fi[1] += ai * pp;
    }
    F[size_t(d) * n_mbf * 2 + T * 2 + 0] = double2{fr[0], fi[0]};
    F[size_t(d) * n_mbf * 2 + T * 2 + 1] = double2{fr[1], fi[1]};
}

// A[(2d + c), (i, T)], column-major with leading dimension 2 n_dir
__global__ void __launch_bounds__(256)
    pattern_matrix_kernel(const char* __restrict__ model, const double* __restrict__ theta,
                          const double* __restrict__ phi, int n_dir, const double* __restrict__ x,
                          const double* __restrict__ y, int n_ant, int n_mbf, const double2* __restrict__ F,
                          double2* __restrict__ A) {
    const ModelHeader* h = reinterpret_cast<const ModelHeader*>(model);
    const double k = h->k;
    const double pref = h->omega_mu / (4.0 * kPi);
    const int64_t rows = 2 * int64_t(n_dir);
    const int64_t total = rows * n_ant;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += int64_t(gridDim.x) * blockDim.x) {
        const int64_t i = e / rows;             // antenna
        const int r = int(e % rows);            // 2d + c
        const int d = r >> 1, c = r & 1;
        double st, ct, sp, cp;
        sincos(theta[d], &st, &ct);
        sincos(phi[d], &sp, &cp);
        double sn, cs;
        sincos(k * (st * cp * x[i] + st * sp * y[i]), &sn, &cs);
        for (int T = 0; T < n_mbf; ++T) {
            const double2 f = F[size_t(d) * n_mbf * 2 + T * 2 + c];
            // -j pref f e^{j phase}
            const double fr = f.x * cs - f.y * sn, fi = f.x * sn + f.y * cs;
            A[(i * n_mbf + T) * rows + r] = double2{pref * fi, -pref * fr};
        }
    }
}

size_t patterns_ws_layout(int n_mbf, int n_ant, int n_dir, double2** F, double2** A, char* base) {
    const int64_t fb = align256(int64_t(n_dir) * n_mbf * 2 * 16);
    const int64_t ab = align256(int64_t(2) * n_dir * n_ant * n_mbf * 16);
    if (base) {
        *F = reinterpret_cast<double2*>(base);
        *A = reinterpret_cast<double2*>(base + fb);
    }
    return size_t(fb + ab);
}

}  // namespace
}  // namespace harp

using namespace harp;

extern "C" harp_status embedded_patterns_ws(int32_t n_mbf, int32_t n_ant, int32_t n_dir, size_t* bytes) {
    if (!bytes || n_mbf <= 0 || n_ant <= 0 || n_dir <= 0) return HARP_E_ARG;
    *bytes = patterns_ws_layout(n_mbf, n_ant, n_dir, nullptr, nullptr, nullptr);
    return HARP_OK;
}

extern "C" harp_status embedded_patterns(const void* d_model, int32_t n_mbf, const double* d_x, const double* d_y,
                                         int32_t n_ant, const void* d_X, int64_t ldx, int32_t n_ports,
                                         const double* d_theta, const double* d_phi, int32_t n_dir, void* d_E,
                                         void* d_ws, size_t ws_bytes, hipStream_t stream) {
    if (!d_model || !d_x || !d_y || !d_X || !d_theta || !d_phi || !d_E) return HARP_E_ARG;
    if (n_mbf <= 0 || n_ant <= 0 || n_ports <= 0 || n_dir <= 0) return HARP_E_ARG;
    const int64_t n = int64_t(n_ant) * n_mbf;
    if (ldx < n || 2 * int64_t(n_dir) > INT32_MAX || n > INT32_MAX) return HARP_E_ARG;
    const size_t need = patterns_ws_layout(n_mbf, n_ant, n_dir, nullptr, nullptr, nullptr);
    if (!d_ws || ws_bytes < need) return HARP_E_WORKSPACE;
    double2 *F, *A;
    patterns_ws_layout(n_mbf, n_ant, n_dir, &F, &A, static_cast<char*>(d_ws));
    const char* model = static_cast<const char*>(d_model);
    const int nf = n_dir * n_mbf;
    HARP_PROF_LAUNCH(HARP_K_AUX, stream, 0.0, 0.0,
                     hipLaunchKernelGGL(mbf_pattern_kernel, dim3((nf + 255) / 256), dim3(256), 0, stream, model,
                                        d_theta, d_phi, n_dir, n_mbf, F));
    HARP_LAUNCH_CHECK();
    const int64_t total = 2 * int64_t(n_dir) * n_ant;
    const unsigned blocks = unsigned(std::min<int64_t>((total + 255) / 256, 8192));
    HARP_PROF_LAUNCH(HARP_K_AUX, stream, 0.0, 0.0,
                     hipLaunchKernelGGL(pattern_matrix_kernel, dim3(blocks), dim3(256), 0, stream, model, d_theta,
                                        d_phi, n_dir, d_x, d_y, n_ant, n_mbf, F, A));
    HARP_LAUNCH_CHECK();
    GemmArgs<double> g;
    g.M = 2 * n_dir;
    g.N = n_ports;
    g.K = int(n);
    g.A = reinterpret_cast<const double*>(A);
    g.lda = 2 * int64_t(n_dir);
    g.sA = 0;
    g.B = static_cast<const double*>(d_X);
    g.ldb = ldx;
    g.sB = 0;
    g.C = nullptr;
    g.ldc = 2 * int64_t(n_dir);
    g.sC = 0;
    g.D = static_cast<double*>(d_E);
    g.ldd = 2 * int64_t(n_dir);
    g.sD = 0;
    g.alpha = 1.0;
    g.beta = 0.0;
    g.active = nullptr;
    return cgemm<double>(g, 1, stream);
}
