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

// A[(2d + c), (i, T)], column-major with leading dimension 2 n_dir; with
// HERM its conjugate transpose A^H (n x 2 n_dir, leading dimension n)
template <bool HERM>
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
            if constexpr (HERM)
                A[size_t(r) * n_ant * n_mbf + i * n_mbf + T] = double2{pref * fi, pref * fr};
            else
                A[(i * n_mbf + T) * rows + r] = double2{pref * fi, -pref * fr};
        }
    }
}

// Direct position term of the pattern product: with A = -j pref F e^{j phi_i},
// phi_i = k (u_x x_i + u_y y_i), and K = conj(gE) X^T (2 n_dir x n),
//   dJ/dx_i = Re sum_{(2d+c), T} (jk u_x) A K = k pref Re sum u_x F e^{j phi_i} K
// (and u_y for y).  One workgroup per antenna, fixed-order block reduction.
__global__ void __launch_bounds__(256)
    pattern_position_vjp_kernel(const char* __restrict__ model, const double* __restrict__ theta,
                                const double* __restrict__ phi, int n_dir, const double* __restrict__ x,
                                const double* __restrict__ y, int n_mbf, const double2* __restrict__ F,
                                const double2* __restrict__ K, double* __restrict__ gx, double* __restrict__ gy) {
    const ModelHeader* h = reinterpret_cast<const ModelHeader*>(model);
    const double k = h->k, kp = k * h->omega_mu / (4.0 * kPi);
    const int i = blockIdx.x;
    const int64_t rows = 2 * int64_t(n_dir);
    double sx = 0.0, sy = 0.0;
    for (int d = threadIdx.x; d < n_dir; d += blockDim.x) {
        double st, ct, sp, cp;
        sincos(theta[d], &st, &ct);
        sincos(phi[d], &sp, &cp);
        const double ux = st * cp, uy = st * sp;
        double sn, cs;
        sincos(k * (ux * x[i] + uy * y[i]), &sn, &cs);
        double re = 0.0;
        for (int T = 0; T < n_mbf; ++T) {
            for (int c = 0; c < 2; ++c) {
                const double2 f = F[size_t(d) * n_mbf * 2 + T * 2 + c];
                const double fr = f.x * cs - f.y * sn, fi = f.x * sn + f.y * cs;
                const double2 kk = K[(size_t(i) * n_mbf + T) * rows + 2 * d + c];
                re += fr * kk.x - fi * kk.y;
            }
        }
        sx += kp * ux * re;
        sy += kp * uy * re;
    }
    __shared__ double red[2][256];
    red[0][threadIdx.x] = sx;
    red[1][threadIdx.x] = sy;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (int(threadIdx.x) < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] += red[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        gx[i] += red[0][0];
        gy[i] += red[1][0];
    }
}

struct PatVjpWs {
    double2 *F, *Ah, *gEc, *Xt, *K;
};
size_t patterns_vjp_ws_layout(int n_mbf, int n_ant, int n_dir, int n_ports, PatVjpWs* w, char* base) {
    const int64_t n = int64_t(n_ant) * n_mbf, rows = 2 * int64_t(n_dir);
    const int64_t sz[5] = {align256(int64_t(n_dir) * n_mbf * 2 * 16), align256(n * rows * 16),
                           align256(rows * n_ports * 16), align256(int64_t(n_ports) * n * 16),
                           align256(rows * n * 16)};
    int64_t off = 0;
    double2** dst[5] = {w ? &w->F : nullptr, w ? &w->Ah : nullptr, w ? &w->gEc : nullptr, w ? &w->Xt : nullptr,
                        w ? &w->K : nullptr};
    for (int q = 0; q < 5; ++q) {
        if (base) *dst[q] = reinterpret_cast<double2*>(base + off);
        off += sz[q];
    }
    return size_t(off);
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
                     hipLaunchKernelGGL(pattern_matrix_kernel<false>, dim3(blocks), dim3(256), 0, stream, model, d_theta,
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

extern "C" harp_status embedded_patterns_vjp_ws(int32_t n_mbf, int32_t n_ant, int32_t n_dir, int32_t n_ports,
                                                size_t* bytes) {
    if (!bytes || n_mbf <= 0 || n_ant <= 0 || n_dir <= 0 || n_ports <= 0) return HARP_E_ARG;
    *bytes = patterns_vjp_ws_layout(n_mbf, n_ant, n_dir, n_ports, nullptr, nullptr);
    return HARP_OK;
}

extern "C" harp_status embedded_patterns_vjp(const void* d_model, int32_t n_mbf, const double* d_x, const double* d_y,
                                             int32_t n_ant, const void* d_X, int64_t ldx, int32_t n_ports,
                                             const double* d_theta, const double* d_phi, int32_t n_dir,
                                             const void* d_gE, void* d_gX, int64_t ldgx, double* d_gx, double* d_gy,
                                             void* d_ws, size_t ws_bytes, hipStream_t stream) {
    if (!d_model || !d_x || !d_y || !d_X || !d_theta || !d_phi || !d_gE || !d_gX || !d_gx || !d_gy)
        return HARP_E_ARG;
    if (n_mbf <= 0 || n_ant <= 0 || n_ports <= 0 || n_dir <= 0) return HARP_E_ARG;
    const int64_t n = int64_t(n_ant) * n_mbf, rows = 2 * int64_t(n_dir);
    if (ldx < n || ldgx < n || rows > INT32_MAX || n > INT32_MAX) return HARP_E_ARG;
    const size_t need = patterns_vjp_ws_layout(n_mbf, n_ant, n_dir, n_ports, nullptr, nullptr);
    if (!d_ws || ws_bytes < need) return HARP_E_WORKSPACE;
    PatVjpWs w;
    patterns_vjp_ws_layout(n_mbf, n_ant, n_dir, n_ports, &w, static_cast<char*>(d_ws));
    const char* model = static_cast<const char*>(d_model);
    const int nf = n_dir * n_mbf;
    HARP_PROF_LAUNCH(HARP_K_AUX, stream, 0.0, 0.0,
                     hipLaunchKernelGGL(mbf_pattern_kernel, dim3((nf + 255) / 256), dim3(256), 0, stream, model,
                                        d_theta, d_phi, n_dir, n_mbf, w.F));
    HARP_LAUNCH_CHECK();
    const int64_t total = rows * n_ant;
    const unsigned blocks = unsigned(std::min<int64_t>((total + 255) / 256, 8192));
    HARP_PROF_LAUNCH(HARP_K_AUX, stream, 0.0, 0.0,
                     hipLaunchKernelGGL(pattern_matrix_kernel<true>, dim3(blocks), dim3(256), 0, stream, model,
                                        d_theta, d_phi, n_dir, d_x, d_y, n_ant, n_mbf, w.F, w.Ah));
    HARP_LAUNCH_CHECK();
    harp_status s;
    // gX += A^H gE
    GemmArgs<double> g{};
    g.M = int(n);
    g.N = n_ports;
    g.K = int(rows);
    g.A = reinterpret_cast<const double*>(w.Ah);
    g.lda = n;
    g.B = static_cast<const double*>(d_gE);
    g.ldb = rows;
    g.C = static_cast<const double*>(d_gX);
    g.ldc = ldgx;
    g.D = static_cast<double*>(d_gX);
    g.ldd = ldgx;
    g.alpha = 1.0;
    g.beta = 1.0;
    g.active = nullptr;
    if ((s = cgemm<double>(g, 1, stream)) != HARP_OK) return s;
    // K = conj(gE) X^T
    if ((s = harp_cmatrix_copy(int(rows), n_ports, 1, d_gE, rows, 0, w.gEc, rows, 0, 0, 1, stream)) != HARP_OK)
        return s;
    if ((s = harp_cmatrix_copy(int(n), n_ports, 1, d_X, ldx, 0, w.Xt, n_ports, 0, 1, 0, stream)) != HARP_OK) return s;
    GemmArgs<double> k{};
    k.M = int(rows);
    k.N = int(n);
    k.K = n_ports;
    k.A = reinterpret_cast<const double*>(w.gEc);
    k.lda = rows;
    k.B = reinterpret_cast<const double*>(w.Xt);
    k.ldb = n_ports;
    k.C = nullptr;
    k.ldc = rows;
    k.D = reinterpret_cast<double*>(w.K);
    k.ldd = rows;
    k.alpha = 1.0;
    k.beta = 0.0;
    k.active = nullptr;
    if ((s = cgemm<double>(k, 1, stream)) != HARP_OK) return s;
    HARP_PROF_LAUNCH(HARP_K_AUX, stream, 0.0, 0.0,
                     hipLaunchKernelGGL(pattern_position_vjp_kernel, dim3(unsigned(n_ant)), dim3(256), 0, stream,
                                        model, d_theta, d_phi, n_dir, d_x, d_y, n_mbf, w.F, w.K, d_gx, d_gy));
    HARP_LAUNCH_CHECK();
    return HARP_OK;
}
